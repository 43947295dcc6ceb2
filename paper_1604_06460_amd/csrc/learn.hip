// Learned cost model and plan selection for batches.
//
// The model is a 24 -> 64 -> 64 -> 4 perceptron with ReLU activations,
// FP32, y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 (row-major, x @ W). Its
// four outputs predict the log device time of a segment under each plan
// option (fuse at k = 2, 4, 6; emulate). Training minimises the masked mean
// squared error sum(mask (y - t)^2) / sum(mask) with Adam; the forward pass,
// the layer-wise backward pass and the Adam update are the kernels below.
//
// Plan selection picks, per segment, the option with the smallest predicted
// time among the valid ones. The fallback policies are the plain rules: a
// fixed fusion width with every subroutine emulated, or the paper's cost
// models (Eq. 1 for the FFT against Eq. 2 for the gate-level QFT on one
// device; arithmetic is always emulated, Sec. III-A and IV-B) with a
// roofline estimate of the fused sweeps.
#include "qs_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

namespace {

using namespace qs;

constexpr int kIn = QS_N_FEATURES, kH = 64, kOut = 4;
constexpr int kW1 = 0, kB1 = kW1 + kIn * kH, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH,
              kB3 = kW3 + kH * kOut, kParams = kB3 + kOut;
static_assert(kParams == QS_MLP_PARAMS, "parameter count");
constexpr int kT = 256;

// forward for a batch of rows: one thread per row; parameters staged in LDS
__global__ __launch_bounds__(kT) void k_mlp_forward(int n, const float *__restrict__ x,
                                                    const int *__restrict__ rows,
                                                    const float *__restrict__ p,
                                                    const float *__restrict__ mean,
                                                    const float *__restrict__ istd,
                                                    float *__restrict__ xs, float *__restrict__ a1,
                                                    float *__restrict__ a2, float *__restrict__ y)
{
    __shared__ float P[kParams];
    for (int i = threadIdx.x; i < kParams; i += kT) P[i] = p[i];
    __syncthreads();
    const int s = blockIdx.x * kT + threadIdx.x;
    if (s >= n) return;
    const int r = rows ? rows[s] : s;
    float xi[kIn], h1[kH];
#pragma unroll
    for (int i = 0; i < kIn; ++i) {
        xi[i] = (x[size_t(r) * kIn + i] - mean[i]) * istd[i];
        xs[size_t(s) * kIn + i] = xi[i];
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = P[kB1 + j];
#pragma unroll
        for (int i = 0; i < kIn; ++i) acc = fmaf(xi[i], P[kW1 + i * kH + j], acc);
        a1[size_t(s) * kH + j] = acc;
        h1[j] = fmaxf(acc, 0.f);
    }
    float h2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = P[kB2 + j];
#pragma unroll
        for (int i = 0; i < kH; ++i) acc = fmaf(h1[i], P[kW2 + i * kH + j], acc);
        a2[size_t(s) * kH + j] = acc;
        h2[j] = fmaxf(acc, 0.f);
    }
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
        float acc = P[kB3 + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) acc = fmaf(h2[i], P[kW3 + i * kOut + o], acc);
        y[size_t(s) * kOut + o] = acc;
    }
}

// dy = 2 mask (y - t) / sum(mask); per-block partial loss sums
__global__ __launch_bounds__(kT) void k_mlp_dy(int n, const int *__restrict__ rows,
                                               const float *__restrict__ y, const float *__restrict__ t,
                                               const float *__restrict__ mask, float inv_msum,
                                               float *__restrict__ dy, float *__restrict__ loss_part)
{
    __shared__ float red[kT];
    const int s = blockIdx.x * kT + threadIdx.x;
    float l = 0.f;
    if (s < n) {
        const int r = rows ? rows[s] : s;
        for (int o = 0; o < kOut; ++o) {
            const float mk = mask[size_t(r) * kOut + o];
            const float d = y[size_t(s) * kOut + o] - t[size_t(r) * kOut + o];
            dy[size_t(s) * kOut + o] = 2.f * mk * d * inv_msum;
            l += mk * d * d;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0] * inv_msum;
}

// da2 = (dy W3^T) . [a2 > 0];  da1 = (da2 W2^T) . [a1 > 0]
__global__ __launch_bounds__(kT) void k_mlp_back(int n, const float *__restrict__ p,
                                                 const float *__restrict__ dy, const float *__restrict__ a1,
                                                 const float *__restrict__ a2, float *__restrict__ da1,
                                                 float *__restrict__ da2)
{
    __shared__ float P[kParams];
    for (int i = threadIdx.x; i < kParams; i += kT) P[i] = p[i];
    __syncthreads();
    const int s = blockIdx.x * kT + threadIdx.x;
    if (s >= n) return;
    float g2[kH];
    for (int j = 0; j < kH; ++j) {
        float acc = 0.f;
        for (int o = 0; o < kOut; ++o) acc = fmaf(dy[size_t(s) * kOut + o], P[kW3 + j * kOut + o], acc);
        g2[j] = a2[size_t(s) * kH + j] > 0.f ? acc : 0.f;
        da2[size_t(s) * kH + j] = g2[j];
    }
    for (int i = 0; i < kH; ++i) {
        float acc = 0.f;
        for (int j = 0; j < kH; ++j) acc = fmaf(g2[j], P[kW2 + i * kH + j], acc);
        da1[size_t(s) * kH + i] = a1[size_t(s) * kH + i] > 0.f ? acc : 0.f;
    }
}

// parameter gradients: one thread per parameter, sum over the rows
__global__ __launch_bounds__(kT) void k_mlp_wgrad(int n, const float *__restrict__ xs,
                                                  const float *__restrict__ a1, const float *__restrict__ a2,
                                                  const float *__restrict__ dy, const float *__restrict__ da1,
                                                  const float *__restrict__ da2, float *__restrict__ g)
{
    const int q = blockIdx.x * kT + threadIdx.x;
    if (q >= kParams) return;
    float acc = 0.f;
    if (q < kB1) {                       // W1[i][j] = sum xs[i] da1[j]
        const int i = q / kH, j = q % kH;
        for (int s = 0; s < n; ++s) acc = fmaf(xs[size_t(s) * kIn + i], da1[size_t(s) * kH + j], acc);
    } else if (q < kW2) {                // b1[j]
        const int j = q - kB1;
        for (int s = 0; s < n; ++s) acc += da1[size_t(s) * kH + j];
    } else if (q < kB2) {                // W2[i][j] = sum relu(a1[i]) da2[j]
        const int i = (q - kW2) / kH, j = (q - kW2) % kH;
        for (int s = 0; s < n; ++s) acc = fmaf(fmaxf(a1[size_t(s) * kH + i], 0.f), da2[size_t(s) * kH + j], acc);
    } else if (q < kW3) {                // b2[j]
        const int j = q - kB2;
        for (int s = 0; s < n; ++s) acc += da2[size_t(s) * kH + j];
    } else if (q < kB3) {                // W3[i][o] = sum relu(a2[i]) dy[o]
        const int i = (q - kW3) / kOut, o = (q - kW3) % kOut;
        for (int s = 0; s < n; ++s) acc = fmaf(fmaxf(a2[size_t(s) * kH + i], 0.f), dy[size_t(s) * kOut + o], acc);
    } else {                             // b3[o]
        const int o = q - kB3;
        for (int s = 0; s < n; ++s) acc += dy[size_t(s) * kOut + o];
    }
    g[q] = acc;
}

// Adam (Kingma and Ba), bias-corrected, step t >= 1
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * kT + threadIdx.x;
    if (q >= kParams) return;
    const float gg = g[q];
    const float mm = b1 * m[q] + (1.f - b1) * gg;
    const float vv = b2 * v[q] + (1.f - b2) * gg * gg;
    m[q] = mm;
    v[q] = vv;
    p[q] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace

struct qs_mlp_t {
    hipStream_t stream = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *mean = nullptr, *istd = nullptr;
    int adam_t = 0;
    // raw feature range of the training rows (host); unset: no range check
    bool have_range = false;
    float lo[QS_N_FEATURES] = {0}, hi[QS_N_FEATURES] = {0};
    // segments of the last learned choice: [learned, out of range,
    // non-finite prediction, gain below the margin]
    int choose_counts[4] = {0, 0, 0, 0};
    // work buffers sized for `cap` rows
    int cap = 0;
    float *x = nullptr, *t = nullptr, *mask = nullptr, *xs = nullptr, *a1 = nullptr, *a2 = nullptr,
          *y = nullptr, *dy = nullptr, *da1 = nullptr, *da2 = nullptr, *lp = nullptr;
    int *rows = nullptr;
};

namespace {

void free_work(qs_mlp_t *m)
{
    float **bufs[] = {&m->x, &m->t, &m->mask, &m->xs, &m->a1, &m->a2, &m->y, &m->dy, &m->da1, &m->da2, &m->lp};
    for (float **b : bufs)
        if (*b) {
            (void)hipFree(*b);
            *b = nullptr;
        }
    if (m->rows) (void)hipFree(m->rows);
    m->rows = nullptr;
    m->cap = 0;
}

int ensure_work(qs_mlp_t *m, int n)
{
    if (n <= m->cap) return QS_OK;
    QS_HIP(hipStreamSynchronize(m->stream));
    free_work(m);
    const size_t N = size_t(std::max(n, 256));
    struct {
        float **p;
        size_t cols;
    } plan[] = {{&m->x, kIn}, {&m->t, kOut}, {&m->mask, kOut}, {&m->xs, kIn}, {&m->a1, kH}, {&m->a2, kH},
                {&m->y, kOut}, {&m->dy, kOut}, {&m->da1, kH}, {&m->da2, kH}, {&m->lp, 1}};
    for (auto &e : plan) QS_HIP(hipMalloc(reinterpret_cast<void **>(e.p), sizeof(float) * N * e.cols));
    QS_HIP(hipMalloc(reinterpret_cast<void **>(&m->rows), sizeof(int) * N));
    m->cap = int(N);
    return QS_OK;
}

unsigned blocks(int n) { return unsigned(std::max(1, (n + kT - 1) / kT)); }

// forward + backward on rows[0..n) of the uploaded (x, t, mask); returns the loss
int grad_pass(qs_mlp_t *m, int n, const int *d_rows, float msum, float *loss)
{
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(n)), dim3(kT), 0, m->stream, n, m->x, d_rows, m->p, m->mean,
                       m->istd, m->xs, m->a1, m->a2, m->y);
    hipLaunchKernelGGL(k_mlp_dy, dim3(blocks(n)), dim3(kT), 0, m->stream, n, d_rows, m->y, m->t, m->mask,
                       1.f / msum, m->dy, m->lp);
    hipLaunchKernelGGL(k_mlp_back, dim3(blocks(n)), dim3(kT), 0, m->stream, n, m->p, m->dy, m->a1, m->a2,
                       m->da1, m->da2);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks(kParams)), dim3(kT), 0, m->stream, n, m->xs, m->a1, m->a2,
                       m->dy, m->da1, m->da2, m->g);
    QS_HIP(hipGetLastError());
    if (loss) {
        std::vector<float> lp(blocks(n));
        QS_HIP(hipMemcpyAsync(lp.data(), m->lp, sizeof(float) * lp.size(), hipMemcpyDeviceToHost, m->stream));
        QS_HIP(hipStreamSynchronize(m->stream));
        double s = 0.0;
        for (float f : lp) s += f;
        *loss = float(s);
    }
    return QS_OK;
}

int upload_data(qs_mlp_t *m, int n, const float *x, const float *t, const float *mask)
{
    if (int rc = ensure_work(m, n)) return rc;
    QS_HIP(hipMemcpyAsync(m->x, x, sizeof(float) * size_t(n) * kIn, hipMemcpyHostToDevice, m->stream));
    if (t) QS_HIP(hipMemcpyAsync(m->t, t, sizeof(float) * size_t(n) * kOut, hipMemcpyHostToDevice, m->stream));
    if (mask) QS_HIP(hipMemcpyAsync(m->mask, mask, sizeof(float) * size_t(n) * kOut, hipMemcpyHostToDevice, m->stream));
    return QS_OK;
}

}  // namespace

extern "C" {

int qs_mlp_create(const float *params, uint64_t seed, void *hip_stream, qs_mlp *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "NULL output model");
    *out = nullptr;
    qs_mlp_t *m = new (std::nothrow) qs_mlp_t();
    if (!m) return fail(QS_ENOMEM, "host allocation failed");
    m->stream = static_cast<hipStream_t>(hip_stream);
    std::vector<float> init(kParams, 0.f);
    if (params) {
        std::copy(params, params + kParams, init.begin());
    } else {
        // He initialisation for the weights, zero biases
        std::mt19937_64 rng(seed);
        std::normal_distribution<float> nd(0.f, 1.f);
        for (int i = 0; i < kIn * kH; ++i) init[size_t(kW1 + i)] = nd(rng) * std::sqrt(2.f / kIn);
        for (int i = 0; i < kH * kH; ++i) init[size_t(kW2 + i)] = nd(rng) * std::sqrt(2.f / kH);
        for (int i = 0; i < kH * kOut; ++i) init[size_t(kW3 + i)] = nd(rng) * std::sqrt(2.f / kH);
    }
    std::vector<float> zeros(kParams, 0.f), ones(kIn, 1.f);
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void **>(&m->p), sizeof(float) * kParams)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&m->g), sizeof(float) * kParams)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&m->m), sizeof(float) * kParams)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&m->v), sizeof(float) * kParams)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&m->mean), sizeof(float) * kIn)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&m->istd), sizeof(float) * kIn)) != hipSuccess) {
        int rc = hip_fail(e, "hipMalloc(model)");
        qs_mlp_free(m);
        return rc;
    }
    if ((e = hipMemcpy(m->p, init.data(), sizeof(float) * kParams, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(m->m, zeros.data(), sizeof(float) * kParams, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(m->v, zeros.data(), sizeof(float) * kParams, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(m->mean, zeros.data(), sizeof(float) * kIn, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(m->istd, ones.data(), sizeof(float) * kIn, hipMemcpyHostToDevice)) != hipSuccess) {
        int rc = hip_fail(e, "hipMemcpy(model)");
        qs_mlp_free(m);
        return rc;
    }
    *out = m;
    return QS_OK;
}

int qs_mlp_get_params(qs_mlp m, float *params)
{
    clear_error();
    if (!m || !params) return fail(QS_EINVAL, "NULL argument");
    QS_HIP(hipStreamSynchronize(m->stream));
    QS_HIP(hipMemcpy(params, m->p, sizeof(float) * kParams, hipMemcpyDeviceToHost));
    return QS_OK;
}

int qs_mlp_set_norm(qs_mlp m, const float *mean, const float *inv_std)
{
    clear_error();
    if (!m || !mean || !inv_std) return fail(QS_EINVAL, "NULL argument");
    for (int i = 0; i < kIn; ++i)
        if (!std::isfinite(mean[i]) || !std::isfinite(inv_std[i])) return fail(QS_EINVAL, "non-finite normalisation");
    QS_HIP(hipMemcpyAsync(m->mean, mean, sizeof(float) * kIn, hipMemcpyHostToDevice, m->stream));
    QS_HIP(hipMemcpyAsync(m->istd, inv_std, sizeof(float) * kIn, hipMemcpyHostToDevice, m->stream));
    QS_HIP(hipStreamSynchronize(m->stream));
    return QS_OK;
}

int qs_mlp_forward(qs_mlp m, int n, const float *x, float *y)
{
    clear_error();
    if (!m || !x || !y || n < 0) return fail(QS_EINVAL, "bad argument");
    if (n == 0) return QS_OK;
    if (int rc = upload_data(m, n, x, nullptr, nullptr)) return rc;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(n)), dim3(kT), 0, m->stream, n, m->x, nullptr, m->p, m->mean,
                       m->istd, m->xs, m->a1, m->a2, m->y);
    QS_HIP(hipGetLastError());
    QS_HIP(hipMemcpyAsync(y, m->y, sizeof(float) * size_t(n) * kOut, hipMemcpyDeviceToHost, m->stream));
    QS_HIP(hipStreamSynchronize(m->stream));
    return QS_OK;
}

int qs_mlp_loss_grad(qs_mlp m, int n, const float *x, const float *t, const float *mask, float *loss, float *grad)
{
    clear_error();
    if (!m || !x || !t || !mask || n < 1) return fail(QS_EINVAL, "bad argument");
    double msum = 0.0;
    for (size_t i = 0; i < size_t(n) * kOut; ++i) msum += mask[i];
    if (msum <= 0.0) return fail(QS_EINVAL, "mask selects nothing");
    if (int rc = upload_data(m, n, x, t, mask)) return rc;
    float l = 0.f;
    if (int rc = grad_pass(m, n, nullptr, float(msum), &l)) return rc;
    if (loss) *loss = l;
    if (grad) {
        QS_HIP(hipMemcpyAsync(grad, m->g, sizeof(float) * kParams, hipMemcpyDeviceToHost, m->stream));
        QS_HIP(hipStreamSynchronize(m->stream));
    }
    return QS_OK;
}

int qs_mlp_adam_step(qs_mlp m, float lr)
{
    clear_error();
    if (!m) return fail(QS_EINVAL, "NULL model");
    ++m->adam_t;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, float(m->adam_t)), c2 = 1.f - std::pow(b2, float(m->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(kParams)), dim3(kT), 0, m->stream, m->p, m->g, m->m, m->v, lr, b1, b2,
                       1e-8f, c1, c2);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

int qs_mlp_train(qs_mlp m, int n, const float *x, const float *t, const float *mask, int epochs, int batch,
                 float lr, uint64_t seed, float *final_loss)
{
    clear_error();
    if (!m || !x || !t || !mask || n < 1 || epochs < 0 || batch < 1 || !(lr > 0.f))
        return fail(QS_EINVAL, "bad argument");
    if (int rc = upload_data(m, n, x, t, mask)) return rc;
    std::vector<int> perm(static_cast<size_t>(n));
    std::iota(perm.begin(), perm.end(), 0);
    std::mt19937_64 rng(seed);
    for (int ep = 0; ep < epochs; ++ep) {
        std::shuffle(perm.begin(), perm.end(), rng);
        QS_HIP(hipMemcpyAsync(m->rows, perm.data(), sizeof(int) * size_t(n), hipMemcpyHostToDevice, m->stream));
        QS_HIP(hipStreamSynchronize(m->stream));
        for (int s0 = 0; s0 < n; s0 += batch) {
            const int nb = std::min(batch, n - s0);
            double msum = 0.0;
            for (int s = s0; s < s0 + nb; ++s)
                for (int o = 0; o < kOut; ++o) msum += mask[size_t(perm[size_t(s)]) * kOut + o];
            if (msum <= 0.0) continue;
            if (int rc = grad_pass(m, nb, m->rows + s0, float(msum), nullptr)) return rc;
            if (int rc = qs_mlp_adam_step(m, lr)) return rc;
        }
    }
    if (final_loss) {
        double msum = 0.0;
        for (size_t i = 0; i < size_t(n) * kOut; ++i) msum += mask[i];
        if (int rc = grad_pass(m, n, nullptr, float(std::max(msum, 1.0)), final_loss)) return rc;
    }
    QS_HIP(hipStreamSynchronize(m->stream));
    return QS_OK;
}

int qs_mlp_set_range(qs_mlp m, const float *lo, const float *hi)
{
    clear_error();
    if (!m) return fail(QS_EINVAL, "NULL model");
    if (!lo && !hi) {
        m->have_range = false;
        return QS_OK;
    }
    if (!lo || !hi) return fail(QS_EINVAL, "NULL range bound");
    for (int i = 0; i < kIn; ++i)
        if (!std::isfinite(lo[i]) || !std::isfinite(hi[i]) || lo[i] > hi[i])
            return fail(QS_EINVAL, "feature %d: bad range [%g, %g]", i, double(lo[i]), double(hi[i]));
    std::copy(lo, lo + kIn, m->lo);
    std::copy(hi, hi + kIn, m->hi);
    m->have_range = true;
    return QS_OK;
}

int qs_mlp_choose_stats(qs_mlp m, int *counts)
{
    clear_error();
    if (!m || !counts) return fail(QS_EINVAL, "NULL argument");
    std::copy(m->choose_counts, m->choose_counts + 4, counts);
    return QS_OK;
}

int qs_mlp_free(qs_mlp m)
{
    clear_error();
    if (!m) return QS_OK;
    (void)hipStreamSynchronize(m->stream);
    free_work(m);
    float *bufs[] = {m->p, m->g, m->m, m->v, m->mean, m->istd};
    for (float *b : bufs)
        if (b) (void)hipFree(b);
    delete m;
    return QS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Plan selection
// ---------------------------------------------------------------------------
namespace {

// One-device constants of the plain cost models.
constexpr double kBmem = 8.0e12;        // HBM bytes/s
constexpr double kF32 = 78.6e12;        // FP32 vector flop/s (no packed FP32)
constexpr double kF32Peak = 157.3e12;   // FP32 peak flop/s (Eq. 1's FLOPS_peak)
constexpr double kEffFft = 0.15;        // FFT efficiency in Eq. 1 (10-20% per Sec. III-B)

double blocks_from_feature(float f) { return std::max(1.0, std::expm1(double(f))); }

// Eq. (2)-style roofline estimate of a fused sweep sequence.
double fused_cost(double blocks, int k, int n)
{
    const double N = std::ldexp(1.0, n);
    return blocks * (2.0 * 8.0 * N / kBmem + 8.0 * std::ldexp(1.0, k) * N / kF32);
}

// The paper's rules for one segment (QS_POLICY_HEURISTIC): arithmetic is
// always emulated (Sec. III-A, IV-B); a QFT is emulated when Eq. (1) with one
// device and no exchange does not exceed Eq. (2); a gate list takes the
// fusion width with the lowest roofline estimate.
int heuristic_option(int kind, int n, const float *fs)
{
    if (kind == QS_SEG_MODMUL) return QS_PLAN_EMULATE;
    if (kind == QS_SEG_QFT) {
        const double N = std::ldexp(1.0, n), m = double(fs[14]);
        const double t_fft = 5.0 * N * m / (kEffFft * kF32Peak);
        const double t_qft = 4.0 * N * m * m / kBmem;
        if (t_fft <= t_qft) return QS_PLAN_EMULATE;
    }
    int best = 0;
    double bc = 0.0;
    for (int o = 0; o < 3; ++o) {
        const double c = fused_cost(blocks_from_feature(fs[17 + o]), 2 + 2 * o, n);
        if (o == 0 || c < bc) {
            bc = c;
            best = o;
        }
    }
    return best;
}

// A learned choice departs from the heuristic only when the model predicts
// it at least this much faster (natural-log time, ~5%).
constexpr float kLearnedMargin = 0.05f;
// Features may lie this fraction of the training range outside it.
constexpr float kRangeSlack = 0.05f;

}  // namespace

extern "C" int qs_batch_choose(qs_batch b, int policy, qs_mlp model, int *options)
{
    clear_error();
    if (!b || !options) return fail(QS_EINVAL, "NULL argument");
    if (policy < QS_POLICY_HEURISTIC || policy > QS_POLICY_FIXED_K6) return fail(QS_EINVAL, "unknown policy %d", policy);
    if (policy == QS_POLICY_LEARNED && !model) return fail(QS_EINVAL, "learned policy needs a model");
    int ns = 0;
    if (int rc = qs_batch_info(b, &ns, nullptr)) return rc;
    const size_t nss = static_cast<size_t>(ns);
    std::vector<int> kind(nss), circ(nss), nq(nss);
    if (int rc = qs_batch_segment_info(b, kind.data(), circ.data(), nq.data())) return rc;
    std::vector<float> f(size_t(ns) * QS_N_FEATURES);
    if (int rc = qs_batch_features(b, f.data())) return rc;
    if (policy == QS_POLICY_FIXED_K2 || policy == QS_POLICY_FIXED_K4 || policy == QS_POLICY_FIXED_K6) {
        for (int s = 0; s < ns; ++s)
            options[s] = kind[size_t(s)] == QS_SEG_GATES ? policy - QS_POLICY_FIXED_K2 : QS_PLAN_EMULATE;
        return QS_OK;
    }
    for (int s = 0; s < ns; ++s)
        options[s] = heuristic_option(kind[size_t(s)], nq[size_t(s)], f.data() + size_t(s) * QS_N_FEATURES);
    if (policy == QS_POLICY_HEURISTIC) return QS_OK;
    // learned: the predicted fastest option, with the heuristic as fallback
    // for segments the model has not seen the like of (features outside the
    // training range), cannot rate (non-finite outputs) or rates as no
    // clear gain over the heuristic's own option
    std::vector<float> y(size_t(ns) * 4);
    if (int rc = qs_mlp_forward(model, ns, f.data(), y.data())) return rc;
    int cnt[4] = {0, 0, 0, 0};
    for (int s = 0; s < ns; ++s) {
        const float *fs = f.data() + size_t(s) * QS_N_FEATURES;
        const float *ys = y.data() + size_t(s) * 4;
        const int nopt = kind[size_t(s)] == QS_SEG_GATES ? 3 : 4;
        bool finite = true;
        for (int o = 0; o < nopt; ++o) finite = finite && std::isfinite(ys[o]);
        if (!finite) {
            ++cnt[2];
            continue;
        }
        bool inside = true;
        if (model->have_range)
            for (int i = 0; i < QS_N_FEATURES && inside; ++i) {
                const float slack = kRangeSlack * (model->hi[i] - model->lo[i]);
                inside = fs[i] >= model->lo[i] - slack && fs[i] <= model->hi[i] + slack;
            }
        if (!inside) {
            ++cnt[1];
            continue;
        }
        int best = 0;
        for (int o = 1; o < nopt; ++o)
            if (ys[o] < ys[best]) best = o;
        const int heur = options[s];
        if (best != heur && ys[heur] - ys[best] < kLearnedMargin) {
            ++cnt[3];
            continue;
        }
        options[s] = best;
        ++cnt[0];
    }
    std::copy(cnt, cnt + 4, model->choose_counts);
    return QS_OK;
}
