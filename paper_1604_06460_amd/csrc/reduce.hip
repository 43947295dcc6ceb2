// Measurement quantities read directly off the state (Sec. III-D): the
// whole distribution or an expectation value in one pass, no sampling of
// repeated runs. Probabilities are |alpha_i|^2 (Sec. II). All accumulation
// is FP64, also for FP32 states. Partial sums are combined in a fixed order
// so repeated calls give identical results.
#include "qs_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace qs {
namespace {

constexpr int kThreads = 256;
constexpr int kReduceBlocks = 2048;

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / 64; ++w) t += sh[w];
    __syncthreads();
    return t;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_norm2(const typename V2<R>::T *__restrict__ psi,
                                                    uint64_t dim, double *__restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    double s = 0.0;
    for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < dim;
         i += uint64_t(gridDim.x) * kThreads) {
        const double x = double(psi[i].x), y = double(psi[i].y);
        s = fma(x, x, fma(y, y, s));
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// <psi|P|psi> for a Pauli string: P|i> = c_i |i ^ f>, f = x|y,
// c_i = i^{|y|} (-1)^{popcount(i & (y|z))}. For f != 0 the pair (i, i^f) is
// visited once through its member with the top bit of f clear, and both
// terms conj(psi_{i^f}) c_i psi_i and conj(psi_i) c_{i^f} psi_{i^f} are
// added; the common factor i^{|y|} is applied on the host.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_pauli(const typename V2<R>::T *__restrict__ psi,
                                                    uint64_t n_items, uint64_t f, int hbit,
                                                    uint64_t sgn_mask, double *__restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    double sre = 0.0, sim = 0.0;
    for (uint64_t g = uint64_t(blockIdx.x) * kThreads + threadIdx.x; g < n_items;
         g += uint64_t(gridDim.x) * kThreads) {
        if (f == 0) {
            const double x = double(psi[g].x), y = double(psi[g].y);
            const double p = fma(x, x, y * y);
            sre += (__popcll(g & sgn_mask) & 1) ? -p : p;
            continue;
        }
        const uint64_t i = ((g >> hbit) << (hbit + 1)) | (g & ((1ull << hbit) - 1));
        const uint64_t j = i ^ f;
        const double ar = double(psi[i].x), ai = double(psi[i].y);
        const double br = double(psi[j].x), bi = double(psi[j].y);
        const double si = (__popcll(i & sgn_mask) & 1) ? -1.0 : 1.0;
        const double sj = (__popcll(j & sgn_mask) & 1) ? -1.0 : 1.0;
        // conj(b) * a * si + conj(a) * b * sj
        const double cr = br * ar + bi * ai;  // Re(conj(b) a) = Re(conj(a) b)
        const double ci = br * ai - bi * ar;  // Im(conj(b) a) = -Im(conj(a) b)
        sre += (si + sj) * cr;
        sim += (si - sj) * ci;
    }
    sre = block_sum(sre, sh);
    sim = block_sum(sim, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sre;
        partial[2 * blockIdx.x + 1] = sim;
    }
}

// Fixed-order final sum of `count` interleaved tuples of width w.
__global__ void k_finish(const double *__restrict__ partial, int count, int w,
                         double *__restrict__ out)
{
    __shared__ double sh[kThreads / 64];
    for (int c = 0; c < w; ++c) {
        double s = 0.0;
        for (int i = threadIdx.x; i < count; i += kThreads) s += partial[size_t(i) * w + c];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) out[c] = s;
    }
}

struct QArgs {
    int m;
    int q[20];
};

__device__ __forceinline__ uint32_t outcome_of(uint64_t i, const QArgs &qa)
{
    uint32_t o = 0;
    for (int r = 0; r < qa.m; ++r) o |= uint32_t((i >> qa.q[r]) & 1) << r;
    return o;
}

// Marginals, small m: per-workgroup histogram in LDS, one row of partials
// per workgroup. Workgroup b sweeps one contiguous chunk of the state, 256
// consecutive amplitudes per step, so a thread's outcome changes only when
// a measured qubit at bit 8 or above flips: the thread accumulates in a
// register and adds to the LDS bin only when its outcome changes. When
// every measured qubit is 6 or above (wave_uniform) all 64 lanes of a wave
// share the outcome, and the wave sums its lanes before one atomic.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_hist_lds(const typename V2<R>::T *__restrict__ psi,
                                                       uint64_t dim, QArgs qa, int wave_uniform,
                                                       double *__restrict__ partial)
{
    extern __shared__ double hist[];
    const int M = 1 << qa.m;
    for (int o = threadIdx.x; o < M; o += kThreads) hist[o] = 0.0;
    __syncthreads();
    const uint64_t chunk = (dim + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = uint64_t(blockIdx.x) * chunk;
    const uint64_t hi = lo + chunk < dim ? lo + chunk : dim;
    uint32_t cur = 0;
    double acc = 0.0;
    bool any = false;
    auto flush = [&]() {
        if (wave_uniform) {
            const double s = wave_sum(acc);
            if ((threadIdx.x & 63) == 0) atomicAdd(&hist[cur], s);
        } else {
            atomicAdd(&hist[cur], acc);
        }
    };
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
        const double x = double(psi[i].x), y = double(psi[i].y);
        const uint32_t o = outcome_of(i, qa);
        if (any && o != cur) {       // wave-uniform when wave_uniform is set
            flush();
            acc = 0.0;
        }
        cur = o;
        any = true;
        acc = fma(x, x, fma(y, y, acc));
    }
    if (any) flush();
    __syncthreads();
    for (int o = threadIdx.x; o < M; o += kThreads) partial[size_t(blockIdx.x) * M + o] = hist[o];
}

__global__ void k_hist_cols(const double *__restrict__ partial, int rows, int M,
                            double *__restrict__ p)
{
    for (int o = blockIdx.x * kThreads + threadIdx.x; o < M; o += gridDim.x * kThreads) {
        double s = 0.0;
        for (int r = 0; r < rows; ++r) s += partial[size_t(r) * M + o];
        p[o] = s;
    }
}

// Marginals, larger m: one thread per outcome sums its 2^(n-m) members.
struct RestArgs {
    int nr;
    int pos[64];  // ascending positions of the measured qubits (inserted zeros)
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_hist_gather(const typename V2<R>::T *__restrict__ psi,
                                                          uint64_t rest_count, QArgs qa,
                                                          RestArgs ra, double *__restrict__ p)
{
    const uint32_t M = 1u << qa.m;
    for (uint32_t o = blockIdx.x * kThreads + threadIdx.x; o < M; o += gridDim.x * kThreads) {
        uint64_t head = 0;
        for (int r = 0; r < qa.m; ++r) head |= uint64_t((o >> r) & 1) << qa.q[r];
        double s = 0.0;
        for (uint64_t rr = 0; rr < rest_count; ++rr) {
            uint64_t i = rr;
            for (int t = 0; t < ra.nr; ++t) {
                const int pp = ra.pos[t];
                i = ((i >> pp) << (pp + 1)) | (i & ((1ull << pp) - 1));
            }
            i |= head;
            const double x = double(psi[i].x), y = double(psi[i].y);
            s = fma(x, x, fma(y, y, s));
        }
        p[o] = s;
    }
}

// Inclusive prefix sum of p (single workgroup, fixed order): each thread
// scans a contiguous chunk, chunk totals are scanned serially.
__global__ __launch_bounds__(kThreads) void k_cdf(const double *__restrict__ p, int M,
                                                  double *__restrict__ cdf)
{
    __shared__ double tot[kThreads];
    const int chunk = (M + kThreads - 1) / kThreads;
    const int lo = threadIdx.x * chunk, hi = min(M, lo + chunk);
    double s = 0.0;
    for (int o = lo; o < hi; ++o) s += p[o];
    tot[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < kThreads; ++t) {
            const double v = tot[t];
            tot[t] = run;
            run += v;
        }
    }
    __syncthreads();
    double run = tot[threadIdx.x];
    for (int o = lo; o < hi; ++o) {
        run += p[o];
        cdf[o] = run;
    }
}

// Smallest o with cdf[o] > u * total (binary search).
__global__ void k_sample(const double *__restrict__ cdf, int M, const double *__restrict__ u,
                         int shots, uint64_t *__restrict__ out)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= shots) return;
    const double target = u[s] * cdf[M - 1];
    int lo = 0, hi = M - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    out[s] = uint64_t(lo);
}

// Project onto outcome `o` and rescale by 1/sqrt(p_o) (p_o read on device).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_collapse(typename V2<R>::T *__restrict__ psi,
                                                       uint64_t dim, QArgs qa,
                                                       const uint64_t *__restrict__ outcome,
                                                       const double *__restrict__ p)
{
    using C2 = typename V2<R>::T;
    const uint32_t o = uint32_t(outcome[0]);
    const double sc = 1.0 / sqrt(p[o]);
    for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < dim;
         i += uint64_t(gridDim.x) * kThreads) {
        if (outcome_of(i, qa) == o) {
            const C2 a = psi[i];
            psi[i] = C2{R(double(a.x) * sc), R(double(a.y) * sc)};
        } else {
            psi[i] = C2{R(0), R(0)};
        }
    }
}

template <typename R>
__global__ void k_gather_amps(const typename V2<R>::T *__restrict__ psi,
                              const uint64_t *__restrict__ idx, int count,
                              typename V2<R>::T *__restrict__ out)
{
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t < count) out[t] = psi[idx[t]];
}

// Fixed-order final sum of the Pauli partials (as k_finish), times
// i^{popcount(y)} (y_pow = popcount(y) mod 4), written to device memory.
__global__ void k_finish_pauli(const double *__restrict__ partial, int count, int y_pow, double *__restrict__ out)
{
    __shared__ double sh[kThreads / 64];
    double s[2];
    for (int c = 0; c < 2; ++c) {
        double v = 0.0;
        for (int i = threadIdx.x; i < count; i += kThreads) v += partial[size_t(i) * 2 + c];
        s[c] = block_sum(v, sh);
    }
    if (threadIdx.x == 0) {
        double r = s[0], im = s[1];
        switch (y_pow) {
        case 0: break;
        case 1: { const double t = r; r = -im; im = t; break; }
        case 2: r = -r; im = -im; break;
        default: { const double t = r; r = im; im = -t; break; }
        }
        out[0] = r;
        out[1] = im;
    }
}

// Scratch of the allocation-free expectation (qs_expectation_noalloc): the
// per-block partial sums of one Pauli expectation, two doubles for each of
// at most kReduceBlocks blocks (32 KiB). Each GPU holds one copy from the
// library's load until the process ends; calls that overlap on one GPU race
// on it. Host code reaches it only through the per-device address that
// hipGetSymbolAddress returns (the array's name is a host-side stand-in).
constexpr size_t kNoAllocDoubles = 2 * size_t(kReduceBlocks);
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on `device`, resolved once per device with
// that device current.
int scratch_address(int device, double **out)
{
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return fail(QS_EUNSUPPORTED, "device %d outside [0, %d)", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        QS_HIP(hipGetDevice(&cur));
        if (cur != device) QS_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(QS_EDEVICE, "no device address for the expectation scratch");
        addr[device] = static_cast<double *>(p);
    }
    *out = addr[device];
    return QS_OK;
}

unsigned red_grid(uint64_t items)
{
    uint64_t b = (items + kThreads - 1) / kThreads;
    return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(b, kReduceBlocks)));
}

int finish_to_host(qs_state *h, int count, int w, double *out)
{
    double *fin = h->partials + size_t(kReduceBlocks) * 2;
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, h->stream, h->partials, count, w, fin);
    QS_HIP(hipGetLastError());
    if (int rc = ensure_host_out(h, sizeof(double) * size_t(w))) return rc;
    QS_HIP(hipMemcpyAsync(h->host_out, fin, sizeof(double) * size_t(w), hipMemcpyDeviceToHost,
                          h->stream));
    QS_HIP(hipStreamSynchronize(h->stream));
    for (int c = 0; c < w; ++c) out[c] = h->host_out[c];
    return QS_OK;
}

}  // namespace

int reduce_norm2(qs_state *h, double *out)
{
    if (int rc = ensure_partials(h, size_t(kReduceBlocks) * 2 + 8)) return rc;
    const unsigned g = red_grid(h->dim());
    if (h->dtype == QS_C128)
        hipLaunchKernelGGL(k_norm2<double>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const double2 *>(h->psi), h->dim(), h->partials);
    else
        hipLaunchKernelGGL(k_norm2<float>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const float2 *>(h->psi), h->dim(), h->partials);
    QS_HIP(hipGetLastError());
    return finish_to_host(h, int(g), 1, out);
}

int reduce_pauli(qs_state *h, uint64_t xm, uint64_t ym, uint64_t zm, double *re, double *im)
{
    if (int rc = ensure_partials(h, size_t(kReduceBlocks) * 2 + 8)) return rc;
    const uint64_t f = xm | ym;
    const uint64_t sgn = ym | zm;
    int hbit = 0;
    uint64_t items = h->dim();
    if (f) {
        hbit = 63 - __builtin_clzll(f);
        items >>= 1;
    }
    const unsigned g = red_grid(items);
    if (h->dtype == QS_C128)
        hipLaunchKernelGGL(k_pauli<double>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const double2 *>(h->psi), items, f, hbit, sgn, h->partials);
    else
        hipLaunchKernelGGL(k_pauli<float>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const float2 *>(h->psi), items, f, hbit, sgn, h->partials);
    QS_HIP(hipGetLastError());
    double s[2];
    if (int rc = finish_to_host(h, int(g), 2, s)) return rc;
    // multiply by i^{popcount(y)}
    double r = s[0], i = s[1];
    switch (__builtin_popcountll(ym) & 3) {
    case 0: break;
    case 1: { double t = r; r = -i; i = t; break; }
    case 2: r = -r; i = -i; break;
    case 3: { double t = r; r = i; i = -t; break; }
    }
    *re = r;
    *im = i;
    return QS_OK;
}

int reduce_pauli_noalloc(qs_state *h, uint64_t xm, uint64_t ym, uint64_t zm, double *device_out)
{
    double *part = nullptr;
    if (int rc = scratch_address(h->device, &part)) return rc;
    const uint64_t f = xm | ym;
    const uint64_t sgn = ym | zm;
    int hbit = 0;
    uint64_t items = h->dim();
    if (f) {
        hbit = 63 - __builtin_clzll(f);
        items >>= 1;
    }
    const unsigned g = red_grid(items);
    if (size_t(g) * 2 > kNoAllocDoubles)
        return fail(QS_EUNSUPPORTED, "%u partial sums exceed the %zu-double scratch", g, kNoAllocDoubles);
    if (h->dtype == QS_C128)
        hipLaunchKernelGGL(k_pauli<double>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const double2 *>(h->psi), items, f, hbit, sgn, part);
    else
        hipLaunchKernelGGL(k_pauli<float>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const float2 *>(h->psi), items, f, hbit, sgn, part);
    QS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_pauli, dim3(1), dim3(kThreads), 0, h->stream, part, int(g),
                       __builtin_popcountll(ym) & 3, device_out);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

int gather_amplitudes(qs_state *h, int count, const uint64_t *indices, void *host_dst)
{
    void *didx = nullptr, *dout = nullptr;
    if (int rc = h->stage.put(h->stream, indices, sizeof(uint64_t) * size_t(count), &didx)) return rc;
    if (int rc = h->stage.reserve(h->stream, h->amp_bytes() * size_t(count), &dout)) return rc;
    const unsigned g = unsigned((count + kThreads - 1) / kThreads);
    if (h->dtype == QS_C128)
        hipLaunchKernelGGL(k_gather_amps<double>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const double2 *>(h->psi), static_cast<const uint64_t *>(didx),
                           count, static_cast<double2 *>(dout));
    else
        hipLaunchKernelGGL(k_gather_amps<float>, dim3(g), dim3(kThreads), 0, h->stream,
                           static_cast<const float2 *>(h->psi), static_cast<const uint64_t *>(didx),
                           count, static_cast<float2 *>(dout));
    QS_HIP(hipGetLastError());
    if (int rc = ensure_host_out(h, h->amp_bytes() * size_t(count))) return rc;
    QS_HIP(hipMemcpyAsync(h->host_out, dout, h->amp_bytes() * size_t(count), hipMemcpyDeviceToHost,
                          h->stream));
    QS_HIP(hipStreamSynchronize(h->stream));
    std::copy_n(reinterpret_cast<char *>(h->host_out), h->amp_bytes() * size_t(count),
                static_cast<char *>(host_dst));
    return QS_OK;
}

int measure(qs_state *h, int m, const int *qubits, int shots, const double *u, uint64_t *outcomes,
            double *probs, int collapse)
{
    const int M = 1 << m;
    QArgs qa;
    qa.m = m;
    for (int r = 0; r < m; ++r) qa.q[r] = qubits[r];
    const bool lds_path = m <= 12;
    const unsigned g = red_grid(h->dim());
    // device layout: [p (M) | cdf (M) | partial rows | outcomes | uniforms]
    const size_t rows = lds_path ? g : 0;
    const size_t need = size_t(M) * 2 + rows * size_t(M) + size_t(shots) * 2 + 16;
    if (int rc = ensure_partials(h, std::max(need, size_t(kReduceBlocks) * 2 + 8))) return rc;
    double *p = h->partials;
    double *cdf = p + M;
    double *part = cdf + M;
    uint64_t *dout = reinterpret_cast<uint64_t *>(part + rows * size_t(M));
    double *du = reinterpret_cast<double *>(dout + shots);
    if (lds_path) {
        const size_t lds = sizeof(double) * size_t(M);
        int lowest = 64;
        for (int r = 0; r < m; ++r) lowest = std::min(lowest, qubits[r]);
        // wave-uniform bins need whole 64-aligned waves: chunks are powers of
        // two of at least 256 amplitudes once the state has 128 or more
        const int uniform = (lowest >= 6 && h->dim() >= 128) ? 1 : 0;
        if (h->dtype == QS_C128)
            hipLaunchKernelGGL(k_hist_lds<double>, dim3(g), dim3(kThreads), lds, h->stream,
                               static_cast<const double2 *>(h->psi), h->dim(), qa, uniform, part);
        else
            hipLaunchKernelGGL(k_hist_lds<float>, dim3(g), dim3(kThreads), lds, h->stream,
                               static_cast<const float2 *>(h->psi), h->dim(), qa, uniform, part);
        QS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_hist_cols, dim3((M + kThreads - 1) / kThreads), dim3(kThreads), 0,
                           h->stream, part, int(rows), M, p);
    } else {
        RestArgs ra;
        int tmp[20];
        std::copy(qubits, qubits + m, tmp);
        std::sort(tmp, tmp + m);
        ra.nr = m;
        for (int r = 0; r < m; ++r) ra.pos[r] = tmp[r];
        const uint64_t rest = h->dim() >> m;
        if (h->dtype == QS_C128)
            hipLaunchKernelGGL(k_hist_gather<double>, dim3((M + kThreads - 1) / kThreads),
                               dim3(kThreads), 0, h->stream, static_cast<const double2 *>(h->psi),
                               rest, qa, ra, p);
        else
            hipLaunchKernelGGL(k_hist_gather<float>, dim3((M + kThreads - 1) / kThreads),
                               dim3(kThreads), 0, h->stream, static_cast<const float2 *>(h->psi),
                               rest, qa, ra, p);
    }
    QS_HIP(hipGetLastError());
    if (shots > 0) {
        hipLaunchKernelGGL(k_cdf, dim3(1), dim3(kThreads), 0, h->stream, p, M, cdf);
        QS_HIP(hipGetLastError());
        void *du_staged = nullptr;
        if (int rc = h->stage.put(h->stream, u, sizeof(double) * size_t(shots), &du_staged)) return rc;
        QS_HIP(hipMemcpyAsync(du, du_staged, sizeof(double) * size_t(shots),
                              hipMemcpyDeviceToDevice, h->stream));
        hipLaunchKernelGGL(k_sample, dim3((shots + kThreads - 1) / kThreads), dim3(kThreads), 0,
                           h->stream, cdf, M, du, shots, dout);
        QS_HIP(hipGetLastError());
        if (collapse) {
            const unsigned cg = unsigned(std::min<uint64_t>((h->dim() + kThreads - 1) / kThreads, 1u << 20));
            if (h->dtype == QS_C128)
                hipLaunchKernelGGL(k_collapse<double>, dim3(cg), dim3(kThreads), 0, h->stream,
                                   static_cast<double2 *>(h->psi), h->dim(), qa, dout, p);
            else
                hipLaunchKernelGGL(k_collapse<float>, dim3(cg), dim3(kThreads), 0, h->stream,
                                   static_cast<float2 *>(h->psi), h->dim(), qa, dout, p);
            QS_HIP(hipGetLastError());
        }
    }
    const size_t hb = (probs ? sizeof(double) * size_t(M) : 0) + sizeof(uint64_t) * size_t(shots);
    if (int rc = ensure_host_out(h, hb + 16)) return rc;
    char *ho = reinterpret_cast<char *>(h->host_out);
    if (shots > 0)
        QS_HIP(hipMemcpyAsync(ho, dout, sizeof(uint64_t) * size_t(shots), hipMemcpyDeviceToHost,
                              h->stream));
    if (probs)
        QS_HIP(hipMemcpyAsync(ho + sizeof(uint64_t) * size_t(shots), p, sizeof(double) * size_t(M),
                              hipMemcpyDeviceToHost, h->stream));
    QS_HIP(hipStreamSynchronize(h->stream));
    if (shots > 0) std::copy_n(reinterpret_cast<uint64_t *>(ho), shots, outcomes);
    if (probs) std::copy_n(reinterpret_cast<double *>(ho + sizeof(uint64_t) * size_t(shots)), M, probs);
    return QS_OK;
}

}  // namespace qs
