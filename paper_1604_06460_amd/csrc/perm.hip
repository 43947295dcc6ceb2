// Arithmetic emulated as a permutation of basis states (Sec. III-A): instead
// of simulating the Toffoli network of a reversible multiplier, evaluate the
// classical function on every basis-state index and move the amplitude.
//
// Controlled modular multiplication |c>|x> -> |c>|a^c x mod N> (x < N; x >= N
// fixed) is applied in gather form: output index with work value x' reads
// the input at x = a^(-c) x' mod N. Every output amplitude is written once,
// so the output stream is fully coalesced; inputs are read once each, in an
// order scattered only inside one control block (2^w amplitudes).
// Amplitudes are copied without arithmetic, so the result is bit-exact.
#include "qs_internal.h"

#include <algorithm>
#include <numeric>

namespace qs {
namespace {

constexpr int kThreads = 256;

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

// (x * y) mod N for x, y < N < 2^32 via a 64-bit Barrett reduction with
// mu = floor((2^64 - 1) / N); the quotient estimate is at most two short.
__device__ __forceinline__ uint64_t mulmod(uint64_t x, uint64_t y, uint64_t N, uint64_t mu)
{
    const uint64_t p = x * y;
    const uint64_t q = __umul64hi(p, mu);
    uint64_t r = p - q * N;
    while (r >= N) r -= N;
    return r;
}

// inv_pow[c] = a^(-c) mod N for c in [0, 2^cbits): ainv = a^(-1) mod N by
// the extended Euclidean algorithm, then square-and-multiply.
__global__ void k_inv_powers(uint64_t a, uint64_t N, uint64_t mu, int count,
                             uint64_t *__restrict__ inv_pow)
{
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= count) return;
    int64_t t0 = 0, t1 = 1;
    int64_t r0 = int64_t(N), r1 = int64_t(a % N);
    while (r1 != 0) {
        const int64_t q = r0 / r1;
        int64_t tmp = r0 - q * r1;
        r0 = r1;
        r1 = tmp;
        tmp = t0 - q * t1;
        t0 = t1;
        t1 = tmp;
    }
    uint64_t base = uint64_t(t0 < 0 ? t0 + int64_t(N) : t0) % N;
    uint64_t res = 1 % N;
    for (uint64_t e = uint64_t(c); e; e >>= 1) {
        if (e & 1) res = mulmod(res, base, N, mu);
        base = mulmod(base, base, N, mu);
    }
    inv_pow[c] = res;
}

struct ModmulArgs {
    int work_lo, w, ctrl_lo, c;
    uint64_t N, mu;
};

template <typename R, typename IT>
__global__ __launch_bounds__(kThreads) void k_modmul_gather(
    const typename V2<R>::T *__restrict__ in, typename V2<R>::T *__restrict__ out, IT dim,
    ModmulArgs ma, const uint64_t *__restrict__ inv_pow)
{
    const IT wmask = (IT(1) << ma.w) - 1;
    const IT cmask = (IT(1) << ma.c) - 1;
    const IT stride = IT(gridDim.x) * kThreads;
    for (IT i = IT(blockIdx.x) * kThreads + threadIdx.x; i < dim; i += stride) {
        const IT xp = (i >> ma.work_lo) & wmask;
        IT src = i;
        if (uint64_t(xp) < ma.N) {
            const IT cc = ma.c ? ((i >> ma.ctrl_lo) & cmask) : IT(0);
            const uint64_t x = mulmod(inv_pow[cc], uint64_t(xp), ma.N, ma.mu);
            src = (i & ~(wmask << ma.work_lo)) | (IT(x) << ma.work_lo);
        }
        out[i] = in[src];
    }
}

template <typename R, typename IT>
__global__ __launch_bounds__(kThreads) void k_table_gather(
    const typename V2<R>::T *__restrict__ in, typename V2<R>::T *__restrict__ out, IT dim, int lo,
    int nbits, const uint64_t *__restrict__ src_of)
{
    const IT fmask = (IT(1) << nbits) - 1;
    const IT stride = IT(gridDim.x) * kThreads;
    for (IT i = IT(blockIdx.x) * kThreads + threadIdx.x; i < dim; i += stride) {
        const IT f = (i >> lo) & fmask;
        out[i] = in[(i & ~(fmask << lo)) | (IT(src_of[f]) << lo)];
    }
}

// src_of[dest[f]] = f
__global__ void k_invert_table(const uint64_t *__restrict__ dest, uint64_t count,
                               uint64_t *__restrict__ src_of)
{
    for (uint64_t f = uint64_t(blockIdx.x) * kThreads + threadIdx.x; f < count;
         f += uint64_t(gridDim.x) * kThreads)
        src_of[dest[f]] = f;
}

unsigned grid_for(uint64_t items)
{
    uint64_t b = (items + kThreads - 1) / kThreads;
    return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(b, 1ull << 22)));
}

template <typename R, typename IT>
void launch_modmul(qs_state *h, const ModmulArgs &ma, const uint64_t *inv)
{
    using C2 = typename V2<R>::T;
    hipLaunchKernelGGL((k_modmul_gather<R, IT>), dim3(grid_for(h->dim())), dim3(kThreads), 0,
                       h->stream, static_cast<const C2 *>(h->psi), static_cast<C2 *>(h->scratch),
                       IT(h->dim()), ma, inv);
}

template <typename R, typename IT>
void launch_table(qs_state *h, int lo, int nbits, const uint64_t *src_of)
{
    using C2 = typename V2<R>::T;
    hipLaunchKernelGGL((k_table_gather<R, IT>), dim3(grid_for(h->dim())), dim3(kThreads), 0,
                       h->stream, static_cast<const C2 *>(h->psi), static_cast<C2 *>(h->scratch),
                       IT(h->dim()), lo, nbits, src_of);
}

// The permuted state sits in the scratch buffer: make it the state.
int adopt_scratch(qs_state *h)
{
    if (h->borrowed) {
        QS_HIP(hipMemcpyAsync(h->psi, h->scratch, h->dim() * h->amp_bytes(),
                              hipMemcpyDeviceToDevice, h->stream));
    } else {
        std::swap(h->psi, h->scratch);
    }
    return QS_OK;
}

uint64_t barrett_mu(uint64_t N) { return ~0ull / N; }

}  // namespace

int emulate_modmul(qs_state *h, const qs_perm *p)
{
    if (int rc = ensure_scratch(h)) return rc;
    const int cnt = 1 << p->c;
    void *dinv = nullptr;
    if (int rc = h->stage.reserve(h->stream, sizeof(uint64_t) * size_t(cnt), &dinv)) return rc;
    const uint64_t mu = barrett_mu(p->N);
    hipLaunchKernelGGL(k_inv_powers, dim3((cnt + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       h->stream, p->a, p->N, mu, cnt, static_cast<uint64_t *>(dinv));
    QS_HIP(hipGetLastError());
    ModmulArgs ma{p->work_lo, p->w, p->ctrl_lo, p->c, p->N, mu};
    const bool small = h->n <= 31;
    const uint64_t *inv = static_cast<const uint64_t *>(dinv);
    if (h->dtype == QS_C128) {
        if (small) launch_modmul<double, uint32_t>(h, ma, inv);
        else launch_modmul<double, uint64_t>(h, ma, inv);
    } else {
        if (small) launch_modmul<float, uint32_t>(h, ma, inv);
        else launch_modmul<float, uint64_t>(h, ma, inv);
    }
    QS_HIP(hipGetLastError());
    return adopt_scratch(h);
}

int emulate_table(qs_state *h, const qs_perm *p)
{
    if (int rc = ensure_scratch(h)) return rc;
    const uint64_t cnt = 1ull << p->nbits;
    void *tables = nullptr;
    QS_HIP(hipMalloc(&tables, sizeof(uint64_t) * cnt * 2));
    uint64_t *ddest = static_cast<uint64_t *>(tables), *dsrc = ddest + cnt;
    hipError_t e = hipMemcpyAsync(ddest, p->dest, sizeof(uint64_t) * cnt, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_invert_table, dim3(grid_for(cnt)), dim3(kThreads), 0, h->stream, ddest,
                           cnt, dsrc);
        const bool small = h->n <= 31;
        if (h->dtype == QS_C128) {
            if (small) launch_table<double, uint32_t>(h, p->lo, p->nbits, dsrc);
            else launch_table<double, uint64_t>(h, p->lo, p->nbits, dsrc);
        } else {
            if (small) launch_table<float, uint32_t>(h, p->lo, p->nbits, dsrc);
            else launch_table<float, uint64_t>(h, p->lo, p->nbits, dsrc);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(tables);
    if (e != hipSuccess) return hip_fail(e, "table permutation");
    return adopt_scratch(h);
}

}  // namespace qs

namespace {
uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}
}  // namespace

extern "C" int qs_emulate_permutation(qs_handle h, const qs_perm *p)
{
    using namespace qs;
    clear_error();
    if (!h) return fail(QS_EINVAL, "NULL handle");
    if (!p) return fail(QS_EINVAL, "NULL permutation");
    if (p->kind == QS_PERM_MODMUL) {
        if (p->w < 1 || p->c < 0 || p->c > 20 || p->work_lo < 0 || p->work_lo + p->w > h->n)
            return fail(QS_EINVAL, "work register [%d, %d) outside the state", p->work_lo, p->work_lo + p->w);
        if (p->c > 0 && (p->ctrl_lo < 0 || p->ctrl_lo + p->c > h->n))
            return fail(QS_EINVAL, "control register outside the state");
        if (p->c > 0 && !(p->ctrl_lo >= p->work_lo + p->w || p->ctrl_lo + p->c <= p->work_lo))
            return fail(QS_EINVAL, "control and work registers overlap");
        if (p->N < 2 || p->N >= (1ull << 32) || p->N > (1ull << p->w))
            return fail(QS_EINVAL, "modulus N=%llu outside [2, min(2^w, 2^32))", (unsigned long long)p->N);
        if (gcd_u64(p->a % p->N, p->N) != 1)
            return fail(QS_EINVAL, "gcd(a, N) != 1: not a permutation");
        return emulate_modmul(h, p);
    }
    if (p->kind == QS_PERM_TABLE) {
        if (p->nbits < 1 || p->nbits > 24 || p->lo < 0 || p->lo + p->nbits > h->n)
            return fail(QS_EINVAL, "table field outside the state or wider than 24 bits");
        if (!p->dest) return fail(QS_EINVAL, "NULL table");
        const uint64_t cnt = 1ull << p->nbits;
        std::vector<uint8_t> seen(cnt, 0);
        for (uint64_t f = 0; f < cnt; ++f) {
            if (p->dest[f] >= cnt || seen[p->dest[f]]) return fail(QS_EINVAL, "table is not a permutation");
            seen[p->dest[f]] = 1;
        }
        return emulate_table(h, p);
    }
    return fail(QS_EINVAL, "unknown permutation kind %d", p->kind);
}
