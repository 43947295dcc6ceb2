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

// ---------------------------------------------------------------------------
// Integer multiplication and division into a third register (Sec. III-A).
// Three m-bit fields a, b, c of the index. Multiplication keeps a and b and
// rotates c by a*b; division maps the 2m-bit pair (a, c) given b. Both run in
// gather form: each output index computes where its amplitude came from.
// ---------------------------------------------------------------------------
struct ArithArgs {
    int a_lo, b_lo, c_lo, m;
};

// Source (a, c) of the output (a', c') under division. One step of the
// forward map acts on the (m+1)-bit window W of Y = a + 2^m c at bit s: with
// W < b it is kept; with b <= W < b + 2^m it becomes W - b + 2^m (quotient
// bit 1); with W >= b + 2^m its top bit is cleared. The three images are
// [0, b), [2^m, 2^(m+1)) and [b, 2^m), so the step is undone by reading the
// case off the output window W': top bit set -> W' - 2^m + b; W' < b -> W';
// otherwise W' + 2^m. Steps are undone from s = 0 up. Y has 2m <= 22 bits
// (at most 34 qubits hold three registers), so 32-bit arithmetic is exact.
__device__ __forceinline__ void div_source(uint32_t &a, uint32_t &c, uint32_t b, int m)
{
    const uint32_t M1 = (2u << m) - 1, top = 1u << m;
    uint32_t Y = a | (c << m);
    for (int s = 0; s < m; ++s) {
        const uint32_t W = (Y >> s) & M1;
        const uint32_t delta = (W & top) ? b - top : (W < b ? 0u : top);
        Y += delta << s;
    }
    a = Y & (top - 1);
    c = Y >> m;
}

// Output order. Neither map changes b, so the outputs with one b value take
// their inputs from the same 2^(n-m) indices. With bmajor set, thread t
// handles the output whose b field is the top m bits of t and whose other
// bits are the rest of t in order: the whole device then works inside one or
// two such slices at a time, which stay in cache while their scattered reads
// are served. It pays for division when a sits above c: every input of a
// clean-c output lies in another a row. Multiplication walks the blocks in
// chunked XCD order (runs of 128), which on 30 qubits with c lowest takes
// 5.5 instead of 6.2 ms; the same order makes division slower (20 instead of
// 15 ms), so division keeps the launch order.
template <typename R, typename IT, int KIND>
__global__ __launch_bounds__(kThreads) void k_arith_gather(
    const typename V2<R>::T *__restrict__ in, typename V2<R>::T *__restrict__ out, IT dim,
    ArithArgs aa, int n, int bmajor)
{
    const uint32_t M0 = (1u << aa.m) - 1;
    const IT clear = ~((IT(M0) << aa.a_lo) | (IT(M0) << aa.c_lo));
    const IT stride = IT(gridDim.x) * kThreads;
    const int nrest = n - aa.m;
    const IT below_b = (IT(1) << aa.b_lo) - 1;
    const IT first = KIND == QS_ARITH_MUL ? xcd_order<IT, 128>(blockIdx.x, gridDim.x) : IT(blockIdx.x);
    for (IT t = first * kThreads + threadIdx.x; t < dim; t += stride) {
        IT i = t;
        if (bmajor) {
            const IT r = t & ((IT(1) << nrest) - 1);
            i = (r & below_b) | ((r >> aa.b_lo) << (aa.b_lo + aa.m)) | ((t >> nrest) << aa.b_lo);
        }
        uint32_t a = uint32_t(i >> aa.a_lo) & M0;
        const uint32_t b = uint32_t(i >> aa.b_lo) & M0;
        uint32_t c = uint32_t(i >> aa.c_lo) & M0;
        if (KIND == QS_ARITH_MUL) c = (c - a * b) & M0;
        else div_source(a, c, b, aa.m);
        out[i] = in[(i & clear) | (IT(a) << aa.a_lo) | (IT(c) << aa.c_lo)];
    }
}

// Multiplication only moves amplitudes inside the c field, and how far
// depends on a and b alone. A tile is every c value times the 2^t lowest
// index bits (one 128-byte line of amplitudes), all other bits fixed: the map
// keeps each tile, so the tile is read into LDS and written back rotated,
// with every global access a whole line. Requires c_lo >= t.
constexpr int kTileThreads = 1024;
constexpr size_t kTileLdsMax = 128 * 1024;

template <typename R, typename IT>
__global__ __launch_bounds__(kTileThreads) void k_mul_tile(
    const typename V2<R>::T *__restrict__ in, typename V2<R>::T *__restrict__ out, IT n_tiles,
    ArithArgs aa, int t)
{
    using C2 = typename V2<R>::T;
    extern __shared__ unsigned char lds_raw[];
    C2 *tile = reinterpret_cast<C2 *>(lds_raw);
    constexpr int VPT = int(kTileLdsMax / sizeof(C2) / kTileThreads);   // 8 (complex128), 16 (complex64)
    const int per = 1 << (t + aa.m);            // a multiple of kTileThreads, at most VPT of them
    const int lmask = (1 << t) - 1;
    const int gap = aa.c_lo - t;
    const uint32_t M0 = (1u << aa.m) - 1;
    auto index = [&](IT T, int e) {
        const IT base = ((T & ((IT(1) << gap) - 1)) << t) | ((T >> gap) << (aa.c_lo + aa.m));
        return base | IT(e & lmask) | (IT(e >> t) << aa.c_lo);
    };
    // Each thread holds its share of the next tile in registers while the
    // current one is written out, so loads stay in flight across tiles.
    C2 v[VPT];
    IT T = blockIdx.x;
    if (T < n_tiles) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int e = threadIdx.x + k * kTileThreads;
            if (e < per) v[k] = in[index(T, e)];
        }
    }
    for (; T < n_tiles; T += gridDim.x) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int e = threadIdx.x + k * kTileThreads;
            if (e < per) tile[e] = v[k];
        }
        __syncthreads();
        const IT Tn = T + gridDim.x;
        if (Tn < n_tiles) {
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                const int e = threadIdx.x + k * kTileThreads;
                if (e < per) v[k] = in[index(Tn, e)];
            }
        }
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int e = threadIdx.x + k * kTileThreads;
            if (e < per) {
                const IT j = index(T, e);
                const uint32_t a = uint32_t(j >> aa.a_lo) & M0;
                const uint32_t b = uint32_t(j >> aa.b_lo) & M0;
                const uint32_t cs = (uint32_t(e >> t) - a * b) & M0;
                out[j] = tile[int(cs << t) | (e & lmask)];
            }
        }
        __syncthreads();
    }
}

template <typename R, typename IT>
int launch_arith(qs_state *h, int kind, const ArithArgs &aa)
{
    using C2 = typename V2<R>::T;
    const int t = sizeof(R) == 8 ? 3 : 4;          // amplitudes per 128-byte line: 2^t
    const size_t tile_bytes = (size_t(1) << (t + aa.m)) * sizeof(C2);
    const bool tiled = kind == QS_ARITH_MUL && aa.c_lo >= t && tile_bytes <= kTileLdsMax &&
                       (1 << (t + aa.m)) >= kTileThreads;
    const C2 *in = static_cast<const C2 *>(h->psi);
    C2 *out = static_cast<C2 *>(h->scratch);
    if (tiled) {
        static bool lds_ok = false;
        if (!lds_ok) {
            QS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_mul_tile<R, IT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(kTileLdsMax)));
            lds_ok = true;
        }
        const IT n_tiles = IT(h->dim() >> (t + aa.m));
        // persistent: as many workgroups as fit at once (LDS, and at most two
        // of 1024 threads per compute unit)
        const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(2, (160 * 1024) / tile_bytes));
        const unsigned grid = unsigned(std::min<uint64_t>(n_tiles, uint64_t(device_cus()) * per_cu));
        hipLaunchKernelGGL((k_mul_tile<R, IT>), dim3(grid), dim3(kTileThreads), tile_bytes, h->stream, in,
                           out, n_tiles, aa, t);
    } else if (kind == QS_ARITH_MUL) {
        hipLaunchKernelGGL((k_arith_gather<R, IT, QS_ARITH_MUL>), dim3(grid_for(h->dim())), dim3(kThreads),
                           0, h->stream, in, out, IT(h->dim()), aa, h->n, 0);
    } else {
        // b-major order when a lies above c and whole lines of outputs stay
        // contiguous (b clear of the lowest t bits)
        const int bmajor = aa.a_lo > aa.c_lo && aa.b_lo >= t;
        hipLaunchKernelGGL((k_arith_gather<R, IT, QS_ARITH_DIV>), dim3(grid_for(h->dim())), dim3(kThreads),
                           0, h->stream, in, out, IT(h->dim()), aa, h->n, bmajor);
    }
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace

int emulate_arith(qs_state *h, int kind, int a_lo, int b_lo, int c_lo, int m)
{
    if (int rc = ensure_scratch(h)) return rc;
    const ArithArgs aa{a_lo, b_lo, c_lo, m};
    const bool small = h->n <= 31;
    int rc;
    if (h->dtype == QS_C128) rc = small ? launch_arith<double, uint32_t>(h, kind, aa) : launch_arith<double, uint64_t>(h, kind, aa);
    else rc = small ? launch_arith<float, uint32_t>(h, kind, aa) : launch_arith<float, uint64_t>(h, kind, aa);
    if (rc) return rc;
    return adopt_scratch(h);
}

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

extern "C" int qs_emulate_arith(qs_handle h, int kind, int a_lo, int b_lo, int c_lo, int m)
{
    using namespace qs;
    clear_error();
    if (!h) return fail(QS_EINVAL, "NULL handle");
    if (kind != QS_ARITH_MUL && kind != QS_ARITH_DIV) return fail(QS_EINVAL, "unknown arithmetic kind %d", kind);
    if (m < 1 || 3 * m > h->n) return fail(QS_EINVAL, "three %d-bit registers do not fit %d qubits", m, h->n);
    const int lo[3] = {a_lo, b_lo, c_lo};
    for (int r = 0; r < 3; ++r) {
        if (lo[r] < 0 || lo[r] + m > h->n)
            return fail(QS_EINVAL, "register [%d, %d) outside the state", lo[r], lo[r] + m);
        for (int q = 0; q < r; ++q)
            if (lo[r] < lo[q] + m && lo[q] < lo[r] + m) return fail(QS_EINVAL, "registers overlap");
    }
    return emulate_arith(h, kind, a_lo, b_lo, c_lo, m);
}
