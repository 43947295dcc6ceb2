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
#include <vector>

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

// (x + y) mod N for x, y < N
__device__ __forceinline__ uint64_t addmod(uint64_t x, uint64_t y, uint64_t N)
{
    const uint64_t s = x + y;
    return s >= N ? s - N : s;
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

// ---------------------------------------------------------------------------
// Tiled gather for a work register at the bottom of the index (work_lo = 0).
// The plain gather reads one 16-byte amplitude per output from a scattered
// source, and every source line is fetched again for each of its
// amplitudes. The tiled form uses the structure of x -> A x mod N: the
// outputs y = P_j + i, with P_j = j A mod N, read the sources
// x = A^(-1) y = j + B i, so for a fixed i consecutive rows j read
// consecutive sources, while for a fixed j consecutive i write consecutive
// outputs. The R points P_j (j < R) split the circle Z_N into R arcs
// (rows); by the three-gap theorem the arc after P_j has length
//   d1 if j + jp < R, else d2 if j >= jm, else d1 + d2,
// where jp / jm index the points nearest 0 from above / below, d1 = P_jp
// and d2 = N - P_jm. R is the denominator q_k of a continued-fraction
// convergent of A / N: then only two arc lengths occur and both are near
// N / R, so rows are balanced. jp and jm are q_(k-1) and q_k - q_(k-1) (in
// the order fixed by the sign of q_(k-1) A - p_(k-1) N). A workgroup owns 64
// consecutive rows (and, when R < 4096, one of 4096 / R-ish segments of
// their columns, so every block keeps 64 busy workgroups) and walks them
// COLS outputs at a time through an LDS tile: COLS reads of 64 consecutive
// sources, 64 writes of COLS consecutive outputs, each row continued by the
// next tile of the same workgroup. The default tile is 64 x 128 (1024
// threads; 130 KB of LDS for complex128, one workgroup per CU): its writes
// run over 2 KB (complex128), which pays more than longer reads (128 x 64
// tiles are slower). Indices
// x >= N are fixed points and are copied. A control value without a
// convergent denominator in [64, min(4096, N / 64)] keeps the plain gather
// for its blocks.
// ---------------------------------------------------------------------------
constexpr int kTileRows = 64;                            // tile: 64 rows x COLS outputs
constexpr int kMaxRows = 4096, kMinRows = 64;
constexpr int kWgPerBlock = kMaxRows / kTileRows;        // workgroups per control block

struct ModRows {
    uint64_t A, B;          // a^c mod N and a^(-c) mod N
    uint32_t R, jp, jm;     // row count (0: plain gather), points nearest 0 from above / below
    uint32_t d1, d2;        // P_jp and N - P_jm
    uint32_t pad;
};

__device__ __forceinline__ uint64_t row_len(uint32_t j, const ModRows &r)
{
    if (j + r.jp < r.R) return r.d1;
    if (j >= r.jm) return r.d2;
    return uint64_t(r.d1) + r.d2;
}

// grid: kWgPerBlock workgroups per control block (a block = 2^w consecutive
// amplitudes sharing all other bits); workgroups past the block's rows only
// copy their share of the fixed points. NT threads.
template <typename R, int COLS, int NT, int ROWS = kTileRows>
__global__ __launch_bounds__(NT) void k_modmul_tiled(const typename V2<R>::T *__restrict__ in,
                                                      typename V2<R>::T *__restrict__ out, ModmulArgs ma,
                                                      const ModRows *__restrict__ rows)
{
    using C2 = typename V2<R>::T;
    constexpr int kTileCols = COLS, kThreads = NT;
    __shared__ C2 tile[kTileCols][ROWS + 1];
    const uint64_t blk = blockIdx.x / kWgPerBlock;
    const uint32_t jb = blockIdx.x % kWgPerBlock;
    const uint64_t base = blk << ma.w;
    const uint64_t W = uint64_t(1) << ma.w;
    const uint32_t cc = ma.c ? uint32_t((base >> ma.ctrl_lo) & ((uint64_t(1) << ma.c) - 1)) : 0u;
    const ModRows r = rows[cc];
    const uint64_t N = ma.N;
    const int t = threadIdx.x;
    // fixed points x in [N, 2^w): this workgroup's share, copied
    {
        const uint64_t span = W - N, share = (span + kWgPerBlock - 1) / kWgPerBlock;
        const uint64_t lo = N + uint64_t(jb) * share, hi = min(W, lo + share);
        for (uint64_t y = lo + t; y < hi; y += kThreads) out[base + y] = in[base + y];
    }
    if (r.R == 0) {
        // plain gather over this workgroup's share of [0, N)
        const uint64_t share = (N + kWgPerBlock - 1) / kWgPerBlock;
        const uint64_t lo = uint64_t(jb) * share, hi = min(N, lo + share);
        for (uint64_t y = lo + t; y < hi; y += kThreads) out[base + y] = in[base + mulmod(r.B, y, N, ma.mu)];
        return;
    }
    // the block's rows form nrb groups of ROWS; when there are fewer than 64
    // groups, each group's columns are split into seg = 64 / nrb segments so
    // that all 64 workgroups of the block carry work
    const uint32_t nrb = (r.R + ROWS - 1) / ROWS;
    const uint32_t nseg = kWgPerBlock / nrb;
    if (jb >= nrb * nseg) return;
    const uint32_t j0 = (jb % nrb) * ROWS, sg = jb / nrb;
    const uint32_t j1 = min(r.R, j0 + ROWS);
    // longest row of the group: rows have one of two lengths
    uint64_t maxlen = 0;
    for (uint32_t j = j0; j < j1; ++j) maxlen = max(maxlen, row_len(j, r));
    const uint64_t ntiles = (maxlen + kTileCols - 1) / kTileCols;
    const uint64_t tlo = ntiles * sg / nseg, thi = ntiles * (sg + 1) / nseg;
    // element e of a tile: load view (col = e / ROWS, row = e % ROWS), store
    // view (row = e / COLS, col = e % COLS). The next tile's sources are
    // loaded into registers while the current tile is written out.
    //
    // Index arithmetic without a product per element: a thread's load
    // elements share row j = j0 + t mod ROWS and step the column by
    // NT / ROWS, so their sources j + B i step by B (NT / ROWS) mod N; its store
    // elements share column t mod COLS and step the row by NT / COLS, so
    // their destinations P_j + i step by A (NT / COLS) mod N. From tile to
    // tile the sources advance by B COLS and the destinations by COLS. One
    // modular product per thread sets each chain up.
    constexpr int kPer = ROWS * kTileCols / kThreads;
    constexpr int kLStep = kThreads / ROWS, kSStep = kThreads / kTileCols;
    const uint32_t lrow = uint32_t(t) % ROWS, lcol = uint32_t(t) / ROWS;
    const uint32_t jl = j0 + lrow;
    const uint64_t llen = jl < j1 ? row_len(jl, r) : 0;
    const uint64_t lstep = mulmod(r.B, kLStep, N, ma.mu), ltile = mulmod(r.B, kTileCols, N, ma.mu);
    const uint32_t srow = uint32_t(t) / kTileCols, scol = uint32_t(t) % kTileCols;
    const uint64_t sstep = mulmod(r.A, kSStep, N, ma.mu);
    // chain heads at tile tlo: source of load element 0, destination of store element 0
    uint64_t xh = addmod(mulmod(r.B, tlo * kTileCols + lcol, N, ma.mu), uint64_t(jl) % N, N);
    uint64_t yh = addmod(mulmod(uint64_t(j0 + srow), r.A, N, ma.mu), (tlo * kTileCols + scol) % N, N);
    C2 pre[kPer];
    auto fetch = [&](uint64_t i0, uint64_t x) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const uint64_t i = i0 + lcol + uint64_t(q) * kLStep;
            pre[q] = i < llen ? in[base + x] : C2{R(0), R(0)};   // zeros are never stored
            x = addmod(x, lstep, N);
        }
    };
    if (tlo < thi) fetch(tlo * kTileCols, xh);
    for (uint64_t i0 = tlo * kTileCols; i0 < thi * kTileCols; i0 += kTileCols) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = t + q * kThreads;
            tile[e / ROWS][e % ROWS] = pre[q];
        }
        __syncthreads();
        xh = addmod(xh, ltile, N);
        if (i0 + kTileCols < thi * kTileCols) fetch(i0 + kTileCols, xh);
        uint64_t y = yh;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const uint32_t row = srow + uint32_t(q) * kSStep;
            const uint32_t j = j0 + row;
            if (j < j1 && i0 + scol < row_len(j, r)) out[base + y] = tile[scol][row];
            y = addmod(y, sstep, N);
        }
        yh = addmod(yh, kTileCols % N, N);
        __syncthreads();
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

// Tile width of the tiled gather: 64 x 64 tiles with 512 threads (the
// default: 7.9 ms at 30 qubits complex128, against 8.5 ms for 64 x 32,
// 9.4 ms for 64 x 16 with 256 threads and 12.6-13.4 ms for the plain
// gather), 64 x 32 (tuning value 3) or 64 x 16 (tuning value 2).
template <typename R>
void launch_tiled(qs_state *h, int kern, unsigned blocks, const ModmulArgs &ma, const ModRows *tab)
{
    using C2 = typename V2<R>::T;
    const C2 *src = static_cast<const C2 *>(h->psi);
    C2 *dst = static_cast<C2 *>(h->scratch);
    if (kern == 2)
        hipLaunchKernelGGL((k_modmul_tiled<R, 16, 256>), dim3(blocks), dim3(256), 0, h->stream, src, dst, ma, tab);
    else if (kern == 3)
        hipLaunchKernelGGL((k_modmul_tiled<R, 32, 512>), dim3(blocks), dim3(512), 0, h->stream, src, dst, ma, tab);
    else if (kern == 4)
        hipLaunchKernelGGL((k_modmul_tiled<R, 64, 512>), dim3(blocks), dim3(512), 0, h->stream, src, dst, ma, tab);
    else
        hipLaunchKernelGGL((k_modmul_tiled<R, 128, 1024>), dim3(blocks), dim3(1024), 0, h->stream, src, dst, ma, tab);
}

// Row tables of the tiled gather, per control value c: A = a^c mod N, its
// inverse, and R = the largest continued-fraction denominator q_k of A / N
// with q_k <= min(4096, N / 64) (0 if it is below 64, then the block keeps
// the plain gather), with jp, jm, d1, d2 of the three-gap rule.
void mod_rows_table(uint64_t a, uint64_t N, int count, ModRows *out)
{
    const uint64_t rmax = std::min<uint64_t>(kMaxRows, N / 64);
    unsigned __int128 A = 1 % N;
    for (int c = 0; c < count; ++c) {
        ModRows r{};
        r.A = uint64_t(A);
        // inverse of A by the extended Euclidean algorithm
        int64_t t0 = 0, t1 = 1, r0 = int64_t(N), r1 = int64_t(r.A);
        while (r1) {
            const int64_t q = r0 / r1;
            int64_t tmp = r0 - q * r1;
            r0 = r1;
            r1 = tmp;
            tmp = t0 - q * t1;
            t0 = t1;
            t1 = tmp;
        }
        r.B = uint64_t(t0 < 0 ? t0 + int64_t(N) : t0);
        // convergents p_k / q_k of A / N; keep the last q_k <= rmax with
        // the preceding one (q_(k-1), p_(k-1))
        int64_t pm2 = 0, qm2 = 1, pm1 = 1, qm1 = 0;   // k = -2, -1
        int64_t num = int64_t(r.A), den = int64_t(N);
        int64_t bp = -1, bq = 0, bpp = 0, bqq = 0;   // chosen (p_k, q_k) and (p_(k-1), q_(k-1))
        while (den) {
            const int64_t tq = num / den;
            const int64_t rem = num - tq * den;
            num = den;
            den = rem;
            const int64_t pk = tq * pm1 + pm2, qk = tq * qm1 + qm2;
            if (qk > int64_t(rmax)) break;
            bp = pk;
            bq = qk;
            bpp = pm1;
            bqq = qm1;
            pm2 = pm1;
            qm2 = qm1;
            pm1 = pk;
            qm1 = qk;
        }
        if (bp >= 0 && bq >= kMinRows && bqq >= 1) {
            const int64_t e = bqq * int64_t(r.A) - bpp * int64_t(N);   // signed offset of point q_(k-1)
            r.R = uint32_t(bq);
            const uint64_t pq = uint64_t(bqq) * r.A % N;                 // P at q_(k-1)
            const uint64_t po = uint64_t(bq - bqq) * r.A % N;            // P at q_k - q_(k-1)
            if (e > 0) {
                r.jp = uint32_t(bqq);
                r.jm = uint32_t(bq - bqq);
                r.d1 = uint32_t(pq);
                r.d2 = uint32_t(N - po);
            } else {
                r.jp = uint32_t(bq - bqq);
                r.jm = uint32_t(bqq);
                r.d1 = uint32_t(po);
                r.d2 = uint32_t(N - pq);
            }
        }
        out[c] = r;
        A = A * (a % N) % N;
    }
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
    // tiled gather: work register at the bottom of the index, a modulus
    // well above the row counts, at most 2^12 control values (one row table
    // entry each)
    const int kern = tune_value(QS_TUNE_MODMUL_KERNEL, h->dtype, 0, 0, 0);
    if (p->work_lo == 0 && p->N >= (uint64_t(kMinRows) << 6) && p->c <= 12 && kern != 1) {
        std::vector<ModRows> tab(static_cast<size_t>(cnt));
        mod_rows_table(p->a % p->N, p->N, cnt, tab.data());
        void *drows = nullptr;
        if (int rc = h->stage.put(h->stream, tab.data(), sizeof(ModRows) * tab.size(), &drows)) return rc;
        const uint64_t blocks = (h->dim() >> p->w) * uint64_t(kWgPerBlock);
        if (blocks > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "modmul grid too large");
        const auto *tabp = static_cast<const ModRows *>(drows);
        if (h->dtype == QS_C128)
            launch_tiled<double>(h, kern, unsigned(blocks), ma, tabp);
        else
            launch_tiled<float>(h, kern, unsigned(blocks), ma, tabp);
        QS_HIP(hipGetLastError());
        return adopt_scratch(h);
    }
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
