// Device building blocks of the QFT emulation (Sec. III-B), shared by the
// standalone FFT passes (fft.hip) and the batched persistent kernel
// (batch.hip). See fft.hip for the decomposition.
#pragma once

#include "qs_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace qs {
namespace fftdev {

constexpr int kRmax = 10;                 // digit width limit (bits)
constexpr size_t kLdsMax = 160 * 1024;    // LDS of a CU (largest tile budget)
constexpr size_t kLdsBytes = 80 * 1024;   // default tile budget: two workgroups per CU
constexpr int kMaxCols = 16;

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <typename C2> struct NtVec;
template <> struct NtVec<double2> { typedef double __attribute__((ext_vector_type(2))) T; };
template <> struct NtVec<float2> { typedef float __attribute__((ext_vector_type(2))) T; };

template <typename C2>
__device__ __forceinline__ C2 load_amp(const C2 *p, int nt)
{
    if (nt & 2) {
        using T = typename NtVec<C2>::T;
        const T v = __builtin_nontemporal_load(reinterpret_cast<const T *>(p));
        return C2{v.x, v.y};
    }
    return *p;
}

template <typename C2>
__device__ __forceinline__ void store_amp(C2 *p, C2 v, int nt)
{
    if (nt & 1) {
        using T = typename NtVec<C2>::T;
        const T w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<T *>(p));
    } else {
        *p = v;
    }
}

template <typename C2>
__device__ __forceinline__ C2 cmul(C2 a, C2 b)
{
    return C2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

struct PassArgs {
    int r;              // digit width
    int dig_lo;         // absolute position of the digit
    int cb;             // number of column bits
    int col_pos[6];     // absolute source positions of the column bits
    int nrest;
    int rest_pos[40];   // remaining bits (ascending), enumerated by tile index
    int nst;            // in-LDS stages
    int rho[4], sigma[4];
    // pass twiddle (tw_bits == 0: none)
    int tw_bits;        // log2 N_j
    int krest_lo, krest_bits;
    int sgn;            // +1 forward QFT, -1 inverse
    double scale;
    // final pass: destination field index from the position digits
    int final_pass;
    int q_lo, m;
    int ndig;
    int dpos[8], dw[8], doff[8];
    uint64_t tiles;     // number of tiles of this pass
    int nt;             // cache policy: bit 0 nontemporal stores, bit 1 nontemporal loads
};

// Column pad (elements) of the LDS tile: a column stride congruent to
// W/C modulo W = 256 B / amplitude puts C columns x W/C consecutive rows on
// distinct banks of a 256-byte bank row, the shape of every tile access.
__host__ __device__ inline int col_pad(int cb, int amp)
{
    const int w = 256 / amp;
    return std::min(16, std::max(1, w >> cb));
}

// LDS bytes of a tile of 2^r x 2^cb: padded tile, the twiddle tables, and
// per digit value its LDS row after the stages (u16) and its destination
// bits (u64)
inline size_t lds_need(int r, int cb, size_t amp)
{
    const size_t C = size_t(1) << cb, L = size_t(1) << r;
    return amp * (size_t(L + col_pad(cb, int(amp))) * C + 64 + 64 * C) + 2 * L + 8 + 8 * L;
}

inline size_t pass_lds_bytes(const PassArgs &pa, size_t amp) { return lds_need(pa.r, pa.cb, amp); }

// LDS slot of row p of column c (S = padded column stride); the low 4 row
// bits are XOR-swizzled by the next 4 for the strided stage accesses.
__device__ __forceinline__ int phys(int c, int p, int S)
{
    return c * S + (p ^ ((p >> 4) & 15));
}

// exp(s 2 pi i num / 2^bits) with num already reduced below 2^bits.
template <typename C2, typename R>
__device__ __forceinline__ C2 unit_root(uint64_t num, int bits, int sgn)
{
    double sn, cs;
    sincospi(double(sgn) * 2.0 * (double(num) / double(1ull << bits)), &sn, &cs);
    return C2{R(cs), R(sn)};
}

// Stage twiddle exp(s 2 pi i y / 1024) from the two 32-entry tables.
template <typename C2>
__device__ __forceinline__ C2 stw(const C2 *__restrict__ ta, const C2 *__restrict__ tb, int y)
{
    return (y & 31) ? ((y >> 5) ? cmul(ta[y & 31], tb[y >> 5]) : ta[y & 31]) : tb[y >> 5];
}

// Natural-order DFT of RAD register values (radix-2 decimation in frequency
// followed by a compile-time bit reversal of the register names).
template <typename C2, int RAD>
__device__ __forceinline__ void dft_reg(C2 (&v)[RAD], const C2 *__restrict__ tb)
{
#pragma unroll
    for (int h = RAD / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int b = 0; b < RAD; b += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const C2 a = v[b + j], c = v[b + j + h];
                v[b + j] = C2{a.x + c.x, a.y + c.y};
                const C2 d{a.x - c.x, a.y - c.y};
                // exp(s 2 pi i j / (2h)) = 1024-table entry j * 512 / h
                v[b + j + h] = (j == 0) ? d : cmul(d, tb[(j * (512 / h)) >> 5]);
            }
        }
    }
    C2 t[RAD];
#pragma unroll
    for (int l = 0; l < RAD; ++l) {
        int rv = 0;
#pragma unroll
        for (int b = 0; (1 << b) < RAD; ++b) rv |= ((l >> b) & 1) << (__builtin_ctz(RAD) - 1 - b);
        t[l] = v[rv];
    }
#pragma unroll
    for (int l = 0; l < RAD; ++l) v[l] = t[l];
}

// One radix-RAD stage over the tile in LDS: digit at sigma (within r bits),
// then the twiddle exp(s 2 pi i k' l / 2^(sigma+rho)) with k' = bits below.
template <typename C2, int RHO, int NT>
__device__ void lds_stage(C2 *lds, int r, int cb, int S, int sigma, const C2 *__restrict__ ta,
                          const C2 *__restrict__ tb)
{
    constexpr int RAD = 1 << RHO;
    const int items = 1 << (cb + r - RHO);
    const int tw_shift = kRmax - (sigma + RHO);
    for (int it = threadIdx.x; it < items; it += NT) {
        const int c = it & ((1 << cb) - 1);
        const int o = it >> cb;
        const int lo = o & ((1 << sigma) - 1);
        const int hi = (o >> sigma) << (sigma + RHO);
        C2 v[RAD];
#pragma unroll
        for (int d = 0; d < RAD; ++d) v[d] = lds[phys(c, hi | (d << sigma) | lo, S)];
        dft_reg<C2, RAD>(v, tb);
        if (sigma > 0) {
#pragma unroll
            for (int l = 1; l < RAD; ++l) {
                const int y = ((lo * l) << tw_shift) & 1023;
                v[l] = cmul(v[l], stw(ta, tb, y));
            }
        }
#pragma unroll
        for (int d = 0; d < RAD; ++d) lds[phys(c, hi | (d << sigma) | lo, S)] = v[d];
    }
}

// Pieces of one tile of one pass, each executed by a whole workgroup of NT
// threads. A tile is the 2^r values of the pass digit for C = 2^cb columns
// (C consecutive values of the lowest available bits) at one value of the
// remaining bits.
__device__ __forceinline__ uint64_t tile_base(const PassArgs &pa, uint64_t tile)
{
    uint64_t base = 0;
    for (int i = 0; i < pa.nrest; ++i) base |= ((tile >> i) & 1ull) << pa.rest_pos[i];
    return base;
}

__device__ __forceinline__ uint64_t tile_colbits(const PassArgs &pa, int c)
{
    uint64_t v = 0;
    for (int i = 0; i < pa.cb; ++i) v |= uint64_t((c >> i) & 1) << pa.col_pos[i];
    return v;
}

// Source index of tile element e (column = low cb bits of e, digit value =
// the rest), so consecutive threads read consecutive columns.
__device__ __forceinline__ uint64_t tile_src(const PassArgs &pa, uint64_t base, int e)
{
    const int c = e & ((1 << pa.cb) - 1), p = e >> pa.cb;
    return base | (uint64_t(p) << pa.dig_lo) | tile_colbits(pa, c);
}

// LDS carve-up: tile, then the stage and pass twiddle tables.
template <typename C2>
struct TileLds {
    C2 *tile, *ta, *tb, *ga, *gb;
    uint16_t *row;   // [L] LDS row holding output digit value l after the stages
    uint64_t *dbits; // [L] destination index bits of output digit value l
    int S;           // padded column stride (elements)
    __device__ TileLds(unsigned char *raw, int r, int cb)
    {
        S = (1 << r) + col_pad(cb, int(sizeof(C2)));
        const int C = 1 << cb;
        tile = reinterpret_cast<C2 *>(raw);
        ta = tile + size_t(C) * S;                 // exp(s 2 pi i j / 1024), j < 32
        tb = ta + 32;                              // exp(s 2 pi i 32 j / 1024), j < 32
        ga = tb + 32;                              // [C][32] pass twiddle, low 5 bits of l
        gb = ga + 32 * C;                          // [C][32] pass twiddle, high bits of l
        row = reinterpret_cast<uint16_t *>(gb + 32 * C);
        dbits = reinterpret_cast<uint64_t *>((reinterpret_cast<uintptr_t>(row + (1 << r)) + 7) & ~uintptr_t(7));
    }
};

// Destination of source index x on a final pass: the field's digits in
// reversed order (a bit permutation of the field, identity elsewhere).
__device__ __forceinline__ uint64_t final_dest(const PassArgs &pa, uint64_t x)
{
    const uint64_t fmask = ((1ull << pa.m) - 1) << pa.q_lo;
    uint64_t f = 0;
    for (int d = 0; d < pa.ndig; ++d) f |= ((x >> pa.dpos[d]) & ((1ull << pa.dw[d]) - 1)) << pa.doff[d];
    return (x & ~fmask) | (f << pa.q_lo);
}

// Per-pass tables: LDS row of every output digit value (the stages leave
// the digit's sub-digits in reversed order) and its destination bits.
template <int NT>
__device__ void tile_index_tables(const PassArgs &pa, uint16_t *row, uint64_t *dbits)
{
    for (int l = threadIdx.x; l < (1 << pa.r); l += NT) {
        int p = 0, sh = 0;
        for (int s = 0; s < pa.nst; ++s) {
            p |= ((l >> sh) & ((1 << pa.rho[s]) - 1)) << pa.sigma[s];
            sh += pa.rho[s];
        }
        row[l] = uint16_t(p);
        const uint64_t x = uint64_t(l) << pa.dig_lo;
        dbits[l] = pa.final_pass ? final_dest(pa, x) : x;
    }
}

template <typename R, int NT>
__device__ void tile_tables(const PassArgs &pa, uint64_t base, const TileLds<typename V2<R>::T> &T)
{
    using C2 = typename V2<R>::T;
    const int C = 1 << pa.cb;
    for (int t = threadIdx.x; t < 64 + (pa.tw_bits ? 64 * C : 0); t += NT) {
        if (t < 32) {
            T.ta[t] = unit_root<C2, R>(uint64_t(t), kRmax, pa.sgn);
        } else if (t < 64) {
            T.tb[t - 32] = unit_root<C2, R>(uint64_t(t - 32) << 5, kRmax, pa.sgn);
        } else {
            const int u = t - 64, c = u >> 6, j = u & 31, hi = (u >> 5) & 1;
            const uint64_t kr = ((base | tile_colbits(pa, c)) >> pa.krest_lo) & ((1ull << pa.krest_bits) - 1);
            const uint64_t mask = (1ull << pa.tw_bits) - 1;
            const uint64_t e2 = (kr * (uint64_t(j) << (hi ? 5 : 0))) & mask;
            (hi ? T.gb : T.ga)[c * 32 + j] = unit_root<C2, R>(e2, pa.tw_bits, pa.sgn);
        }
    }
}

// Register stages over the tile in LDS (expects the tile and tables
// written and a barrier passed; ends with a barrier). MAXRHO bounds the
// radix the kernel is compiled for (the plan must respect it).
template <typename R, int NT, int MAXRHO = 4>
__device__ void tile_stages(const PassArgs &pa, const TileLds<typename V2<R>::T> &T)
{
    using C2 = typename V2<R>::T;
    const int r = pa.r;
    for (int s = 0; s < pa.nst; ++s) {
        const int rho = pa.rho[s];
        if (rho == 1) lds_stage<C2, 1, NT>(T.tile, r, pa.cb, T.S, pa.sigma[s], T.ta, T.tb);
        else if (rho == 2) lds_stage<C2, 2, NT>(T.tile, r, pa.cb, T.S, pa.sigma[s], T.ta, T.tb);
        else if (MAXRHO == 3 || rho == 3) lds_stage<C2, 3, NT>(T.tile, r, pa.cb, T.S, pa.sigma[s], T.ta, T.tb);
        else if constexpr (MAXRHO >= 4) lds_stage<C2, 4, NT>(T.tile, r, pa.cb, T.S, pa.sigma[s], T.ta, T.tb);
        __syncthreads();
    }
}

// Thread geometry of a tile: element e = tid + i*NT has column tid mod C
// (NT is a multiple of C) and digit value tid/C + i*NT/C, so a thread's
// elements share their column bits and step through the digit.
struct TileThread {
    int c0, l0, lstep, reps;
    __device__ TileThread(const PassArgs &pa, int NT)
    {
        c0 = int(threadIdx.x) & ((1 << pa.cb) - 1);
        l0 = int(threadIdx.x) >> pa.cb;
        lstep = NT >> pa.cb;
        reps = ((1 << (pa.r + pa.cb)) + NT - 1) / NT;
    }
};

// Load a tile into LDS. Loads go out in batches of 8 into registers before
// any is written to LDS, so a thread has up to 8 reads in flight instead of
// waiting for each one.
template <typename R, int NT>
__device__ void tile_load(const typename V2<R>::T *__restrict__ src, const PassArgs &pa, uint64_t base,
                          const TileLds<typename V2<R>::T> &T, const TileThread &th)
{
    using C2 = typename V2<R>::T;
    constexpr int B = 8;
    const C2 *s0 = src + (base | tile_colbits(pa, th.c0));
    const int L = 1 << pa.r;
    for (int i0 = 0; i0 < th.reps; i0 += B) {
        C2 v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int l = th.l0 + (i0 + k) * th.lstep;
            if (i0 + k < th.reps && l < L) v[k] = load_amp(s0 + (uint64_t(l) << pa.dig_lo), pa.nt);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int l = th.l0 + (i0 + k) * th.lstep;
            if (i0 + k < th.reps && l < L) T.tile[phys(th.c0, l, T.S)] = v[k];
        }
    }
}

// Pass twiddle, scale and store (with the digit reversal on a final pass).
template <typename R, int NT>
__device__ void tile_store(typename V2<R>::T *__restrict__ dst, const PassArgs &pa, uint64_t base,
                           const TileLds<typename V2<R>::T> &T, const TileThread &th)
{
    using C2 = typename V2<R>::T;
    const int L = 1 << pa.r, c0 = th.c0;
    const uint64_t x0 = base | tile_colbits(pa, c0);
    C2 *d0 = dst + (pa.final_pass ? final_dest(pa, x0) : x0);
    const C2 *ga = T.ga + c0 * 32, *gb = T.gb + c0 * 32;
    for (int i = 0; i < th.reps; ++i) {
        const int l = th.l0 + i * th.lstep;
        if (l >= L) break;
        C2 v = T.tile[phys(c0, T.row[l], T.S)];
        if (pa.tw_bits) v = cmul(v, (l >> 5) ? cmul(ga[l & 31], gb[l >> 5]) : ga[l]);
        if (pa.scale != 1.0) v = C2{R(double(v.x) * pa.scale), R(double(v.y) * pa.scale)};
        store_amp(d0 + T.dbits[l], v, pa.nt);
    }
}

// One whole tile: load, tables, stages, store. Ends with a workgroup
// barrier so the LDS can be reused at once.
template <typename R, int NT, int MAXRHO = 4>
__device__ void fft_tile(const typename V2<R>::T *__restrict__ src, typename V2<R>::T *__restrict__ dst,
                         const PassArgs &pa, uint64_t tile, unsigned char *lds_raw)
{
    const TileLds<typename V2<R>::T> T(lds_raw, pa.r, pa.cb);
    const TileThread th(pa, NT);
    const uint64_t base = tile_base(pa, tile);
    tile_load<R, NT>(src, pa, base, T, th);
    tile_tables<R, NT>(pa, base, T);
    tile_index_tables<NT>(pa, T.row, T.dbits);
    __syncthreads();
    tile_stages<R, NT, MAXRHO>(pa, T);
    tile_store<R, NT>(dst, pa, base, T, th);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Host: pass plan for an m-qubit field at q_lo of an n-qubit state.
// P = ceil(m / digit) digits from the top of the field; all passes but the
// last are in place; with P > 1 the last writes out of place and reverses
// the digit order.
// ---------------------------------------------------------------------------
inline void stage_plan(int r, PassArgs &pa, int max_rho = 4)
{
    pa.nst = 0;
    int top = r;
    while (top > 0) {
        const int rho = std::min(max_rho, top);
        pa.rho[pa.nst] = rho;
        pa.sigma[pa.nst] = top - rho;
        ++pa.nst;
        top -= rho;
    }
}

// reg_cb >= 0 asks for exactly reg_cb column bits on every pass whose digit
// is kRmax bits wide (the register-tile kernels), where the state has that
// many bits outside the digit; other passes size their columns to the LDS
// budget.
inline int plan_passes(int n, int q_lo, int m, int inverse, int digit, size_t lds_budget, size_t amp,
                       std::vector<PassArgs> &out, int max_rho = 4, int reg_cb = -1)
{
    const int P = (m + digit - 1) / digit;
    if (P > 8) return fail(QS_EUNSUPPORTED, "QFT field needs more than 8 passes");
    int width[8], pos[8];
    {
        int rem = m;
        for (int j = 0; j < P; ++j) {
            width[j] = (rem + (P - j) - 1) / (P - j);
            rem -= width[j];
        }
        int top = q_lo + m;
        for (int j = 0; j < P; ++j) {
            top -= width[j];
            pos[j] = top;
        }
    }
    out.clear();
    for (int j = 0; j < P; ++j) {
        PassArgs pa;
        std::memset(&pa, 0, sizeof pa);
        pa.r = width[j];
        pa.dig_lo = pos[j];
        pa.sgn = inverse ? -1 : 1;
        pa.scale = 1.0;
        pa.q_lo = q_lo;
        pa.m = m;
        stage_plan(pa.r, pa, max_rho);
        const bool last = (j == P - 1);
        int maxcb = 0;
        while ((2 << maxcb) <= kMaxCols && lds_need(pa.r, maxcb + 1, amp) <= lds_budget) ++maxcb;
        int want = std::max(0, std::min(maxcb, n - pa.r));
        const int avail = (last && P > 1) ? q_lo + width[0] : n - pa.r;
        if (reg_cb >= 0 && pa.r == kRmax && avail >= reg_cb) want = reg_cb;
        std::vector<int> cols;
        if (last && P > 1) {
            // destination-contiguous bits: spectators below the field, then the
            // low bits of the top digit (they become the lowest field bits)
            for (int b = 0; b < q_lo && int(cols.size()) < want; ++b) cols.push_back(b);
            for (int b = 0; b < width[0] && int(cols.size()) < want; ++b) cols.push_back(pos[0] + b);
        } else {
            for (int b = 0; b < n && int(cols.size()) < want; ++b)
                if (b < pa.dig_lo || b >= pa.dig_lo + pa.r) cols.push_back(b);
        }
        pa.cb = int(cols.size());
        for (int i = 0; i < pa.cb; ++i) pa.col_pos[i] = cols[size_t(i)];
        std::vector<int> rest;
        for (int b = 0; b < n; ++b) {
            const bool in_dig = (b >= pa.dig_lo && b < pa.dig_lo + pa.r);
            const bool in_col = std::find(cols.begin(), cols.end(), b) != cols.end();
            if (!in_dig && !in_col) rest.push_back(b);
        }
        pa.nrest = int(rest.size());
        for (int i = 0; i < pa.nrest; ++i) pa.rest_pos[i] = rest[size_t(i)];
        if (!last) {
            pa.tw_bits = pos[j] + width[j] - q_lo;  // bits of the current sub-problem
            pa.krest_lo = q_lo;
            pa.krest_bits = pos[j] - q_lo;
        }
        if (last) pa.scale = 1.0 / std::sqrt(std::ldexp(1.0, m));
        if (last && P > 1) {
            pa.final_pass = 1;
            pa.ndig = P;
            int off = 0;
            for (int d = 0; d < P; ++d) {
                pa.dpos[d] = pos[d];
                pa.dw[d] = width[d];
                pa.doff[d] = off;   // digit d holds output digit d (lowest first)
                off += width[d];
            }
        }
        pa.tiles = (1ull << n) >> (pa.r + pa.cb);
        out.push_back(pa);
    }
    return QS_OK;
}

}  // namespace fftdev
}  // namespace qs
