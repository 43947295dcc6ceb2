// QFT emulated as a fast Fourier transform (Sec. III-B). The QFT maps
//   alpha_l -> 2^(-m/2) sum_k alpha_k exp(+2 pi i k l / 2^m)
// on an m-qubit field of the index; the gate-level circuit needs m
// Hadamards and m(m-1)/2 conditional phase shifts, each a full sweep, while
// the emulator performs the same transform as an FFT in a handful of sweeps.
//
// Decomposition (decimation in frequency). The field is split into P digits
// of at most 10 bits, processed from the most significant one. A pass over
// digit j computes, for every fixed value of the other index bits, the DFT
// over that digit, multiplies by the twiddle exp(s 2 pi i k_rest l_j / N_j)
// (k_rest = field bits below the digit, N_j = 2^(bits up to the digit's
// top)) and stores output digit l_j in the digit's place. After the last
// pass the output digits sit in reversed digit order; the last pass writes
// out of place and performs that reversal in its store, so a P-pass
// transform moves the state P times. The passes alternate between the
// state and a scratch buffer so that the last one lands in the state.
//
// Passes over a 10-bit digit (every pass of a 30-qubit QFT) run on
// register-tile kernels: a tile is the 1024 digit values of C columns with
// C amplitudes = 128 bytes per row (8 complex128, 16 complex64), the
// shortest row that a DRAM burst serves in full; rows of the top digit lie
// 16 MiB apart. The tile is held in registers, and LDS serves only the
// exchanges of the 16 x 64 (or 8 x 128) split of the 1024-point DFT. The
// default (k_fft_reg_stream) is persistent, one workgroup per CU: it
// transforms one tile while the next one loads into registers. The
// register-tile kernels are described with their code below.
//
// Other passes (and every pass under FFT kernel options 1 and 2) use an
// LDS tile of 2^r digit values x C columns (C consecutive values of the
// lowest available bits; the 80 KB budget gives a 10-bit digit C = 4
// complex128 or 8 complex64 columns, 64 bytes) and perform the 2^r-point
// DFT as radix-2^rho register stages (rho <= 3 for complex128, 4 for
// complex64), again decimation in frequency: one workgroup per tile
// (k_fft_pass) in an XCD-aware order, or persistent workgroups streaming
// tiles (k_fft_stream). Their LDS layout is column-major with a 4-element
// pad per column and the low 4 bits of the row XOR-swizzled by the next 4,
// which keeps both the strided and the contiguous stage accesses free of
// bank conflicts.
//
// Twiddles. LDS-tile kernels: products of two table entries in LDS (stage:
// exp(s 2 pi i y / 1024) = A[y mod 32] * B[y / 32]; pass: per column
// GA[l mod 32] * GB[l / 32]). Register-tile kernels: butterfly twiddles of
// the 8- and 16-point DFTs are compile-time constants, the inter-stage
// twiddles are powers of one per-thread root, and the pass twiddle is the
// product of a per-pass column table and a per-tile table. The exponents
// (k_rest * l) are always reduced exactly in integers before an angle is
// formed; every table entry and root is one FP64 sincospi call or a
// product of such entries, and FP32 states round the FP64 values. The
// device code of the LDS-tile kernels lives in fft_dev.h (shared with the
// batched kernel).
#include "fft_dev.h"

#include <cstdlib>

namespace qs {
namespace {

using namespace fftdev;

constexpr unsigned kXcds = 8;   // XCDs of an MI355X

// 512 threads per workgroup; complex128 stages stop at radix 8 so that
// two 512-thread workgroups fit a CU's registers.
template <typename R> struct FftThreads { static constexpr int value = 512; };
template <typename R> struct FftRho { static constexpr int value = 3; };
template <> struct FftRho<float> { static constexpr int value = 4; };

// One workgroup per tile. Workgroups are dispatched round-robin over the 8
// XCDs (each with its own L2), while consecutive tiles share cache lines
// when a tile's columns span less than a line; the block -> tile map hands
// consecutive tiles to consecutive workgroups of the same XCD, so both
// halves of a line are read through one L2 at about the same time.
template <typename R, int NT = FftThreads<R>::value>
__global__ __launch_bounds__(NT) void k_fft_pass(const typename V2<R>::T *__restrict__ src,
                                                 typename V2<R>::T *__restrict__ dst, PassArgs pa)
{
    extern __shared__ unsigned char lds_raw[];
    const unsigned b = blockIdx.x, g = gridDim.x;
    const uint64_t tile = (g % kXcds) ? b : uint64_t(b % kXcds) * (g / kXcds) + b / kXcds;
    fft_tile<R, NT, FftRho<R>::value>(src, dst, pa, tile, lds_raw);
}

// Streaming pass: 512 threads, at most V tile elements per thread (the
// largest tile, 2^10 x 8 complex128 or 2^10 x 16 complex64, is 16 x 512 or
// 32 x 512 elements). Workgroup b owns tiles [b*per_wg, (b+1)*per_wg).
// Complex128 stages stop at radix 8 so that the prefetched tile and the
// stage registers fit the register file without spills.
constexpr int kStreamNT = 512;
template <typename R> struct StreamV { static constexpr int value = 16; };
template <> struct StreamV<float> { static constexpr int value = 32; };
template <typename R> struct StreamRho { static constexpr int value = 3; };
template <> struct StreamRho<float> { static constexpr int value = 4; };

template <typename R>
__global__ __launch_bounds__(kStreamNT) void k_fft_stream(const typename V2<R>::T *__restrict__ src,
                                                          typename V2<R>::T *__restrict__ dst, PassArgs pa,
                                                          uint64_t per_wg)
{
    using C2 = typename V2<R>::T;
    constexpr int NT = kStreamNT, V = StreamV<R>::value;
    extern __shared__ unsigned char lds_raw[];
    const uint64_t t0 = uint64_t(blockIdx.x) * per_wg;
    const uint64_t t1 = t0 + per_wg < pa.tiles ? t0 + per_wg : pa.tiles;
    if (t0 >= t1) return;
    const int L = 1 << pa.r, E = L << pa.cb;
    const TileLds<C2> T(lds_raw, pa.r, pa.cb);
    const TileThread th(pa, NT);
    // the thread's elements: column c0, digit values l0 + i*lstep, so the
    // source index is base + off0 + i*step (disjoint bit fields)
    const uint64_t off0 = tile_colbits(pa, th.c0) | (uint64_t(th.l0) << pa.dig_lo);
    const uint64_t step = uint64_t(th.lstep) << pa.dig_lo;
    tile_index_tables<NT>(pa, T.row, T.dbits);
    C2 pre[V];
    auto fetch = [&](uint64_t t) {
        const C2 *s0 = src + (tile_base(pa, t) | off0);
#pragma unroll
        for (int i = 0; i < V; ++i)
            if (int(threadIdx.x) + i * NT < E) pre[i] = s0[uint64_t(i) * step];
    };
    fetch(t0);
    for (uint64_t t = t0; t < t1; ++t) {
        const uint64_t base = tile_base(pa, t);
#pragma unroll
        for (int i = 0; i < V; ++i)
            if (int(threadIdx.x) + i * NT < E) T.tile[phys(th.c0, th.l0 + i * th.lstep, T.S)] = pre[i];
        tile_tables<R, NT>(pa, base, T);
        __syncthreads();
        if (t + 1 < t1) fetch(t + 1);   // in flight during the stages and the store
        tile_stages<R, NT, StreamRho<R>::value>(pa, T);
        tile_store<R, NT>(dst, pa, base, T, th);
        __syncthreads();
    }
}

// A register copy the compiler cannot coalesce: the destination is an
// early-clobber operand, so it never shares the source's registers.
__device__ __forceinline__ double2 copy_reg(double2 x)
{
    double2 r;
    asm("v_mov_b64 %0, %1" : "=&v"(r.x) : "v"(x.x));
    asm("v_mov_b64 %0, %1" : "=&v"(r.y) : "v"(x.y));
    return r;
}
__device__ __forceinline__ float2 copy_reg(float2 x)
{
    float2 r;
    asm("v_mov_b32 %0, %1" : "=&v"(r.x) : "v"(x.x));
    asm("v_mov_b32 %0, %1" : "=&v"(r.y) : "v"(x.y));
    return r;
}

// Register-tile passes for 10-bit digits. A tile is the 1024 digit values
// of C columns, C amplitudes of 128 bytes in all, so every global access of
// the tile runs over whole 128-byte lines (the LDS-tile kernel above reaches
// only 64-byte runs with 10-bit digits). The tile lives in registers:
// thread t holds column c = t mod C at the 16 digit values j + 64 i
// (j = t / C, i = 0..15). The 1024-point DFT is split 16 x 64:
//   X[k1 + 16 k2] = sum_j w64^(j k2) [ w1024^(j k1) sum_i x[j + 64 i] w16^(i k1) ]
// The inner 16-point DFT and its twiddle are register work; the 64-point
// DFTs over j (8 x 8, again decimation in frequency) exchange the values
// through LDS, one half of the k1 values at a time (k_fft_reg, two
// workgroups per CU) or the whole tile at once (k_fft_reg_stream). Output
// digit k1 + 16 k2 gets the pass twiddle and is stored in the digit's place,
// or at its reversed-digit destination on a final pass.
//
// Memory ordering in the persistent kernels: the vector-memory counter
// counts loads and stores together and completes in order, so any global
// load issued inside the tile loop after a tile's stores would make its
// consumer wait for those stores. The loop therefore issues exactly one
// batch of global loads per tile (the next tile's values, right at the top)
// and reads every twiddle root from LDS tables built once per workgroup.
constexpr int kRegCols128 = 8;    // complex128: 8 columns of 16 bytes
constexpr int kRegCols64 = 16;    // complex64: 16 columns of 8 bytes
template <typename R> struct RegCols { static constexpr int value = kRegCols128; };
template <> struct RegCols<float> { static constexpr int value = kRegCols64; };

// Natural-order forward DFT (exp(+2 pi i k l / RAD)) of RAD = 8 or 16
// register values: radix-2 decimation in frequency with the butterfly
// twiddles exp(2 pi i u / 16) as compile-time constants (u = 4: a swap;
// u = 2, 6: one multiplication by sqrt(1/2)), then a compile-time bit
// reversal of the register names.
template <typename C2, int U>
__device__ __forceinline__ C2 tw16(C2 d)
{
    using R = decltype(d.x);
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
    if constexpr (U == 0) return d;
    else if constexpr (U == 4) return C2{-d.y, d.x};
    else if constexpr (U == 2) return C2{R(h) * (d.x - d.y), R(h) * (d.x + d.y)};
    else if constexpr (U == 6) return C2{R(-h) * (d.x + d.y), R(h) * (d.x - d.y)};
    else {
        constexpr double cs = U == 1 ? c1 : U == 3 ? s1 : U == 5 ? -s1 : -c1;
        constexpr double sn = U == 1 ? s1 : U == 3 ? c1 : U == 5 ? c1 : s1;
        return C2{R(cs) * d.x - R(sn) * d.y, R(cs) * d.y + R(sn) * d.x};
    }
}

template <typename C2, int RAD, int H, int J>
__device__ __forceinline__ void dft_level_j(C2 (&v)[RAD])
{
    if constexpr (J < H) {
#pragma unroll
        for (int b = 0; b < RAD; b += 2 * H) {
            const C2 a = v[b + J], c = v[b + J + H];
            v[b + J] = C2{a.x + c.x, a.y + c.y};
            v[b + J + H] = tw16<C2, J * (8 / H)>(C2{a.x - c.x, a.y - c.y});
        }
        dft_level_j<C2, RAD, H, J + 1>(v);
    }
}

template <typename C2, int RAD, int H = RAD / 2>
__device__ __forceinline__ void dft_fwd(C2 (&v)[RAD])
{
    if constexpr (H >= 1) {
        dft_level_j<C2, RAD, H, 0>(v);
        dft_fwd<C2, RAD, H / 2>(v);
    } else {
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
}

// LDS slot of (k1 within the round, column, j); j's bit 0 is flipped by
// bit 3 so that the three access shapes (rows j, j + 1; stride-8 reads in
// both exchange steps) fall on distinct banks.
template <int C>
__device__ __forceinline__ int reg_slot(int q, int c, int j)
{
    return ((q << 6) + (j ^ ((j >> 3) & 1))) * C + c;
}

// The pass twiddle exp(2 pi i k_rest L / 2^tw) of output digit L in column
// c factors into a column part (k_rest bits that are column bits: the same
// for every tile of the pass) and a tile part (k_rest bits of the tile
// base), each split by L = l + 32 h into two 32-entry tables.
template <typename R, int C>
struct RegLds {
    using C2 = typename V2<R>::T;
    C2 *xs;         // exchange area [kq][rows][C]
    C2 *gac, *gbc;  // [C][32]: column part at l and at 32 h
    C2 *gat, *gbt;  // [32]: tile part at l and at 32 h
    C2 *roots;      // LDS root tables (persistent kernels) or nullptr
    __device__ RegLds(C2 *tables, C2 *x, C2 *rt = nullptr) : xs(x), roots(rt)
    {
        gac = tables;
        gbc = gac + 32 * C;
        gat = gbc + 32 * C;
        gbt = gat + 32;
    }
    // pass twiddle at L0 and the factor for L0 -> L0 + 128
    __device__ __forceinline__ void twiddle(int c, int L0, C2 &g0, C2 &g128) const
    {
        g0 = cmul(gac[c * 32 + (L0 & 31)], gat[L0 & 31]);
        if (L0 >> 5) g0 = cmul(g0, cmul(gbc[c * 32 + (L0 >> 5)], gbt[L0 >> 5]));
        g128 = cmul(gbc[c * 32 + 4], gbt[4]);
    }
};

inline size_t reg_table_bytes(int C, size_t amp) { return amp * (64 * size_t(C) + 64); }
inline size_t reg_lds_bytes(int kq, int C, size_t amp) { return amp * size_t(kq) * 64 * C + reg_table_bytes(C, amp); }

// Root tables of a pass with pass-twiddle width tw: level k holds
// exp(2 pi i x 2^(12k) / 2^tw) for x < 4096 (k = 0, 1, 2), so any
// exp(2 pi i e / 2^tw) with e < 2^36 is the product of three entries. One
// FP64 sincospi per entry, rounded for complex64.
constexpr int kRootBits = 12, kRootLevels = 3;
template <typename R>
__global__ void k_root_tables(typename V2<R>::T *__restrict__ T, int tw)
{
    using C2 = typename V2<R>::T;
    const int u = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (u >= kRootLevels << kRootBits) return;
    const int k = u >> kRootBits, x = u & ((1 << kRootBits) - 1);
    const int sh = kRootBits * k;
    const uint64_t e = sh >= tw ? 0 : (uint64_t(x) << sh) & ((1ull << tw) - 1);
    T[u] = unit_root<C2, R>(e, tw, 1);
}

template <typename C2>
__device__ __forceinline__ C2 root_from_tables(const C2 *__restrict__ T, uint64_t e, int tw)
{
    C2 r = T[e & ((1u << kRootBits) - 1)];
    if (tw > kRootBits) r = cmul(r, T[(1 << kRootBits) + ((e >> kRootBits) & ((1u << kRootBits) - 1))]);
    if (tw > 2 * kRootBits) r = cmul(r, T[(2 << kRootBits) + ((e >> (2 * kRootBits)) & ((1u << kRootBits) - 1))]);
    return r;
}

// LDS root tables of the persistent kernels: level k holds
// exp(2 pi i x 2^(8k) / 2^tw) for x < 256 (k < 5, so e < 2^40), 20 KB for
// complex128. Reading them inside the tile loop uses the LDS counter, not
// the vector-memory counter that the tile's loads and stores share.
constexpr int kLRootBits = 8, kLRootLevels = 5;
inline size_t lroot_bytes(size_t amp) { return amp * (size_t(kLRootLevels) << kLRootBits); }

template <typename R, int NT>
__device__ void lroots_init(typename V2<R>::T *rt, int tw)
{
    using C2 = typename V2<R>::T;
    for (int u = int(threadIdx.x); u < (kLRootLevels << kLRootBits); u += NT) {
        const int sh = kLRootBits * (u >> kLRootBits), x = u & ((1 << kLRootBits) - 1);
        const uint64_t e = sh >= tw ? 0 : (uint64_t(x) << sh) & ((1ull << tw) - 1);
        rt[u] = unit_root<C2, R>(e, tw, 1);
    }
}

template <typename C2>
__device__ __forceinline__ C2 lroot(const C2 *rt, uint64_t e, int tw)
{
    C2 r = rt[e & ((1u << kLRootBits) - 1)];
#pragma unroll
    for (int k = 1; k < kLRootLevels; ++k)
        if (kLRootBits * k < tw) r = cmul(r, rt[(k << kLRootBits) + ((e >> (kLRootBits * k)) & ((1u << kLRootBits) - 1))]);
    return r;
}

// Pass twiddle tables, for the forward sign (an inverse pass conjugates its
// values on entry and exit), from the root tables (no sincospi near the
// tile loop, whose registers it would raise). Column part once per
// workgroup, tile part per tile (64 entries); the caller places a barrier
// before they are read.
template <typename R, int C, int NT, bool LDS_ROOTS>
__device__ void reg_col_tables(const PassArgs &pa, const RegLds<R, C> &T, const typename V2<R>::T *__restrict__ roots)
{
    if (!pa.tw_bits) return;
    const uint64_t kmask = (1ull << pa.krest_bits) - 1, mask = (1ull << pa.tw_bits) - 1;
    for (int w = int(threadIdx.x); w < 64 * C; w += NT) {
        const int c = w >> 6, j = w & 31, hi = (w >> 5) & 1;
        const uint64_t kr = (tile_colbits(pa, c) >> pa.krest_lo) & kmask;
        const uint64_t e = (kr * (uint64_t(j) << (hi ? 5 : 0))) & mask;
        (hi ? T.gbc : T.gac)[c * 32 + j] = LDS_ROOTS ? lroot(roots, e, pa.tw_bits) : root_from_tables(roots, e, pa.tw_bits);
    }
}

// Tile part from the LDS roots (persistent kernels): thread w < 64 writes
// entry w; the caller places it between two barriers of the tile.
template <typename R, int C>
__device__ __forceinline__ void reg_tile_tables_lds(const PassArgs &pa, uint64_t base, const RegLds<R, C> &T,
                                                    int w)
{
    if (pa.tw_bits && w < 64) {
        const int j = w & 31, hi = w >> 5;
        const uint64_t kr = (base >> pa.krest_lo) & ((1ull << pa.krest_bits) - 1);
        const uint64_t e = (kr * (uint64_t(j) << (hi ? 5 : 0))) & ((1ull << pa.tw_bits) - 1);
        (hi ? T.gbt : T.gat)[j] = lroot(T.roots, e, pa.tw_bits);
    }
}

// Tile part of the pass twiddle: thread w < 64 forms entry w (l = w mod 32
// at 32^(w / 32)) as the product of up to three root-table entries. The
// loads are issued at the top of a tile and the product is formed only
// after the first exchange step: the vector-memory counter also counts
// stores and completes in order, so consuming the loads right away would
// wait for the previous tile's stores and for the next tile's prefetch.
template <typename R>
struct TileRoot {
    using C2 = typename V2<R>::T;
    C2 a{1, 0}, b{1, 0}, c{1, 0};
    __device__ __forceinline__ void load(const PassArgs &pa, uint64_t base, const C2 *__restrict__ roots)
    {
        const int w = int(threadIdx.x);
        if (pa.tw_bits && w < 64) {
            const int j = w & 31, hi = w >> 5;
            const uint64_t kr = (base >> pa.krest_lo) & ((1ull << pa.krest_bits) - 1);
            const uint64_t e = (kr * (uint64_t(j) << (hi ? 5 : 0))) & ((1ull << pa.tw_bits) - 1);
            constexpr uint64_t m = (1u << kRootBits) - 1;
            a = roots[e & m];
            if (pa.tw_bits > kRootBits) b = roots[(1 << kRootBits) + ((e >> kRootBits) & m)];
            if (pa.tw_bits > 2 * kRootBits) c = roots[(2 << kRootBits) + ((e >> (2 * kRootBits)) & m)];
        }
    }
    template <int C>
    __device__ __forceinline__ void store(const PassArgs &pa, const RegLds<R, C> &T) const
    {
        const int w = int(threadIdx.x);
        if (pa.tw_bits && w < 64) (w < 32 ? T.gat : T.gbt)[w & 31] = cmul(cmul(a, b), c);
    }
};

// Load the thread's 16 values of a tile (plain loads: the register-tile
// passes ignore the cache-policy option).
template <typename R, int C>
__device__ __forceinline__ void reg_load(typename V2<R>::T (&v)[16], const typename V2<R>::T *__restrict__ src,
                                         const PassArgs &pa, uint64_t base, int t)
{
    const int c = t % C, j = t / C;
    const typename V2<R>::T *s0 = src + (base | tile_colbits(pa, c));
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = s0[uint64_t(j + 64 * i) << pa.dig_lo];
}

// x * w^k for k = 1..K-1 given w: the powers are formed from w, w^2, w^4,
// w^8 (repeated squaring) and products of those, a few roundings each, so
// no twiddle table entry has to be read (and held) per value.
// The root is routed through an empty asm statement that also reads v[0],
// so the powers are formed where they are used: without it the compiler
// computes them early (or once outside a tile loop) and keeps all of them
// live across the whole transform, which makes the kernels spill.
template <typename C2, int K>
__device__ __forceinline__ void apply_powers(C2 (&v)[K], C2 w, int first = 1)
{
    asm volatile("" : "+v"(w.x), "+v"(w.y) : "v"(v[0].x));
    const C2 w2 = cmul(w, w), w4 = cmul(w2, w2);
    C2 w8 = w4;
    if constexpr (K > 8) w8 = cmul(w4, w4);
#pragma unroll
    for (int k = 1; k < K; ++k) {
        if (k < first) continue;
        C2 p = (k & 1) ? w : ((k & 2) ? w2 : ((k & 4) ? w4 : w8));
        const int rest = k & (k - 1);   // k without its lowest set bit
        if (rest & 2) p = cmul(p, w2);
        if (rest & 4) p = cmul(p, w4);
        if (rest & 8) p = cmul(p, w8);
        v[k] = cmul(v[k], p);
    }
}

// Per-thread roots: exp(2 pi i j / 1024) and exp(2 pi i (j mod 8) / 64)
// for the thread's j = t / C.
template <typename R, int C>
struct RegRoots {
    using C2 = typename V2<R>::T;
    C2 wj, w64;
    __device__ RegRoots()
    {
        const int j = int(threadIdx.x) / C;
        wj = unit_root<C2, R>(uint64_t(j), kRmax, 1);
        w64 = unit_root<C2, R>(uint64_t(j & 7), 6, 1);
    }
};

// Transform and store one tile whose values are in v (the tile's pass
// twiddle tables are written here). The 16-point DFT starts with its first
// decimation-in-frequency level, which splits it into an 8-point DFT of the
// sums (even k1) and one of the twiddled differences (odd k1); the two
// halves then go through the exchange one after the other (KQ = 8, two
// rounds, half the tile in LDS) or together (KQ = 16, one round), so only
// half the tile is in flight in registers at a time. LDS slot q of a round
// holds k1 = 2q + h (KQ = 8) or k1 = q (KQ = 16). Leaves the LDS in use:
// the caller places a barrier before writing it again.
template <typename R, int C, int KQ>
__device__ __forceinline__ void reg_tile(typename V2<R>::T (&v)[16], typename V2<R>::T *__restrict__ dst,
                                         const PassArgs &pa, uint64_t base, const RegLds<R, C> &T,
                                         const RegRoots<R, C> &W, int dsh, const TileRoot<R> *troot, int t,
                                         bool lead_barrier = false)
{
    using C2 = typename V2<R>::T;
    constexpr int NT = 64 * C, ROUNDS = 16 / KQ, ITEMS = KQ * 8 * C;
    const int c = t % C, j = t / C;
    const bool inv = pa.sgn < 0;
    if (inv) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i].y = -v[i].y;
    }
    // first level: sums stay in v[0..7], differences times w16^i go to v[8..15]
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const C2 a = v[i], b = v[i + 8];
        v[i] = C2{a.x + b.x, a.y + b.y};
        v[i + 8] = C2{a.x - b.x, a.y - b.y};
    }
    v[9] = tw16<C2, 1>(v[9]);
    v[10] = tw16<C2, 2>(v[10]);
    v[11] = tw16<C2, 3>(v[11]);
    v[12] = tw16<C2, 4>(v[12]);
    v[13] = tw16<C2, 5>(v[13]);
    v[14] = tw16<C2, 6>(v[14]);
    v[15] = tw16<C2, 7>(v[15]);
    const C2 wj2 = cmul(W.wj, W.wj);
    const uint64_t xc = base | tile_colbits(pa, c);
    C2 *d0 = dst + (pa.final_pass ? final_dest(pa, xc) : xc);
    // half h: 8-point DFT -> k1 = 2m + h, times w1024^(j k1) = w^(j h) (w^(2j))^m
    auto half = [&](int h, C2 (&x)[8]) {
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = v[8 * h + m];
        dft_fwd<C2, 8>(x);
        if (h) {
#pragma unroll
            for (int m = 0; m < 8; ++m) x[m] = cmul(x[m], W.wj);
        }
        apply_powers<C2, 8>(x, wj2);
    };
    if (lead_barrier) __syncthreads();   // persistent use: the previous tile no longer reads the LDS
#pragma unroll
    for (int h = 0; h < ROUNDS; ++h) {
        if (h) __syncthreads();
        if constexpr (KQ == 8) {
            C2 x[8];
            half(h, x);
#pragma unroll
            for (int q = 0; q < 8; ++q) T.xs[reg_slot<C>(q, c, j)] = x[q];
        } else {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                C2 x[8];
                half(hh, x);
#pragma unroll
                for (int m = 0; m < 8; ++m) T.xs[reg_slot<C>(2 * m + hh, c, j)] = x[m];
            }
        }
        __syncthreads();
        // 8-point DFTs over a of the values j = jl + 8 a, then w64^(jl b);
        // every item of the thread has jl = j mod 8
#pragma unroll
        for (int k = 0; k < ITEMS / NT; ++k) {
            const int it = t + k * NT, jl = (it / C) & 7, q = it / (8 * C);
            C2 z[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) z[a] = T.xs[reg_slot<C>(q, c, jl + 8 * a)];
            dft_fwd<C2, 8>(z);
            apply_powers<C2, 8>(z, W.w64);
#pragma unroll
            for (int b = 0; b < 8; ++b) T.xs[reg_slot<C>(q, c, jl + 8 * b)] = z[b];
        }
        if (h == 0) {
            if (troot) troot->store(pa, T);
            else reg_tile_tables_lds<R, C>(pa, base, T, t);
        }
        __syncthreads();
        // 8-point DFTs over jl of the values jl + 8 b: output k2 = b + 8 e,
        // digit L = k1 + 16 b + 128 e; pass twiddle g(L0) g(128)^e
#pragma unroll
        for (int k = 0; k < ITEMS / NT; ++k) {
            const int it = t + k * NT, b = (it / C) & 7, q = it / (8 * C);
            C2 u[8];
#pragma unroll
            for (int jl = 0; jl < 8; ++jl) u[jl] = T.xs[reg_slot<C>(q, c, jl + 8 * b)];
            dft_fwd<C2, 8>(u);
            const int k1 = KQ == 8 ? 2 * q + h : q;
            const int L0 = k1 + 16 * b;
            if (pa.tw_bits) {
                C2 g0, g128;
                T.twiddle(c, L0, g0, g128);
#pragma unroll
                for (int e = 0; e < 8; ++e) u[e] = cmul(u[e], g0);
                apply_powers<C2, 8>(u, g128);
            }
            C2 *dp = d0 + (uint64_t(L0) << dsh);
            const uint64_t step = uint64_t(128) << dsh;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                C2 x = u[e];
                if (pa.scale != 1.0) x = C2{R(double(x.x) * pa.scale), R(double(x.y) * pa.scale)};
                if (inv) x.y = -x.y;
                dp[e * step] = x;
            }
        }
    }
}

// Position of the output digit's lowest bit in the destination index.
__device__ __forceinline__ int reg_dest_shift(const PassArgs &pa)
{
    return pa.final_pass ? __builtin_ctzll(final_dest(pa, 1ull << pa.dig_lo)) : pa.dig_lo;
}

// One workgroup per tile, half the tile exchanged per round (two
// workgroups share a CU), XCD-aware tile order as in k_fft_pass.
template <typename R, int C = RegCols<R>::value>
__global__ __launch_bounds__(64 * C, 4) void k_fft_reg(const typename V2<R>::T *__restrict__ src,
                                                      typename V2<R>::T *__restrict__ dst, PassArgs pa,
                                                      const typename V2<R>::T *__restrict__ roots)
{
    using C2 = typename V2<R>::T;
    extern __shared__ unsigned char lds_raw[];
    C2 *tabs = reinterpret_cast<C2 *>(lds_raw);
    const RegLds<R, C> T(tabs, tabs + 64 * C + 64);
    const unsigned b = blockIdx.x, g = gridDim.x;
    const uint64_t tile = (g % kXcds) ? b : uint64_t(b % kXcds) * (g / kXcds) + b / kXcds;
    const uint64_t base = tile_base(pa, tile);
    reg_col_tables<R, C, 64 * C, false>(pa, T, roots);
    const RegRoots<R, C> W;
    typename V2<R>::T v[16];
    reg_load<R, C>(v, src, pa, base, int(threadIdx.x));
    TileRoot<R> tr;
    tr.load(pa, base, roots);
    reg_tile<R, C, 8>(v, dst, pa, base, T, W, reg_dest_shift(pa), &tr, int(threadIdx.x));
}

// Persistent: one workgroup per CU walks tiles b', b' + G, ... (G = grid,
// b' the XCD-aware rank), with the next tile's values loaded into registers
// while the current one is transformed; the whole tile is exchanged at once.
template <typename R, int C = RegCols<R>::value>
__global__ __launch_bounds__(64 * C, 1) void k_fft_reg_stream(const typename V2<R>::T *__restrict__ src,
                                                             typename V2<R>::T *__restrict__ dst, PassArgs pa)
{
    using C2 = typename V2<R>::T;
    extern __shared__ unsigned char lds_raw[];
    C2 *tabs = reinterpret_cast<C2 *>(lds_raw);
    C2 *rt = tabs + 64 * C + 64;
    const RegLds<R, C> T(tabs, rt + (kLRootLevels << kLRootBits), rt);
    const unsigned b = blockIdx.x, g = gridDim.x;
    const uint64_t first = (g % kXcds) ? b : uint64_t(b % kXcds) * (g / kXcds) + b / kXcds;
    if (first >= pa.tiles) return;
    const int dsh = reg_dest_shift(pa);
    C2 p[16];
    reg_load<R, C>(p, src, pa, tile_base(pa, first), int(threadIdx.x));
    if (pa.tw_bits) lroots_init<R, 64 * C>(rt, pa.tw_bits);
    __syncthreads();
    reg_col_tables<R, C, 64 * C, true>(pa, T, rt);
    const RegRoots<R, C> W;
    auto body = [&](uint64_t tile) {
        int t = int(threadIdx.x);
        asm volatile("" : "+v"(t));   // keeps per-thread offsets from being hoisted out of the loop
        const uint64_t base = tile_base(pa, tile);
        // the tile's values move out of the prefetch registers (a real copy,
        // see k_fft_reg8_stream), then the next tile is requested at once
        C2 v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = copy_reg(p[i]);
        if (tile + g < pa.tiles) reg_load<R, C>(p, src, pa, tile_base(pa, tile + g), t);
        reg_tile<R, C, 16>(v, dst, pa, base, T, W, dsh, nullptr, t, true);
    };
    // The first tile is peeled so that every entry into the loop comes after
    // a tile's stores, as the back edge does: the compiler then waits for
    // the prefetched values alone at the top of a tile, not for the stores.
    body(first);
    for (uint64_t tile = first + g; tile < pa.tiles; tile += g) body(tile);
}

// Eight values per thread: the persistent kernel for complex128. A
// workgroup of 128 C threads (C = 8: 1024 threads, four waves per SIMD)
// holds one tile in registers, rows j + 128 i (i = 0..7) of column c for
// thread t = c + C j, and the next tile's values in flight behind it. The
// 1024-point DFT is split 8 x 128, the 128-point part 8 x 16:
//   X[k1 + 8 (b + 8 e)] = sum_jl w16^(jl e) w128^(jl b) sum_a w8^(a b)
//                         [ w1024^(j k1) sum_i x[j + 128 i] w8^(i k1) ]_(j = jl + 16 a)
// with one LDS exchange of the whole tile after the first 8-point DFT and
// one after the second. The last 16-point DFT is shared by two threads:
// its first decimation level gives the even e to one (sums) and the odd e
// to the other (differences), each then an 8-point DFT.
template <int C>
__device__ __forceinline__ int reg8_slot(int k1, int c, int j)
{
    return ((k1 << 7) + (j ^ ((j >> 4) & 1))) * C + c;
}

template <typename R, int C>
__device__ __forceinline__ void reg8_load(typename V2<R>::T (&v)[8], const typename V2<R>::T *__restrict__ src,
                                          const PassArgs &pa, uint64_t base, int t)
{
    const int c = t % C, j = t / C;
    const typename V2<R>::T *s0 = src + (base | tile_colbits(pa, c));
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = s0[uint64_t(j + 128 * i) << pa.dig_lo];
}

template <typename R, int C>
__global__ __launch_bounds__(128 * C) void k_fft_reg8_stream(const typename V2<R>::T *__restrict__ src,
                                                            typename V2<R>::T *__restrict__ dst, PassArgs pa)
{
    using C2 = typename V2<R>::T;
    constexpr int NT = 128 * C;
    extern __shared__ unsigned char lds_raw[];
    C2 *tabs = reinterpret_cast<C2 *>(lds_raw);
    C2 *rt = tabs + 64 * C + 64;
    const RegLds<R, C> T(tabs, rt + (kLRootLevels << kLRootBits), rt);
    C2 *xs = T.xs;   // [8][128][C]
    const unsigned blk = blockIdx.x, g = gridDim.x;
    const uint64_t first = (g % kXcds) ? blk : uint64_t(blk % kXcds) * (g / kXcds) + blk / kXcds;
    if (first >= pa.tiles) return;
    const bool inv = pa.sgn < 0;
    const int dsh = reg_dest_shift(pa);
    // per-thread roots: w1024^j (first twiddle), w128^jl for the B1 items
    // (jl = j mod 16), w16^jl is a constant per register. Per tile, the B1
    // item of the thread is (column c, jl = (t / C) mod 16, k1 = t / 16C)
    // and its B2 item (c, b = (t / C) mod 8, parity (t / 8C) mod 2, k1).
    const C2 wj = unit_root<C2, R>(uint64_t(threadIdx.x / C), kRmax, 1);
    const C2 w128 = unit_root<C2, R>(uint64_t((threadIdx.x / C) & 15), 7, 1);
    C2 p[8];
    reg8_load<R, C>(p, src, pa, tile_base(pa, first), int(threadIdx.x));
    if (pa.tw_bits) lroots_init<R, NT>(rt, pa.tw_bits);
    __syncthreads();
    reg_col_tables<R, C, NT, true>(pa, T, rt);
    auto body = [&](uint64_t tile) {
        // the thread's indices, opaque per tile: keeps the compiler from
        // hoisting every LDS and global offset out of the loop into live
        // registers
        int t = int(threadIdx.x);
        asm volatile("" : "+v"(t));
        const uint64_t base = tile_base(pa, tile);
        const int c = t % C, j = t / C;
        const int b2 = (t / C) & 7, par = (t / (8 * C)) & 1, k1b = t / (16 * C);
        const int jl1 = (t / C) & 15;
        // the tile's values move out of the prefetch registers (a real copy,
        // so the next tile can load into the same registers and the loop
        // carries no register shuffle that would wait for that load), then
        // the next tile is requested at once
        C2 v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = copy_reg(p[i]);
        if (tile + g < pa.tiles) reg8_load<R, C>(p, src, pa, tile_base(pa, tile + g), t);
        if (inv) {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i].y = -v[i].y;
        }
        dft_fwd<C2, 8>(v);
        apply_powers<C2, 8>(v, wj);
        __syncthreads();   // the previous tile no longer reads the LDS
#pragma unroll
        for (int k = 0; k < 8; ++k) xs[reg8_slot<C>(k, c, j)] = v[k];
        __syncthreads();
        {   // B1: 8-point DFT over a of j = jl + 16 a, times w128^(jl b)
            C2 z[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) z[a] = xs[reg8_slot<C>(k1b, c, jl1 + 16 * a)];
            dft_fwd<C2, 8>(z);
            apply_powers<C2, 8>(z, w128);
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) xs[reg8_slot<C>(k1b, c, jl1 + 16 * bb)] = z[bb];
        }
        reg_tile_tables_lds<R, C>(pa, base, T, t);
        __syncthreads();
        {   // B2: half of the 16-point DFT over jl of the values jl + 16 b
            C2 u[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const C2 x0 = xs[reg8_slot<C>(k1b, c, i + 16 * b2)];
                const C2 x1 = xs[reg8_slot<C>(k1b, c, i + 8 + 16 * b2)];
                u[i] = par ? C2{x0.x - x1.x, x0.y - x1.y} : C2{x0.x + x1.x, x0.y + x1.y};
            }
            if (par) {
                u[1] = tw16<C2, 1>(u[1]);
                u[2] = tw16<C2, 2>(u[2]);
                u[3] = tw16<C2, 3>(u[3]);
                u[4] = tw16<C2, 4>(u[4]);
                u[5] = tw16<C2, 5>(u[5]);
                u[6] = tw16<C2, 6>(u[6]);
                u[7] = tw16<C2, 7>(u[7]);
            }
            dft_fwd<C2, 8>(u);
            // output e = 2 m + par: digit L = k1 + 8 b + 64 par + 128 m
            const int L0 = k1b + 8 * b2 + 64 * par;
            if (pa.tw_bits) {
                C2 g0, g128;
                T.twiddle(c, L0, g0, g128);
#pragma unroll
                for (int m = 0; m < 8; ++m) u[m] = cmul(u[m], g0);
                apply_powers<C2, 8>(u, g128);
            }
            const uint64_t xc = base | tile_colbits(pa, c);
            C2 *dp = dst + (pa.final_pass ? final_dest(pa, xc) : xc) + (uint64_t(L0) << dsh);
            const uint64_t step = uint64_t(128) << dsh;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                C2 x = u[m];
                if (pa.scale != 1.0) x = C2{R(double(x.x) * pa.scale), R(double(x.y) * pa.scale)};
                if (inv) x.y = -x.y;
                dp[m * step] = x;
            }
        }
    };
    // The first tile is peeled so that every entry into the loop comes after
    // a tile's stores, as the back edge does: the compiler then waits for
    // the prefetched values alone at the top of a tile, not for the stores.
    body(first);
    for (uint64_t tile = first + g; tile < pa.tiles; tile += g) body(tile);
}

inline size_t reg8_lds_bytes(int C, size_t amp) { return amp * size_t(8) * 128 * C + reg_table_bytes(C, amp) + lroot_bytes(amp); }

// Pass shape: widest digit and LDS bytes per workgroup tile. Narrower digits
// mean more passes but longer contiguous runs per global access (the tile
// holds LDS/(2^r * amplitude) columns). Both come from the tuning table
// (per dtype and n bucket), else the widest digit and the full budget.
struct FftShape {
    int digit = kRmax;
    size_t lds = kLdsBytes;
};

FftShape fft_shape(int dtype, int n)
{
    FftShape s;
    const int nb = tune_nbucket(n);
    if (const int dg = tune_value(QS_TUNE_FFT_DIGIT, dtype, 0, 0, nb)) s.digit = std::min(kRmax, dg);
    if (const int kb = tune_value(QS_TUNE_FFT_LDS_KB, dtype, 0, 0, nb)) s.lds = std::min(kLdsMax, size_t(kb) * 1024);
    return s;
}

template <typename R>
int run_fft(qs_state *h, int q_lo, int m, int inverse)
{
    using C2 = typename V2<R>::T;
    const FftShape shape = fft_shape(h->dtype, h->n);
    // 1 LDS tile per workgroup, 2 streaming LDS tiles, 3 register tile per
    // workgroup, 4 persistent register tile (the default), 5 persistent
    // register tile with eight values per thread; passes whose digit is not
    // 10 bits wide take the LDS-tile kernel of option 1 or 2
    int kern = tune_value(QS_TUNE_FFT_KERNEL, h->dtype, 0, 0, tune_nbucket(h->n));
    if (kern == 0) kern = 4;
    const bool stream = kern == 2;
    const bool reg = kern == 3 || kern == 4 || kern == 5;
    constexpr int RC = RegCols<R>::value;
    constexpr int RC8 = 8;   // columns of the eight-value kernel (1024 threads)
    const int reg_cb = !reg ? -1 : (kern == 5 ? __builtin_ctz(RC8) : __builtin_ctz(RC));
    std::vector<PassArgs> passes;
    if (int rc = plan_passes(h->n, q_lo, m, inverse, shape.digit, shape.lds, sizeof(C2), passes,
                             stream ? StreamRho<R>::value : FftRho<R>::value, reg_cb))
        return rc;
    const int nt = tune_value(QS_TUNE_FFT_NT, h->dtype, 0, 0, tune_nbucket(h->n));
    for (auto &pa : passes) pa.nt = nt;
    const int P = int(passes.size());
    if (P > 1)
        if (int rc = ensure_scratch(h)) return rc;
    // With P > 1 the last passes alternate between the state and the scratch
    // buffer, an even number of them, so the last (which reverses the digits
    // and cannot run in place) writes the state itself; an odd leading pass
    // runs in place. Out-of-place passes are also faster than in-place ones
    // at the middle digit's stride, and no copy back is needed.
    const int k_oop = P > 1 ? (P & ~1) : 0;
    C2 *cur = static_cast<C2 *>(h->psi), *oth = static_cast<C2 *>(h->scratch);
    for (int j = 0; j < P; ++j) {
        const PassArgs &pa = passes[size_t(j)];
        const C2 *src = cur;
        C2 *dst = cur;
        if (j >= P - k_oop) {
            dst = oth;
            std::swap(cur, oth);
        }
        const size_t lds = pass_lds_bytes(pa, sizeof(C2));
        const uint64_t elems = uint64_t(1) << (pa.r + pa.cb);
        if (reg && pa.r == kRmax && pa.cb == reg_cb) {
            const C2 *roots = nullptr;
            if (pa.tw_bits && kern == 3) {
                if (!h->fft_roots)
                    QS_HIP(hipMalloc(&h->fft_roots, (size_t(kRootLevels) << kRootBits) * sizeof(double2)));
                roots = static_cast<const C2 *>(h->fft_roots);
                hipLaunchKernelGGL(k_root_tables<R>, dim3((kRootLevels << kRootBits) / 256), dim3(256), 0, h->stream,
                                   static_cast<C2 *>(h->fft_roots), pa.tw_bits);
            }
            if (kern == 5) {
                const uint64_t grid = std::min<uint64_t>(pa.tiles, uint64_t(device_cus()));
                hipLaunchKernelGGL((k_fft_reg8_stream<R, RC8>), dim3(unsigned(grid)), dim3(128 * RC8),
                                   reg8_lds_bytes(RC8, sizeof(C2)), h->stream, src, dst, pa);
            } else if (kern == 4) {
                const uint64_t grid = std::min<uint64_t>(pa.tiles, uint64_t(device_cus()));
                hipLaunchKernelGGL((k_fft_reg_stream<R, RC>), dim3(unsigned(grid)), dim3(64 * RC),
                                   reg_lds_bytes(16, RC, sizeof(C2)) + lroot_bytes(sizeof(C2)), h->stream, src, dst, pa);
            } else {
                if (pa.tiles > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "FFT tile count too large");
                hipLaunchKernelGGL((k_fft_reg<R, RC>), dim3(unsigned(pa.tiles)), dim3(64 * RC),
                                   reg_lds_bytes(8, RC, sizeof(C2)), h->stream, src, dst, pa, roots);
            }
        } else if (stream && elems <= uint64_t(kStreamNT) * StreamV<R>::value) {
            int per_cu = 0;
            QS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(k_fft_stream<R>), kStreamNT, lds));
            const uint64_t grid = std::min<uint64_t>(pa.tiles, uint64_t(std::max(per_cu, 1)) * device_cus());
            const uint64_t per_wg = (pa.tiles + grid - 1) / grid;
            const uint64_t used = (pa.tiles + per_wg - 1) / per_wg;
            hipLaunchKernelGGL(k_fft_stream<R>, dim3(unsigned(used)), dim3(kStreamNT), lds, h->stream, src, dst,
                               pa, per_wg);
        } else {
            if (pa.tiles > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "FFT tile count too large");
            hipLaunchKernelGGL(k_fft_pass<R>, dim3(unsigned(pa.tiles)), dim3(FftThreads<R>::value), lds,
                               h->stream, src, dst, pa);
        }
        QS_HIP(hipGetLastError());
    }
    return QS_OK;
}

}  // namespace

int emulate_qft(qs_state *h, int q_lo, int m, int inverse)
{
    static bool lds_ok = false;
    if (!lds_ok) {
        const int cap = int(kLdsMax);
        const void *fns[] = {reinterpret_cast<const void *>(k_fft_pass<double>),
                             reinterpret_cast<const void *>(k_fft_pass<float>),
                             reinterpret_cast<const void *>(k_fft_stream<double>),
                             reinterpret_cast<const void *>(k_fft_stream<float>),
                             reinterpret_cast<const void *>(k_fft_reg<double>),
                             reinterpret_cast<const void *>(k_fft_reg<float>),
                             reinterpret_cast<const void *>(k_fft_reg_stream<double>),
                             reinterpret_cast<const void *>(k_fft_reg_stream<float>),
                             reinterpret_cast<const void *>(k_fft_reg8_stream<double, 8>),
                             reinterpret_cast<const void *>(k_fft_reg8_stream<float, 8>)};
        for (const void *f : fns) QS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, cap));
        lds_ok = true;
    }
    return h->dtype == QS_C128 ? run_fft<double>(h, q_lo, m, inverse) : run_fft<float>(h, q_lo, m, inverse);
}

}  // namespace qs

extern "C" int qs_emulate_qft(qs_handle h, int q_lo, int m, int inverse)
{
    qs::clear_error();
    if (!h) return qs::fail(QS_EINVAL, "NULL handle");
    if (m < 1 || q_lo < 0 || q_lo + m > h->n)
        return qs::fail(QS_EINVAL, "QFT field [%d, %d) outside the %d-qubit state", q_lo, q_lo + m, h->n);
    return qs::emulate_qft(h, q_lo, m, inverse);
}
