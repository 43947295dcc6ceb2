// Fused 5- and 6-qubit blocks on complex64 states as a batched GEMM on the
// matrix cores. A sweep computes Y = M X for every group X of 2^k
// amplitudes that agree outside the block's qubits (the Kronecker structure
// of Sec. II). In real block form
//   [Yr]   [Mr  -Mi] [Xr]
//   [Yi] = [Mi   Mr] [Xi]
// a 6-qubit block is a 128 x 128 real matrix times 128 x G real columns,
// 8 flops per complex multiply-add and 32 flop per byte moved: past the
// FP32 vector ridge, so the FP32 MFMA units (FP32 inputs, FP32
// accumulation) carry it.
//
// Every kernel here: workgroups of 4 waves, persistent over tiles of 4096
// amplitudes (32 KiB). A tile spans index bits 0..5, the block qubits above
// bit 5 and the lowest free bits above 5 (12 bits in all), so loads and
// stores move runs of 64 consecutive amplitudes per wave instruction. Each
// wave keeps its slice of the block matrix in registers for the whole
// kernel.
//
// k_dense_mfma_3m (the default) forms Re Y = Mr Xr - Mi Xi and
// Im Y = (Mr + Mi)(Xr + Xi) - Mr Xr - Mi Xi from three real products
// (Gauss), 3/4 of the real block form's matrix-core work, on
// v_mfma_f32_16x16x4_f32. k_dense_mfma_pair runs the real block form on
// v_mfma_f32_32x32x2_f32. Both stage the tile once, as (re, im) pairs in a
// swizzled 32 KiB LDS layout with no bank conflicts; each wave owns the real
// and imaginary parts of 16 outputs, so its results leave as pairs. Four
// workgroups fit on a compute unit, and the next tile's loads go out as soon
// as a tile's outputs are staged.
//
// k_dense_mfma6 (QS_TUNE_MFMA_KERNEL = 1, 6-qubit blocks) is the first
// layout: it stages the tile in load order, regroups it into a second
// 32 KiB buffer in real form and owns real output rows [32w, 32w + 32) per
// wave (a 32 x 128 slice of the real block matrix in 64 VGPRs; A operand:
// lane l holds row l%32 at k = 2s + l/32; accumulator register v of lane l
// holds row 8(v/4) + 4(l/32) + v%4 and column l%32 of its 32 x 32 output
// block); 194 VGPRs and 64 KiB LDS leave room for two workgroups per compute
// unit, and the next tile is prefetched into registers during the k loop.
#include "qs_internal.h"

#include <algorithm>
#include <cstdlib>

namespace qs {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;

struct TileArgs {
    int nfix;
    int pos[40];           // tile bit positions (ascending), removed from the tile index
    uint64_t offl[64];     // global offset of load-layout register r (bits of the tile above 5)
    int lane_pos[6];       // compact position of each group bit
    int offc_even[32];     // compact offset of local index 2t (t < 32)
    int bit0_pos;          // compact position of local bit 0
};

template <typename IT, typename Args>
__device__ __forceinline__ IT expand_tile(IT g, const Args &ta)
{
    for (int i = 0; i < ta.nfix; ++i) {
        const int p = ta.pos[i];
        g = ((g >> p) << (p + 1)) | (g & ((IT(1) << p) - IT(1)));
    }
    return g;
}

__device__ __forceinline__ int slot(int p) { return p ^ ((p >> 5) & 31); }

template <typename IT>
__global__ __launch_bounds__(64 * kWaves, 2) void k_dense_mfma6(float2 *__restrict__ psi,
                                                             const float *__restrict__ mat,
                                                             IT n_tiles, TileArgs ta)
{
    // tile: the 4096 amplitudes in compact order (swizzled slots);
    // xb: the same tile in real form, xb[k * 64 + col], k < 128 (re rows
    // 0..63, im rows 64..127), so step s of the MFMA loop reads a constant
    // offset from one base address.
    __shared__ float2 tile[4096];
    __shared__ float xb[128 * 64];
    float *tf = reinterpret_cast<float *>(tile);
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = threadIdx.x & 63;
    const int hi = lane >> 5, lo = lane & 31;

    // A slice of the real block matrix: row i = 32 wave + lo, k = 2s + hi
    float a[64];
    {
        const int i = 32 * wave + lo;
        const int jr = i & 63;
        const bool iim = i >= 64;
#pragma unroll
        for (int s = 0; s < 64; ++s) {
            const int k = 2 * s + hi;
            const int jc = k & 63;
            const bool kim = k >= 64;
            const float mr = mat[2 * (jr * 64 + jc)], mi = mat[2 * (jr * 64 + jc) + 1];
            a[s] = iim ? (kim ? mr : mi) : (kim ? -mi : mr);
        }
    }
    // compact positions of this lane's two B columns (groups lo and 32 + lo)
    int colpos[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int col = 32 * h + lo;
        int p = 0;
#pragma unroll
        for (int b = 0; b < 6; ++b) p |= ((col >> b) & 1) << ta.lane_pos[b];
        colpos[h] = p;
    }

    // load layout: lane = bits 0..5, register r = 16 wave + q; the next
    // tile's amplitudes are fetched into registers while this one runs on
    // the matrix cores
    float2 pre[16];
    auto fetch = [&](IT tt) {
        const float2 *gs = psi + expand_tile<IT>(tt, ta) + lane;
#pragma unroll
        for (int q = 0; q < 16; ++q) pre[q] = gs[ta.offl[16 * wave + q]];
    };
    if (IT(blockIdx.x) < n_tiles) fetch(IT(blockIdx.x));
    for (IT t = IT(blockIdx.x); t < n_tiles; t += IT(gridDim.x)) {
        float2 *g = psi + expand_tile<IT>(t, ta) + lane;
#pragma unroll
        for (int q = 0; q < 16; ++q) tile[slot(lane + 64 * (16 * wave + q))] = pre[q];
        __syncthreads();
        // regroup into real form: thread -> (local index j, group col), lanes
        // take consecutive groups so the xb writes are conflict free
#pragma unroll 4
        for (int e = threadIdx.x; e < 4096; e += 64 * kWaves) {
            const int col = e & 63, j = e >> 6;
            int p = 0;
#pragma unroll
            for (int b = 0; b < 6; ++b) p |= ((col >> b) & 1) << ta.lane_pos[b];
            p |= ta.offc_even[j >> 1] | ((j & 1) << ta.bit0_pos);
            const float2 x = tile[slot(p)];
            xb[j * 64 + col] = x.x;
            xb[(j + 64) * 64 + col] = x.y;
        }
        __syncthreads();
        if (t + IT(gridDim.x) < n_tiles) fetch(t + IT(gridDim.x));   // each tile has one owner
        v16f acc[2] = {v16f{0}, v16f{0}};
        const float *bp = xb + hi * 64 + lo;
        // two independent accumulation chains (column halves) interleaved;
        // the scheduling barrier every 8 steps bounds how many B operands the
        // compiler prefetches into registers
#pragma unroll
        for (int s = 0; s < 64; ++s) {
            // B[k][col] with k = 2s + hi, col = 32h + lo
            const float b0 = bp[s * 128], b1 = bp[s * 128 + 32];
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b1, acc[1], 0, 0, 0);
            if ((s & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        // write Y back in place of X (compute layout)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 32 * wave + 8 * (v >> 2) + 4 * hi + (v & 3);
                const int j = i & 63;
                const int p = colpos[h] | ta.offc_even[j >> 1] | ((j & 1) << ta.bit0_pos);
                tf[2 * slot(p) + (i >> 6)] = acc[h][v];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = 16 * wave + q;
            g[ta.offl[r]] = tile[slot(lane + 64 * r)];
        }
        __syncthreads();
    }
}

// Pair layout. The tile is staged in LDS once, as (re, im) pairs at
// position (m << CB) | (col ^ sw(m)): m the block's local index (bit i of m
// is the i-th lowest block qubit), col the group (CB = 12 - k column bits).
// sw(m) puts the bits of m that come from block qubits below 6 back on those
// qubits' positions, so the load-layout element of lane l lands at
// (m << CB) | (l ^ c_r): every staging write and read moves 64 distinct bank
// pairs. Wave w owns the real and the imaginary output rows of m in
// [16 rb, 16 rb + 16) for the groups [64 ch, 64 ch + 64) (rb = w, ch = 0 for
// 6-qubit blocks; rb = w % 2, ch = w / 2 for 5-qubit blocks): local row
// i < 16 is Re y, i >= 16 is Im y of m = 16 rb + (i & 15). Step s = 2t + p of
// the k loop takes part p of input m = 2t + l/32, so one 8-byte LDS read
// feeds two steps, and accumulator registers v and v + 8 hold the real and
// imaginary parts of one output. The staging buffer is 32 KiB, which leaves
// room for three or four workgroups per compute unit.
struct PairArgs {
    int nfix;
    int pos[40];           // tile bit positions (ascending), removed from the tile index
    uint64_t offl[64];     // global offset of load-layout register r (tile bits above 5)
    uint32_t offr[64];     // LDS byte offset part of register r: ((m_r << 6) | c_r) * 8
    uint32_t sw[64];       // swizzle of local index m, in bytes (sw(m) * 8)
    int lane_m[6];         // local-index bit carried by lane bit b, or -1
    int upos[6];           // position in the caller's target list of local bit i
};

// PF: 0 loads each tile when it starts, 1 prefetches the next tile into
// registers during the k loop, 2 issues the next tile's loads after the
// outputs are staged (into the accumulators' registers, free by then).
template <typename IT, int K, int PF, int MINW>
__global__ __launch_bounds__(64 * kWaves, MINW) void k_dense_mfma_pair(float2 *__restrict__ psi,
                                                                      const float *__restrict__ mat,
                                                                      IT n_tiles, PairArgs pa)
{
    __shared__ float2 xs[4096];
    char *xb = reinterpret_cast<char *>(xs);
    auto lds = [&](int byte_off) -> float2 & { return *reinterpret_cast<float2 *>(xb + byte_off); };
    // M local indices, 4096 / M groups per tile: CB column bits; wave w owns
    // outputs [16 rb, 16 rb + 16) of the groups [64 ch, 64 ch + 64)
    constexpr int M = 1 << K, NT = M / 2, CB = 12 - K, NRB = M / 16;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = threadIdx.x & 63;
    const int hi = lane >> 5, lo = lane & 31;
    const int rb = wave % NRB, ch = wave / NRB;

    // A slice: output row i = lo of this wave, input (m = 2t + hi, part p)
    // at step s = 2t + p
    float a[2 * NT];
    {
        const int mo = 16 * rb + (lo & 15);
        const bool oim = lo >= 16;
        int uo = 0;
#pragma unroll
        for (int b = 0; b < K; ++b) uo |= ((mo >> b) & 1) << pa.upos[b];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int mi = 2 * t + hi;
            int ui = 0;
#pragma unroll
            for (int b = 0; b < K; ++b) ui |= ((mi >> b) & 1) << pa.upos[b];
            const float mr = mat[2 * (uo * M + ui)], mim = mat[2 * (uo * M + ui) + 1];
            a[2 * t] = oim ? mim : mr;         // input real part
            a[2 * t + 1] = oim ? mr : -mim;    // input imaginary part
        }
    }
    // byte offsets (8 bytes per pair); staging position of this lane in the
    // load layout: (m_l << CB) | l
    int ml = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if (pa.lane_m[b] >= 0) ml |= ((lane >> b) & 1) << pa.lane_m[b];
    const int base0 = ((ml << CB) | lane) << 3;
    // B reads: pair (m = 2t + hi, col = 64ch + 32h + lo); sw is linear in m,
    // so sw(2t + hi) = sw(2t) ^ sw(hi)
    const int bl0 = (((hi << CB) | (64 * ch + lo)) << 3) ^ int(pa.sw[hi]);
    // output writes: (m = 16rb + 8(v/4) + 4hi + v%4, col = 64ch + 32h + lo)
    const int ol0 = ((((4 * hi) << CB) | (64 * ch + lo)) << 3) ^ int(pa.sw[4 * hi]);

    // loaded amplitudes: pre (PF 0, 1) or, under PF 2, the accumulator
    // registers, which are free between the staging of one tile's outputs
    // and the next tile's k loop
    float2 pre[16];
    v16f acc[2] = {v16f{0}, v16f{0}};
    auto put = [&](int q, float2 x) {
        if (PF == 2) {
            acc[q >> 3][(2 * q) & 15] = x.x;
            acc[q >> 3][(2 * q + 1) & 15] = x.y;
        } else {
            pre[q] = x;
        }
    };
    auto got = [&](int q) -> float2 {
        if (PF == 2) return make_float2(acc[q >> 3][(2 * q) & 15], acc[q >> 3][(2 * q + 1) & 15]);
        return pre[q];
    };
    auto fetch = [&](IT tt) {
        const float2 *gs = psi + expand_tile<IT>(tt, pa) + lane;
#pragma unroll
        for (int q = 0; q < 16; ++q) put(q, gs[pa.offl[16 * wave + q]]);
    };
    if (PF && IT(blockIdx.x) < n_tiles) fetch(IT(blockIdx.x));
    for (IT t = IT(blockIdx.x); t < n_tiles; t += IT(gridDim.x)) {
        float2 *g = psi + expand_tile<IT>(t, pa) + lane;
        const bool more = t + IT(gridDim.x) < n_tiles;
        if (!PF) fetch(t);
        // the per-lane bases are made opaque once per tile, so the compiler
        // recomputes the staging addresses instead of holding 100 of them
        int base = base0, bl = bl0, ol = ol0;
        asm volatile("" : "+v"(base), "+v"(bl), "+v"(ol));
#pragma unroll
        for (int q = 0; q < 16; ++q) lds(base ^ int(pa.offr[16 * wave + q])) = got(q);
        __syncthreads();
        if (PF == 1 && more) fetch(t + IT(gridDim.x));   // each tile has one owner
        acc[0] = v16f{0};
        acc[1] = v16f{0};
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
            const int sx = int(pa.sw[2 * tt]);
            const float2 b0 = lds((tt << (CB + 4)) + (bl ^ sx));
            const float2 b1 = lds((tt << (CB + 4)) + ((bl ^ sx) ^ 256));
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2 * tt], b0.x, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2 * tt], b1.x, acc[1], 0, 0, 0);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2 * tt + 1], b0.y, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2 * tt + 1], b1.y, acc[1], 0, 0, 0);
            if ((tt & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int mu = 16 * rb + 8 * (v >> 2) + (v & 3);   // m without its lane bit 2
                lds((mu << (CB + 3)) + ((ol ^ int(pa.sw[mu])) ^ (256 * h))) = make_float2(acc[h][v], acc[h][v + 8]);
            }
        }
        if (PF == 2) {
            // keeps the loads after the staging writes, so the loaded
            // values can take the accumulators' registers
            __builtin_amdgcn_sched_barrier(0);
            if (more) fetch(t + IT(gridDim.x));
        }
        __syncthreads();
#pragma unroll
        // no barrier here: a wave reads back exactly the slots it fills with
        // the next tile, so the next staging writes race with no other wave
        for (int q = 0; q < 16; ++q) g[pa.offl[16 * wave + q]] = lds(base ^ int(pa.offr[16 * wave + q]));
    }
}

// Three-product form (Gauss): with T1 = Mr Xr, T2 = Mi Xi and
// T3 = (Mr + Mi)(Xr + Xi), Re Y = T1 - T2 and Im Y = T3 - T1 - T2: three real
// products of 2^K x 2^K blocks where the real block form needs four, so the
// matrix cores do 3/4 of the work. The tile is staged as in the pair layout
// (sw additionally toggles column bit 4 with bit 0 of m unless the lowest
// block qubit sits on bit 4, which keeps the 16-lane halves of every B read
// on distinct banks). v_mfma_f32_16x16x4_f32: wave w owns outputs
// [16 rb, 16 rb + 16) of the groups [64 ch, 64 ch + 64); lane l supplies A
// row l%16 and B column l%16 at k = 4s + l/16, and accumulator register v of
// lane l holds output row 4(l/16) + v. Each of the three products keeps four
// 16-column accumulators; one 8-byte LDS read gives Xr, Xi and, added,
// Xr + Xi for three MFMA steps. With W16 (qubit 0 not in the block) a lane
// moves two neighbouring amplitudes per global access, halving the vector
// memory instructions of a tile.
template <typename IT, int K, int MINW, bool W16>
__global__ __launch_bounds__(64 * kWaves, MINW) void k_dense_mfma_3m(float2 *__restrict__ psi,
                                                                   const float *__restrict__ mat, IT n_tiles,
                                                                   PairArgs pa, int lane_ef)
{
    __shared__ float2 xs[4096];
    char *xb = reinterpret_cast<char *>(xs);
    auto lds = [&](int byte_off) -> float2 & { return *reinterpret_cast<float2 *>(xb + byte_off); };
    constexpr int M = 1 << K, NS = M / 4, CB = 12 - K, NRB = M / 16;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int rb = wave % NRB, ch = wave / NRB;

    float a1[NS], a2[NS], a3[NS];
    {
        const int mo = 16 * rb + c;
        int uo = 0;
#pragma unroll
        for (int b = 0; b < K; ++b) uo |= ((mo >> b) & 1) << pa.upos[b];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int mi = 4 * s + g;
            int ui = 0;
#pragma unroll
            for (int b = 0; b < K; ++b) ui |= ((mi >> b) & 1) << pa.upos[b];
            const float mr = mat[2 * (uo * M + ui)], mim = mat[2 * (uo * M + ui) + 1];
            a1[s] = mr;
            a2[s] = mim;
            a3[s] = mr + mim;
        }
    }
    // W16: a lane moves two neighbouring amplitudes (16 bytes) of row
    // 16w + 2q + l/32 at positions pl, pl + 1; bit 0 is then no block qubit,
    // so the two share m and land in adjacent LDS slots
    // (offl and offr are linear in r, so row 2q + 1 adds offl[1] and
    // toggles offr[1]: folded into the lane's base address and slot)
    const int pl = W16 ? 2 * (lane & 31) : lane, hrow = W16 ? lane >> 5 : 0;
    int ml = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if (pa.lane_m[b] >= 0) ml |= ((pl >> b) & 1) << pa.lane_m[b];
    const int base0 = (((ml << CB) | (pl ^ (lane_ef ? (ml & 1) << 4 : 0))) << 3) ^ (hrow ? int(pa.offr[1]) : 0);
    const uint64_t hoff = hrow ? pa.offl[1] : 0;
    const int swg = ((g & 1) ? int(pa.sw[1]) : 0) ^ ((g & 2) ? int(pa.sw[2]) : 0);
    const int sw4g = ((g & 1) ? int(pa.sw[4]) : 0) ^ ((g & 2) ? int(pa.sw[8]) : 0);
    // B reads: pair (m = 4s + g, col = 64ch + 16cb + c)
    const int bl0 = (((g << CB) | (64 * ch + c)) << 3) ^ swg;
    // output writes: (m = 16rb + 4g + v, col = 64ch + 16cb + c)
    const int ol0 = ((((4 * g) << CB) | (64 * ch + c)) << 3) ^ sw4g;

    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f acc[3][4];
    // the next tile's amplitudes are loaded into the first 32 accumulator
    // registers once a tile's outputs are staged
    auto put = [&](int q, float2 x) {
        acc[q >> 3][(q >> 1) & 3][2 * (q & 1)] = x.x;
        acc[q >> 3][(q >> 1) & 3][2 * (q & 1) + 1] = x.y;
    };
    auto got = [&](int q) -> float2 {
        return make_float2(acc[q >> 3][(q >> 1) & 3][2 * (q & 1)], acc[q >> 3][(q >> 1) & 3][2 * (q & 1) + 1]);
    };
    auto put4 = [&](int q, float4 x) { acc[q >> 2][q & 3] = v4f{x.x, x.y, x.z, x.w}; };
    auto got4 = [&](int q) -> float4 {
        const v4f a = acc[q >> 2][q & 3];
        return make_float4(a[0], a[1], a[2], a[3]);
    };
    auto fetch = [&](IT tt) {
        const float2 *gs = psi + expand_tile<IT>(tt, pa) + pl + hoff;
        if constexpr (W16) {
#pragma unroll
            for (int q = 0; q < 8; ++q) put4(q, *reinterpret_cast<const float4 *>(gs + pa.offl[16 * wave + 2 * q]));
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) put(q, gs[pa.offl[16 * wave + q]]);
        }
    };
    if (IT(blockIdx.x) < n_tiles) fetch(IT(blockIdx.x));
    for (IT t = IT(blockIdx.x); t < n_tiles; t += IT(gridDim.x)) {
        float2 *gp = psi + expand_tile<IT>(t, pa) + pl + hoff;
        const bool more = t + IT(gridDim.x) < n_tiles;
        int base = base0, bl = bl0, ol = ol0;
        asm volatile("" : "+v"(base), "+v"(bl), "+v"(ol));
        if constexpr (W16) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                *reinterpret_cast<float4 *>(xb + (base ^ int(pa.offr[16 * wave + 2 * q]))) = got4(q);
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) lds(base ^ int(pa.offr[16 * wave + q])) = got(q);
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[p][cb] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int sx = int(pa.sw[4 * s]);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const float2 b = lds((s << (CB + 5)) + ((bl ^ sx) ^ (cb << 7)));
                acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], b.x, acc[0][cb], 0, 0, 0);
                acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[s], b.y, acc[1][cb], 0, 0, 0);
                acc[2][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[s], b.x + b.y, acc[2][cb], 0, 0, 0);
            }
            if ((s & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int mu = 16 * rb + v;   // m without its lane bits 2, 3
                const float t1 = acc[0][cb][v], t2 = acc[1][cb][v], t3 = acc[2][cb][v];
                lds((mu << (CB + 3)) + ((ol ^ int(pa.sw[mu])) ^ (cb << 7))) = make_float2(t1 - t2, t3 - t1 - t2);
            }
        }
        // loads after the staging writes, into the accumulators' registers
        __builtin_amdgcn_sched_barrier(0);
        if (more) fetch(t + IT(gridDim.x));
        __syncthreads();
        // no barrier after this: a wave reads back exactly the slots it
        // fills with the next tile
        if constexpr (W16) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                *reinterpret_cast<float4 *>(gp + pa.offl[16 * wave + 2 * q]) =
                    *reinterpret_cast<const float4 *>(xb + (base ^ int(pa.offr[16 * wave + 2 * q])));
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) gp[pa.offl[16 * wave + q]] = lds(base ^ int(pa.offr[16 * wave + q]));
        }
    }
}

template <typename IT>
int launch_t(qs_state *h, const GateDesc &d, const float *dmat)
{
    constexpr int K = 6;
    uint64_t tmask = 0;
    for (int i = 0; i < K; ++i) tmask |= 1ull << d.targets[i];
    int klo = 0;
    for (int i = 0; i < K; ++i) klo += d.targets[i] < 6;
    std::vector<int> extra;
    for (int b = 6; b < h->n && int(extra.size()) < klo; ++b)
        if (!((tmask >> b) & 1)) extra.push_back(b);
    std::vector<int> P = {0, 1, 2, 3, 4, 5};
    for (int i = 0; i < K; ++i)
        if (d.targets[i] >= 6) P.push_back(d.targets[i]);
    for (int b : extra) P.push_back(b);
    std::sort(P.begin(), P.end());
    auto compact = [&](int b) { return int(std::lower_bound(P.begin(), P.end(), b) - P.begin()); };
    TileArgs ta;
    ta.nfix = int(P.size());
    for (int i = 0; i < ta.nfix; ++i) ta.pos[i] = P[size_t(i)];
    for (int r = 0; r < 64; ++r) {
        uint64_t o = 0;
        for (int i = 0; i < K; ++i)
            if ((r >> i) & 1) o |= 1ull << P[size_t(6 + i)];
        ta.offl[r] = o;
    }
    std::vector<int> lane_bits;
    for (int b = 0; b < 6; ++b)
        if (!((tmask >> b) & 1)) lane_bits.push_back(b);
    for (int b : extra) lane_bits.push_back(b);
    for (int b = 0; b < 6; ++b) ta.lane_pos[b] = compact(lane_bits[size_t(b)]);
    auto offc = [&](int j) {
        int o = 0;
        for (int i = 0; i < K; ++i)
            if ((j >> i) & 1) o |= 1 << compact(d.targets[i]);
        return o;
    };
    for (int t = 0; t < 32; ++t) ta.offc_even[t] = offc(2 * t);
    ta.bit0_pos = compact(d.targets[0]);
    const IT n_tiles = IT(h->dim() >> 12);
    // persistent grid: tuned workgroups per CU (default 4)
    const int per_cu = tune_value(QS_TUNE_MFMA_WG_PER_CU, QS_C64, 6, 0, tune_nbucket(h->n));
    const uint64_t grid = std::min<uint64_t>(uint64_t(n_tiles), uint64_t(device_cus()) * uint64_t(per_cu ? per_cu : 4));
    hipLaunchKernelGGL((k_dense_mfma6<IT>), dim3(unsigned(grid)), dim3(64 * kWaves), 0, h->stream,
                       static_cast<float2 *>(h->psi), dmat, n_tiles, ta);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

template <typename IT, int K, int PF, int MINW>
int launch_pair_k(qs_state *h, const float *dmat, IT n_tiles, const PairArgs &pa)
{
    auto kern = k_dense_mfma_pair<IT, K, PF, MINW>;
    int resident = 0;
    QS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, reinterpret_cast<const void *>(kern), 64 * kWaves, 0));
    const int per_cu = tune_value(QS_TUNE_MFMA_WG_PER_CU, QS_C64, K, 0, tune_nbucket(h->n));
    const int wg = std::max(1, per_cu ? std::min(per_cu, resident) : resident);
    const uint64_t grid = std::min<uint64_t>(uint64_t(n_tiles), uint64_t(device_cus()) * uint64_t(wg));
    hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(64 * kWaves), 0, h->stream, static_cast<float2 *>(h->psi),
                       dmat, n_tiles, pa);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

template <typename IT, int K, int MINW, bool W16>
int launch_3m_k(qs_state *h, const float *dmat, IT n_tiles, const PairArgs &pa, int lane_ef)
{
    auto kern = k_dense_mfma_3m<IT, K, MINW, W16>;
    int resident = 0;
    QS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, reinterpret_cast<const void *>(kern), 64 * kWaves, 0));
    const int per_cu = tune_value(QS_TUNE_MFMA_WG_PER_CU, QS_C64, K, 0, tune_nbucket(h->n));
    const int wg = std::max(1, per_cu ? std::min(per_cu, resident) : resident);
    const uint64_t grid = std::min<uint64_t>(uint64_t(n_tiles), uint64_t(device_cus()) * uint64_t(wg));
    hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(64 * kWaves), 0, h->stream, static_cast<float2 *>(h->psi),
                       dmat, n_tiles, pa, lane_ef);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

template <typename IT, int K>
int launch_pair(qs_state *h, const GateDesc &d, const float *dmat, int variant)
{
    uint64_t tmask = 0;
    for (int i = 0; i < K; ++i) tmask |= 1ull << d.targets[i];
    std::vector<int> T(d.targets, d.targets + K);
    std::sort(T.begin(), T.end());
    int klo = 0;
    for (int i = 0; i < K; ++i) klo += T[size_t(i)] < 6;
    // the tile: bits 0..5, the block qubits above 5 and the lowest free bits
    // above 5, 12 bits in all; the free bits carry the groups' remaining
    // column bits (col bit T_i for the i-th of them while i < klo, then 6, 7)
    std::vector<int> extra;
    for (int b = 6; b < h->n && int(extra.size()) < 6 - (K - klo); ++b)
        if (!((tmask >> b) & 1)) extra.push_back(b);
    std::vector<int> P = {0, 1, 2, 3, 4, 5};
    for (int i = klo; i < K; ++i) P.push_back(T[size_t(i)]);
    for (int b : extra) P.push_back(b);
    std::sort(P.begin(), P.end());
    auto compact = [&](int b) { return int(std::lower_bound(P.begin(), P.end(), b) - P.begin()); };
    constexpr int CB = 12 - K;
    PairArgs pa;
    pa.nfix = int(P.size());
    for (int i = 0; i < pa.nfix; ++i) pa.pos[i] = P[size_t(i)];
    for (int i = 0; i < 6; ++i)
        pa.upos[i] = i < K ? int(std::find(d.targets, d.targets + K, T[size_t(i)]) - d.targets) : 0;
    for (int r = 0; r < 64; ++r) {
        uint64_t o = 0;
        for (int i = 0; i < 6; ++i)
            if ((r >> i) & 1) o |= 1ull << P[size_t(6 + i)];
        pa.offl[r] = o;
        uint32_t mr = 0, cr = 0;
        for (int i = klo; i < K; ++i) mr |= uint32_t((r >> (compact(T[size_t(i)]) - 6)) & 1) << i;
        for (int j = 0; j < int(extra.size()); ++j) {
            const int cpos = j < klo ? T[size_t(j)] : 6 + (j - klo);
            cr |= uint32_t((r >> (compact(extra[size_t(j)]) - 6)) & 1) << cpos;
        }
        pa.offr[r] = ((mr << CB) | cr) << 3;
    }
    // the three-product kernel's swizzle also toggles column bit 4 with bit 0
    // of m, unless the lowest block qubit is bit 4 itself
    const bool three = !(variant == 2 || variant == 3 || variant == 4);   // the switch below
    const bool ef = three && (klo == 0 || T[0] != 4);
    auto swz = [&](int m) {
        uint32_t sw = 0;
        for (int i = 0; i < klo; ++i) sw |= uint32_t((m >> i) & 1) << T[size_t(i)];
        if (ef) sw ^= uint32_t(m & 1) << 4;
        return sw;
    };
    for (int m = 0; m < 64; ++m) pa.sw[m] = swz(m) << 3;
    if (three)
        for (int r = 0; r < 64; ++r) {
            const uint32_t mr = (pa.offr[r] >> 3) >> CB;
            pa.offr[r] ^= swz(int(mr)) << 3;
        }
    for (int b = 0; b < 6; ++b) {
        pa.lane_m[b] = -1;
        for (int i = 0; i < klo; ++i)
            if (T[size_t(i)] == b) pa.lane_m[b] = i;
    }
    const IT n_tiles = IT(h->dim() >> 12);
    switch (variant) {
    case 2: return launch_pair_k<IT, K, 1, 3>(h, dmat, n_tiles, pa);
    case 3: return launch_pair_k<IT, K, 2, 4>(h, dmat, n_tiles, pa);
    case 4: return launch_pair_k<IT, K, 0, 4>(h, dmat, n_tiles, pa);
    case 6: return launch_3m_k<IT, K, 4, false>(h, dmat, n_tiles, pa, (klo >= 1 && T[0] != 4) ? 1 : 0);
    default:
        // 16-byte accesses unless bit 0 is a block qubit
        if (T[0] != 0) return launch_3m_k<IT, K, 4, true>(h, dmat, n_tiles, pa, (klo >= 1 && T[0] != 4) ? 1 : 0);
        return launch_3m_k<IT, K, 4, false>(h, dmat, n_tiles, pa, (klo >= 1 && T[0] != 4) ? 1 : 0);
    }
}

}  // namespace

bool mfma_applicable(const qs_state *h, const GateDesc &d)
{
    return h->dtype == QS_C64 && (d.k == 5 || d.k == 6) && d.ctrl_mask == 0 && h->n >= 12;
}

int launch_dense_mfma(qs_state *h, const GateDesc &d, const void *dmat)
{
    const float *m = static_cast<const float *>(dmat);
    const int variant = tune_value(QS_TUNE_MFMA_KERNEL, QS_C64, d.k, 0, tune_nbucket(h->n));
    if (d.k == 5)
        return h->n <= 31 ? launch_pair<uint32_t, 5>(h, d, m, variant) : launch_pair<uint64_t, 5>(h, d, m, variant);
    if (variant == 1) return h->n <= 31 ? launch_t<uint32_t>(h, d, m) : launch_t<uint64_t>(h, d, m);
    return h->n <= 31 ? launch_pair<uint32_t, 6>(h, d, m, variant) : launch_pair<uint64_t, 6>(h, d, m, variant);
}

}  // namespace qs
