// Many independent, uneven circuits in one persistent launch (complex64).
//
// Each circuit is a list of segments (a gate list, a QFT subroutine or a
// modular multiplication). A plan assigns every segment one option: fuse its
// gates into blocks of at most 2, 4 or 6 qubits, or emulate the subroutine
// (FFT for the QFT, Sec. III-B; a basis-state permutation for arithmetic,
// Sec. III-A). Planning turns each circuit into a list of ops; the persistent
// kernel then runs them.
//
// Scheduling: workgroups pop tickets from a queue ordered by estimated time
// per ticket (largest first). Circuits of at most 13 qubits (64 KiB of
// complex64) have one ticket: one workgroup keeps the state in LDS from the
// first op to the last and writes it to HBM once. A larger circuit is swept
// in HBM by a gang of G workgroups (G sized from the plan's cost estimate),
// one ticket per member: each op is split over the members, which meet at a
// cross-workgroup barrier (a monotonic arrival counter per circuit) between
// ops. A gang's tickets are consecutive in the queue, so only the most
// recently opened gang can be waiting for members, and any workgroup that
// finishes its work pops exactly those tickets next; with G no larger than
// the number of co-resident workgroups every gang completes. A second
// buffer serves the out-of-place ops (last FFT pass, permutation).
//
// Every segment's device time is taken with the constant-rate real-time
// counter at segment boundaries inside the kernel; these timings are what
// the learned cost model trains on.
#include "fft_dev.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>
#include <vector>

namespace {

using namespace qs;
using fftdev::PassArgs;

constexpr int kBT = 256;      // threads per workgroup
constexpr int kNS = 13;       // largest LDS-resident circuit (complex64)
constexpr size_t kLds = size_t(8) << kNS;  // 64 KiB
constexpr size_t kFftLds = kLds;           // FFT tile budget inside the batch kernel (its dynamic LDS)

enum OpType { OP_INIT = 0, OP_DENSE = 1, OP_DIAG = 2, OP_FFT_LDS = 3, OP_FFT_PASS = 4, OP_PERM = 5,
              OP_NORM = 6 };

struct BOp {
    int type;
    int k;
    int seg;            // global segment id (timing), -1 for bookkeeping ops
    int src, dst;       // 0: primary buffer, 1: second buffer (HBM circuits)
    int t[6];           // block qubits, ascending (local bit m = t[m])
    int64_t mat;        // offset in floats into the FP32 matrix pool
    int q_lo, m, inv;   // FFT field
    int pass;           // index into the pass table
    int mono;           // OP_DENSE: the block is a monomial (moves and phases), swept exactly on the ALUs
    int work_lo, w, ctrl_lo, c;
    uint32_t N, pad;
    uint64_t a, mu;
};

struct BCirc {
    int n, op0, op1, final_buf;
    uint64_t off_a, off_b;   // element offsets of the two buffers
    int gang;                // workgroups sweeping this circuit together
    int p0;                  // first slot of its norm partials
};

struct Ticket {
    int circ, member;
};

constexpr uint64_t kSpinTicks = 500000000ull;   // 5 s of the 100 MHz counter

// Cross-workgroup barrier of a gang of G workgroups. Every thread releases
// its stores at device scope (L2 write-back) and the workgroup meets; thread
// 0 arrives on the circuit's counter with a device-scope release and polls
// it with relaxed loads (an acquire per poll would invalidate the L2 of the
// XCD over and over) until all G members of this round have arrived; after
// the workgroup meets again every thread acquires once (L1/L2 invalidate).
// The counter only grows (round e completes at (e+1)*G arrivals), so it
// needs no reset between rounds. A wait longer than kSpinTicks sets the
// error flag; once it is set no barrier waits, so the kernel drains.
__device__ __forceinline__ void gang_sync(unsigned *bar, unsigned G, unsigned &epoch, unsigned *err)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = (epoch + 1u) * G;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            // after any timeout every barrier gives way at once
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (wall_clock64() - t0 > kSpinTicks) {
                atomicOr(err, 1u);
                break;
            }
        }
    }
    ++epoch;
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// ---------------------------------------------------------------------------
// device helpers (all executed by a whole workgroup; st may point to LDS or
// to global memory through the flat address space)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t deposit_zero(uint32_t g, const int *t, int k)
{
    for (int i = 0; i < k; ++i) {
        const int p = t[i];
        g = ((g >> p) << (p + 1)) | (g & ((1u << p) - 1u));
    }
    return g;
}

template <int D, int L0>
__device__ __forceinline__ void rchunk(const float *__restrict__ row, const float2 (&v)[D], float &re, float &im)
{
#pragma unroll
    for (int l = L0; l < L0 + (D < 8 ? D : 8); ++l) {
        const float mr = row[2 * l], mi = row[2 * l + 1];
        re = fmaf(mr, v[l].x, re);
        re = fmaf(-mi, v[l].y, re);
        im = fmaf(mr, v[l].y, im);
        im = fmaf(mi, v[l].x, im);
    }
}

template <int D>
__device__ __forceinline__ void rdot(const float *__restrict__ row, const float2 (&v)[D], float &re, float &im)
{
    if constexpr (D <= 8) {
        rchunk<D, 0>(row, v, re, im);
    } else {
#pragma unroll 1
        for (int c = 0; c < D / 8; ++c) {
            switch (c) {
            case 0: rchunk<D, 0>(row, v, re, im); break;
            case 1: rchunk<D, 8>(row, v, re, im); break;
            case 2: if constexpr (D > 16) rchunk<D, 16>(row, v, re, im); break;
            case 3: if constexpr (D > 16) rchunk<D, 24>(row, v, re, im); break;
            case 4: if constexpr (D > 32) rchunk<D, 32>(row, v, re, im); break;
            case 5: if constexpr (D > 32) rchunk<D, 40>(row, v, re, im); break;
            case 6: if constexpr (D > 32) rchunk<D, 48>(row, v, re, im); break;
            default: if constexpr (D > 32) rchunk<D, 56>(row, v, re, im); break;
            }
        }
    }
}

template <int K>
__device__ void op_dense(float2 *st, int n, const BOp &op, const float *__restrict__ mat, uint32_t r, uint32_t G)
{
    constexpr int D = 1 << K;
    // offset of local index j inside a group (uniform across the workgroup)
    auto off = [&](int j) {
        uint32_t o = 0;
#pragma unroll
        for (int m = 0; m < K; ++m)
            if ((j >> m) & 1) o |= 1u << op.t[m];
        return o;
    };
    const uint32_t groups = 1u << (n - K);
    for (uint32_t g = r * kBT + threadIdx.x; g < groups; g += G * kBT) {
        float2 *p = st + deposit_zero(g, op.t, K);
        float2 v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = p[off(j)];
#pragma unroll 1
        for (int j = 0; j < D; ++j) {
            float re = 0.f, im = 0.f;
            rdot<D>(mat + 2 * j * D, v, re, im);
            p[off(j)] = float2{re, im};
        }
    }
}

// Dense 4- to 6-qubit blocks on states in HBM (14 qubits or more) run on
// the FP32 matrix cores as three real products per complex product (blocks
// of moves and phases stay on the ALUs, whose one-term sums are exact):
// Re Y = Mr Xr - Mi Xi, Im Y = (Mr + Mi)(Xr + Xi) - Mr Xr - Mi Xi, over
// tiles of 4096 amplitudes (the block's qubits and the 12 - K lowest other
// bits, which number the C = 4096 / 2^K columns). A tile is staged in the
// dynamic LDS, m-major with rows of C + 16 pairs, so that the two 16-lane
// halves of every B read fall on distinct banks; outputs go straight back
// to HBM. Wave w owns outputs [16 rb, 16 rb + 16) of the columns
// [64 ch, 64 ch + 64), in two passes of 32 columns; v_mfma_f32_16x16x4_f32,
// lane l supplying A row l%16 and B column l%16 at k = 4s + l/16, and
// holding output rows 4(l/16) + v of its 16-column block.
__device__ __forceinline__ uint32_t pdep_bits(uint32_t x, uint32_t mask, int nbits)
{
    uint32_t o = 0;
    for (int i = 0; i < nbits; ++i) {
        const uint32_t low = mask & (0u - mask);
        if ((x >> i) & 1u) o |= low;
        mask ^= low;
    }
    return o;
}

template <int K>
__device__ void op_dense_mfma(float2 *st, int n, const BOp &op, const float *__restrict__ mat, uint32_t r,
                              uint32_t G, float2 *xs)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    constexpr int M = 1 << K, NS = M / 4, C = 4096 / M, NRB = M / 16, PAD = C + 16, NF = 12 - K;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int rb = wave % NRB, ch = wave / NRB;
    uint32_t tmask = 0;
#pragma unroll
    for (int m = 0; m < K; ++m) tmask |= 1u << op.t[m];
    uint32_t fmask = 0;                       // the NF lowest bits outside the block
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const uint32_t x = tmask | fmask;
        fmask |= ~x & (x + 1u);
    }
    const uint32_t tile_mask = tmask | fmask;
    auto mbits = [&](int m) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) o |= uint32_t((m >> i) & 1) << op.t[i];
        return o;
    };
    float a1[NS], a2[NS], a3[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int idx = 2 * ((16 * rb + c) * M + 4 * s + g);
        a1[s] = mat[idx];
        a2[s] = mat[idx + 1];
        a3[s] = a1[s] + a2[s];
    }
    const uint32_t mg4 = mbits(4 * g);
    // staging: thread tid takes column tid % C of rows tid / C + (256 / C) q
    const uint32_t scol = threadIdx.x % C, srow = threadIdx.x / C, scoff = pdep_bits(scol, fmask, NF);
    const uint32_t n_tiles = 1u << (n - 12);
    for (uint32_t tt = r; tt < n_tiles; tt += G) {
        uint32_t tb = tt;
        for (uint32_t msk = tile_mask; msk; msk &= msk - 1u) {
            const int p = __builtin_ctz(msk);
            tb = ((tb >> p) << (p + 1)) | (tb & ((1u << p) - 1u));
        }
#pragma unroll 4
        for (int q = 0; q < 4096 / kBT; ++q) {
            const int m = int(srow) + (kBT / C) * q;
            xs[m * PAD + int(scol)] = st[tb | scoff | mbits(m)];
        }
        __syncthreads();
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
            v4f acc[3][2];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[p][h] = v4f{0.f, 0.f, 0.f, 0.f};
            const int col0 = 64 * ch + 32 * half + c;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float2 b = xs[(4 * s + g) * PAD + col0 + 16 * h];
                    acc[0][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], b.x, acc[0][h], 0, 0, 0);
                    acc[1][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[s], b.y, acc[1][h], 0, 0, 0);
                    acc[2][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[s], b.x + b.y, acc[2][h], 0, 0, 0);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t co = tb | pdep_bits(uint32_t(col0 + 16 * h), fmask, NF) | mg4;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float t1 = acc[0][h][v], t2 = acc[1][h][v], t3 = acc[2][h][v];
                    st[co | mbits(16 * rb + v)] = float2{t1 - t2, t3 - t1 - t2};
                }
            }
        }
        __syncthreads();   // every wave is done with the staged tile
    }
}

__device__ void op_diag(float2 *st, int n, const BOp &op, const float *__restrict__ mat, uint32_t r, uint32_t G)
{
    const int D = 1 << op.k;
    for (uint32_t i = r * kBT + threadIdx.x; i < (1u << n); i += G * kBT) {
        int j = 0;
#pragma unroll
        for (int m = 0; m < 6; ++m)
            if (m < op.k) j |= int((i >> op.t[m]) & 1) << m;
        const float dr = mat[2 * (j * D + j)], di = mat[2 * (j * D + j) + 1];
        const float2 a = st[i];
        st[i] = float2{dr * a.x - di * a.y, dr * a.y + di * a.x};
    }
}

// In-LDS QFT of the field [q_lo, q_lo+m) of an n <= 13 qubit state:
// radix-2 decimation in frequency from the top field bit, then the
// bit-reversal of the field staged through registers, then 2^(-m/2).
__device__ void op_fft_lds(float2 *st, int n, const BOp &op)
{
    const int sgn = op.inv ? -1 : 1;
    for (int b = op.m - 1; b >= 0; --b) {
        const int bit = op.q_lo + b;
        for (uint32_t t = threadIdx.x; t < (1u << (n - 1)); t += kBT) {
            const uint32_t i = ((t >> bit) << (bit + 1)) | (t & ((1u << bit) - 1u));
            const uint32_t j = i | (1u << bit);
            const uint32_t kk = (i >> op.q_lo) & ((1u << b) - 1u);
            double sn, cs;
            sincospi(double(sgn) * double(kk) / double(1u << b), &sn, &cs);
            const float2 x = st[i], y = st[j];
            st[i] = float2{x.x + y.x, x.y + y.y};
            const float dr = x.x - y.x, di = x.y - y.y;
            st[j] = float2{float(dr * cs - di * sn), float(dr * sn + di * cs)};
        }
        __syncthreads();
    }
    const float scale = float(1.0 / sqrt(double(1u << op.m)));
    const uint32_t fmask = ((1u << op.m) - 1u) << op.q_lo;
    float2 v[(1 << kNS) / kBT];
    const int per = (1 << n) / kBT > 0 ? (1 << n) / kBT : 1;
#pragma unroll
    for (int q = 0; q < (1 << kNS) / kBT; ++q) {
        const uint32_t e = threadIdx.x + uint32_t(q) * kBT;
        if (q < per && e < (1u << n)) {
            const uint32_t f = (e & fmask) >> op.q_lo;
            uint32_t rf = 0;
            for (int b = 0; b < op.m; ++b) rf |= ((f >> b) & 1u) << (op.m - 1 - b);
            v[q] = st[(e & ~fmask) | (rf << op.q_lo)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (1 << kNS) / kBT; ++q) {
        const uint32_t e = threadIdx.x + uint32_t(q) * kBT;
        if (q < per && e < (1u << n)) st[e] = float2{v[q].x * scale, v[q].y * scale};
    }
}

__device__ __forceinline__ uint64_t mulmod_b(uint64_t x, uint64_t y, uint64_t N, uint64_t mu)
{
    const uint64_t p = x * y;
    const uint64_t q = __umul64hi(p, mu);
    uint64_t r = p - q * N;
    while (r >= N) r -= N;
    return r;
}

// a^(-c) mod N for c < 2^cb into tbl (threads c < 2^cb)
__device__ void inv_powers(const BOp &op, uint32_t *tbl)
{
    const int cnt = 1 << op.c;
    for (int c = threadIdx.x; c < cnt; c += kBT) {
        int64_t t0 = 0, t1 = 1, r0 = int64_t(op.N), r1 = int64_t(op.a % op.N);
        while (r1 != 0) {
            const int64_t q = r0 / r1;
            int64_t tmp = r0 - q * r1;
            r0 = r1;
            r1 = tmp;
            tmp = t0 - q * t1;
            t0 = t1;
            t1 = tmp;
        }
        uint64_t base = uint64_t(t0 < 0 ? t0 + int64_t(op.N) : t0) % op.N, res = 1 % op.N;
        for (uint64_t e = uint64_t(c); e; e >>= 1) {
            if (e & 1) res = mulmod_b(res, base, op.N, op.mu);
            base = mulmod_b(base, base, op.N, op.mu);
        }
        tbl[c] = uint32_t(res);
    }
}

__device__ __forceinline__ uint32_t perm_src(uint32_t i, const BOp &op, const uint32_t *tbl)
{
    const uint32_t wm = (1u << op.w) - 1u;
    const uint32_t xp = (i >> op.work_lo) & wm;
    if (xp >= op.N) return i;
    const uint32_t cc = op.c ? ((i >> op.ctrl_lo) & ((1u << op.c) - 1u)) : 0u;
    const uint32_t x = uint32_t(mulmod_b(tbl[cc], xp, op.N, op.mu));
    return (i & ~(wm << op.work_lo)) | (x << op.work_lo);
}

// counter[0]: queue head, counter[1]: error flag, then one barrier counter
// per circuit
__global__ void k_reset(unsigned *counter, int n, uint64_t *ticks, int n_ticks)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counter[i] = 0;
    // segments without ops (an empty gate list) report zero time
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_ticks; i += gridDim.x * blockDim.x) ticks[i] = 0;
}

__global__ __launch_bounds__(kBT, 2) void k_batch(float2 *__restrict__ A, float2 *__restrict__ B,
                                                   const BCirc *__restrict__ circ,
                                                   const Ticket *__restrict__ tickets, int n_tickets,
                                                   const BOp *__restrict__ ops,
                                                   const float *__restrict__ pool,
                                                   const PassArgs *__restrict__ passes,
                                                   unsigned *__restrict__ counter,
                                                   uint64_t *__restrict__ seg_ticks,
                                                   double2 *__restrict__ partials,
                                                   double *__restrict__ norms, double *__restrict__ z0,
                                                   ulonglong2 *__restrict__ trace)
{
    extern __shared__ unsigned char lds_raw[];
    __shared__ int s_idx;
    __shared__ uint32_t s_tbl[64];
    __shared__ double s_red[2][kBT / 64];
    unsigned *const err = counter + 1;
    unsigned *const bars = counter + 2;
    for (;;) {
        if (threadIdx.x == 0) s_idx = int(atomicAdd(counter, 1u));
        __syncthreads();
        const int qi = __builtin_amdgcn_readfirstlane(s_idx);
        __syncthreads();
        if (qi >= n_tickets) break;
        const Ticket tk = tickets[qi];
        const BCirc cc = circ[tk.circ];
        const uint32_t G = uint32_t(cc.gang), r = uint32_t(tk.member);
        const bool in_lds = cc.n <= kNS;
        const bool lead = r == 0 && threadIdx.x == 0;
        const uint64_t t_ticket = wall_clock64();
        unsigned epoch = 0;
        float2 *const buf_a = A + cc.off_a, *const buf_b = B + cc.off_b;
        float2 *lst = reinterpret_cast<float2 *>(lds_raw);
        int cur_seg = -1;
        uint64_t t_seg = 0;
        for (int o = cc.op0; o < cc.op1; ++o) {
            const BOp op = ops[o];
            if (op.seg != cur_seg) {
                if (lead) {
                    const uint64_t now = wall_clock64();
                    if (cur_seg >= 0) seg_ticks[cur_seg] = now - t_seg;
                    t_seg = now;
                }
                cur_seg = op.seg;
            }
            float2 *src = in_lds ? lst : (op.src ? buf_b : buf_a);
            float2 *dst = in_lds ? lst : (op.dst ? buf_b : buf_a);
            switch (op.type) {
            case OP_INIT:
                for (uint32_t i = r * kBT + threadIdx.x; i < (1u << cc.n); i += G * kBT)
                    dst[i] = float2{i == 0 ? 1.f : 0.f, 0.f};
                break;
            case OP_DENSE: {
                const float *m = pool + op.mat;
                if (op.k >= 4 && !in_lds && !op.mono) {
                    float2 *xs = reinterpret_cast<float2 *>(lds_raw);   // staging: the LDS no HBM state uses
                    if (op.k == 4) op_dense_mfma<4>(dst, cc.n, op, m, r, G, xs);
                    else if (op.k == 5) op_dense_mfma<5>(dst, cc.n, op, m, r, G, xs);
                    else op_dense_mfma<6>(dst, cc.n, op, m, r, G, xs);
                    break;
                }
                switch (op.k) {
                case 1: op_dense<1>(dst, cc.n, op, m, r, G); break;
                case 2: op_dense<2>(dst, cc.n, op, m, r, G); break;
                case 3: op_dense<3>(dst, cc.n, op, m, r, G); break;
                case 4: op_dense<4>(dst, cc.n, op, m, r, G); break;
                case 5: op_dense<5>(dst, cc.n, op, m, r, G); break;
                default: op_dense<6>(dst, cc.n, op, m, r, G); break;
                }
                break;
            }
            case OP_DIAG:
                op_diag(dst, cc.n, op, pool + op.mat, r, G);
                break;
            case OP_FFT_LDS:
                op_fft_lds(dst, cc.n, op);
                break;
            case OP_FFT_PASS: {
                const PassArgs &pa = passes[op.pass];
                for (uint64_t t = r; t < pa.tiles; t += G)
                    fftdev::fft_tile<float, kBT>(src, dst, pa, t, lds_raw);
                break;
            }
            case OP_PERM: {
                inv_powers(op, s_tbl);
                __syncthreads();
                if (in_lds) {
                    float2 v[(1 << kNS) / kBT];
#pragma unroll
                    for (int q = 0; q < (1 << kNS) / kBT; ++q) {
                        const uint32_t e = threadIdx.x + uint32_t(q) * kBT;
                        if (e < (1u << cc.n)) v[q] = lst[perm_src(e, op, s_tbl)];
                    }
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < (1 << kNS) / kBT; ++q) {
                        const uint32_t e = threadIdx.x + uint32_t(q) * kBT;
                        if (e < (1u << cc.n)) lst[e] = v[q];
                    }
                } else {
                    for (uint32_t i = r * kBT + threadIdx.x; i < (1u << cc.n); i += G * kBT)
                        dst[i] = src[perm_src(i, op, s_tbl)];
                }
                break;
            }
            case OP_NORM: {
                double s = 0.0, z = 0.0;
                for (uint32_t i = r * kBT + threadIdx.x; i < (1u << cc.n); i += G * kBT) {
                    const float2 a = src[i];
                    const double p = double(a.x) * a.x + double(a.y) * a.y;
                    s += p;
                    z += (i & 1u) ? -p : p;
                }
                for (int d = 32; d > 0; d >>= 1) {
                    s += __shfl_xor(s, d, 64);
                    z += __shfl_xor(z, d, 64);
                }
                if ((threadIdx.x & 63) == 0) {
                    s_red[0][threadIdx.x >> 6] = s;
                    s_red[1][threadIdx.x >> 6] = z;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    double ts = 0.0, tz = 0.0;
                    for (int w = 0; w < kBT / 64; ++w) {
                        ts += s_red[0][w];
                        tz += s_red[1][w];
                    }
                    partials[cc.p0 + int(r)] = double2{ts, tz};
                }
                if (G > 1) gang_sync(bars + tk.circ, G, epoch, err);
                if (lead) {
                    // members summed in a fixed order: the result does not
                    // depend on which workgroup finished first
                    double ts = 0.0, tz = 0.0;
                    for (uint32_t m = 0; m < G; ++m) {
                        const double2 pm = partials[cc.p0 + int(m)];
                        ts += pm.x;
                        tz += pm.y;
                    }
                    norms[tk.circ] = ts;
                    z0[tk.circ] = tz;
                }
                break;
            }
            default:
                break;
            }
            if (G > 1 && o + 1 < cc.op1)
                gang_sync(bars + tk.circ, G, epoch, err);
            else
                __syncthreads();
        }
        if (lead && cur_seg >= 0) seg_ticks[cur_seg] = wall_clock64() - t_seg;
        if (in_lds) {
            float2 *out = buf_a;
            for (uint32_t i = threadIdx.x; i < (1u << cc.n); i += kBT) out[i] = lst[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) trace[qi] = ulonglong2{t_ticket, (wall_clock64() << 12) | (blockIdx.x & 4095u)};
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct GateList {
    std::vector<int> k, targets;
    std::vector<double> mats;
    std::vector<uint64_t> cm, cv;
    std::vector<size_t> toff, moff;
    int n_gates() const { return int(k.size()); }
};

struct SegInfo {
    int kind, circuit, list;
    int q_lo, m, inv;
    qs_perm perm;
    float feat[QS_N_FEATURES];
};

struct FusedList {       // a gate list fused at some k, composed into the pool
    std::vector<int> blk_k;
    std::vector<std::vector<int>> blk_q;
    std::vector<int> blk_diag, blk_mono;
    std::vector<int64_t> blk_mat;   // pool offset (floats)
};

struct qs_batch_t {
    hipStream_t stream = nullptr;
    int n_circ = 0;
    std::vector<int> cn;                 // qubits per circuit
    std::vector<std::vector<int>> cseg;  // segment ids per circuit
    std::vector<SegInfo> segs;
    std::vector<GateList> lists;
    std::map<std::tuple<const double *, const int *, const int *, int>, int> list_of_ptr;
    std::map<std::pair<int, int>, std::vector<float>> list_stats;   // (list, n) -> cached statistics
    std::vector<uint64_t> off_a, off_b;
    float2 *A = nullptr, *B = nullptr;
    size_t a_elems = 0, b_elems = 0;
    // plan
    std::map<std::pair<int, int>, FusedList> fused;   // (list, k) -> blocks
    std::vector<float> pool_host_dummy;
    float *pool = nullptr;
    size_t pool_floats = 0, pool_cap = 0;
    BOp *d_ops = nullptr;
    BCirc *d_circ = nullptr;
    Ticket *d_tickets = nullptr;
    double2 *d_partials = nullptr;
    ulonglong2 *d_trace = nullptr;   // per ticket: start tick, end tick << 12 | workgroup
    std::vector<Ticket> tickets;     // host copy of the queue
    int n_tickets = 0;
    int grid = 0;                 // co-resident workgroups of the persistent launch
    PassArgs *d_passes = nullptr;
    unsigned *d_counter = nullptr;
    uint64_t *d_ticks = nullptr;
    double *d_norm = nullptr, *d_z0 = nullptr;
    std::vector<int> final_buf;
    bool planned = false;
    double clock_khz = 100000.0;
};

namespace {

int gcd_ok(uint64_t a, uint64_t N)
{
    while (N) {
        const uint64_t t = a % N;
        a = N;
        N = t;
    }
    return a == 1;
}

void seg_features(qs_batch_t *b, SegInfo &s, double batch_bytes)
{
    const GateList &L = b->lists[size_t(s.list)];
    const int n = b->cn[size_t(s.circuit)];
    const auto skey = std::make_pair(s.list, n);
    auto hit = b->list_stats.find(skey);
    if (hit != b->list_stats.end()) {
        std::memcpy(s.feat, hit->second.data(), sizeof(float) * QS_N_FEATURES);
        s.feat[3] = s.feat[4] = s.feat[5] = 0.f;
        s.feat[3 + s.kind] = 1.f;
        s.feat[14] = s.kind == QS_SEG_QFT ? float(s.m) : 0.f;
        s.feat[15] = s.kind == QS_SEG_MODMUL ? float(s.perm.w) : 0.f;
        s.feat[16] = s.kind == QS_SEG_MODMUL ? float(s.perm.c) : 0.f;
        s.feat[21] = float(std::log2(std::max(batch_bytes, 1.0)));
        return;
    }
    int n1 = 0, n2 = 0, nd = 0, nc = 0, tot = 0, lo = 0, hi = 0;
    double tsum = 0.0;
    uint64_t span = 0;
    for (int g = 0; g < L.n_gates(); ++g) {
        const int k = L.k[size_t(g)];
        const uint64_t cm = L.cm[size_t(g)];
        const int width = k + __builtin_popcountll(cm);
        (width == 1 ? n1 : n2)++;
        if (cm) ++nc;
        GateDesc d;
        classify(L.mats.data() + L.moff[size_t(g)], k, d);
        if (d.cls == GC_IDENTITY || d.cls == GC_PHASE1 || d.cls == GC_DIAG) ++nd;
        for (int m = 0; m < k; ++m) {
            const int t = L.targets[L.toff[size_t(g)] + size_t(m)];
            ++tot;
            lo += t < 6;
            hi += t >= 14;
            tsum += t;
            span |= 1ull << t;
        }
        span |= cm;
    }
    int blocks[3] = {0, 0, 0};
    const int ks[3] = {2, 4, 6};
    for (int i = 0; i < 3; ++i) {
        Plan p;
        plan_fusion(n, L.n_gates(), L.k.data(), L.targets.data(), L.cm.data(), ks[i], p);
        blocks[i] = int(p.block_gates.size());
    }
    float *f = s.feat;
    for (int i = 0; i < QS_N_FEATURES; ++i) f[i] = 0.f;
    f[0] = float(n);
    f[1] = float(n + 3);
    f[2] = n <= kNS ? 1.f : 0.f;
    f[3 + s.kind] = 1.f;
    f[6] = float(std::log1p(double(L.n_gates())));
    f[7] = float(std::log1p(double(n1)));
    f[8] = float(std::log1p(double(n2)));
    f[9] = float(std::log1p(double(nd)));
    f[10] = float(std::log1p(double(nc)));
    f[11] = tot ? float(lo) / float(tot) : 0.f;
    f[12] = tot ? float(hi) / float(tot) : 0.f;
    f[13] = tot ? float(tsum / tot / n) : 0.f;
    f[14] = s.kind == QS_SEG_QFT ? float(s.m) : 0.f;
    f[15] = s.kind == QS_SEG_MODMUL ? float(s.perm.w) : 0.f;
    f[16] = s.kind == QS_SEG_MODMUL ? float(s.perm.c) : 0.f;
    f[17] = float(std::log1p(double(blocks[0])));
    f[18] = float(std::log1p(double(blocks[1])));
    f[19] = float(std::log1p(double(blocks[2])));
    f[20] = float(__builtin_popcountll(span)) / float(n);
    f[21] = float(std::log2(std::max(batch_bytes, 1.0)));
    f[22] = float(std::log2(double(std::max(blocks[1], 1))) + n + 4);
    f[23] = float(std::log2(double(std::max(blocks[2], 1))) + n + 9);
    b->list_stats[skey] = std::vector<float>(f, f + QS_N_FEATURES);
}

// Workgroups of k_batch that fit on the device at once (the persistent grid;
// also the bound a gang must stay under so that all its members run).
int resident_grid(int &grid)
{
    static int cached = 0;
    if (!cached) {
        QS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(kLds)));
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        QS_HIP(hipGetDevice(&dev));
        QS_HIP(hipGetDeviceProperties(&prop, dev));
        QS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_batch), kBT, kLds));
        if (per_cu < 1) return fail(QS_EDEVICE, "the batch kernel does not fit on a compute unit");
        cached = std::min(per_cu, 2) * prop.multiProcessorCount;
    }
    grid = cached;
    return QS_OK;
}

// Gang size of an HBM circuit: the smallest power of two that brings its
// time per member under a quarter (tunable) of the average work per workgroup
// (`share`), so that gangs remove the tail of a batch with few large
// circuits and stay small (few barriers) when many circuits already keep
// every workgroup busy. At least 2^12 amplitudes per member, at most a
// quarter of the co-resident workgroups.
int gang_size(int n, double cost, double share, int grid)
{
    if (n <= kNS) return 1;
    const int tuned = tune_value(QS_TUNE_BATCH_GANG_SHARE, QS_C64, 0, 0, 0);
    const double want = double(tuned ? tuned : 4) * cost / std::max(share, 1.0);
    int g = 1;
    while (g < want && g < (1 << std::min(n - 12, 20))) g <<= 1;
    return std::max(1, std::min(g, grid / 4));
}

int free_plan(qs_batch_t *b)
{
    if (b->d_ops) (void)hipFree(b->d_ops);
    if (b->d_circ) (void)hipFree(b->d_circ);
    if (b->d_tickets) (void)hipFree(b->d_tickets);
    if (b->d_partials) (void)hipFree(b->d_partials);
    if (b->d_trace) (void)hipFree(b->d_trace);
    if (b->d_passes) (void)hipFree(b->d_passes);
    b->d_ops = nullptr;
    b->d_circ = nullptr;
    b->d_tickets = nullptr;
    b->d_partials = nullptr;
    b->d_trace = nullptr;
    b->d_passes = nullptr;
    b->planned = false;
    return QS_OK;
}

// Fuse and compose (on the GPU, FP64, rounded into the FP32 pool) every
// (list, k) pair that the plan needs and the cache does not hold yet.
int compose_lists(qs_batch_t *b, const std::vector<std::pair<int, int>> &need)
{
    std::vector<ComposeGate> cg;
    std::vector<ComposeBlock> cb;
    std::vector<double> gm;
    std::vector<std::pair<std::pair<int, int>, FusedList>> fresh;
    int64_t out_off = 0;
    int kmax = 1;
    for (const auto &key : need) {
        if (b->fused.count(key)) continue;
        const GateList &L = b->lists[size_t(key.first)];
        Plan p;
        int n_q = 0;
        for (int g = 0; g < L.n_gates(); ++g) {
            for (int m = 0; m < L.k[size_t(g)]; ++m) n_q = std::max(n_q, L.targets[L.toff[size_t(g)] + size_t(m)] + 1);
            if (L.cm[size_t(g)]) n_q = std::max(n_q, 64 - __builtin_clzll(L.cm[size_t(g)]));
        }
        plan_fusion(std::max(n_q, 1), L.n_gates(), L.k.data(), L.targets.data(), L.cm.data(), key.second, p);
        FusedList F;
        for (size_t bi = 0; bi < p.block_gates.size(); ++bi) {
            const auto &qs = p.block_qubits[bi];
            const int kb = int(qs.size());
            if (kb > QS_MAX_K) return fail(QS_EUNSUPPORTED, "a gate spans more than %d qubits", QS_MAX_K);
            kmax = std::max(kmax, kb);
            auto local = [&](int q) { return int(std::lower_bound(qs.begin(), qs.end(), q) - qs.begin()); };
            ComposeBlock B;
            B.k = kb;
            B.g0 = int(cg.size());
            bool diag = true, mono = true;
            for (int g : p.block_gates[bi]) {
                ComposeGate G;
                std::memset(&G, 0, sizeof G);
                G.k = L.k[size_t(g)];
                for (int m = 0; m < G.k; ++m) G.local_t[m] = local(L.targets[L.toff[size_t(g)] + size_t(m)]);
                for (int q = 0; q < 64; ++q)
                    if ((L.cm[size_t(g)] >> q) & 1) {
                        G.ctrl_mask |= 1u << local(q);
                        if ((L.cv[size_t(g)] >> q) & 1) G.ctrl_vals |= 1u << local(q);
                    }
                G.mat_off = int64_t(gm.size());
                const double *src = L.mats.data() + L.moff[size_t(g)];
                gm.insert(gm.end(), src, src + (size_t(2) << (2 * G.k)));
                GateDesc tmp;
                classify(src, G.k, tmp);
                if (!(tmp.cls == GC_IDENTITY || tmp.cls == GC_PHASE1 || tmp.cls == GC_DIAG)) diag = false;
                if (!(tmp.cls == GC_IDENTITY || tmp.cls == GC_PHASE1 || tmp.cls == GC_DIAG || tmp.cls == GC_MONOMIAL))
                    mono = false;
                cg.push_back(G);
            }
            B.g1 = int(cg.size());
            B.pad = 0;
            B.out_off = out_off;
            cb.push_back(B);
            F.blk_k.push_back(kb);
            F.blk_q.push_back(qs);
            F.blk_diag.push_back(diag ? 1 : 0);
            F.blk_mono.push_back(mono ? 1 : 0);
            F.blk_mat.push_back(int64_t(b->pool_floats) + out_off);
            out_off += int64_t(2) << (2 * kb);
        }
        fresh.emplace_back(key, std::move(F));
    }
    if (cb.empty()) {
        for (auto &fr : fresh) b->fused[fr.first] = std::move(fr.second);
        return QS_OK;
    }
    // grow the pool (device-to-device copy of what it holds)
    const size_t need_floats = b->pool_floats + size_t(out_off);
    if (need_floats > b->pool_cap) {
        const size_t cap = std::max(need_floats, b->pool_cap * 2);
        float *np = nullptr;
        QS_HIP(hipMalloc(reinterpret_cast<void **>(&np), cap * sizeof(float)));
        if (b->pool) {
            QS_HIP(hipMemcpyAsync(np, b->pool, b->pool_floats * sizeof(float), hipMemcpyDeviceToDevice, b->stream));
            QS_HIP(hipStreamSynchronize(b->stream));
            (void)hipFree(b->pool);
        }
        b->pool = np;
        b->pool_cap = cap;
    }
    void *dcg = nullptr, *dcb = nullptr, *dgm = nullptr, *dout = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        if (dcg) (void)hipFree(dcg);
        if (dcb) (void)hipFree(dcb);
        if (dgm) (void)hipFree(dgm);
        if (dout) (void)hipFree(dout);
    };
    if ((e = hipMalloc(&dcg, sizeof(ComposeGate) * cg.size())) != hipSuccess ||
        (e = hipMalloc(&dcb, sizeof(ComposeBlock) * cb.size())) != hipSuccess ||
        (e = hipMalloc(&dgm, sizeof(double) * gm.size())) != hipSuccess ||
        (e = hipMalloc(&dout, sizeof(double) * size_t(out_off))) != hipSuccess) {
        cleanup();
        return hip_fail(e, "hipMalloc(batch compose)");
    }
    if ((e = hipMemcpyAsync(dcg, cg.data(), sizeof(ComposeGate) * cg.size(), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(dcb, cb.data(), sizeof(ComposeBlock) * cb.size(), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(dgm, gm.data(), sizeof(double) * gm.size(), hipMemcpyHostToDevice, b->stream)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "hipMemcpyAsync(batch compose)");
    }
    int rc = launch_compose(b->stream, int(cb.size()), static_cast<ComposeBlock *>(dcb),
                            static_cast<ComposeGate *>(dcg), static_cast<double *>(dgm),
                            static_cast<double *>(dout), kmax);
    if (!rc) rc = launch_cast_f64_to_f32(b->stream, static_cast<double *>(dout), b->pool + b->pool_floats, size_t(out_off));
    if (!rc && (e = hipStreamSynchronize(b->stream)) != hipSuccess) rc = hip_fail(e, "batch compose");
    cleanup();
    if (rc) return rc;
    b->pool_floats += size_t(out_off);
    for (auto &fr : fresh) b->fused[fr.first] = std::move(fr.second);
    return QS_OK;
}

}  // namespace

extern "C" {

int qs_batch_create(int n_circuits, const qs_batch_circuit *circuits, void *hip_stream, qs_batch *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "NULL output batch");
    *out = nullptr;
    if (n_circuits < 1 || !circuits) return fail(QS_EINVAL, "empty batch");
    qs_batch_t *b = new (std::nothrow) qs_batch_t();
    if (!b) return fail(QS_ENOMEM, "host allocation failed");
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->n_circ = n_circuits;
    b->cn.resize(size_t(n_circuits));
    b->cseg.resize(size_t(n_circuits));
    auto bail = [&](int rc) {
        delete b;
        return rc;
    };
    double batch_bytes = 0.0;
    for (int c = 0; c < n_circuits; ++c) {
        const qs_batch_circuit &C = circuits[c];
        if (C.n_qubits < 2 || C.n_qubits > 26) return bail(fail(QS_EINVAL, "circuit %d: n=%d outside [2, 26]", c, C.n_qubits));
        if (C.n_segments < 0 || (C.n_segments > 0 && !C.segments)) return bail(fail(QS_EINVAL, "circuit %d: bad segments", c));
        b->cn[size_t(c)] = C.n_qubits;
        batch_bytes += 8.0 * double(1ull << C.n_qubits);
        for (int s = 0; s < C.n_segments; ++s) {
            const qs_segment &S = C.segments[s];
            const qs_circuit &G = S.gates;
            if (S.kind < QS_SEG_GATES || S.kind > QS_SEG_MODMUL)
                return bail(fail(QS_EINVAL, "circuit %d segment %d: unknown kind", c, s));
            // validate the gate list against this circuit
            if (G.n_gates < 0 || (G.n_gates > 0 && (!G.k || !G.targets || !G.matrices)))
                return bail(fail(QS_EINVAL, "circuit %d segment %d: bad gate list", c, s));
            size_t toff = 0;
            for (int g = 0; g < G.n_gates; ++g) {
                const int k = G.k[g];
                if (k < 1 || k > QS_MAX_K) return bail(fail(QS_EINVAL, "circuit %d segment %d gate %d: width", c, s, g));
                uint64_t tm = 0;
                for (int m = 0; m < k; ++m) {
                    const int t = G.targets[toff + size_t(m)];
                    if (t < 0 || t >= C.n_qubits || ((tm >> t) & 1))
                        return bail(fail(QS_EINVAL, "circuit %d segment %d gate %d: target", c, s, g));
                    tm |= 1ull << t;
                }
                const uint64_t cm = G.ctrl_mask ? G.ctrl_mask[g] : 0, cv = G.ctrl_vals ? G.ctrl_vals[g] : 0;
                if ((cm >> C.n_qubits) || (cm & tm) || (cv & ~cm) || k + __builtin_popcountll(cm) > QS_MAX_K)
                    return bail(fail(QS_EINVAL, "circuit %d segment %d gate %d: controls", c, s, g));
                toff += size_t(k);
            }
            SegInfo si;
            std::memset(&si, 0, sizeof si);
            si.kind = S.kind;
            si.circuit = c;
            if (S.kind == QS_SEG_QFT) {
                if (S.m < 1 || S.q_lo < 0 || S.q_lo + S.m > C.n_qubits)
                    return bail(fail(QS_EINVAL, "circuit %d segment %d: QFT field", c, s));
                si.q_lo = S.q_lo;
                si.m = S.m;
                si.inv = S.inverse ? 1 : 0;
            } else if (S.kind == QS_SEG_MODMUL) {
                const qs_perm &P = S.perm;
                if (P.kind != QS_PERM_MODMUL || P.w < 1 || P.c < 0 || P.c > 6 || P.work_lo < 0 ||
                    P.work_lo + P.w > C.n_qubits || (P.c && (P.ctrl_lo < 0 || P.ctrl_lo + P.c > C.n_qubits)) ||
                    (P.c && !(P.ctrl_lo >= P.work_lo + P.w || P.ctrl_lo + P.c <= P.work_lo)) ||
                    P.N < 2 || P.N > (1ull << P.w) || !gcd_ok(P.a % P.N, P.N))
                    return bail(fail(QS_EINVAL, "circuit %d segment %d: modular multiplication", c, s));
                si.perm = P;
                si.perm.dest = nullptr;
            }
            // the gate list (shared lists are stored once)
            const auto key = std::make_tuple(G.matrices, G.targets, G.k, G.n_gates);
            auto it = b->list_of_ptr.find(key);
            if (it == b->list_of_ptr.end() || G.n_gates == 0) {
                GateList L;
                size_t t = 0, mo = 0;
                for (int g = 0; g < G.n_gates; ++g) {
                    const int k = G.k[g];
                    L.k.push_back(k);
                    L.toff.push_back(t);
                    L.moff.push_back(mo);
                    for (int m = 0; m < k; ++m) L.targets.push_back(G.targets[t + size_t(m)]);
                    const size_t cnt = size_t(2) << (2 * k);
                    L.mats.insert(L.mats.end(), G.matrices + mo, G.matrices + mo + cnt);
                    L.cm.push_back(G.ctrl_mask ? G.ctrl_mask[g] : 0);
                    L.cv.push_back(G.ctrl_vals ? G.ctrl_vals[g] : 0);
                    t += size_t(k);
                    mo += cnt;
                }
                b->lists.push_back(std::move(L));
                si.list = int(b->lists.size()) - 1;
                if (G.n_gates > 0) b->list_of_ptr[key] = si.list;
            } else {
                si.list = it->second;
            }
            b->cseg[size_t(c)].push_back(int(b->segs.size()));
            b->segs.push_back(si);
        }
    }
    for (auto &s : b->segs) seg_features(b, s, batch_bytes);
    // buffers
    b->off_a.resize(size_t(n_circuits));
    b->off_b.resize(size_t(n_circuits));
    for (int c = 0; c < n_circuits; ++c) {
        const size_t d = size_t(1) << b->cn[size_t(c)];
        b->off_a[size_t(c)] = b->a_elems;
        b->a_elems += (d + 31) & ~size_t(31);
        b->off_b[size_t(c)] = b->b_elems;
        if (b->cn[size_t(c)] > kNS) b->b_elems += (d + 31) & ~size_t(31);
    }
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void **>(&b->A), sizeof(float2) * b->a_elems)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->B), sizeof(float2) * std::max<size_t>(b->b_elems, 32))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_counter), sizeof(unsigned) * (2 + size_t(n_circuits)))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_ticks), sizeof(uint64_t) * std::max<size_t>(b->segs.size(), 1))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_norm), sizeof(double) * size_t(n_circuits))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_z0), sizeof(double) * size_t(n_circuits))) != hipSuccess) {
        int rc = hip_fail(e, "hipMalloc(batch)");
        qs_batch_free(b);
        return rc;
    }
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        b->clock_khz = double(khz);
    *out = b;
    return QS_OK;
}

int qs_batch_info(qs_batch b, int *n_segments, double *state_bytes)
{
    clear_error();
    if (!b) return fail(QS_EINVAL, "NULL batch");
    if (n_segments) *n_segments = int(b->segs.size());
    if (state_bytes) *state_bytes = 8.0 * double(b->a_elems);
    return QS_OK;
}

int qs_batch_segment_info(qs_batch b, int *kind, int *circuit, int *n_qubits)
{
    clear_error();
    if (!b) return fail(QS_EINVAL, "NULL batch");
    for (size_t s = 0; s < b->segs.size(); ++s) {
        if (kind) kind[s] = b->segs[s].kind;
        if (circuit) circuit[s] = b->segs[s].circuit;
        if (n_qubits) n_qubits[s] = b->cn[size_t(b->segs[s].circuit)];
    }
    return QS_OK;
}

int qs_batch_features(qs_batch b, float *features)
{
    clear_error();
    if (!b || !features) return fail(QS_EINVAL, "NULL argument");
    for (size_t s = 0; s < b->segs.size(); ++s)
        std::memcpy(features + s * QS_N_FEATURES, b->segs[s].feat, sizeof(float) * QS_N_FEATURES);
    return QS_OK;
}

int qs_batch_set_plan(qs_batch b, const int *options)
{
    clear_error();
    if (!b || !options) return fail(QS_EINVAL, "NULL argument");
    for (size_t s = 0; s < b->segs.size(); ++s) {
        const int o = options[s];
        if (o < QS_PLAN_K2 || o > QS_PLAN_EMULATE) return fail(QS_EINVAL, "segment %zu: unknown option %d", s, o);
        if (o == QS_PLAN_EMULATE && b->segs[s].kind == QS_SEG_GATES)
            return fail(QS_EINVAL, "segment %zu: a plain gate list has no emulated form", s);
    }
    const int kof[3] = {2, 4, 6};
    std::vector<std::pair<int, int>> need;
    for (size_t s = 0; s < b->segs.size(); ++s)
        if (options[s] != QS_PLAN_EMULATE) need.emplace_back(b->segs[s].list, kof[options[s]]);
    if (int rc = compose_lists(b, need)) return rc;
    // op lists
    std::vector<BOp> ops;
    std::vector<BCirc> circ(size_t(b->n_circ));
    std::vector<PassArgs> passes;
    std::vector<double> cost(size_t(b->n_circ), 0.0);
    b->final_buf.assign(size_t(b->n_circ), 0);
    for (int c = 0; c < b->n_circ; ++c) {
        const int n = b->cn[size_t(c)];
        const bool in_lds = n <= kNS;
        int cur = 0;
        BCirc C;
        C.n = n;
        C.op0 = int(ops.size());
        C.off_a = b->off_a[size_t(c)];
        C.off_b = b->off_b[size_t(c)];
        BOp init;
        std::memset(&init, 0, sizeof init);
        init.type = OP_INIT;
        init.seg = -1;
        ops.push_back(init);
        for (int sid : b->cseg[size_t(c)]) {
            const SegInfo &S = b->segs[size_t(sid)];
            const int o = options[sid];
            if (o != QS_PLAN_EMULATE) {
                const FusedList &F = b->fused.at(std::make_pair(S.list, kof[o]));
                for (size_t bi = 0; bi < F.blk_k.size(); ++bi) {
                    BOp op;
                    std::memset(&op, 0, sizeof op);
                    op.type = F.blk_diag[bi] ? OP_DIAG : OP_DENSE;
                    op.mono = F.blk_mono[bi];
                    op.k = F.blk_k[bi];
                    op.seg = sid;
                    op.src = op.dst = cur;
                    for (int m = 0; m < op.k; ++m) op.t[m] = F.blk_q[bi][size_t(m)];
                    op.mat = F.blk_mat[bi];
                    ops.push_back(op);
                    cost[size_t(c)] += double(1ull << n) * (1.0 + 0.25 * op.k);
                }
            } else if (S.kind == QS_SEG_QFT) {
                BOp op;
                std::memset(&op, 0, sizeof op);
                op.seg = sid;
                op.q_lo = S.q_lo;
                op.m = S.m;
                op.inv = S.inv;
                if (in_lds) {
                    op.type = OP_FFT_LDS;
                    ops.push_back(op);
                } else {
                    std::vector<PassArgs> pl;
                    if (int rc = fftdev::plan_passes(n, S.q_lo, S.m, S.inv, fftdev::kRmax, kFftLds, sizeof(float2), pl))
                        return rc;
                    for (size_t j = 0; j < pl.size(); ++j) {
                        op.type = OP_FFT_PASS;
                        op.pass = int(passes.size());
                        passes.push_back(pl[j]);
                        op.src = cur;
                        const bool out_of_place = pl.size() > 1 && j + 1 == pl.size();
                        op.dst = out_of_place ? 1 - cur : cur;
                        ops.push_back(op);
                        cur = op.dst;
                    }
                }
                cost[size_t(c)] += double(1ull << n) * 3.0;
            } else {
                BOp op;
                std::memset(&op, 0, sizeof op);
                op.type = OP_PERM;
                op.seg = sid;
                op.work_lo = S.perm.work_lo;
                op.w = S.perm.w;
                op.ctrl_lo = S.perm.ctrl_lo;
                op.c = S.perm.c;
                op.N = uint32_t(S.perm.N);
                op.a = S.perm.a;
                op.mu = ~0ull / S.perm.N;
                op.src = cur;
                op.dst = in_lds ? cur : 1 - cur;
                ops.push_back(op);
                cur = op.dst;
                cost[size_t(c)] += double(1ull << n);
            }
        }
        BOp nrm;
        std::memset(&nrm, 0, sizeof nrm);
        nrm.type = OP_NORM;
        nrm.seg = -2;
        nrm.src = nrm.dst = cur;
        ops.push_back(nrm);
        C.op1 = int(ops.size());
        C.final_buf = in_lds ? 0 : cur;
        b->final_buf[size_t(c)] = C.final_buf;
        circ[size_t(c)] = C;
    }
    // seg -2 (final norm) must not overwrite a segment time: map to -1
    for (auto &op : ops)
        if (op.seg < 0) op.seg = -1;
    // gangs, tickets (largest time per member first), norm partial slots
    int grid = 0;
    if (int rc = resident_grid(grid)) return rc;
    int p0 = 0;
    const double share = std::accumulate(cost.begin(), cost.end(), 0.0) / grid;
    for (int c = 0; c < b->n_circ; ++c) {
        circ[size_t(c)].gang = gang_size(b->cn[size_t(c)], cost[size_t(c)], share, grid);
        circ[size_t(c)].p0 = p0;
        p0 += circ[size_t(c)].gang;
    }
    // time per ticket, in amplitude-op units: the member's share of the
    // work plus, for a gang, one barrier per op (about as long as sweeping
    // kBarrierAmps amplitudes)
    const int tuned_bar = tune_value(QS_TUNE_BATCH_BARRIER_AMPS, QS_C64, 0, 0, 0);
    const double kBarrierAmps = tuned_bar ? double(tuned_bar) : 4096.0;
    std::vector<double> per_ticket(size_t(b->n_circ));
    for (int c = 0; c < b->n_circ; ++c) {
        const BCirc &C = circ[size_t(c)];
        per_ticket[size_t(c)] = cost[size_t(c)] / C.gang + (C.gang > 1 ? kBarrierAmps * (C.op1 - C.op0) : 0.0);
    }
    std::vector<int> order(size_t(b->n_circ));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return per_ticket[size_t(x)] > per_ticket[size_t(y)]; });
    std::vector<Ticket> tickets;
    tickets.reserve(size_t(p0));
    for (int c : order)
        for (int m = 0; m < circ[size_t(c)].gang; ++m) tickets.push_back(Ticket{c, m});
    free_plan(b);
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_ops), sizeof(BOp) * ops.size())) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_circ), sizeof(BCirc) * circ.size())) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_tickets), sizeof(Ticket) * tickets.size())) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_partials), sizeof(double2) * tickets.size())) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_trace), sizeof(ulonglong2) * tickets.size())) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->d_passes), sizeof(PassArgs) * std::max<size_t>(passes.size(), 1))) != hipSuccess)
        return hip_fail(e, "hipMalloc(batch plan)");
    b->n_tickets = int(tickets.size());
    b->tickets = tickets;
    b->grid = grid;
    QS_HIP(hipMemcpyAsync(b->d_ops, ops.data(), sizeof(BOp) * ops.size(), hipMemcpyHostToDevice, b->stream));
    QS_HIP(hipMemcpyAsync(b->d_circ, circ.data(), sizeof(BCirc) * circ.size(), hipMemcpyHostToDevice, b->stream));
    QS_HIP(hipMemcpyAsync(b->d_tickets, tickets.data(), sizeof(Ticket) * tickets.size(), hipMemcpyHostToDevice, b->stream));
    if (!passes.empty())
        QS_HIP(hipMemcpyAsync(b->d_passes, passes.data(), sizeof(PassArgs) * passes.size(), hipMemcpyHostToDevice, b->stream));
    QS_HIP(hipStreamSynchronize(b->stream));
    b->planned = true;
    return QS_OK;
}

int qs_batch_run(qs_batch b, double *wall_ms, double *seg_us, double *norms, double *z0)
{
    clear_error();
    if (!b) return fail(QS_EINVAL, "NULL batch");
    if (!b->planned) return fail(QS_EINVAL, "batch has no plan (qs_batch_set_plan)");
    // the grid never exceeds what is co-resident (each gang fits in it)
    const int grid = std::min(b->n_tickets, b->grid);
    const int n_cnt = 2 + b->n_circ;
    hipEvent_t e0, e1;
    QS_HIP(hipEventCreate(&e0));
    QS_HIP(hipEventCreate(&e1));
    const int n_ticks = int(b->segs.size());
    hipLaunchKernelGGL(k_reset, dim3(std::min((std::max(n_cnt, n_ticks) + 255) / 256, 1024)), dim3(256), 0, b->stream,
                       b->d_counter, n_cnt, b->d_ticks, n_ticks);
    QS_HIP(hipGetLastError());
    QS_HIP(hipEventRecord(e0, b->stream));
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBT), kLds, b->stream, b->A, b->B, b->d_circ, b->d_tickets,
                       b->n_tickets, b->d_ops, b->pool, b->d_passes, b->d_counter, b->d_ticks, b->d_partials,
                       b->d_norm, b->d_z0, b->d_trace);
    QS_HIP(hipGetLastError());
    QS_HIP(hipEventRecord(e1, b->stream));
    QS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    unsigned flags[2] = {0, 0};
    QS_HIP(hipMemcpy(flags, b->d_counter, sizeof flags, hipMemcpyDeviceToHost));
    if (flags[1]) return fail(QS_EDEVICE, "a gang barrier of the batch kernel timed out; results are invalid");
    if (wall_ms) *wall_ms = double(ms);
    if (seg_us) {
        std::vector<uint64_t> t(b->segs.size());
        QS_HIP(hipMemcpy(t.data(), b->d_ticks, sizeof(uint64_t) * t.size(), hipMemcpyDeviceToHost));
        for (size_t s = 0; s < t.size(); ++s) seg_us[s] = double(t[s]) * 1000.0 / b->clock_khz;
    }
    if (norms) QS_HIP(hipMemcpy(norms, b->d_norm, sizeof(double) * size_t(b->n_circ), hipMemcpyDeviceToHost));
    if (z0) QS_HIP(hipMemcpy(z0, b->d_z0, sizeof(double) * size_t(b->n_circ), hipMemcpyDeviceToHost));
    return QS_OK;
}

int qs_batch_trace(qs_batch b, int capacity, int *n_tickets, double *start_us, double *end_us, int *circuit,
                   int *member, int *workgroup)
{
    clear_error();
    if (!b || !n_tickets) return fail(QS_EINVAL, "NULL argument");
    if (!b->planned) return fail(QS_EINVAL, "batch has no plan (qs_batch_set_plan)");
    *n_tickets = b->n_tickets;
    const int cnt = std::min(std::max(capacity, 0), b->n_tickets);
    if (cnt == 0) return QS_OK;
    std::vector<ulonglong2> t(size_t(b->n_tickets));
    QS_HIP(hipStreamSynchronize(b->stream));
    QS_HIP(hipMemcpy(t.data(), b->d_trace, sizeof(ulonglong2) * t.size(), hipMemcpyDeviceToHost));
    uint64_t t0 = ~0ull;
    for (const auto &x : t) t0 = std::min<uint64_t>(t0, x.x);
    const double us = 1000.0 / b->clock_khz;
    for (int i = 0; i < cnt; ++i) {
        const ulonglong2 &x = t[size_t(i)];
        if (start_us) start_us[i] = double(x.x - t0) * us;
        if (end_us) end_us[i] = double((x.y >> 12) - t0) * us;
        if (workgroup) workgroup[i] = int(x.y & 4095u);
        if (circuit) circuit[i] = b->tickets[size_t(i)].circ;
        if (member) member[i] = b->tickets[size_t(i)].member;
    }
    return QS_OK;
}

int qs_batch_get_state(qs_batch b, int circuit, void *host_dst)
{
    clear_error();
    if (!b || !host_dst) return fail(QS_EINVAL, "NULL argument");
    if (circuit < 0 || circuit >= b->n_circ) return fail(QS_EINVAL, "circuit %d outside the batch", circuit);
    const size_t d = size_t(1) << b->cn[size_t(circuit)];
    const float2 *src = (b->final_buf.empty() || b->final_buf[size_t(circuit)] == 0)
                            ? b->A + b->off_a[size_t(circuit)]
                            : b->B + b->off_b[size_t(circuit)];
    QS_HIP(hipStreamSynchronize(b->stream));
    QS_HIP(hipMemcpy(host_dst, src, sizeof(float2) * d, hipMemcpyDeviceToHost));
    return QS_OK;
}

int qs_batch_free(qs_batch b)
{
    clear_error();
    if (!b) return QS_OK;
    (void)hipStreamSynchronize(b->stream);
    free_plan(b);
    if (b->A) (void)hipFree(b->A);
    if (b->B) (void)hipFree(b->B);
    if (b->pool) (void)hipFree(b->pool);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->d_ticks) (void)hipFree(b->d_ticks);
    if (b->d_norm) (void)hipFree(b->d_norm);
    if (b->d_z0) (void)hipFree(b->d_z0);
    delete b;
    return QS_OK;
}

}  // extern "C"
