// Gate sweeps over a 2^n state (Sec. II): the 2^n x 2^n operator of a k-qubit
// gate is the Kronecker product of its 2^k x 2^k matrix with identities, so a
// sweep visits every group of 2^k amplitudes that agree outside the targets
// and multiplies it by the small matrix. Structure is exploited as Sec. II
// and Sec. III-B describe: multiplications by one and zero are skipped, a
// conditional phase shift touches only the indices that carry the phase,
// and permutation gates only move amplitudes.
//
// Index mapping. The "fixed" bit positions of a sweep (targets, and control
// qubits whose value is pinned) are removed from the index space; a work
// item g in [0, 2^(n - nfix)) is expanded back by inserting a zero at every
// fixed position (ascending) and OR-ing the pinned control values. Lanes of a
// wave take consecutive g, so they walk the lowest free bits and global
// accesses coalesce whenever no target sits in the lowest bits.
#include "qs_internal.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace qs {
namespace {

constexpr int kMaxFix = 40;
constexpr int kBlock = 256;

struct FixArgs {
    int nfix;
    int pos[kMaxFix];  // ascending
    uint64_t vals;     // pinned bits OR-ed after expansion
};

template <int D>
struct OffArgs {
    uint64_t o[D];     // offset of local index j inside a group
};

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

// Nontemporal (streaming) loads and stores of one amplitude, selected by a
// tuning flag: bit 0 stores, bit 1 loads. The phase and diagonal kernels
// always stream: on 30-qubit complex128 states a controlled phase takes
// 1.26-1.36 ms that way and 1.43 ms with plain accesses. Monomial gates
// keep plain accesses: they write partial lines, which streaming stores
// made 10% slower (controlled X gates of a 31-qubit adder network).
template <typename C2> struct NtVec;
template <> struct NtVec<double2> { typedef double __attribute__((ext_vector_type(2))) T; };
template <> struct NtVec<float2> { typedef float __attribute__((ext_vector_type(2))) T; };

// Kernels take the policy as a template parameter: a runtime flag puts a
// branch around every access and serialises the stores.
template <typename F>
void with_nt(int nt, F &&f)
{
    switch (nt & 3) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 3>{}); break;
    }
}

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

// Chunked XCD workgroup order (xcd_order, qs_internal.h): C = 64 for the
// dense block sweeps and C = 128 for the elementwise gate kernels beat both
// the launch order (6.37 -> 6.01 ms per 4-qubit block, 1015 -> 969 ms for
// the gate-level QFT on 30-qubit complex128 states) and one contiguous
// eighth per XCD.
constexpr unsigned kXcdRunDense = 64, kXcdRunElem = 128;

template <typename IT>
__device__ __forceinline__ IT expand(IT g, const FixArgs &f)
{
    for (int i = 0; i < f.nfix; ++i) {
        const int p = f.pos[i];
        const IT lo = g & ((IT(1) << p) - IT(1));
        g = ((g >> p) << (p + 1)) | lo;
    }
    return g | IT(f.vals);
}

// Dense sweep: one thread owns one group, holds its 2^K amplitudes in
// registers and writes out_j = sum_l M[j][l] in_l. The matrix pointer and
// every index into it are uniform, so the entries are read through scalar
// loads and used as SGPR operands of the FMAs. Loops over output rows and
// over 8-entry chunks of a row are kept rolled, so at most one chunk (16
// reals) is resident in SGPRs; fully unrolled, the compiler hoists the whole
// matrix and spills scalar registers into vector lanes.
template <typename R, typename C2, int D, int L0>
__device__ __forceinline__ void row_chunk(const R *__restrict__ row, const C2 (&v)[D], R &re, R &im)
{
#pragma unroll
    for (int l = L0; l < L0 + (D < 8 ? D : 8); ++l) {
        const R mr = row[2 * l];
        const R mi = row[2 * l + 1];
        re = fma(mr, v[l].x, re);
        re = fma(-mi, v[l].y, re);
        im = fma(mr, v[l].y, im);
        im = fma(mi, v[l].x, im);
    }
}

template <typename R, typename C2, int D>
__device__ __forceinline__ void row_dot(const R *__restrict__ row, const C2 (&v)[D], R &re, R &im)
{
    if constexpr (D <= 8) {
        row_chunk<R, C2, D, 0>(row, v, re, im);
    } else {
#pragma unroll 1
        for (int c = 0; c < D / 8; ++c) {
            switch (c) {
            case 0: row_chunk<R, C2, D, 0>(row, v, re, im); break;
            case 1: row_chunk<R, C2, D, 8>(row, v, re, im); break;
            case 2: if constexpr (D > 16) row_chunk<R, C2, D, 16>(row, v, re, im); break;
            case 3: if constexpr (D > 16) row_chunk<R, C2, D, 24>(row, v, re, im); break;
            case 4: if constexpr (D > 32) row_chunk<R, C2, D, 32>(row, v, re, im); break;
            case 5: if constexpr (D > 32) row_chunk<R, C2, D, 40>(row, v, re, im); break;
            case 6: if constexpr (D > 32) row_chunk<R, C2, D, 48>(row, v, re, im); break;
            default: if constexpr (D > 32) row_chunk<R, C2, D, 56>(row, v, re, im); break;
            }
        }
    }
}

template <typename R, int K, typename IT, int NT>
__global__ __launch_bounds__(kBlock) void k_dense(typename V2<R>::T *__restrict__ psi,
                                                  const R *__restrict__ mat, IT n_groups,
                                                  FixArgs fx, OffArgs<(1 << K)> off)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K;
    const IT stride = IT(gridDim.x) * kBlock;
    const IT first = xcd_order<IT, kXcdRunDense>(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    for (IT g = first; g < n_groups; g += stride) {
        C2 *p = psi + expand<IT>(g, fx);
        C2 v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = load_amp(p + off.o[j], NT);
#pragma unroll 1
        for (int j = 0; j < D; ++j) {
            R re = R(0), im = R(0);
            row_dot<R, C2, D>(mat + 2 * j * D, v, re, im);
            store_amp(p + off.o[j], C2{re, im}, NT);
        }
    }
}

// Dense sweep for blocks with targets inside a cache line. A wave owns a
// tile of 2^(6+K) amplitudes spanned by index bits 0..5, the targets above
// bit 5, and the lowest free bits above bit 5 ("extra" bits), as many as
// there are targets below bit 6. Loads and stores use the layout lane =
// bits 0..5, register = the other tile bits, so every wave-wide access is
// 64 consecutive amplitudes. An LDS transpose regroups the tile so each lane
// owns one whole group (lane = the free tile bits, register = the local
// index), the group is multiplied in registers, and the transpose is undone
// before the store. Positions are compact tile indices; the LDS slot of
// position p XORs its low bits with the next ones, which spreads both
// layouts over distinct banks.
template <int D>
struct LdsArgs {
    int lane_pos[6];   // compact position of each lane bit in the compute layout
    int offc[D];       // compact position offset of local index j
};

template <typename C2>
__device__ __forceinline__ int lds_slot(int p)
{
    constexpr int SW = 256 / int(sizeof(C2));  // elements per 256-byte bank row
    return p ^ ((p / SW) & (SW - 1));
}

template <typename R, int K, typename IT, int NT>
__global__ __launch_bounds__(64) void k_dense_lds(typename V2<R>::T *__restrict__ psi,
                                                  const R *__restrict__ mat, IT n_tiles,
                                                  FixArgs fx, OffArgs<(1 << K)> offl,
                                                  LdsArgs<(1 << K)> la)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K;
    __shared__ C2 tile[64 * D];
    const int lane = threadIdx.x;
    int lp = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) lp |= ((lane >> b) & 1) << la.lane_pos[b];
    for (IT t = xcd_order<IT, kXcdRunDense>(blockIdx.x, gridDim.x); t < n_tiles; t += IT(gridDim.x)) {
        C2 *p = psi + expand<IT>(t, fx) + lane;
        C2 v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v[r] = load_amp(p + offl.o[r], NT);
#pragma unroll
        for (int r = 0; r < D; ++r) tile[lds_slot<C2>(lane + 64 * r)] = v[r];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = tile[lds_slot<C2>(lp | la.offc[j])];
#pragma unroll 1
        for (int j = 0; j < D; ++j) {
            R re = R(0), im = R(0);
            row_dot<R, C2, D>(mat + 2 * j * D, v, re, im);
            tile[lds_slot<C2>(lp | la.offc[j])] = C2{re, im};
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < D; ++r) store_amp(p + offl.o[r], tile[lds_slot<C2>(lane + 64 * r)], NT);
        __syncthreads();
    }
}

// Dense sweep for blocks of 2 to 4 qubits with the tile shared by a
// workgroup of 256 threads. A tile is 1024 amplitudes: the 2^K values of the
// targets times the 2^(10-K) values of the lowest free bits (the columns).
// Tile entry e lives at the address that deposits e's ten bits into the ten
// tile bits (ascending), and thread tid loads entries tid + 256u, u = 0..3:
// bits 0-5 are always tile bits, so each wave reads 1 KiB of consecutive
// amplitudes per load, and each lane has four loads in flight where a lane
// that owns a whole group has 2^K. After a barrier, thread tid computes
// four output rows of one column from LDS; the rows are uniform across the
// wave, so the matrix entries are scalar operands. The outputs go to a
// second LDS tile and leave with the load pattern. One tile per workgroup
// (the grid is the tile count): with a tile loop the compiler hoists the
// four matrix rows out of it and spills scalar registers.
template <int K>
struct TileArgs {
    int tb[10];          // absolute tile bit positions, ascending
    int cpos[10 - K];    // tile-index position of each column bit, ascending
    int offc[1 << K];    // tile-index offset of local index j (bit m <-> target m)
};

template <typename R, int K, typename IT, int NT>
__global__ __launch_bounds__(256) void k_dense_tile(typename V2<R>::T *__restrict__ psi,
                                                    const R *__restrict__ mat, IT n_tiles,
                                                    FixArgs ft, TileArgs<K> ta)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K, NG = D / 4, WPG = 4 / NG;   // row groups, waves per row group
    static_assert(K >= 2 && K <= 4, "four output rows per thread, 1024-entry tile");
    __shared__ C2 tin[1024];
    __shared__ C2 tout[1024];
    const int tid = int(threadIdx.x);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = wave / WPG;                          // output rows 4g .. 4g + 3
    const int col = (wave % WPG) * 64 + (tid & 63);
    int ct = 0;
#pragma unroll
    for (int i = 0; i < 10 - K; ++i) ct |= ((col >> i) & 1) << ta.cpos[i];
    IT off[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u;
        IT o = 0;
#pragma unroll
        for (int i = 0; i < 10; ++i) o |= IT((e >> i) & 1) << ta.tb[i];
        off[u] = o;
    }
    const R *rows = mat + 2 * (4 * g) * D;
    const IT t = xcd_order<IT, kXcdRunDense>(blockIdx.x, gridDim.x);
    if (t >= n_tiles) return;   // whole workgroup: the barriers below stay uniform
    C2 *p = psi + expand<IT>(t, ft);
    C2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = load_amp(p + off[u], NT);
#pragma unroll
    for (int u = 0; u < 4; ++u) tin[lds_slot<C2>(tid + 256 * u)] = v[u];
    __syncthreads();
    R re[4] = {R(0), R(0), R(0), R(0)}, im[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int c = 0; c < D; ++c) {
        const C2 x = tin[lds_slot<C2>(ct | ta.offc[c])];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const R mr = rows[2 * (q * D + c)], mi = rows[2 * (q * D + c) + 1];
            re[q] = fma(mr, x.x, re[q]);
            re[q] = fma(-mi, x.y, re[q]);
            im[q] = fma(mr, x.y, im[q]);
            im[q] = fma(mi, x.x, im[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) tout[lds_slot<C2>(ct | ta.offc[4 * g + q])] = C2{re[q], im[q]};
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = tout[lds_slot<C2>(tid + 256 * u)];
#pragma unroll
    for (int u = 0; u < 4; ++u) store_amp(p + off[u], v[u], NT);
}

// Dense sweep for wide blocks (K = 5, 6) whose groups do not fit one
// thread's registers. A workgroup of 4 waves shares the tile of k_dense_lds
// (2^(6+K) amplitudes, loaded and stored 64 consecutive amplitudes per
// instruction) in LDS; lane l owns group l of the tile and wave w computes
// output rows [w D/4, (w+1) D/4) of all 64 groups. The group's inputs are
// read from LDS 8 at a time and each output row's 8-entry matrix chunk
// arrives through scalar loads (SGPR operands), issued one row ahead; a
// scheduling barrier after each row keeps the compiler from hoisting every
// chunk into SGPRs.
template <typename R, int K, typename IT>
__global__ __launch_bounds__(256) void k_dense_wide(typename V2<R>::T *__restrict__ psi,
                                                    const R *__restrict__ mat, IT n_tiles,
                                                    FixArgs fx, OffArgs<(1 << K)> offl,
                                                    LdsArgs<(1 << K)> la)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K, RW = D / 4;
    __shared__ C2 tile[64 * D];
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = int(threadIdx.x) & 63;
    int lp = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) lp |= ((lane >> b) & 1) << la.lane_pos[b];
    for (IT t = IT(blockIdx.x); t < n_tiles; t += IT(gridDim.x)) {
        C2 *p = psi + expand<IT>(t, fx) + lane;
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int rr = wave * RW + q;
            tile[lds_slot<C2>(lane + 64 * rr)] = p[offl.o[rr]];
        }
        __syncthreads();
        R re[RW], im[RW];
#pragma unroll
        for (int jj = 0; jj < RW; ++jj) re[jj] = im[jj] = R(0);
#pragma unroll 1
        for (int c = 0; c < D / 8; ++c) {
            C2 x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = tile[lds_slot<C2>(lp | la.offc[8 * c + i])];
            // row chunks one ahead: the next row's scalar loads are in
            // flight while the current row's FMAs run
            const R *rows = mat + 2 * (wave * RW * D + 8 * c);
            R cur[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) cur[i] = rows[i];
#pragma unroll
            for (int jj = 0; jj < RW; ++jj) {
                R nxt[16];
                if (jj + 1 < RW) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) nxt[i] = rows[2 * D * (jj + 1) + i];
                }
                // four independent FMA chains per row
                R ra = re[jj], rb = R(0), ia = im[jj], ib = R(0);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const R mr = cur[2 * i], mi = cur[2 * i + 1];
                    ra = fma(mr, x[i].x, ra);
                    rb = fma(-mi, x[i].y, rb);
                    ia = fma(mr, x[i].y, ia);
                    ib = fma(mi, x[i].x, ib);
                }
                re[jj] = ra + rb;
                im[jj] = ia + ib;
                if (jj + 1 < RW) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) cur[i] = nxt[i];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();   // every wave has read the inputs of the tile
#pragma unroll
        for (int jj = 0; jj < RW; ++jj) tile[lds_slot<C2>(lp | la.offc[wave * RW + jj])] = C2{re[jj], im[jj]};
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int rr = wave * RW + q;
            p[offl.o[rr]] = tile[lds_slot<C2>(lane + 64 * rr)];
        }
        __syncthreads();
    }
}

// Dense sweep for groups too wide to keep in one thread's registers: the
// 2^K outputs of a group are split over D/OUTS lanes of the same wave. Every
// lane reads the whole group (cache hits after the first lane) and the
// matrix rows it owns; a wave retires all of its loads before any store, so
// the in-place update is race free.
template <typename R, int K, int OUTS, typename IT>
__global__ __launch_bounds__(kBlock) void k_dense_split(typename V2<R>::T *__restrict__ psi,
                                                        const R *__restrict__ mat, IT n_groups,
                                                        FixArgs fx, OffArgs<(1 << K)> off)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K;
    constexpr int LPG = D / OUTS;
    static_assert(LPG <= 64 && (64 % LPG) == 0, "group must stay inside one wave");
    const IT total = n_groups * LPG;
    const IT stride = IT(gridDim.x) * kBlock;
    for (IT t = IT(blockIdx.x) * kBlock + threadIdx.x; t < total; t += stride) {
        const IT g = t / LPG;
        const int r = int(t % LPG);
        C2 *p = psi + expand<IT>(g, fx);
        R acc[OUTS][2];
#pragma unroll
        for (int o = 0; o < OUTS; ++o) acc[o][0] = acc[o][1] = R(0);
        for (int l = 0; l < D; ++l) {
            const C2 x = p[off.o[l]];
#pragma unroll
            for (int o = 0; o < OUTS; ++o) {
                const int j = r * OUTS + o;
                const R mr = mat[2 * (j * D + l)];
                const R mi = mat[2 * (j * D + l) + 1];
                acc[o][0] = fma(mr, x.x, fma(-mi, x.y, acc[o][0]));
                acc[o][1] = fma(mr, x.y, fma(mi, x.x, acc[o][1]));
            }
        }
#pragma unroll
        for (int o = 0; o < OUTS; ++o) p[off.o[r * OUTS + o]] = C2{acc[o][0], acc[o][1]};
    }
}

// Multiply the amplitudes whose fixed bits match the pinned pattern by one
// phase (a conditional phase shift, Sec. III-B: with both bits pinned only
// a quarter of the vector is read and written).
template <typename R, typename IT>
__global__ __launch_bounds__(kBlock) void k_phase1(typename V2<R>::T *__restrict__ psi, IT n_items,
                                                   FixArgs fx, R pr, R pi)
{
    using C2 = typename V2<R>::T;
    const IT stride = IT(gridDim.x) * kBlock;
    const IT first = xcd_order<IT, kXcdRunElem>(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    for (IT g = first; g < n_items; g += stride) {
        C2 *p = psi + expand<IT>(g, fx);
        const C2 a = load_amp(p, 3);
        store_amp(p, C2{pr * a.x - pi * a.y, pr * a.y + pi * a.x}, 3);
    }
}

// The same phase when some pinned bits lie inside a 128-byte line: writing
// only the selected amplitudes would leave every line partly written, which
// the memory turns into read-modify-writes. Instead every amplitude of the
// lines whose pinned bits above the line match is read and written back,
// multiplied where the in-line bits match too (unchanged amplitudes are
// stored as read, bit for bit).
template <typename R, typename IT>
__global__ __launch_bounds__(kBlock) void k_phase1_lines(typename V2<R>::T *__restrict__ psi, IT n_items,
                                                         FixArgs fx, uint64_t low_mask, uint64_t low_vals, R pr,
                                                         R pi)
{
    using C2 = typename V2<R>::T;
    const IT stride = IT(gridDim.x) * kBlock;
    const IT first = xcd_order<IT, kXcdRunElem>(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    for (IT g = first; g < n_items; g += stride) {
        C2 *p = psi + expand<IT>(g, fx);
        C2 a = load_amp(p, 3);
        if ((uint64_t(p - psi) & low_mask) == low_vals) a = C2{pr * a.x - pi * a.y, pr * a.y + pi * a.x};
        store_amp(p, a, 3);
    }
}

// Diagonal gate: one elementwise pass; the entry is picked by the target
// bits of the index. Controls are pinned as fixed bits.
template <typename R, int K, typename IT>
__global__ __launch_bounds__(kBlock) void k_diag(typename V2<R>::T *__restrict__ psi,
                                                 const R *__restrict__ mat, int row_stride,
                                                 IT n_items, FixArgs fx, OffArgs<K> tg)
{
    using C2 = typename V2<R>::T;
    __shared__ R dsh[2 << K];
    for (int j = threadIdx.x; j < (1 << K); j += kBlock) {
        dsh[2 * j] = mat[2 * (size_t(j) * row_stride + j)];
        dsh[2 * j + 1] = mat[2 * (size_t(j) * row_stride + j) + 1];
    }
    __syncthreads();
    const IT stride = IT(gridDim.x) * kBlock;
    const IT first = xcd_order<IT, kXcdRunElem>(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    for (IT g = first; g < n_items; g += stride) {
        const IT i = expand<IT>(g, fx);
        int j = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) j |= int((i >> tg.o[m]) & 1) << m;
        const R dr = dsh[2 * j], di = dsh[2 * j + 1];
        const C2 a = load_amp(psi + i, 3);
        store_amp(psi + i, C2{dr * a.x - di * a.y, dr * a.y + di * a.x}, 3);
    }
}

// Monomial gate (one nonzero per row and column): out[dst[j]] = c_j in[j].
// Only moved or rescaled entries are touched; entries equal to exactly one
// are moved without arithmetic, so permutation gates are bit-exact.
template <typename R, int K>
struct MonoArgs {
    uint64_t touched;       // bit j: local index j is read and written
    uint64_t unit;          // bit j: c_j == 1 exactly
    uint8_t dst[1 << K];
    R coef[2 << K];
};

template <typename R, int K, typename IT>
__global__ __launch_bounds__(kBlock) void k_monomial(typename V2<R>::T *__restrict__ psi,
                                                     IT n_groups, FixArgs fx,
                                                     OffArgs<(1 << K)> off, MonoArgs<R, K> ma)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K;
    const IT stride = IT(gridDim.x) * kBlock;
    const IT first = xcd_order<IT, kXcdRunElem>(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    for (IT g = first; g < n_groups; g += stride) {
        C2 *p = psi + expand<IT>(g, fx);
        C2 v[D];
#pragma unroll
        for (int j = 0; j < D; ++j)
            if ((ma.touched >> j) & 1) v[j] = p[off.o[j]];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (!((ma.touched >> j) & 1)) continue;
            C2 x = v[j];
            if (!((ma.unit >> j) & 1)) {
                const R cr = ma.coef[2 * j], ci = ma.coef[2 * j + 1];
                x = C2{cr * v[j].x - ci * v[j].y, cr * v[j].y + ci * v[j].x};
            }
            p[off.o[ma.dst[j]]] = x;
        }
    }
}

__global__ void k_cast(const double *__restrict__ src, float *__restrict__ dst, size_t count)
{
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < count;
         i += size_t(gridDim.x) * kBlock)
        dst[i] = float(src[i]);
}

template <typename R>
__global__ void k_fill_basis(typename V2<R>::T *__restrict__ psi, uint64_t dim, uint64_t index)
{
    using C2 = typename V2<R>::T;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < dim;
         i += uint64_t(gridDim.x) * kBlock)
        psi[i] = C2{R(i == index ? 1 : 0), R(0)};
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
unsigned grid_for(uint64_t items)
{
    uint64_t b = (items + kBlock - 1) / kBlock;
    const uint64_t cap = 1ull << 22;  // grid-stride beyond 2^30 threads
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return unsigned(b);
}

int make_fix(const int *pos, int npos, uint64_t vals, FixArgs &f)
{
    if (npos > kMaxFix) return fail(QS_EUNSUPPORTED, "more than %d fixed qubits", kMaxFix);
    f.nfix = npos;
    int tmp[64];
    std::copy(pos, pos + npos, tmp);
    std::sort(tmp, tmp + npos);
    for (int i = 0; i < npos; ++i) f.pos[i] = tmp[i];
    f.vals = vals;
    return QS_OK;
}

int fixed_positions(const GateDesc &d, bool with_targets, int *out)
{
    int c = 0;
    if (with_targets)
        for (int m = 0; m < d.k; ++m) out[c++] = d.targets[m];
    for (int q = 0; q < 64; ++q)
        if ((d.ctrl_mask >> q) & 1) out[c++] = q;
    return c;
}

template <int D>
void make_off(const GateDesc &d, OffArgs<D> &o)
{
    for (int j = 0; j < D; ++j) {
        uint64_t v = 0;
        for (int m = 0; m < d.k; ++m)
            if ((j >> m) & 1) v |= 1ull << d.targets[m];
        o.o[j] = v;
    }
}

template <typename R, typename IT, int K>
int dense_k(qs_state *h, const GateDesc &d, const void *dmat)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K;
    FixArgs fx;
    int pos[64];
    int np = fixed_positions(d, true, pos);
    if (int rc = make_fix(pos, np, d.ctrl_vals, fx)) return rc;
    OffArgs<D> off;
    make_off<D>(d, off);
    const IT n_groups = IT(h->dim() >> np);
    C2 *psi = static_cast<C2 *>(h->psi);
    const R *m = static_cast<const R *>(dmat);
    int mint = 64;
    for (int i = 0; i < K; ++i) mint = std::min(mint, d.targets[i]);
    // tuned choices for this (dtype, k, target class, n bucket); 0 = default
    const int cls = tune_class(mint, h->dtype), nb = tune_nbucket(h->n);
    const int path = tune_value(QS_TUNE_SWEEP_PATH, h->dtype, K, cls, nb);
    const int wg_per_cu = tune_value(QS_TUNE_SWEEP_WG_PER_CU, h->dtype, K, cls, nb);
    const int nt = tune_value(QS_TUNE_SWEEP_NT, h->dtype, K, cls, nb);
    auto capped = [&](uint64_t g) {
        if (wg_per_cu) g = std::min<uint64_t>(g, uint64_t(wg_per_cu) * uint64_t(device_cus()));
        return unsigned(std::max<uint64_t>(g, 1));
    };
    // 5- and 6-qubit blocks on complex64 states: batched GEMM on the matrix
    // cores
    if constexpr (sizeof(R) == 4 && K >= 5) {
        if ((path == 0 || path == 3) && mfma_applicable(h, d)) return launch_dense_mfma(h, d, dmat);
    }
    // complex128 blocks of 2 to 4 qubits on states of 20 qubits or more
    // default to the workgroup-shared 1024-amplitude tile
    if constexpr (K >= 2 && K <= 4) {
        const bool wt_ok = d.ctrl_mask == 0 && h->n >= 10;
        if (wt_ok && (path == 5 || (path == 0 && sizeof(R) == 8 && h->n >= 20))) {
            uint64_t tmask = 0;
            for (int i = 0; i < K; ++i) tmask |= 1ull << d.targets[i];
            std::vector<int> tb(d.targets, d.targets + K), cols;
            for (int b = 0; int(cols.size()) < 10 - K; ++b)
                if (!((tmask >> b) & 1)) cols.push_back(b);
            tb.insert(tb.end(), cols.begin(), cols.end());
            std::sort(tb.begin(), tb.end());
            auto tpos = [&](int b) { return int(std::lower_bound(tb.begin(), tb.end(), b) - tb.begin()); };
            TileArgs<K> ta;
            for (int i = 0; i < 10; ++i) ta.tb[i] = tb[size_t(i)];
            for (int i = 0; i < 10 - K; ++i) ta.cpos[i] = tpos(cols[size_t(i)]);
            for (int j = 0; j < D; ++j) {
                int o = 0;
                for (int m = 0; m < K; ++m)
                    if ((j >> m) & 1) o |= 1 << tpos(d.targets[m]);
                ta.offc[j] = o;
            }
            FixArgs ft;
            if (int rc = make_fix(tb.data(), 10, 0, ft)) return rc;
            const IT n_tiles = IT(h->dim() >> 10);
            if (uint64_t(n_tiles) > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "tile grid of %llu workgroups", (unsigned long long)n_tiles);
            const unsigned grid = unsigned(n_tiles);   // one tile per workgroup; no grid cap
            with_nt(nt, [&](auto c) {
                hipLaunchKernelGGL((k_dense_tile<R, K, IT, decltype(c)::value>), dim3(grid), dim3(256), 0,
                                   h->stream, psi, m, n_tiles, ft, ta);
            });
            QS_HIP(hipGetLastError());
            return QS_OK;
        }
    }
    // by default, targets inside a 128-byte line stage the tile through LDS
    // (one wave per tile); wide complex128 blocks share a tile per workgroup
    constexpr int kLineBits = sizeof(R) == 8 ? 3 : 4;
    constexpr bool lds_capable = (sizeof(R) == 8) ? (K <= 5) : (K <= 6);
    constexpr bool wide_capable = K >= 5;
    constexpr bool wide_default = K >= 5;
    const bool tile_ok = d.ctrl_mask == 0 && h->n >= 6 + K;
    const bool use_wide = wide_capable && tile_ok && (path == 4 || (path == 0 && wide_default));
    const bool use_lds = lds_capable && tile_ok && !use_wide && (path == 2 || (path != 1 && path != 4 && mint < kLineBits));
    if (use_wide || use_lds) {
        {
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
            OffArgs<D> offl;
            for (int r = 0; r < D; ++r) {
                uint64_t o = 0;
                for (int i = 0; i < K; ++i)
                    if ((r >> i) & 1) o |= 1ull << P[size_t(6 + i)];
                offl.o[r] = o;
            }
            LdsArgs<D> la;
            std::vector<int> lane_bits;
            for (int b = 0; b < 6; ++b)
                if (!((tmask >> b) & 1)) lane_bits.push_back(b);
            for (int b : extra) lane_bits.push_back(b);
            for (int b = 0; b < 6; ++b) la.lane_pos[b] = compact(lane_bits[size_t(b)]);
            for (int j = 0; j < D; ++j) {
                int o = 0;
                for (int i = 0; i < K; ++i)
                    if ((j >> i) & 1) o |= 1 << compact(d.targets[i]);
                la.offc[j] = o;
            }
            FixArgs ft;
            if (int rc = make_fix(P.data(), int(P.size()), 0, ft)) return rc;
            const IT n_tiles = IT(h->dim() >> (6 + K));
            const unsigned grid = capped(std::min<uint64_t>(uint64_t(n_tiles), 1ull << 22));
            if (use_wide) {
                if constexpr (wide_capable)
                    hipLaunchKernelGGL((k_dense_wide<R, K, IT>), dim3(grid), dim3(256), 0, h->stream, psi, m,
                                       n_tiles, ft, offl, la);
            } else if constexpr (lds_capable) {
                with_nt(nt, [&](auto c) {
                    hipLaunchKernelGGL((k_dense_lds<R, K, IT, decltype(c)::value>), dim3(grid), dim3(64), 0,
                                       h->stream, psi, m, n_tiles, ft, offl, la);
                });
            }
            QS_HIP(hipGetLastError());
            return QS_OK;
        }
    }
    constexpr bool split = (sizeof(R) == 8 && K >= 6);
    if constexpr (split) {
        hipLaunchKernelGGL((k_dense_split<R, K, 8, IT>), dim3(capped(grid_for(uint64_t(n_groups) * (D / 8)))),
                           dim3(kBlock), 0, h->stream, psi, m, n_groups, fx, off);
    } else {
        with_nt(nt, [&](auto c) {
            hipLaunchKernelGGL((k_dense<R, K, IT, decltype(c)::value>), dim3(capped(grid_for(n_groups))),
                               dim3(kBlock), 0, h->stream, psi, m, n_groups, fx, off);
        });
    }
    QS_HIP(hipGetLastError());
    return QS_OK;
}

template <typename R, typename IT>
int dense_dispatch(qs_state *h, const GateDesc &d, const void *dmat)
{
    switch (d.k) {
    case 1: return dense_k<R, IT, 1>(h, d, dmat);
    case 2: return dense_k<R, IT, 2>(h, d, dmat);
    case 3: return dense_k<R, IT, 3>(h, d, dmat);
    case 4: return dense_k<R, IT, 4>(h, d, dmat);
    case 5: return dense_k<R, IT, 5>(h, d, dmat);
    case 6: return dense_k<R, IT, 6>(h, d, dmat);
    default: return fail(QS_EUNSUPPORTED, "dense gate width %d", d.k);
    }
}

template <typename R, typename IT, int K>
int diag_k(qs_state *h, const GateDesc &d, const void *dmat, int row_stride)
{
    using C2 = typename V2<R>::T;
    FixArgs fx;
    int pos[64];
    int np = fixed_positions(d, false, pos);
    if (int rc = make_fix(pos, np, d.ctrl_vals, fx)) return rc;
    OffArgs<K> tg;
    for (int m = 0; m < K; ++m) tg.o[m] = uint64_t(d.targets[m]);
    const IT n_items = IT(h->dim() >> np);
    hipLaunchKernelGGL((k_diag<R, K, IT>), dim3(grid_for(n_items)), dim3(kBlock), 0, h->stream,
                       static_cast<C2 *>(h->psi), static_cast<const R *>(dmat), row_stride,
                       n_items, fx, tg);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

// The same kernel restricted to the amplitudes whose high target bits (and
// controls) equal one pinned pattern: those bits join the fixed positions,
// so a launch touches 2^-npin of the state. Targets inside a 128-byte line
// stay free and pick their entry from the table, so whole lines are read
// and written.
template <typename R, typename IT, int K>
int diag_pinned_k(qs_state *h, const GateDesc &d, const void *dmat, int row_stride, const int *pin,
                  int npin, uint64_t pin_vals)
{
    using C2 = typename V2<R>::T;
    FixArgs fx;
    if (int rc = make_fix(pin, npin, pin_vals, fx)) return rc;
    OffArgs<K> tg;
    for (int m = 0; m < K; ++m) tg.o[m] = uint64_t(d.targets[m]);
    const IT n_items = IT(h->dim() >> npin);
    hipLaunchKernelGGL((k_diag<R, K, IT>), dim3(grid_for(n_items)), dim3(kBlock), 0, h->stream,
                       static_cast<C2 *>(h->psi), static_cast<const R *>(dmat), row_stride,
                       n_items, fx, tg);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

template <typename R, typename IT>
int diag_pinned_dispatch(qs_state *h, const GateDesc &d, const void *dmat, int row_stride, const int *pin,
                         int npin, uint64_t pin_vals)
{
    switch (d.k) {
    case 1: return diag_pinned_k<R, IT, 1>(h, d, dmat, row_stride, pin, npin, pin_vals);
    case 2: return diag_pinned_k<R, IT, 2>(h, d, dmat, row_stride, pin, npin, pin_vals);
    case 3: return diag_pinned_k<R, IT, 3>(h, d, dmat, row_stride, pin, npin, pin_vals);
    case 4: return diag_pinned_k<R, IT, 4>(h, d, dmat, row_stride, pin, npin, pin_vals);
    case 5: return diag_pinned_k<R, IT, 5>(h, d, dmat, row_stride, pin, npin, pin_vals);
    case 6: return diag_pinned_k<R, IT, 6>(h, d, dmat, row_stride, pin, npin, pin_vals);
    default: return fail(QS_EUNSUPPORTED, "diagonal gate width %d", d.k);
    }
}

template <typename R, typename IT>
int diag_dispatch(qs_state *h, const GateDesc &d, const void *dmat, int row_stride)
{
    switch (d.k) {
    case 1: return diag_k<R, IT, 1>(h, d, dmat, row_stride);
    case 2: return diag_k<R, IT, 2>(h, d, dmat, row_stride);
    case 3: return diag_k<R, IT, 3>(h, d, dmat, row_stride);
    case 4: return diag_k<R, IT, 4>(h, d, dmat, row_stride);
    case 5: return diag_k<R, IT, 5>(h, d, dmat, row_stride);
    case 6: return diag_k<R, IT, 6>(h, d, dmat, row_stride);
    default: return fail(QS_EUNSUPPORTED, "diagonal gate width %d", d.k);
    }
}

template <typename R, typename IT, int K>
int mono_k(qs_state *h, const GateDesc &d, const double *hmat)
{
    using C2 = typename V2<R>::T;
    constexpr int D = 1 << K;
    FixArgs fx;
    int pos[64];
    int np = fixed_positions(d, true, pos);
    if (int rc = make_fix(pos, np, d.ctrl_vals, fx)) return rc;
    OffArgs<D> off;
    make_off<D>(d, off);
    MonoArgs<R, K> ma;
    std::memset(&ma, 0, sizeof ma);
    for (int j = 0; j < D; ++j) {
        const int dj = d.perm_dst[j];
        const double cr = hmat[2 * (size_t(dj) * D + j)], ci = hmat[2 * (size_t(dj) * D + j) + 1];
        ma.dst[j] = uint8_t(dj);
        ma.coef[2 * j] = R(cr);
        ma.coef[2 * j + 1] = R(ci);
        const bool unit = (cr == 1.0 && ci == 0.0);
        if (unit) ma.unit |= 1ull << j;
        if (!unit || dj != j) ma.touched |= 1ull << j;
    }
    const IT n_groups = IT(h->dim() >> np);
    hipLaunchKernelGGL((k_monomial<R, K, IT>), dim3(grid_for(n_groups)), dim3(kBlock), 0, h->stream,
                       static_cast<C2 *>(h->psi), n_groups, fx, off, ma);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

template <typename R, typename IT>
int mono_dispatch(qs_state *h, const GateDesc &d, const double *hmat)
{
    switch (d.k) {
    case 1: return mono_k<R, IT, 1>(h, d, hmat);
    case 2: return mono_k<R, IT, 2>(h, d, hmat);
    case 3: return mono_k<R, IT, 3>(h, d, hmat);
    case 4: return mono_k<R, IT, 4>(h, d, hmat);
    case 5: return mono_k<R, IT, 5>(h, d, hmat);
    case 6: return mono_k<R, IT, 6>(h, d, hmat);
    default: return fail(QS_EUNSUPPORTED, "monomial gate width %d", d.k);
    }
}

template <typename R, typename IT>
int phase1_t(qs_state *h, const GateDesc &d, double pr, double pi)
{
    using C2 = typename V2<R>::T;
    FixArgs fx;
    int pos[64];
    int np = fixed_positions(d, true, pos);
    uint64_t vals = d.ctrl_vals;
    for (int m = 0; m < d.k; ++m)
        if ((d.phase_index >> m) & 1) vals |= 1ull << d.targets[m];
    constexpr int kLineBits = sizeof(R) == 8 ? 3 : 4;
    int hi[64], nhi = 0;
    uint64_t low_mask = 0;
    for (int i = 0; i < np; ++i) {
        if (pos[i] < kLineBits) low_mask |= 1ull << pos[i];
        else hi[nhi++] = pos[i];
    }
    if (low_mask) {
        uint64_t hi_vals = vals & ~low_mask;
        if (int rc = make_fix(hi, nhi, hi_vals, fx)) return rc;
        const IT n_items = IT(h->dim() >> nhi);
        hipLaunchKernelGGL((k_phase1_lines<R, IT>), dim3(grid_for(n_items)), dim3(kBlock), 0, h->stream,
                           static_cast<C2 *>(h->psi), n_items, fx, low_mask, vals & low_mask, R(pr), R(pi));
        QS_HIP(hipGetLastError());
        return QS_OK;
    }
    if (int rc = make_fix(pos, np, vals, fx)) return rc;
    const IT n_items = IT(h->dim() >> np);
    hipLaunchKernelGGL((k_phase1<R, IT>), dim3(grid_for(n_items)), dim3(kBlock), 0, h->stream,
                       static_cast<C2 *>(h->psi), n_items, fx, R(pr), R(pi));
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Exact structure classification (no tolerance: a structured gate must be
// structured bit for bit, otherwise the dense sweep is used).
// ---------------------------------------------------------------------------
void classify(const double *m, int k, GateDesc &d)
{
    const int D = 1 << k;
    auto re = [&](int r, int c) { return m[2 * (size_t(r) * D + c)]; };
    auto im = [&](int r, int c) { return m[2 * (size_t(r) * D + c) + 1]; };
    auto nz = [&](int r, int c) { return re(r, c) != 0.0 || im(r, c) != 0.0; };
    bool diag = true;
    for (int r = 0; r < D && diag; ++r)
        for (int c = 0; c < D; ++c)
            if (r != c && nz(r, c)) { diag = false; break; }
    if (diag) {
        int nonunit = 0, idx = 0;
        for (int j = 0; j < D; ++j)
            if (!(re(j, j) == 1.0 && im(j, j) == 0.0)) { ++nonunit; idx = j; }
        if (nonunit == 0) { d.cls = GC_IDENTITY; return; }
        if (nonunit == 1) { d.cls = GC_PHASE1; d.phase_index = idx; return; }
        d.cls = GC_DIAG;
        return;
    }
    // monomial: exactly one nonzero in every column and every row
    std::vector<int> row_used(D, 0);
    for (int c = 0; c < D; ++c) {
        int cnt = 0, rr = -1;
        for (int r = 0; r < D; ++r)
            if (nz(r, c)) { ++cnt; rr = r; }
        if (cnt != 1 || row_used[rr]) { d.cls = GC_DENSE; return; }
        row_used[rr] = 1;
        d.perm_dst[c] = rr;
    }
    d.cls = GC_MONOMIAL;
}

int launch_dense(qs_state *h, const GateDesc &d, const void *dmat)
{
    const bool small = h->n <= 31;
    if (h->dtype == QS_C128)
        return small ? dense_dispatch<double, uint32_t>(h, d, dmat)
                     : dense_dispatch<double, uint64_t>(h, d, dmat);
    return small ? dense_dispatch<float, uint32_t>(h, d, dmat)
                 : dense_dispatch<float, uint64_t>(h, d, dmat);
}

int launch_diag(qs_state *h, const GateDesc &d, const void *dmat, int row_stride)
{
    const bool small = h->n <= 31;
    if (h->dtype == QS_C128)
        return small ? diag_dispatch<double, uint32_t>(h, d, dmat, row_stride)
                     : diag_dispatch<double, uint64_t>(h, d, dmat, row_stride);
    return small ? diag_dispatch<float, uint32_t>(h, d, dmat, row_stride)
                 : diag_dispatch<float, uint64_t>(h, d, dmat, row_stride);
}

// Fraction of the state a diagonal block must change: the local indices
// whose entry is not exactly one, over 2^k.
double diag_changed_fraction(const double *hdiag, int k)
{
    int cnt = 0;
    for (int j = 0; j < (1 << k); ++j)
        if (!(hdiag[2 * j] == 1.0 && hdiag[2 * j + 1] == 0.0)) ++cnt;
    return double(cnt) / double(1 << k);
}

// A diagonal block whose entries are known on the host (hdiag: 2^k complex
// FP64 values, the block matrix's diagonal). A conditional phase shift moves
// only the amplitudes that carry its phase (Sec. III-B); a product of them
// (CZ layers, controlled phases fused into one block) is treated the same
// way: only the patterns of the targets whose entry differs from one are
// swept. With all entries one nothing is launched; with one entry the phase
// kernel runs; otherwise every distinct pattern of the targets above the
// 128-byte line (those inside a line pick their entry per amplitude, so
// whole lines are rewritten) gets one pinned launch, unless the pinned
// launches together would touch more than half the state, in which case one
// elementwise pass over the state is cheaper.
int launch_phase1_host(qs_state *h, const GateDesc &d, double pr, double pi);

int launch_diag_block(qs_state *h, const GateDesc &din, const void *dmat, int row_stride, const double *hdiag)
{
    const int K = din.k, D = 1 << K;
    std::vector<int> changed;
    for (int j = 0; j < D; ++j)
        if (!(hdiag[2 * j] == 1.0 && hdiag[2 * j + 1] == 0.0)) changed.push_back(j);
    if (changed.empty()) return QS_OK;
    if (changed.size() == 1) {
        GateDesc d = din;
        d.cls = GC_PHASE1;
        d.phase_index = changed[0];
        const size_t j = size_t(changed[0]);
        return launch_phase1_host(h, d, hdiag[2 * j], hdiag[2 * j + 1]);
    }
    const int line_bits = h->amp_bytes() == 16 ? 3 : 4;
    int hi_bit[QS_MAX_K], nhi = 0;
    uint32_t hi_mask = 0;
    for (int m = 0; m < K; ++m)
        if (din.targets[m] >= line_bits) {
            hi_bit[nhi++] = m;
            hi_mask |= 1u << m;
        }
    std::vector<uint32_t> pats;
    for (int j : changed) pats.push_back(uint32_t(j) & hi_mask);
    std::sort(pats.begin(), pats.end());
    pats.erase(std::unique(pats.begin(), pats.end()), pats.end());
    GateDesc d = din;
    d.cls = GC_DIAG;
    if (2 * pats.size() > (size_t(1) << nhi)) return launch_diag(h, d, dmat, row_stride);
    int pin[64], npin = 0;
    for (int i = 0; i < nhi; ++i) pin[npin++] = din.targets[hi_bit[i]];
    for (int q = 0; q < 64; ++q)
        if ((din.ctrl_mask >> q) & 1) pin[npin++] = q;
    const bool small = h->n <= 31;
    for (uint32_t pt : pats) {
        uint64_t vals = din.ctrl_vals;
        for (int i = 0; i < nhi; ++i)
            if ((pt >> hi_bit[i]) & 1) vals |= 1ull << din.targets[hi_bit[i]];
        int rc;
        if (h->dtype == QS_C128)
            rc = small ? diag_pinned_dispatch<double, uint32_t>(h, d, dmat, row_stride, pin, npin, vals)
                       : diag_pinned_dispatch<double, uint64_t>(h, d, dmat, row_stride, pin, npin, vals);
        else
            rc = small ? diag_pinned_dispatch<float, uint32_t>(h, d, dmat, row_stride, pin, npin, vals)
                       : diag_pinned_dispatch<float, uint64_t>(h, d, dmat, row_stride, pin, npin, vals);
        if (rc) return rc;
    }
    return QS_OK;
}

int launch_monomial_host(qs_state *h, const GateDesc &d, const double *hmat)
{
    const bool small = h->n <= 31;
    if (h->dtype == QS_C128)
        return small ? mono_dispatch<double, uint32_t>(h, d, hmat)
                     : mono_dispatch<double, uint64_t>(h, d, hmat);
    return small ? mono_dispatch<float, uint32_t>(h, d, hmat)
                 : mono_dispatch<float, uint64_t>(h, d, hmat);
}

int launch_phase1_host(qs_state *h, const GateDesc &d, double pr, double pi)
{
    const bool small = h->n <= 31;
    if (h->dtype == QS_C128)
        return small ? phase1_t<double, uint32_t>(h, d, pr, pi) : phase1_t<double, uint64_t>(h, d, pr, pi);
    return small ? phase1_t<float, uint32_t>(h, d, pr, pi) : phase1_t<float, uint64_t>(h, d, pr, pi);
}

int launch_cast_f64_to_f32(hipStream_t s, const double *src, float *dst, size_t count)
{
    hipLaunchKernelGGL(k_cast, dim3(grid_for(count)), dim3(kBlock), 0, s, src, dst, count);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

int launch_set_basis(qs_state *h, uint64_t index)
{
    if (h->dtype == QS_C128)
        hipLaunchKernelGGL(k_fill_basis<double>, dim3(grid_for(h->dim())), dim3(kBlock), 0,
                           h->stream, static_cast<double2 *>(h->psi), h->dim(), index);
    else
        hipLaunchKernelGGL(k_fill_basis<float>, dim3(grid_for(h->dim())), dim3(kBlock), 0,
                           h->stream, static_cast<float2 *>(h->psi), h->dim(), index);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

// One gate with its FP64 matrix on the host: classify, stage what the
// chosen kernel reads, launch.
int enqueue_gate(qs_state *h, const GateDesc &din, const double *hmat)
{
    GateDesc d = din;
    classify(hmat, d.k, d);
    const size_t D = size_t(1) << d.k;
    switch (d.cls) {
    case GC_IDENTITY:
        return QS_OK;
    case GC_PHASE1: {
        const size_t j = size_t(d.phase_index);
        return launch_phase1_host(h, d, hmat[2 * (j * D + j)], hmat[2 * (j * D + j) + 1]);
    }
    case GC_MONOMIAL:
        return launch_monomial_host(h, d, hmat);
    default:
        break;
    }
    // dense and diagonal kernels read the matrix from device memory
    const size_t count = 2 * D * D;
    void *dm = nullptr;
    if (int rc = h->stage.put(h->stream, hmat, count * sizeof(double), &dm)) return rc;
    if (h->dtype == QS_C64) {
        void *d32 = nullptr;
        if (int rc = h->stage.reserve(h->stream, count * sizeof(float), &d32)) return rc;
        if (int rc = launch_cast_f64_to_f32(h->stream, static_cast<double *>(dm),
                                            static_cast<float *>(d32), count))
            return rc;
        dm = d32;
    }
    if (d.cls == GC_DIAG) {
        std::vector<double> hdiag(2 * D);
        for (size_t j = 0; j < D; ++j) {
            hdiag[2 * j] = hmat[2 * (j * D + j)];
            hdiag[2 * j + 1] = hmat[2 * (j * D + j) + 1];
        }
        return launch_diag_block(h, d, dm, int(D), hdiag.data());
    }
    return launch_dense(h, d, dm);
}

}  // namespace qs
