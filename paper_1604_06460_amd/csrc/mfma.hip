// Fused 6-qubit blocks on complex64 states as a batched GEMM on the matrix
// cores. A sweep computes Y = M X for every group X of 64 amplitudes that
// agree outside the block's qubits (the Kronecker structure of Sec. II). In
// real block form
//   [Yr]   [Mr  -Mi] [Xr]
//   [Yi] = [Mi   Mr] [Xi]
// this is a 128 x 128 real matrix times 128 x G real columns, with 8 flops
// per complex multiply-add, 32 flop per byte moved: past the FP32 vector
// ridge, so the FP32 MFMA units (v_mfma_f32_32x32x2_f32, FP32 inputs, FP32
// accumulation) carry it.
//
// Workgroup: 4 waves, persistent over tiles of 64 groups (4096 amplitudes,
// 32 KiB); the next tile is prefetched into registers during the MFMA loop. The tile spans index bits 0..5, the block qubits above bit 5 and
// the lowest free bits above 5 (as many as there are block qubits below 6),
// so loads and stores move 64 consecutive amplitudes per wave instruction;
// an LDS layout switch regroups the tile into 64 columns of 64 amplitudes.
// Wave w owns real output rows [32w, 32w+32) and keeps its 32 x 128 slice of
// the real block matrix in 64 VGPRs for the whole kernel (A operand: lane l
// holds row l%32 of the slice at k = 2s + l/32). For each half of the tile
// (32 groups) it runs 64 MFMA steps over k; the B operand of step s is the
// real-form element k = 2s + l/32 of group 32h + l%32, read from LDS.
// Accumulator register v of lane l holds row 8(v/4) + 4(l/32) + v%4 of the
// 32 x 32 output block and column l%32.
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

template <typename IT>
__device__ __forceinline__ IT expand_tile(IT g, const TileArgs &ta)
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

}  // namespace

bool mfma_applicable(const qs_state *h, const GateDesc &d)
{
    return h->dtype == QS_C64 && d.k == 6 && d.ctrl_mask == 0 && h->n >= 12;
}

int launch_dense_mfma(qs_state *h, const GateDesc &d, const void *dmat)
{
    const float *m = static_cast<const float *>(dmat);
    return h->n <= 31 ? launch_t<uint32_t>(h, d, m) : launch_t<uint64_t>(h, d, m);
}

}  // namespace qs
