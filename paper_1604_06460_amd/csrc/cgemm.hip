// Complex GEMM on the matrix cores for the dense-unitary route of phase
// estimation (Sec. III-C): C = op(A) B with A square-ish (M x K), B and C
// given as column lists (so strided-batched products over a state are one
// launch). Complex128 runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), complex64 on the FP32 ones
// (v_mfma_f32_16x16x4f32); the complex product is four real products,
// Re C = Re A Re B - Im A Im B, Im C = Re A Im B + Im A Re B, so the real
// work equals the complex work (8 flops per complex multiply-add).
//
// Tiling: a 256-thread workgroup owns a BM x BM tile of C (BM = 128, or 64
// when 128-tiles would leave compute units idle); its four waves each own a
// quarter as (BM/32) x (BM/32) MFMA tiles of 16 x 16, with real and
// imaginary accumulators (128 values per lane at BM = 128). K advances 8
// complex entries at a time: the A and B panels (BM x 8 each) are staged in
// LDS as separate real and imaginary planes laid out [k][row] / [k][col],
// so every fragment read is 16 consecutive values per quarter-wave. The
// next panel is loaded into registers while the current one is multiplied
// and then written to the second of two LDS buffers, so each K step needs
// one barrier.
//
// MFMA lane layouts (16x16x4, checked on the device): A[i][k] in lane
// i + 16k and B[k][j] in lane j + 16k for both precisions; D[i][j] is in
// lane j + 16 (i / 4), slot i % 4 for FP32 but in lane j + 16 (i % 4), slot
// i / 4 for FP64.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBK = 8, kThreads = 256;

template <typename R> struct Cx;
template <> struct Cx<double> {
    using T = double2;
    typedef double V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mfma(double a, double b, V4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output row of slot r in a lane whose quarter is q = lane / 16
    static __device__ __forceinline__ int row(int q, int r) { return 4 * r + q; }
};
template <> struct Cx<float> {
    using T = float2;
    typedef float V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mfma(float a, float b, V4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
};

__device__ __forceinline__ uint64_t col_off(const ColMap &m, uint64_t c)
{
    return m.base + ((c >> m.runs_log) << m.stride_log) + (c & ((uint64_t(1) << m.runs_log) - 1)) * m.ld;
}

template <typename R, bool CONJ_A, int BM>
__global__ __launch_bounds__(kThreads, BM == 128 ? 1 : 2) void k_cgemm(const typename Cx<R>::T *__restrict__ A, int64_t lda, int M,
                                                        int K, const typename Cx<R>::T *__restrict__ B, ColMap bm,
                                                        typename Cx<R>::T *__restrict__ C, ColMap cm, uint64_t ncols)
{
    using C2 = typename Cx<R>::T;
    using V4 = typename Cx<R>::V4;
    constexpr int kBM = BM, kBN = BM;
    constexpr int TX = BM / 32;          // MFMA tiles per wave and direction
    constexpr int Q = BM / 32;           // panel elements per thread
    constexpr int TPR = kBK / Q;         // threads per k-contiguous panel row
    // two panel buffers: the next panel is written while the current one is
    // read, so one barrier per K step suffices
    __shared__ R a_re[2][kBK * kBM], a_im[2][kBK * kBM], b_re[2][kBK * kBN], b_im[2][kBK * kBN];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * kBM;
    const uint64_t n0 = uint64_t(blockIdx.x) * kBN;
    const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * (BM / 2);

    // global -> register panel loads: 4 complex per thread for A and for B
    // A (op = N): column k of the panel is 128 contiguous rows; thread t
    //   takes k = t / 32, rows 4 (t % 32) .. +3.
    // A (op = C): op(A)[i][k] = conj(A[k][i]); row i of op(A) is column i of A,
    //   contiguous in k; thread t takes i = t / 2, k = 4 (t % 2) .. +3.
    // B: column j contiguous in k; thread t takes j = t / 2, k = 4 (t % 2) .. +3.
    C2 ra[Q], rb[Q];
    const int bj = t / TPR, bk = (t % TPR) * Q;
    const uint64_t bcol = n0 + uint64_t(bj);
    const bool bcol_ok = bcol < ncols;
    const uint64_t boff = bcol_ok ? col_off(bm, bcol) : 0;

    auto load_panel = [&](int k0) {
        if constexpr (!CONJ_A) {
            const int ak = t >> 5, ai = (t & 31) * Q;
            const int k = k0 + ak;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int i = m0 + ai + q;
                ra[q] = (k < K && i < M) ? A[int64_t(i) + int64_t(k) * lda] : C2{0, 0};
            }
        } else {
            const int ai = t / TPR, ak = (t % TPR) * Q;
            const int i = m0 + ai;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int k = k0 + ak + q;
                ra[q] = (k < K && i < M) ? A[int64_t(k) + int64_t(i) * lda] : C2{0, 0};
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = k0 + bk + q;
            rb[q] = (bcol_ok && k < K) ? B[boff + uint64_t(k)] : C2{0, 0};
        }
    };
    auto store_panel = [&](int buf) {
        if constexpr (!CONJ_A) {
            const int ak = t >> 5, ai = (t & 31) * Q;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                a_re[buf][ak * kBM + ai + q] = ra[q].x;
                a_im[buf][ak * kBM + ai + q] = ra[q].y;
            }
        } else {
            const int ai = t / TPR, ak = (t % TPR) * Q;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                a_re[buf][(ak + q) * kBM + ai] = ra[q].x;
                a_im[buf][(ak + q) * kBM + ai] = -ra[q].y;
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            b_re[buf][(bk + q) * kBN + bj] = rb[q].x;
            b_im[buf][(bk + q) * kBN + bj] = rb[q].y;
        }
    };

    V4 acc_re[TX][TX], acc_im[TX][TX];
#pragma unroll
    for (int x = 0; x < TX; ++x)
#pragma unroll
        for (int y = 0; y < TX; ++y) {
            acc_re[x][y] = V4{0, 0, 0, 0};
            acc_im[x][y] = V4{0, 0, 0, 0};
        }

    const int fi = lane & 15, fk = lane >> 4;
    load_panel(0);
    store_panel(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += kBK) {
        const bool more = k0 + kBK < K;
        if (more) load_panel(k0 + kBK);   // in flight during this step's products
#pragma unroll
        for (int ks = 0; ks < kBK; ks += 4) {
            R ar[TX], ai[TX], br[TX], bi[TX], nai[TX];
#pragma unroll
            for (int x = 0; x < TX; ++x) {
                ar[x] = a_re[cur][(ks + fk) * kBM + wr + 16 * x + fi];
                ai[x] = a_im[cur][(ks + fk) * kBM + wr + 16 * x + fi];
                nai[x] = -ai[x];
            }
#pragma unroll
            for (int y = 0; y < TX; ++y) {
                br[y] = b_re[cur][(ks + fk) * kBN + wc + 16 * y + fi];
                bi[y] = b_im[cur][(ks + fk) * kBN + wc + 16 * y + fi];
            }
            // four sweeps over the tiles, so that consecutive updates of one
            // accumulator are 2 TX TY instructions apart (no dependent issue)
#pragma unroll
            for (int x = 0; x < TX; ++x)
#pragma unroll
                for (int y = 0; y < TX; ++y) acc_re[x][y] = Cx<R>::mfma(ar[x], br[y], acc_re[x][y]);
#pragma unroll
            for (int x = 0; x < TX; ++x)
#pragma unroll
                for (int y = 0; y < TX; ++y) acc_im[x][y] = Cx<R>::mfma(ar[x], bi[y], acc_im[x][y]);
#pragma unroll
            for (int x = 0; x < TX; ++x)
#pragma unroll
                for (int y = 0; y < TX; ++y) acc_re[x][y] = Cx<R>::mfma(nai[x], bi[y], acc_re[x][y]);
#pragma unroll
            for (int x = 0; x < TX; ++x)
#pragma unroll
                for (int y = 0; y < TX; ++y) acc_im[x][y] = Cx<R>::mfma(ai[x], br[y], acc_im[x][y]);
        }
        if (more) store_panel(cur ^ 1);   // last read in the previous step
        __syncthreads();
        cur ^= 1;
    }
    // epilogue: lane holds four rows (Cx::row) of column lane % 16 of every
    // 16 x 16 tile
#pragma unroll
    for (int y = 0; y < TX; ++y) {
        const uint64_t col = n0 + uint64_t(wc + 16 * y + fi);
        if (col >= ncols) continue;
        C2 *cp = C + col_off(cm, col);
#pragma unroll
        for (int x = 0; x < TX; ++x)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr + 16 * x + Cx<R>::row(fk, r);
                if (row < M) cp[row] = C2{acc_re[x][y][r], acc_im[x][y][r]};
            }
    }
}

template <typename R, int BM>
void launch_tile(hipStream_t s, bool conj_a, const void *A, int64_t lda, int M, int K, const void *B, ColMap bm,
                 void *C, ColMap cm, uint64_t ncols, dim3 grid)
{
    using C2 = typename Cx<R>::T;
    const auto *a = static_cast<const C2 *>(A);
    const auto *b = static_cast<const C2 *>(B);
    auto *c = static_cast<C2 *>(C);
    if (conj_a)
        hipLaunchKernelGGL((k_cgemm<R, true, BM>), grid, dim3(kThreads), 0, s, a, lda, M, K, b, bm, c, cm, ncols);
    else
        hipLaunchKernelGGL((k_cgemm<R, false, BM>), grid, dim3(kThreads), 0, s, a, lda, M, K, b, bm, c, cm, ncols);
}

}  // namespace

// 128 x 128 tiles when they give every compute unit at least two; 64 x 64
// tiles (four times as many workgroups, two per compute unit) otherwise.
int launch_cgemm(hipStream_t s, int dtype, bool conj_a, const void *A, int64_t lda, int M, int K, const void *B,
                 ColMap bm, void *C, ColMap cm, uint64_t ncols)
{
    if (M < 1 || K < 1 || ncols == 0) return QS_OK;
    const uint64_t big = ((ncols + 127) / 128) * uint64_t((M + 127) / 128);
    const int bmt = big >= 2 * uint64_t(device_cus()) ? 128 : 64;
    const uint64_t gx = (ncols + bmt - 1) / bmt;
    if (gx > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "complex GEMM with %llu columns", (unsigned long long)ncols);
    const dim3 grid(unsigned(gx), unsigned((M + bmt - 1) / bmt));
    if (dtype == QS_C128) {
        if (bmt == 128) launch_tile<double, 128>(s, conj_a, A, lda, M, K, B, bm, C, cm, ncols, grid);
        else launch_tile<double, 64>(s, conj_a, A, lda, M, K, B, bm, C, cm, ncols, grid);
    } else {
        if (bmt == 128) launch_tile<float, 128>(s, conj_a, A, lda, M, K, B, bm, C, cm, ncols, grid);
        else launch_tile<float, 64>(s, conj_a, A, lda, M, K, B, bm, C, cm, ncols, grid);
    }
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace qs
