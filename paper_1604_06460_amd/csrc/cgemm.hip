// Complex GEMM on the matrix cores for the dense-unitary route of phase
// estimation (Sec. III-C): C = op(A) B with A square-ish (M x K), B and C
// given as column lists (so strided-batched products over a state are one
// launch). Complex128 runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), complex64 on the FP32 ones
// (v_mfma_f32_16x16x4f32); the complex product is four real products,
// Re C = Re A Re B - Im A Im B, Im C = Re A Im B + Im A Re B, so the real
// work equals the complex work (8 flops per complex multiply-add).
//
// Tiling: a 256-thread workgroup owns a 128 x 128 tile of C; its four waves
// each own a 64 x 64 quarter as 4 x 4 MFMA tiles of 16 x 16, with real and
// imaginary accumulators (128 values per lane). K advances 8 complex
// entries at a time: the A and B panels (128 x 8 each) are staged in LDS as
// separate real and imaginary planes laid out [k][row] / [k][col], so every
// fragment read is 16 consecutive values per quarter-wave. The next panel
// is loaded into registers while the current one is multiplied.
//
// MFMA lane layouts (16x16x4, checked on the device): A[i][k] in lane
// i + 16k and B[k][j] in lane j + 16k for both precisions; D[i][j] is in
// lane j + 16 (i / 4), slot i % 4 for FP32 but in lane j + 16 (i % 4), slot
// i / 4 for FP64.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBM = 128, kBN = 128, kBK = 8, kThreads = 256;

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

template <typename R, bool CONJ_A>
__global__ __launch_bounds__(kThreads, 1) void k_cgemm(const typename Cx<R>::T *__restrict__ A, int64_t lda, int M,
                                                        int K, const typename Cx<R>::T *__restrict__ B, ColMap bm,
                                                        typename Cx<R>::T *__restrict__ C, ColMap cm, uint64_t ncols)
{
    using C2 = typename Cx<R>::T;
    using V4 = typename Cx<R>::V4;
    __shared__ R a_re[kBK * kBM], a_im[kBK * kBM], b_re[kBK * kBN], b_im[kBK * kBN];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * kBM;
    const uint64_t n0 = uint64_t(blockIdx.x) * kBN;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;

    // global -> register panel loads: 4 complex per thread for A and for B
    // A (op = N): column k of the panel is 128 contiguous rows; thread t
    //   takes k = t / 32, rows 4 (t % 32) .. +3.
    // A (op = C): op(A)[i][k] = conj(A[k][i]); row i of op(A) is column i of A,
    //   contiguous in k; thread t takes i = t / 2, k = 4 (t % 2) .. +3.
    // B: column j contiguous in k; thread t takes j = t / 2, k = 4 (t % 2) .. +3.
    C2 ra[4], rb[4];
    const int bj = t >> 1, bk = (t & 1) * 4;
    const uint64_t bcol = n0 + uint64_t(bj);
    const bool bcol_ok = bcol < ncols;
    const uint64_t boff = bcol_ok ? col_off(bm, bcol) : 0;

    auto load_panel = [&](int k0) {
        if constexpr (!CONJ_A) {
            const int ak = t >> 5, ai = (t & 31) * 4;
            const int k = k0 + ak;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = m0 + ai + q;
                ra[q] = (k < K && i < M) ? A[int64_t(i) + int64_t(k) * lda] : C2{0, 0};
            }
        } else {
            const int ai = t >> 1, ak = (t & 1) * 4;
            const int i = m0 + ai;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + ak + q;
                ra[q] = (k < K && i < M) ? A[int64_t(k) + int64_t(i) * lda] : C2{0, 0};
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + bk + q;
            rb[q] = (bcol_ok && k < K) ? B[boff + uint64_t(k)] : C2{0, 0};
        }
    };
    auto store_panel = [&]() {
        if constexpr (!CONJ_A) {
            const int ak = t >> 5, ai = (t & 31) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a_re[ak * kBM + ai + q] = ra[q].x;
                a_im[ak * kBM + ai + q] = ra[q].y;
            }
        } else {
            const int ai = t >> 1, ak = (t & 1) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a_re[(ak + q) * kBM + ai] = ra[q].x;
                a_im[(ak + q) * kBM + ai] = -ra[q].y;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            b_re[(bk + q) * kBN + bj] = rb[q].x;
            b_im[(bk + q) * kBN + bj] = rb[q].y;
        }
    };

    V4 acc_re[4][4], acc_im[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            acc_re[x][y] = V4{0, 0, 0, 0};
            acc_im[x][y] = V4{0, 0, 0, 0};
        }

    const int fi = lane & 15, fk = lane >> 4;
    load_panel(0);
    for (int k0 = 0; k0 < K; k0 += kBK) {
        __syncthreads();          // the previous panel is no longer read
        store_panel();
        __syncthreads();
        if (k0 + kBK < K) load_panel(k0 + kBK);
#pragma unroll
        for (int ks = 0; ks < kBK; ks += 4) {
            R ar[4], ai[4], br[4], bi[4], nai[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                ar[x] = a_re[(ks + fk) * kBM + wr + 16 * x + fi];
                ai[x] = a_im[(ks + fk) * kBM + wr + 16 * x + fi];
                nai[x] = -ai[x];
            }
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                br[y] = b_re[(ks + fk) * kBN + wc + 16 * y + fi];
                bi[y] = b_im[(ks + fk) * kBN + wc + 16 * y + fi];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    acc_re[x][y] = Cx<R>::mfma(ar[x], br[y], acc_re[x][y]);
                    acc_re[x][y] = Cx<R>::mfma(nai[x], bi[y], acc_re[x][y]);
                    acc_im[x][y] = Cx<R>::mfma(ar[x], bi[y], acc_im[x][y]);
                    acc_im[x][y] = Cx<R>::mfma(ai[x], br[y], acc_im[x][y]);
                }
        }
    }
    // epilogue: lane holds four rows (Cx::row) of column lane % 16 of every
    // 16 x 16 tile
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        const uint64_t col = n0 + uint64_t(wc + 16 * y + fi);
        if (col >= ncols) continue;
        C2 *cp = C + col_off(cm, col);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr + 16 * x + Cx<R>::row(fk, r);
                if (row < M) cp[row] = C2{acc_re[x][y][r], acc_im[x][y][r]};
            }
    }
}

}  // namespace

int launch_cgemm(hipStream_t s, int dtype, bool conj_a, const void *A, int64_t lda, int M, int K, const void *B,
                 ColMap bm, void *C, ColMap cm, uint64_t ncols)
{
    if (M < 1 || K < 1 || ncols == 0) return QS_OK;
    const uint64_t gx = (ncols + kBN - 1) / kBN;
    if (gx > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "complex GEMM with %llu columns", (unsigned long long)ncols);
    const dim3 grid(unsigned(gx), unsigned((M + kBM - 1) / kBM));
    if (dtype == QS_C128) {
        const auto *a = static_cast<const double2 *>(A);
        const auto *b = static_cast<const double2 *>(B);
        auto *c = static_cast<double2 *>(C);
        if (conj_a)
            hipLaunchKernelGGL((k_cgemm<double, true>), grid, dim3(kThreads), 0, s, a, lda, M, K, b, bm, c, cm, ncols);
        else
            hipLaunchKernelGGL((k_cgemm<double, false>), grid, dim3(kThreads), 0, s, a, lda, M, K, b, bm, c, cm, ncols);
    } else {
        const auto *a = static_cast<const float2 *>(A);
        const auto *b = static_cast<const float2 *>(B);
        auto *c = static_cast<float2 *>(C);
        if (conj_a)
            hipLaunchKernelGGL((k_cgemm<float, true>), grid, dim3(kThreads), 0, s, a, lda, M, K, b, bm, c, cm, ncols);
        else
            hipLaunchKernelGGL((k_cgemm<float, false>), grid, dim3(kThreads), 0, s, a, lda, M, K, b, bm, c, cm, ncols);
    }
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace qs
