// FP64 composer of fused blocks. A block acting on k qubits is the ordered
// product of its gates, each embedded in the block's 2^k space as the
// Kronecker product of its small matrix with identities (Sec. II). One
// workgroup builds one block: the 2^k x 2^k matrix lives in LDS (two
// buffers, ping-pong) and every gate is applied to it from the left,
//   U_new[r][c] = sum_l G[j(r)][l] U[r with target bits := l][c]
// for rows r whose control bits match, U_new[r][c] = U[r][c] otherwise.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_compose(const ComposeBlock *__restrict__ blocks,
                                                      const ComposeGate *__restrict__ gates,
                                                      const double *__restrict__ mats,
                                                      double *__restrict__ out)
{
    extern __shared__ double2 lds[];
    const ComposeBlock b = blocks[blockIdx.x];
    const int D = 1 << b.k;
    double2 *U = lds;
    double2 *V = lds + D * D;
    for (int e = threadIdx.x; e < D * D; e += kThreads)
        U[e] = (e / D == e % D) ? double2{1.0, 0.0} : double2{0.0, 0.0};
    __syncthreads();
    for (int gi = b.g0; gi < b.g1; ++gi) {
        const ComposeGate g = gates[gi];
        const int dg = 1 << g.k;
        const double *G = mats + g.mat_off;
        int tmask = 0;
        for (int m = 0; m < g.k; ++m) tmask |= 1 << g.local_t[m];
        for (int e = threadIdx.x; e < D * D; e += kThreads) {
            const int r = e / D, c = e % D;
            if ((r & int(g.ctrl_mask)) != int(g.ctrl_vals)) {
                V[e] = U[e];
                continue;
            }
            int j = 0;
            for (int m = 0; m < g.k; ++m) j |= ((r >> g.local_t[m]) & 1) << m;
            const int rbase = r & ~tmask;
            double re = 0.0, im = 0.0;
            for (int l = 0; l < dg; ++l) {
                int rr = rbase;
                for (int m = 0; m < g.k; ++m) rr |= ((l >> m) & 1) << g.local_t[m];
                const double gr = G[2 * (j * dg + l)], gim = G[2 * (j * dg + l) + 1];
                const double2 u = U[rr * D + c];
                re = fma(gr, u.x, fma(-gim, u.y, re));
                im = fma(gr, u.y, fma(gim, u.x, im));
            }
            V[e] = double2{re, im};
        }
        __syncthreads();
        double2 *t = U;
        U = V;
        V = t;
    }
    double2 *dst = reinterpret_cast<double2 *>(out + b.out_off);
    for (int e = threadIdx.x; e < D * D; e += kThreads) dst[e] = U[e];
}

}  // namespace

int launch_compose(hipStream_t s, int n_blocks, const ComposeBlock *dblocks,
                   const ComposeGate *dgates, const double *dmats, double *dout, int max_k)
{
    if (n_blocks == 0) return QS_OK;
    const size_t D = size_t(1) << max_k;
    const size_t lds = 2 * D * D * sizeof(double2);
    if (lds > 64 * 1024) {
        QS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_compose),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    }
    hipLaunchKernelGGL(k_compose, dim3(n_blocks), dim3(kThreads), lds, s, dblocks, dgates, dmats,
                       dout);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace qs
