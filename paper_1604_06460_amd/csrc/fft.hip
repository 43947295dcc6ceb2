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
// transform moves the state P times.
//
// Inside a pass a workgroup holds a tile of 2^r digit values x C columns
// (C consecutive values of the lowest available bits, so global accesses run
// in C-element segments) in LDS and performs the 2^r-point DFT as radix-2^rho
// register stages (rho <= 4), again decimation in frequency. The LDS layout
// is column-major with a 4-element pad per column and the low 4 bits of the
// row XOR-swizzled by the next 4, which keeps both the strided and the
// contiguous stage accesses free of bank conflicts.
//
// Twiddles are products of two table entries held in LDS. Stage twiddles:
// exp(s 2 pi i y / 1024) = A[y mod 32] * B[y / 32]. Pass twiddles: per
// column, exp(s 2 pi i k_rest l / N_j) = GA[l mod 32] * GB[l / 32] with the
// exponents k_rest * l reduced exactly in integers before the angle is
// formed. Every table entry is one FP64 sincospi call; FP32 states round
// the FP64 values. The device code lives in fft_dev.h (shared with the
// batched kernel).
#include "fft_dev.h"

#include <cstdlib>

namespace qs {
namespace {

using namespace fftdev;

template <typename R> struct FftThreads { static constexpr int value = 256; };
template <> struct FftThreads<float> { static constexpr int value = 512; };

template <typename R, int NT = FftThreads<R>::value>
__global__ __launch_bounds__(NT) void k_fft_pass(const typename V2<R>::T *__restrict__ src,
                                                 typename V2<R>::T *__restrict__ dst, PassArgs pa)
{
    extern __shared__ unsigned char lds_raw[];
    fft_tile<R, NT>(src, dst, pa, blockIdx.x, lds_raw);
}

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
    if (const int kb = tune_value(QS_TUNE_FFT_LDS_KB, dtype, 0, 0, nb)) s.lds = std::min(kLdsBytes, size_t(kb) * 1024);
    return s;
}

template <typename R>
int run_fft(qs_state *h, int q_lo, int m, int inverse)
{
    using C2 = typename V2<R>::T;
    const FftShape shape = fft_shape(h->dtype, h->n);
    std::vector<PassArgs> passes;
    if (int rc = plan_passes(h->n, q_lo, m, inverse, shape.digit, shape.lds, sizeof(C2), passes)) return rc;
    const int P = int(passes.size());
    if (P > 1)
        if (int rc = ensure_scratch(h)) return rc;
    for (int j = 0; j < P; ++j) {
        const PassArgs &pa = passes[size_t(j)];
        const bool last = (j == P - 1);
        const C2 *src = static_cast<const C2 *>(h->psi);
        C2 *dst = (last && P > 1) ? static_cast<C2 *>(h->scratch) : static_cast<C2 *>(h->psi);
        if (pa.tiles > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "FFT tile count too large");
        hipLaunchKernelGGL(k_fft_pass<R>, dim3(unsigned(pa.tiles)), dim3(FftThreads<R>::value),
                           pass_lds_bytes(pa, sizeof(C2)), h->stream, src, dst, pa);
        QS_HIP(hipGetLastError());
    }
    if (P > 1) {
        if (h->borrowed) {
            QS_HIP(hipMemcpyAsync(h->psi, h->scratch, h->dim() * h->amp_bytes(),
                                  hipMemcpyDeviceToDevice, h->stream));
        } else {
            std::swap(h->psi, h->scratch);
        }
    }
    return QS_OK;
}

}  // namespace

int emulate_qft(qs_state *h, int q_lo, int m, int inverse)
{
    static bool lds_ok = false;
    if (!lds_ok) {
        const int cap = int(kLdsBytes + 16 * 1024);
        QS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_fft_pass<double>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, cap));
        QS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_fft_pass<float>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, cap));
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
