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
// in C-element segments; the default 80 KB tile gives a 10-bit digit C = 4
// complex128 or 8 complex64 columns, 64 bytes, and the whole LDS of a CU one
// full 128-byte line) in LDS and performs the 2^r-point DFT as radix-2^rho
// register stages (rho <= 3 for complex128, 4 for complex64), again
// decimation in frequency.
//
// Launch: one workgroup per tile (k_fft_pass, the default; two workgroups
// share a CU with the 80 KB tile) in an XCD-aware order. A persistent
// alternative (k_fft_stream, tuning option 2) walks a contiguous range of
// tiles and prefetches the next tile into registers while the current one is
// transformed; it needs more registers and is slower here. The LDS layout
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
    const int kern = tune_value(QS_TUNE_FFT_KERNEL, h->dtype, 0, 0, tune_nbucket(h->n));
    const bool stream = kern == 2;   // default: one workgroup per tile
    std::vector<PassArgs> passes;
    if (int rc = plan_passes(h->n, q_lo, m, inverse, shape.digit, shape.lds, sizeof(C2), passes,
                             stream ? StreamRho<R>::value : FftRho<R>::value))
        return rc;
    const int nt = tune_value(QS_TUNE_FFT_NT, h->dtype, 0, 0, tune_nbucket(h->n));
    for (auto &pa : passes) pa.nt = nt;
    const int P = int(passes.size());
    if (P > 1)
        if (int rc = ensure_scratch(h)) return rc;
    for (int j = 0; j < P; ++j) {
        const PassArgs &pa = passes[size_t(j)];
        const bool last = (j == P - 1);
        const C2 *src = static_cast<const C2 *>(h->psi);
        C2 *dst = (last && P > 1) ? static_cast<C2 *>(h->scratch) : static_cast<C2 *>(h->psi);
        const size_t lds = pass_lds_bytes(pa, sizeof(C2));
        const uint64_t elems = uint64_t(1) << (pa.r + pa.cb);
        if (stream && elems <= uint64_t(kStreamNT) * StreamV<R>::value) {
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
        const int cap = int(kLdsMax);
        const void *fns[] = {reinterpret_cast<const void *>(k_fft_pass<double>),
                             reinterpret_cast<const void *>(k_fft_pass<float>),
                             reinterpret_cast<const void *>(k_fft_stream<double>),
                             reinterpret_cast<const void *>(k_fft_stream<float>)};
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
