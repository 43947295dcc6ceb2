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
// the FP64 values.
#include "qs_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace qs {
namespace {

template <typename R> struct FftThreads { static constexpr int value = 256; };
template <> struct FftThreads<float> { static constexpr int value = 512; };
constexpr int kRmax = 10;           // digit width limit (bits)
constexpr size_t kLdsBytes = 64 * 1024;
constexpr int kMaxCols = 16;

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <typename C2>
__device__ __forceinline__ C2 cmul(C2 a, C2 b)
{
    return C2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

struct PassArgs {
    int r;              // digit width
    int dig_lo;         // absolute position of the digit
    int cb;             // number of column bits
    int col_pos[6];     // absolute source positions of the column bits
    int nrest;
    int rest_pos[40];   // remaining bits (ascending), enumerated by workgroup
    int nst;            // in-LDS stages
    int rho[4], sigma[4];
    // pass twiddle (tw_bits == 0: none)
    int tw_bits;        // log2 N_j
    int krest_lo, krest_bits;
    int sgn;            // +1 forward QFT, -1 inverse
    double scale;
    // final pass: destination field index from the position digits
    int final_pass;
    int q_lo, m;
    int ndig;
    int dpos[8], dw[8], doff[8];   // absolute position, width, output offset of each digit
};

__device__ __forceinline__ int phys(int c, int p, int L)
{
    return c * (L + 4) + (p ^ ((p >> 4) & 15));
}

// exp(s 2 pi i num / 2^bits) with num already reduced below 2^bits.
template <typename C2, typename R>
__device__ __forceinline__ C2 unit_root(uint64_t num, int bits, int sgn)
{
    double sn, cs;
    sincospi(double(sgn) * 2.0 * (double(num) / double(1ull << bits)), &sn, &cs);
    return C2{R(cs), R(sn)};
}

// Stage twiddle exp(s 2 pi i y / 1024) from the two 32-entry tables.
template <typename C2>
__device__ __forceinline__ C2 stw(const C2 *__restrict__ ta, const C2 *__restrict__ tb, int y)
{
    return (y & 31) ? ((y >> 5) ? cmul(ta[y & 31], tb[y >> 5]) : ta[y & 31]) : tb[y >> 5];
}

// Natural-order DFT of RAD register values (radix-2 decimation in frequency
// followed by a compile-time bit reversal of the register names).
template <typename C2, int RAD>
__device__ __forceinline__ void dft_reg(C2 (&v)[RAD], const C2 *__restrict__ ta,
                                        const C2 *__restrict__ tb)
{
#pragma unroll
    for (int h = RAD / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int b = 0; b < RAD; b += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const C2 a = v[b + j], c = v[b + j + h];
                v[b + j] = C2{a.x + c.x, a.y + c.y};
                const C2 d{a.x - c.x, a.y - c.y};
                // exp(s 2 pi i j / (2h)) = 1024-table entry j * 512 / h
                v[b + j + h] = (j == 0) ? d : cmul(d, tb[(j * (512 / h)) >> 5]);
            }
        }
    }
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

// One radix-RAD stage over the tile in LDS: digit at sigma (within r bits),
// then the twiddle exp(s 2 pi i k' l / 2^(sigma+rho)) with k' = bits below.
template <typename C2, int RHO, int kThreads>
__device__ void lds_stage(C2 *lds, int r, int C, int sigma, const C2 *__restrict__ ta,
                          const C2 *__restrict__ tb)
{
    constexpr int RAD = 1 << RHO;
    const int L = 1 << r;
    const int items = C << (r - RHO);
    const int tw_shift = kRmax - (sigma + RHO);
    for (int it = threadIdx.x; it < items; it += kThreads) {
        const int c = it % C;
        const int o = it / C;
        const int lo = o & ((1 << sigma) - 1);
        const int hi = (o >> sigma) << (sigma + RHO);
        C2 v[RAD];
#pragma unroll
        for (int d = 0; d < RAD; ++d) v[d] = lds[phys(c, hi | (d << sigma) | lo, L)];
        dft_reg<C2, RAD>(v, ta, tb);
        if (sigma > 0) {
#pragma unroll
            for (int l = 1; l < RAD; ++l) {
                const int y = ((lo * l) << tw_shift) & 1023;
                v[l] = cmul(v[l], stw(ta, tb, y));
            }
        }
#pragma unroll
        for (int d = 0; d < RAD; ++d) lds[phys(c, hi | (d << sigma) | lo, L)] = v[d];
    }
}

template <typename R, int kThreads = FftThreads<R>::value>
__global__ __launch_bounds__(kThreads) void k_fft_pass(const typename V2<R>::T *__restrict__ src,
                                                       typename V2<R>::T *__restrict__ dst,
                                                       PassArgs pa)
{
    using C2 = typename V2<R>::T;
    extern __shared__ unsigned char lds_raw[];
    const int r = pa.r, L = 1 << r, C = 1 << pa.cb;
    C2 *lds = reinterpret_cast<C2 *>(lds_raw);
    C2 *ta = lds + size_t(C) * (L + 4);   // exp(s 2 pi i j / 1024), j < 32
    C2 *tb = ta + 32;                      // exp(s 2 pi i 32 j / 1024), j < 32
    C2 *ga = tb + 32;                      // [C][32] pass twiddle, low 5 bits of l
    C2 *gb = ga + 32 * C;                  // [C][32] pass twiddle, high bits of l
    uint64_t base = 0;
    {
        const uint64_t w = blockIdx.x;
        for (int i = 0; i < pa.nrest; ++i) base |= ((w >> i) & 1ull) << pa.rest_pos[i];
    }
    auto colbits = [&](int c) {
        uint64_t v = 0;
        for (int i = 0; i < pa.cb; ++i) v |= uint64_t((c >> i) & 1) << pa.col_pos[i];
        return v;
    };
    // load the tile (consecutive threads take consecutive columns)
    for (int e = threadIdx.x; e < (L << pa.cb); e += kThreads) {
        const int c = e & (C - 1), p = e >> pa.cb;
        lds[phys(c, p, L)] = src[base | (uint64_t(p) << pa.dig_lo) | colbits(c)];
    }
    // twiddle tables (overlap the loads in flight)
    for (int t = threadIdx.x; t < 64 + (pa.tw_bits ? 64 * C : 0); t += kThreads) {
        if (t < 32) {
            ta[t] = unit_root<C2, R>(uint64_t(t), kRmax, pa.sgn);
        } else if (t < 64) {
            tb[t - 32] = unit_root<C2, R>(uint64_t(t - 32) << 5, kRmax, pa.sgn);
        } else {
            const int u = t - 64, c = u >> 6, j = u & 31, hi = (u >> 5) & 1;
            const uint64_t kr = ((base | colbits(c)) >> pa.krest_lo) & ((1ull << pa.krest_bits) - 1);
            const uint64_t mask = (1ull << pa.tw_bits) - 1;
            const uint64_t e2 = (kr * (uint64_t(j) << (hi ? 5 : 0))) & mask;
            (hi ? gb : ga)[c * 32 + j] = unit_root<C2, R>(e2, pa.tw_bits, pa.sgn);
        }
    }
    __syncthreads();
    for (int s = 0; s < pa.nst; ++s) {
        switch (pa.rho[s]) {
        case 1: lds_stage<C2, 1, kThreads>(lds, r, C, pa.sigma[s], ta, tb); break;
        case 2: lds_stage<C2, 2, kThreads>(lds, r, C, pa.sigma[s], ta, tb); break;
        case 3: lds_stage<C2, 3, kThreads>(lds, r, C, pa.sigma[s], ta, tb); break;
        default: lds_stage<C2, 4, kThreads>(lds, r, C, pa.sigma[s], ta, tb); break;
        }
        __syncthreads();
    }
    // store: output digit l sits at the position its stages wrote it to
    const uint64_t fmask = ((1ull << pa.m) - 1) << pa.q_lo;
    for (int e = threadIdx.x; e < (L << pa.cb); e += kThreads) {
        const int c = e & (C - 1), l = e >> pa.cb;
        int p = 0, sh = 0;
        for (int s = 0; s < pa.nst; ++s) {
            p |= ((l >> sh) & ((1 << pa.rho[s]) - 1)) << pa.sigma[s];
            sh += pa.rho[s];
        }
        C2 v = lds[phys(c, p, L)];
        if (pa.tw_bits) {
            const C2 w = (l >> 5) ? cmul(ga[c * 32 + (l & 31)], gb[c * 32 + (l >> 5)]) : ga[c * 32 + l];
            v = cmul(v, w);
        }
        if (pa.scale != 1.0) v = C2{R(double(v.x) * pa.scale), R(double(v.y) * pa.scale)};
        const uint64_t sidx = base | (uint64_t(l) << pa.dig_lo) | colbits(c);
        uint64_t didx = sidx;
        if (pa.final_pass) {
            uint64_t f = 0;
            for (int d = 0; d < pa.ndig; ++d)
                f |= ((sidx >> pa.dpos[d]) & ((1ull << pa.dw[d]) - 1)) << pa.doff[d];
            didx = (sidx & ~fmask) | (f << pa.q_lo);
        }
        dst[didx] = v;
    }
}

void stage_plan(int r, PassArgs &pa)
{
    // radix-16 stages from the top, remainder last
    pa.nst = 0;
    int top = r;
    while (top > 0) {
        const int rho = std::min(4, top);
        pa.rho[pa.nst] = rho;
        pa.sigma[pa.nst] = top - rho;
        ++pa.nst;
        top -= rho;
    }
}

// Pass shape: widest digit and LDS bytes per workgroup tile. Narrower digits
// mean more passes but longer contiguous runs per global access (the tile
// holds LDS/(2^r * amplitude) columns). Overridable for tuning through
// QS_FFT_DIGIT / QS_FFT_LDS_KB.
struct FftShape {
    int digit = 10;
    size_t lds = kLdsBytes;
};

FftShape fft_shape()
{
    FftShape s;
    if (const char *e = getenv("QS_FFT_DIGIT")) s.digit = std::max(1, std::min(kRmax, atoi(e)));
    if (const char *e = getenv("QS_FFT_LDS_KB"))
        s.lds = size_t(std::max(4, std::min(64, atoi(e)))) * 1024;
    return s;
}

template <typename R>
int run_fft(qs_state *h, int q_lo, int m, int inverse)
{
    using C2 = typename V2<R>::T;
    const int n = h->n;
    const FftShape shape = fft_shape();
    const int P = (m + shape.digit - 1) / shape.digit;
    if (P > 8) return fail(QS_EUNSUPPORTED, "QFT field needs more than 8 passes");
    int width[8], pos[8];  // digit j from the top of the field
    {
        int rem = m;
        for (int j = 0; j < P; ++j) {
            width[j] = (rem + (P - j) - 1) / (P - j);
            rem -= width[j];
        }
        int top = q_lo + m;
        for (int j = 0; j < P; ++j) {
            top -= width[j];
            pos[j] = top;
        }
    }
    const int sgn = inverse ? -1 : 1;
    if (P > 1)
        if (int rc = ensure_scratch(h)) return rc;
    for (int j = 0; j < P; ++j) {
        PassArgs pa;
        std::memset(&pa, 0, sizeof pa);
        pa.r = width[j];
        pa.dig_lo = pos[j];
        pa.sgn = sgn;
        pa.scale = 1.0;
        pa.q_lo = q_lo;
        pa.m = m;
        stage_plan(pa.r, pa);
        const bool last = (j == P - 1);
        // columns so that the unpadded tile fills the LDS budget
        int maxcb = 0;
        while ((sizeof(C2) << (pa.r + maxcb + 1)) <= shape.lds && (2 << maxcb) <= kMaxCols) ++maxcb;
        const int want = std::max(0, std::min(maxcb, n - pa.r));
        std::vector<int> cols;
        if (last && P > 1) {
            // destination-contiguous bits: spectators below the field, then the
            // low bits of the top digit (they become the lowest field bits)
            for (int b = 0; b < q_lo && int(cols.size()) < want; ++b) cols.push_back(b);
            for (int b = 0; b < width[0] && int(cols.size()) < want; ++b) cols.push_back(pos[0] + b);
        } else {
            for (int b = 0; b < n && int(cols.size()) < want; ++b)
                if (b < pa.dig_lo || b >= pa.dig_lo + pa.r) cols.push_back(b);
        }
        pa.cb = int(cols.size());
        for (int i = 0; i < pa.cb; ++i) pa.col_pos[i] = cols[size_t(i)];
        std::vector<int> rest;
        for (int b = 0; b < n; ++b) {
            const bool in_dig = (b >= pa.dig_lo && b < pa.dig_lo + pa.r);
            const bool in_col = std::find(cols.begin(), cols.end(), b) != cols.end();
            if (!in_dig && !in_col) rest.push_back(b);
        }
        pa.nrest = int(rest.size());
        for (int i = 0; i < pa.nrest; ++i) pa.rest_pos[i] = rest[size_t(i)];
        if (!last) {
            pa.tw_bits = pos[j] + width[j] - q_lo;  // bits of the current sub-problem
            pa.krest_lo = q_lo;
            pa.krest_bits = pos[j] - q_lo;
        }
        if (last) pa.scale = 1.0 / std::sqrt(std::ldexp(1.0, m));
        if (last && P > 1) {
            pa.final_pass = 1;
            pa.ndig = P;
            int off = 0;
            for (int d = 0; d < P; ++d) {
                pa.dpos[d] = pos[d];
                pa.dw[d] = width[d];
                pa.doff[d] = off;   // digit d holds output digit d (lowest first)
                off += width[d];
            }
        }
        const uint64_t tiles = h->dim() >> (pa.r + pa.cb);
        const size_t C = size_t(1) << pa.cb;
        const size_t lds = sizeof(C2) * (size_t((1 << pa.r) + 4) * C + 64 + 64 * C);
        const C2 *src = static_cast<const C2 *>(h->psi);
        C2 *dst = (last && P > 1) ? static_cast<C2 *>(h->scratch) : static_cast<C2 *>(h->psi);
        if (tiles > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "FFT tile count too large");
        hipLaunchKernelGGL(k_fft_pass<R>, dim3(unsigned(tiles)), dim3(FftThreads<R>::value), lds, h->stream, src,
                           dst, pa);
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
