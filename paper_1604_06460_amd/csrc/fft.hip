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
// Twiddles: exact integer exponents (k * l reduced mod 2^bits) are turned
// into angles and evaluated with sincospi in FP64; stage twiddles come from
// a 2^10-entry table built the same way. FP32 states use the FP64 twiddles
// rounded to FP32.
#include "qs_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace qs {
namespace {

constexpr int kThreads = 256;
constexpr int kRmax = 10;           // digit width limit (bits)
constexpr int kTab = 1 << kRmax;    // stage-twiddle table size
constexpr size_t kLdsBytes = 64 * 1024;

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
    int col_pos[6];     // absolute source positions of the column bits (ascending)
    int nrest;
    int rest_pos[40];   // remaining bits (ascending), enumerated by workgroup
    int nst;            // in-LDS stages
    int rho[4], sigma[4];
    // global twiddle after this pass (tw_bits == 0: none)
    int tw_bits;        // log2 N_j
    int krest_lo, krest_bits;
    int sgn;            // +1 forward QFT, -1 inverse
    double scale;
    // final pass: destination field index from the position digits
    int final_pass;
    int q_lo, m;
    int ndig;
    int dpos[4], dw[4], doff[4];   // absolute position, width, output offset of each digit
};

__device__ __forceinline__ int phys(int c, int p, int L)
{
    return c * (L + 4) + (p ^ ((p >> 4) & 15));
}

// Natural-order DFT of RAD register values (radix-2 decimation in
// frequency followed by a compile-time bit reversal of the register names).
// tab[y * tstride] = exp(s 2 pi i y / RAD).
template <typename C2, int RAD>
__device__ __forceinline__ void dft_reg(C2 (&v)[RAD], const C2 *__restrict__ tab, int tstride)
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
                v[b + j + h] = (j == 0) ? d : cmul(d, tab[j * (RAD / (2 * h)) * tstride]);
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
template <typename C2, int RHO>
__device__ void lds_stage(C2 *lds, int r, int C, int sigma, const C2 *__restrict__ tab)
{
    constexpr int RAD = 1 << RHO;
    const int L = 1 << r;
    const int items = C << (r - RHO);
    const int tstride_dft = kTab >> RHO;
    const int tw_shift = kRmax - (sigma + RHO);
    for (int it = threadIdx.x; it < items; it += kThreads) {
        const int c = it % C;
        const int o = it / C;
        const int lo = o & ((1 << sigma) - 1);
        const int hi = (o >> sigma) << (sigma + RHO);
        C2 v[RAD];
#pragma unroll
        for (int d = 0; d < RAD; ++d) v[d] = lds[phys(c, hi | (d << sigma) | lo, L)];
        dft_reg<C2, RAD>(v, tab, tstride_dft);
        if (sigma > 0) {
#pragma unroll
            for (int l = 1; l < RAD; ++l) {
                const int y = ((lo * l) << tw_shift) & (kTab - 1);
                v[l] = cmul(v[l], tab[y]);
            }
        }
#pragma unroll
        for (int d = 0; d < RAD; ++d) lds[phys(c, hi | (d << sigma) | lo, L)] = v[d];
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_fft_pass(const typename V2<R>::T *__restrict__ src,
                                                       typename V2<R>::T *__restrict__ dst,
                                                       PassArgs pa,
                                                       const typename V2<R>::T *__restrict__ tab)
{
    using C2 = typename V2<R>::T;
    extern __shared__ unsigned char lds_raw[];
    C2 *lds = reinterpret_cast<C2 *>(lds_raw);
    const int r = pa.r, L = 1 << r, C = 1 << pa.cb;
    // tile base: workgroup index deposited into the remaining bit positions
    uint64_t base = 0;
    {
        uint64_t w = blockIdx.x;
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
    __syncthreads();
    for (int s = 0; s < pa.nst; ++s) {
        switch (pa.rho[s]) {
        case 1: lds_stage<C2, 1>(lds, r, C, pa.sigma[s], tab); break;
        case 2: lds_stage<C2, 2>(lds, r, C, pa.sigma[s], tab); break;
        case 3: lds_stage<C2, 3>(lds, r, C, pa.sigma[s], tab); break;
        default: lds_stage<C2, 4>(lds, r, C, pa.sigma[s], tab); break;
        }
        __syncthreads();
    }
    // store: output digit l sits at the position its stages wrote it to
    for (int e = threadIdx.x; e < (L << pa.cb); e += kThreads) {
        const int c = e & (C - 1), l = e >> pa.cb;
        int p = 0, sh = 0;
        for (int s = 0; s < pa.nst; ++s) {
            p |= ((l >> sh) & ((1 << pa.rho[s]) - 1)) << pa.sigma[s];
            sh += pa.rho[s];
        }
        C2 v = lds[phys(c, p, L)];
        const uint64_t sidx = base | (uint64_t(l) << pa.dig_lo) | colbits(c);
        if (pa.tw_bits) {
            const uint64_t kr = (sidx >> pa.krest_lo) & ((1ull << pa.krest_bits) - 1);
            const uint64_t e2 = (kr * uint64_t(l)) & ((1ull << pa.tw_bits) - 1);
            double sn, cs;
            sincospi(double(pa.sgn) * 2.0 * (double(e2) / double(1ull << pa.tw_bits)), &sn, &cs);
            const double vr = double(v.x), vi = double(v.y);
            v = C2{R(vr * cs - vi * sn), R(vr * sn + vi * cs)};
        }
        if (pa.scale != 1.0) v = C2{R(double(v.x) * pa.scale), R(double(v.y) * pa.scale)};
        uint64_t didx = sidx;
        if (pa.final_pass) {
            const uint64_t fmask = ((1ull << pa.m) - 1) << pa.q_lo;
            uint64_t f = 0;
            for (int d = 0; d < pa.ndig; ++d) {
                const uint64_t val = (sidx >> pa.dpos[d]) & ((1ull << pa.dw[d]) - 1);
                f |= val << pa.doff[d];
            }
            didx = (sidx & ~fmask) | (f << pa.q_lo);
        }
        dst[didx] = v;
    }
}

template <typename R>
__global__ void k_twiddle_table(typename V2<R>::T *__restrict__ tab, int sgn)
{
    using C2 = typename V2<R>::T;
    const int y = blockIdx.x * kThreads + threadIdx.x;
    if (y >= kTab) return;
    double sn, cs;
    sincospi(double(sgn) * 2.0 * double(y) / double(kTab), &sn, &cs);
    tab[y] = C2{R(cs), R(sn)};
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

template <typename R>
int run_fft(qs_state *h, int q_lo, int m, int inverse)
{
    using C2 = typename V2<R>::T;
    const int n = h->n;
    const int P = (m + kRmax - 1) / kRmax;
    int width[4], pos[4];  // digit j from the top of the field
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
    void *dtab = nullptr;
    if (int rc = h->stage.reserve(h->stream, sizeof(C2) * kTab, &dtab)) return rc;
    hipLaunchKernelGGL(k_twiddle_table<R>, dim3(kTab / kThreads), dim3(kThreads), 0, h->stream,
                       static_cast<C2 *>(dtab), sgn);
    QS_HIP(hipGetLastError());
    if (P > 1)
        if (int rc = ensure_scratch(h)) return rc;
    for (int j = 0; j < P; ++j) {
        PassArgs pa;
        std::memset(&pa, 0, sizeof pa);
        pa.r = width[j];
        pa.dig_lo = pos[j];
        pa.sgn = sgn;
        pa.scale = 1.0;
        stage_plan(pa.r, pa);
        const bool last = (j == P - 1);
        // column bits
        // columns so that the unpadded tile fills the LDS budget
        int maxcb = 0;
        while ((sizeof(C2) << (pa.r + maxcb + 1)) <= kLdsBytes) ++maxcb;
        const int want = std::max(0, std::min({maxcb, 6, n - pa.r}));
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
            pa.q_lo = q_lo;
            pa.m = m;
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
        const size_t lds = sizeof(C2) * size_t((1 << pa.r) + 4) << pa.cb;
        const C2 *src = static_cast<const C2 *>(h->psi);
        C2 *dst = (last && P > 1) ? static_cast<C2 *>(h->scratch) : static_cast<C2 *>(h->psi);
        if (tiles > 0x7fffffffull) return fail(QS_EUNSUPPORTED, "FFT tile count too large");
        hipLaunchKernelGGL(k_fft_pass<R>, dim3(unsigned(tiles)), dim3(kThreads), lds, h->stream, src,
                           dst, pa, static_cast<const C2 *>(dtab));
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
        QS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_fft_pass<double>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(kLdsBytes + 4096)));
        QS_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_fft_pass<float>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(kLdsBytes + 4096)));
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
