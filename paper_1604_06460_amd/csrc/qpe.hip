// Dense unitaries and the controlled powers of quantum phase estimation
// (Sec. III-C).
//
// A simulator applies U^(2^j) by running the G gates of U 2^j times; an
// emulator may instead build the dense 2^m x 2^m matrix of U once and square
// it, so that U^(2^j) costs one matrix product per bit of precision.
//
// Building U: the identity is laid out as a 2m-qubit work state whose
// amplitude c * 2^m + r is delta(r, c); sweeping the gate list (fused into
// k-qubit blocks) over its low m qubits turns column c into U e_c, so the
// work state holds U column-major with leading dimension 2^m.
//
// Squaring and the controlled application are plain FP64 (complex64 states:
// FP32) GEMMs and go to the BLAS library. For a control qubit q >= m the
// state is a 2^m x 2^(n-m) column-major matrix whose columns with bit q - m
// set come in runs of 2^(q-m) every 2^(q-m+1): one strided-batched GEMM
// computes U times every run into the second buffer, a copy kernel moves the
// other half, and the buffers swap.
#include "qs_internal.h"

#include <rocblas/rocblas.h>

#include <algorithm>
#include <cstring>

using namespace qs;

struct qs_unitary_t {
    int m = 0;
    hipStream_t stream = nullptr;
    double *u = nullptr;     // 2^m x 2^m complex128, column-major
    double *tmp = nullptr;   // squaring target
    float *u32 = nullptr;    // complex64 copy for complex64 states (refreshed on demand)
    bool u32_valid = false;
    size_t dim() const { return size_t(1) << m; }
    size_t elems() const { return dim() * dim(); }
};

namespace {

constexpr int kMaxUnitaryQubits = 15;   // 2^30 entries, 16 GiB per matrix

rocblas_handle blas(int &rc)
{
    static rocblas_handle h = nullptr;
    rc = QS_OK;
    if (!h && rocblas_create_handle(&h) != rocblas_status_success) {
        h = nullptr;
        rc = fail(QS_EDEVICE, "rocblas_create_handle failed");
    }
    return h;
}

int blas_check(rocblas_status s, const char *what)
{
    return s == rocblas_status_success ? QS_OK : fail(QS_EDEVICE, "%s: %s", what, rocblas_status_to_string(s));
}

__global__ void k_identity(double2 *__restrict__ w, int m, uint64_t count)
{
    const uint64_t mask = (1ull << m) - 1;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * blockDim.x)
        w[i] = double2{(i & mask) == (i >> m) ? 1.0 : 0.0, 0.0};
}

// amplitudes whose bit q is 0 (the half the controlled product leaves alone)
template <typename C2>
__global__ void k_copy_ctrl0(const C2 *__restrict__ src, C2 *__restrict__ dst, int q, uint64_t half)
{
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < half;
         t += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t i = ((t >> q) << (q + 1)) | (t & ((1ull << q) - 1));
        dst[i] = src[i];
    }
}

__global__ void k_cast_u(const double *__restrict__ src, float *__restrict__ dst, uint64_t count)
{
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * blockDim.x)
        dst[i] = float(src[i]);
}

// transpose of a complex128 column-major matrix into row-major order
__global__ void k_transpose(const double2 *__restrict__ src, double2 *__restrict__ dst, int m)
{
    const uint64_t d = 1ull << m, count = d * d;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * blockDim.x)
        dst[(i & (d - 1)) * d + (i >> m)] = src[i];
}

unsigned grid_of(uint64_t items)
{
    return unsigned(std::max<uint64_t>(1, std::min<uint64_t>((items + 255) / 256, 1ull << 20)));
}

int check_gates(const qs_circuit *c, int m)
{
    if (!c) return fail(QS_EINVAL, "NULL circuit");
    size_t toff = 0;
    for (int g = 0; g < c->n_gates; ++g) {
        const int k = c->k ? c->k[g] : 0;
        for (int i = 0; i < k; ++i)
            if (c->targets[toff + size_t(i)] >= m)
                return fail(QS_EINVAL, "gate %d acts on qubit %d outside the %d-qubit register", g,
                            c->targets[toff + size_t(i)], m);
        const uint64_t cm = c->ctrl_mask ? c->ctrl_mask[g] : 0;
        if (m < 64 && (cm >> m)) return fail(QS_EINVAL, "gate %d has a control outside the register", g);
        toff += size_t(std::max(k, 0));
    }
    return QS_OK;
}

}  // namespace

extern "C" {

int qs_unitary_build(const qs_circuit *c, int m, int max_k, void *hip_stream, qs_unitary *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "NULL output");
    *out = nullptr;
    if (m < 1 || m > kMaxUnitaryQubits) return fail(QS_EINVAL, "m=%d outside [1, %d]", m, kMaxUnitaryQubits);
    if (int rc = check_gates(c, m)) return rc;
    qs_unitary_t *u = new (std::nothrow) qs_unitary_t();
    if (!u) return fail(QS_ENOMEM, "host allocation failed");
    u->m = m;
    u->stream = static_cast<hipStream_t>(hip_stream);
    auto bail = [&](int rc) {
        qs_unitary_free(u);
        return rc;
    };
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void **>(&u->u), u->elems() * 16)) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc(unitary)"));
    hipLaunchKernelGGL(k_identity, dim3(grid_of(u->elems())), dim3(256), 0, u->stream,
                       reinterpret_cast<double2 *>(u->u), m, uint64_t(u->elems()));
    if ((e = hipGetLastError()) != hipSuccess) return bail(hip_fail(e, "k_identity"));
    // the identity as a 2m-qubit state borrowed by a handle; the gates act on
    // its low m qubits (column index in the high m)
    qs_handle w = nullptr;
    if (int rc = qs_alloc(2 * m, QS_C128, u->u, hip_stream, &w)) return bail(rc);
    int rc = c->n_gates > 0 ? qs_apply_circuit(w, c, max_k) : QS_OK;
    qs_free(w);
    if (rc) return bail(rc);
    if ((e = hipStreamSynchronize(u->stream)) != hipSuccess) return bail(hip_fail(e, "unitary build"));
    *out = u;
    return QS_OK;
}

int qs_unitary_info(qs_unitary u, int *m)
{
    clear_error();
    if (!u) return fail(QS_EINVAL, "NULL unitary");
    if (m) *m = u->m;
    return QS_OK;
}

int qs_unitary_square(qs_unitary u)
{
    clear_error();
    if (!u) return fail(QS_EINVAL, "NULL unitary");
    int rc = QS_OK;
    rocblas_handle b = blas(rc);
    if (rc) return rc;
    if (!u->tmp) QS_HIP(hipMalloc(reinterpret_cast<void **>(&u->tmp), u->elems() * 16));
    if ((rc = blas_check(rocblas_set_stream(b, u->stream), "rocblas_set_stream"))) return rc;
    const rocblas_int d = rocblas_int(u->dim());
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    const auto *A = reinterpret_cast<const rocblas_double_complex *>(u->u);
    auto *C = reinterpret_cast<rocblas_double_complex *>(u->tmp);
    if ((rc = blas_check(rocblas_zgemm(b, rocblas_operation_none, rocblas_operation_none, d, d, d, &one, A, d, A,
                                       d, &zero, C, d),
                         "rocblas_zgemm")))
        return rc;
    std::swap(u->u, u->tmp);
    u->u32_valid = false;
    return QS_OK;
}

int qs_unitary_get(qs_unitary u, double *host_dst)
{
    clear_error();
    if (!u || !host_dst) return fail(QS_EINVAL, "NULL argument");
    if (!u->tmp) QS_HIP(hipMalloc(reinterpret_cast<void **>(&u->tmp), u->elems() * 16));
    hipLaunchKernelGGL(k_transpose, dim3(grid_of(u->elems())), dim3(256), 0, u->stream,
                       reinterpret_cast<const double2 *>(u->u), reinterpret_cast<double2 *>(u->tmp), u->m);
    QS_HIP(hipGetLastError());
    QS_HIP(hipMemcpyAsync(host_dst, u->tmp, u->elems() * 16, hipMemcpyDeviceToHost, u->stream));
    QS_HIP(hipStreamSynchronize(u->stream));
    return QS_OK;
}

int qs_apply_controlled_unitary(qs_handle h, qs_unitary u, int ctrl)
{
    clear_error();
    if (!h || !u) return fail(QS_EINVAL, "NULL argument");
    const int m = u->m;
    if (ctrl < m || ctrl >= h->n)
        return fail(QS_EINVAL, "control qubit %d must lie in [%d, %d) (the register is qubits [0, %d))", ctrl, m,
                    h->n, m);
    if (ctrl - m > 30 || h->n - ctrl - 1 > 30)
        return fail(QS_EUNSUPPORTED, "batched product dimensions exceed 32-bit BLAS sizes");
    int rc = QS_OK;
    rocblas_handle b = blas(rc);
    if (rc) return rc;
    if ((rc = ensure_scratch(h))) return rc;
    // the BLAS library runs on the handle's stream; the unitary must be ready there
    if (u->stream != h->stream) QS_HIP(hipStreamSynchronize(u->stream));
    if ((rc = blas_check(rocblas_set_stream(b, h->stream), "rocblas_set_stream"))) return rc;
    const rocblas_int d = rocblas_int(1) << m;
    const rocblas_int runs = rocblas_int(1) << (ctrl - m);                 // columns per batch
    const rocblas_int batches = rocblas_int(1) << (h->n - ctrl - 1);
    const rocblas_stride stride = rocblas_stride(1) << (ctrl + 1);         // elements between batches
    const size_t first = size_t(1) << ctrl;                                // first column with the control set
    const uint64_t half = h->dim() / 2;
    if (h->dtype == QS_C128) {
        const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
        const auto *A = reinterpret_cast<const rocblas_double_complex *>(u->u);
        const auto *B = reinterpret_cast<const rocblas_double_complex *>(h->psi) + first;
        auto *C = reinterpret_cast<rocblas_double_complex *>(h->scratch) + first;
        if ((rc = blas_check(rocblas_zgemm_strided_batched(b, rocblas_operation_none, rocblas_operation_none, d, runs,
                                                           d, &one, A, d, 0, B, d, stride, &zero, C, d, stride,
                                                           batches),
                             "rocblas_zgemm_strided_batched")))
            return rc;
        hipLaunchKernelGGL(k_copy_ctrl0<double2>, dim3(grid_of(half)), dim3(256), 0, h->stream,
                           static_cast<const double2 *>(h->psi), static_cast<double2 *>(h->scratch), ctrl, half);
    } else {
        if (!u->u32) QS_HIP(hipMalloc(reinterpret_cast<void **>(&u->u32), u->elems() * 8));
        if (!u->u32_valid) {
            hipLaunchKernelGGL(k_cast_u, dim3(grid_of(2 * u->elems())), dim3(256), 0, h->stream, u->u, u->u32,
                               uint64_t(2 * u->elems()));
            QS_HIP(hipGetLastError());
            u->u32_valid = true;
        }
        const rocblas_float_complex one(1.f, 0.f), zero(0.f, 0.f);
        const auto *A = reinterpret_cast<const rocblas_float_complex *>(u->u32);
        const auto *B = reinterpret_cast<const rocblas_float_complex *>(h->psi) + first;
        auto *C = reinterpret_cast<rocblas_float_complex *>(h->scratch) + first;
        if ((rc = blas_check(rocblas_cgemm_strided_batched(b, rocblas_operation_none, rocblas_operation_none, d, runs,
                                                           d, &one, A, d, 0, B, d, stride, &zero, C, d, stride,
                                                           batches),
                             "rocblas_cgemm_strided_batched")))
            return rc;
        hipLaunchKernelGGL(k_copy_ctrl0<float2>, dim3(grid_of(half)), dim3(256), 0, h->stream,
                           static_cast<const float2 *>(h->psi), static_cast<float2 *>(h->scratch), ctrl, half);
    }
    QS_HIP(hipGetLastError());
    if (h->borrowed) {
        QS_HIP(hipMemcpyAsync(h->psi, h->scratch, h->dim() * h->amp_bytes(), hipMemcpyDeviceToDevice, h->stream));
    } else {
        std::swap(h->psi, h->scratch);
    }
    return QS_OK;
}

int qs_unitary_free(qs_unitary u)
{
    clear_error();
    if (!u) return QS_OK;
    if (u->stream) (void)hipStreamSynchronize(u->stream);
    if (u->u) (void)hipFree(u->u);
    if (u->tmp) (void)hipFree(u->tmp);
    if (u->u32) (void)hipFree(u->u32);
    delete u;
    return QS_OK;
}

int qs_emulate_qpe_powers(qs_handle h, const qs_circuit *c, int m, int ctrl_lo, int b, int max_k)
{
    clear_error();
    if (!h) return fail(QS_EINVAL, "NULL handle");
    if (b < 1 || ctrl_lo < m || ctrl_lo + b > h->n)
        return fail(QS_EINVAL, "control register [%d, %d) must lie in [%d, %d)", ctrl_lo, ctrl_lo + b, m, h->n);
    qs_unitary u = nullptr;
    if (int rc = qs_unitary_build(c, m, max_k, h->stream, &u)) return rc;
    int rc = QS_OK;
    for (int j = 0; j < b && !rc; ++j) {
        rc = qs_apply_controlled_unitary(h, u, ctrl_lo + j);
        if (!rc && j + 1 < b) rc = qs_unitary_square(u);
    }
    qs_unitary_free(u);
    return rc;
}

}  // extern "C"
