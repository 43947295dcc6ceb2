// Launch-parameter table consulted by the dispatchers (host only).
//
// Every parameter is an integer; 0 means "built-in default". A value is
// stored per (dtype, k, target class, n bucket) so that a tuner can record
// different choices for, e.g., a 4-qubit complex128 block whose lowest
// target lies inside a cache line of a 30-qubit state and one whose targets
// are all above bit 5. Parameters that do not depend on some of these
// dimensions use index 0 there.
#include "qs_internal.h"

#include <algorithm>

namespace qs {

namespace {

constexpr int kDt = 2, kK = QS_MAX_K + 1, kCls = 3, kNb = 3;
int g_tune[QS_TUNE_COUNT][kDt][kK][kCls][kNb];

struct Range {
    int lo, hi;
};

// accepted non-zero values per parameter
Range range_of(int p)
{
    switch (p) {
    case QS_TUNE_SWEEP_PATH: return {1, 5};
    case QS_TUNE_SWEEP_WG_PER_CU: return {1, 4096};
    case QS_TUNE_FFT_DIGIT: return {2, 10};
    case QS_TUNE_FFT_LDS_KB: return {8, 160};
    case QS_TUNE_MFMA_WG_PER_CU: return {1, 16};
    case QS_TUNE_BATCH_GANG_SHARE: return {1, 256};
    case QS_TUNE_BATCH_BARRIER_AMPS: return {1, 1 << 24};
    case QS_TUNE_FFT_KERNEL: return {1, 5};
    case QS_TUNE_SWEEP_NT: return {1, 3};
    case QS_TUNE_FFT_NT: return {1, 3};
    case QS_TUNE_GEMM_LIB: return {1, 1};
    case QS_TUNE_MODMUL_KERNEL: return {1, 5};
    case QS_TUNE_MFMA_KERNEL: return {1, 6};
    default: return {0, -1};
    }
}

bool index_ok(int v, int n) { return v == -1 || (v >= 0 && v < n); }

}  // namespace

int tune_value(int param, int dtype, int k, int cls, int nb)
{
    if (param < 0 || param >= QS_TUNE_COUNT) return 0;
    return g_tune[param][dtype == QS_C128 ? 1 : 0][std::min(std::max(k, 0), kK - 1)][std::min(std::max(cls, 0), kCls - 1)]
                 [std::min(std::max(nb, 0), kNb - 1)];
}

int tune_class(int min_target, int dtype)
{
    const int line_bits = dtype == QS_C128 ? 3 : 4;   // amplitudes per 128-byte line
    if (min_target < line_bits) return QS_TCLS_SUBLINE;
    return min_target < 6 ? QS_TCLS_SUBWAVE : QS_TCLS_HIGH;
}

int tune_nbucket(int n) { return n < 22 ? 0 : (n < 28 ? 1 : 2); }

int device_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

}  // namespace qs

using namespace qs;

extern "C" {

int qs_tune_set(int param, int dtype, int k, int cls, int nbucket, int value)
{
    clear_error();
    if (param < 0 || param >= QS_TUNE_COUNT) return fail(QS_EINVAL, "unknown tuning parameter %d", param);
    if (!(dtype == -1 || dtype == QS_C64 || dtype == QS_C128)) return fail(QS_EINVAL, "dtype %d", dtype);
    if (!index_ok(k, kK) || !index_ok(cls, kCls) || !index_ok(nbucket, kNb))
        return fail(QS_EINVAL, "tuning index out of range (k=%d cls=%d nbucket=%d)", k, cls, nbucket);
    const Range r = range_of(param);
    if (value != 0 && (value < r.lo || value > r.hi))
        return fail(QS_EINVAL, "value %d outside [%d, %d] for parameter %d (0 = default)", value, r.lo, r.hi, param);
    for (int d = 0; d < kDt; ++d) {
        if (dtype != -1 && d != (dtype == QS_C128 ? 1 : 0)) continue;
        for (int kk = 0; kk < kK; ++kk) {
            if (k != -1 && kk != k) continue;
            for (int c = 0; c < kCls; ++c) {
                if (cls != -1 && c != cls) continue;
                for (int b = 0; b < kNb; ++b)
                    if (nbucket == -1 || b == nbucket) g_tune[param][d][kk][c][b] = value;
            }
        }
    }
    return QS_OK;
}

int qs_tune_get(int param, int dtype, int k, int cls, int nbucket, int *value)
{
    clear_error();
    if (!value) return fail(QS_EINVAL, "NULL output");
    if (param < 0 || param >= QS_TUNE_COUNT) return fail(QS_EINVAL, "unknown tuning parameter %d", param);
    if (!(dtype == QS_C64 || dtype == QS_C128)) return fail(QS_EINVAL, "dtype %d", dtype);
    if (k < 0 || k >= kK || cls < 0 || cls >= kCls || nbucket < 0 || nbucket >= kNb)
        return fail(QS_EINVAL, "tuning index out of range (k=%d cls=%d nbucket=%d)", k, cls, nbucket);
    *value = tune_value(param, dtype, k, cls, nbucket);
    return QS_OK;
}

int qs_tune_reset(void)
{
    clear_error();
    for (int p = 0; p < QS_TUNE_COUNT; ++p)
        for (int d = 0; d < kDt; ++d)
            for (int kk = 0; kk < kK; ++kk)
                for (int c = 0; c < kCls; ++c)
                    for (int b = 0; b < kNb; ++b) g_tune[p][d][kk][c][b] = 0;
    return QS_OK;
}

int qs_tune_classify(int dtype, int n_qubits, int k, const int *targets, int *cls, int *nbucket)
{
    clear_error();
    if (!targets || !cls || !nbucket) return fail(QS_EINVAL, "NULL argument");
    if (!(dtype == QS_C64 || dtype == QS_C128)) return fail(QS_EINVAL, "dtype %d", dtype);
    if (k < 1 || k > QS_MAX_K) return fail(QS_EINVAL, "k=%d", k);
    int mint = 64;
    for (int i = 0; i < k; ++i) mint = std::min(mint, targets[i]);
    *cls = tune_class(mint, dtype);
    *nbucket = tune_nbucket(n_qubits);
    return QS_OK;
}

}  // extern "C"
