// Internal declarations shared by the translation units of libqs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "qs.h"

namespace qs {

// ---------------------------------------------------------------------------
// Errors: thread-local message, integer status across the ABI.
// ---------------------------------------------------------------------------
int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
int hip_fail(hipError_t e, const char *what);

#define QS_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return ::qs::hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// Host -> device staging of small per-call operands (gate matrices, tables).
// A pinned host ring and a device ring of the same size; copies are
// enqueued on the handle's stream, so kernels that read a slot run after it
// is filled. Wrapping synchronises the stream once so no pending copy still
// reads a pinned slot that is about to be overwritten.
// ---------------------------------------------------------------------------
struct Staging {
    char *host = nullptr;
    char *dev = nullptr;
    size_t cap = 0, head = 0;
    int init(size_t bytes);
    void release();
    // Returns a device pointer holding a copy of src (256-byte aligned).
    int put(hipStream_t s, const void *src, size_t bytes, void **dptr);
    // Reserve device space only (for kernel-produced temporaries).
    int reserve(hipStream_t s, size_t bytes, void **dptr);
};

}  // namespace qs

struct qs_state {
    int n = 0;
    int dtype = QS_C128;
    int device = 0;
    void *psi = nullptr;        // current state buffer
    void *scratch = nullptr;    // second buffer for out-of-place passes (library-owned)
    bool borrowed = false;      // psi came from the caller (never swapped, never freed)
    hipStream_t stream = nullptr;
    qs::Staging stage;
    double *partials = nullptr; // reduction partials (device)
    size_t partials_cap = 0;
    void *fft_roots = nullptr;  // root tables of the register-tile FFT passes (device)
    double *host_out = nullptr; // pinned host landing area for small results
    size_t host_out_cap = 0;
    size_t amp_bytes() const { return dtype == QS_C128 ? 16 : 8; }
    uint64_t dim() const { return 1ull << n; }
};

namespace qs {

// ---------------------------------------------------------------------------
// Workgroup order over the 8 XCDs. The dispatcher hands workgroup b to XCD
// b mod 8, so in launch order every XCD takes every eighth tile. xcd_order
// gives XCD x runs of C consecutive tiles instead (tile = run * 8C + x * C +
// offset): each XCD stays on nearby addresses (its own L2, fewer DRAM pages
// open) while all eight stay in the same region of the buffer. Grids that
// are not a multiple of 8C keep the launch order, so the map is always a
// bijection on [0, G).
// ---------------------------------------------------------------------------
template <typename IT, unsigned C>
__device__ __forceinline__ IT xcd_order(unsigned b, unsigned G)
{
    if (G % (8 * C)) return IT(b);
    const unsigned i = b / 8;
    return IT(i / C) * IT(8 * C) + IT(b % 8) * IT(C) + IT(i % C);
}

// ---------------------------------------------------------------------------
// Gate descriptors passed to the sweep launchers (host side).
// ---------------------------------------------------------------------------
enum GateClass { GC_IDENTITY, GC_PHASE1, GC_DIAG, GC_MONOMIAL, GC_DENSE };

struct GateDesc {
    int k = 0;
    int targets[QS_MAX_K] = {0};
    uint64_t ctrl_mask = 0, ctrl_vals = 0;
    int cls = GC_DENSE;
    // GC_PHASE1: the single local index whose diagonal entry is not 1
    int phase_index = 0;
    // GC_MONOMIAL: out[perm_dst[j]] = coef_j * in[j]
    int perm_dst[1 << QS_MAX_K] = {0};
};

// Classify a 2^k x 2^k FP64 interleaved matrix exactly (no tolerance).
void classify(const double *m, int k, GateDesc &d);

// Launchers; dmat points at device data of the handle's precision layout:
// dense/diag/monomial read FP64 (QS_C128) or FP32 (QS_C64) interleaved
// complex matrices. Return a qs_status.
int launch_dense(qs_state *h, const GateDesc &d, const void *dmat);
int launch_diag(qs_state *h, const GateDesc &d, const void *dmat, int stride /*row stride in entries*/);
int launch_phase1(qs_state *h, const GateDesc &d, const void *dmat);
// Diagonal block with its diagonal also on the host (hdiag: 2^k complex
// FP64 entries): sweeps only the target patterns whose entry is not one.
int launch_diag_block(qs_state *h, const GateDesc &d, const void *dmat, int row_stride, const double *hdiag);
double diag_changed_fraction(const double *hdiag, int k);
int launch_monomial(qs_state *h, const GateDesc &d, const void *dmat);
int launch_cast_f64_to_f32(hipStream_t s, const double *src, float *dst, size_t count);
// FP32 MFMA path for dense 6-qubit blocks on complex64 states (mfma.hip)
bool mfma_applicable(const qs_state *h, const GateDesc &d);
int launch_dense_mfma(qs_state *h, const GateDesc &d, const void *dmat);
int launch_set_basis(qs_state *h, uint64_t index);

// Enqueue one gate whose FP64 matrix is on the host (uploads, casts).
int enqueue_gate(qs_state *h, const GateDesc &d, const double *host_mat);

// Composer: see compose.hip.
struct ComposeGate {
    int32_t k;           // gate width (targets only)
    int32_t local_t[QS_MAX_K];  // block-local bit of each target
    uint32_t ctrl_mask;  // block-local control bits
    uint32_t ctrl_vals;
    int64_t mat_off;     // offset (in doubles) of the gate matrix
};
struct ComposeBlock {
    int32_t k;
    int32_t g0, g1;      // gate range in the ComposeGate array
    int32_t pad;
    int64_t out_off;     // offset (in doubles) of the block matrix
};
int launch_compose(hipStream_t s, int n_blocks, const ComposeBlock *dblocks,
                   const ComposeGate *dgates, const double *dmats, double *dout,
                   int max_k);

// Complex GEMM on the matrix cores (cgemm.hip): C = op(A) B, column-major,
// op(A) = A or A^dagger (conj_a), A is M x K with leading dimension lda. B
// and C are given as column lists: column c starts at
// base + ((c >> runs_log) << stride_log) + (c & (2^runs_log - 1)) * ld
// elements, so a strided batch of runs-column blocks is one product. dtype
// QS_C128 runs on FP64 matrix cores, QS_C64 on FP32 ones.
struct ColMap {
    uint64_t base = 0, ld = 0;
    int runs_log = 62, stride_log = 0;
};
int launch_cgemm(hipStream_t s, int dtype, bool conj_a, const void *A, int64_t lda, int M, int K, const void *B,
                 ColMap bm, void *C, ColMap cm, uint64_t ncols);

// Planner (host only)
struct Plan {
    std::vector<int> block_of_gate;
    std::vector<std::vector<int>> block_gates;   // gate ids in circuit order
    std::vector<std::vector<int>> block_qubits;  // ascending
};
// far_lo: lowest qubit whose amplitude rows lie 16 MiB or more apart (bit 24
// of the byte address); the plain greedy plan is compared with one whose
// blocks take at most one such qubit (unless a block's first gate brings
// more) and the cheaper kept. 64 disables the comparison.
int plan_fusion(int n_qubits, int n_gates, const int *k, const int *targets,
                const uint64_t *ctrl_mask, int max_k, Plan &out, int far_lo = 64);
inline int far_qubit(size_t amp_bytes) { return amp_bytes == 16 ? 20 : 21; }

// Reductions (reduce.hip)
int reduce_norm2(qs_state *h, double *out);
int reduce_pauli(qs_state *h, uint64_t xm, uint64_t ym, uint64_t zm, double *re, double *im);
// The same into device memory (out[0] = re, out[1] = im), partial sums in
// the library's static scratch: no allocation, no synchronisation.
int reduce_pauli_noalloc(qs_state *h, uint64_t xm, uint64_t ym, uint64_t zm, double *device_out);
int gather_amplitudes(qs_state *h, int count, const uint64_t *indices, void *host_dst);
int emulate_qft(qs_state *h, int q_lo, int m, int inverse);
int measure(qs_state *h, int m, const int *qubits, int shots, const double *u,
            uint64_t *outcomes, double *probs, int collapse);

// Launch-parameter table (tune.cpp): 0 = built-in default
int tune_value(int param, int dtype, int k, int cls, int nbucket);
int tune_class(int min_target, int dtype);
int tune_nbucket(int n);
int device_cus();

// Device buffers attached to a handle
int ensure_partials(qs_state *h, size_t count);
int ensure_host_out(qs_state *h, size_t bytes);
int ensure_scratch(qs_state *h);
int emulate_arith(qs_state *h, int kind, int a_lo, int b_lo, int c_lo, int m);

}  // namespace qs

struct qs_program_t {
    int n = 0;
    int n_blocks = 0;
    std::vector<int> k;                  // per block
    std::vector<std::vector<int>> qubits;
    std::vector<int> diagonal;           // 1 if the block is diagonal
    std::vector<std::vector<double>> hdiag;  // diagonal blocks: their 2^k FP64 entries (host)
    std::vector<double> changed;         // fraction of amplitudes a block changes (1 for dense)
    std::vector<int64_t> mat_off;        // offset in doubles into dmats
    double *dmats = nullptr;             // FP64 composed matrices (device)
    float *dmats32 = nullptr;            // FP32 copies (device)
    size_t mats_doubles = 0;
    int device = 0;
};
