/*
 * qs.h -- C ABI of the MI355X (gfx950) state-vector library.
 *
 * The library updates a 2^n complex state vector on one GPU: gate-level
 * sweeps (Sec. II of Haener et al., "High Performance Emulation of Quantum
 * Circuits"), fused k-qubit blocks, and the emulator shortcuts of Sec. III:
 * the QFT as an in-place FFT (Sec. III-B), arithmetic as a permutation of
 * basis states (Sec. III-A), and measurement quantities read directly off
 * the state (Sec. III-D).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout. Amplitude i (0 <= i < 2^n) is the coefficient of basis state
 *   |i>; qubit q is bit q of i (qubit 0 = least significant bit). The paper's
 *   Kronecker example (Sec. II) writes qubit 0 as the most significant factor;
 *   relabel q -> n-1-q to go from one to the other. Amplitudes are stored
 *   contiguously, (re, im) interleaved: QS_C128 = two doubles (16 B),
 *   QS_C64 = two floats (8 B). The buffer is at least 256-byte aligned.
 *
 * Gate matrices. A gate on k targets is a 2^k x 2^k complex matrix M given in
 *   FP64, row-major, (re, im) interleaved (2^(2k+1) doubles). Bit m of the
 *   local index is the bit of qubit targets[m]; on every group of 2^k
 *   amplitudes that agree outside the targets the gate computes
 *   out_j = sum_l M[j][l] * in_l (Sec. II: the 2^n x 2^n operator is the
 *   Kronecker product of M with identities). Table 1's two-qubit gates list
 *   the control as the more significant local bit, so CNOT(c -> t) is given
 *   as targets = {t, c}. ctrl_mask/ctrl_vals restrict the gate to indices i
 *   with (i & ctrl_mask) == ctrl_vals. QS_C64 states receive the FP64 matrix
 *   and cast it to FP32 on the device.
 *
 * Ownership. The caller owns every host array it passes (targets, matrices,
 *   uniforms, outputs); the library copies what it needs before returning, so
 *   they may be freed or reused at once. State memory is either allocated by
 *   the library (device_buf == NULL in qs_alloc) or borrowed from the caller
 *   (e.g. a torch tensor's data pointer), in which case the caller keeps it
 *   alive until qs_free.
 *
 * Streams and synchronisation. Every device operation of a handle is
 *   enqueued on the handle's HIP stream. Gate, program and emulation calls
 *   return once enqueued. Calls that produce host results (qs_norm2,
 *   qs_expectation, qs_measure, qs_get_state) and qs_sync wait for the stream.
 *
 * Errors. Every entry point returns a qs_status. Arguments are validated
 *   before anything is enqueued, so on QS_EINVAL / QS_EUNSUPPORTED /
 *   QS_ENOMEM the state is unchanged. Asynchronous device faults surface as
 *   QS_EDEVICE at the next synchronising call. qs_last_error() returns a
 *   message for the calling thread's last failure. Nothing throws across the
 *   ABI.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qs_state *qs_handle;
typedef struct qs_program_t *qs_program;

enum qs_dtype { QS_C64 = 0, QS_C128 = 1 };

enum qs_status {
    QS_OK = 0,
    QS_EINVAL = 1,        /* bad argument */
    QS_ENOMEM = 2,        /* device or host allocation failed */
    QS_EDEVICE = 3,       /* HIP runtime or kernel failure */
    QS_EUNSUPPORTED = 4,  /* valid request this build does not implement */
    QS_ENOTUNITARY = 5    /* matrix failed the optional unitarity check */
};

/* Largest qubit count a handle accepts (2^34 complex128 = 256 GiB). */
#define QS_MAX_QUBITS 34
/* Largest fused-block / gate width accepted by the sweep kernels. */
#define QS_MAX_K 6

/* Message describing the calling thread's last failed call ("" if none). */
const char *qs_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int qs_version(void);

/* ---------------------------------------------------------------------- */
/* State lifetime (Sec. II: 2^n complex amplitudes, sum |alpha_i|^2 = 1)    */
/* ---------------------------------------------------------------------- */

/* Create a handle for an n-qubit state (1 <= n <= QS_MAX_QUBITS) of the given
 * dtype on the current HIP device. device_buf == NULL: the library allocates
 * 2^n amplitudes and sets |0...0>. device_buf != NULL: the caller's buffer
 * (>= 2^n amplitudes, 256-byte aligned) is used as is, contents untouched.
 * hip_stream: a hipStream_t (NULL = the null stream). */
int qs_alloc(int n_qubits, int dtype, void *device_buf, void *hip_stream, qs_handle *out);

/* Release the handle and whatever the library allocated for it; waits for
 * the handle's stream first. A borrowed buffer is not freed. */
int qs_free(qs_handle h);

/* n, dtype and the device address that currently holds the state (it can
 * change after an out-of-place emulation on a library-owned state). */
int qs_info(qs_handle h, int *n_qubits, int *dtype, void **device_ptr);

/* Set the state to |0...0>. */
int qs_set_zero(qs_handle h);

/* Copy the whole state to / from host memory (2^n amplitudes of the
 * handle's dtype). Both wait for the stream. */
int qs_get_state(qs_handle h, void *host_dst);
int qs_set_state(qs_handle h, const void *host_src);

/* Copy 2^n amplitudes of the handle's dtype from device memory (e.g. a
 * resident input state) into the state, enqueued on the handle's stream.
 * The source must not overlap the state. */
int qs_load_device(qs_handle h, const void *device_src);

/* Copy the amplitudes at `count` indices (each < 2^n) to host_dst (count
 * amplitudes of the handle's dtype). For spot checks of large states
 * without a full copy. Waits for the stream. */
int qs_get_amplitudes(qs_handle h, int count, const uint64_t *indices, void *host_dst);

/* Wait for all work enqueued on the handle; reports deferred device faults. */
int qs_sync(qs_handle h);

/* ---------------------------------------------------------------------- */
/* Gates (Sec. II, Table 1)                                                */
/* ---------------------------------------------------------------------- */

/* Apply one gate on k targets (1 <= k <= QS_MAX_K), see "Gate matrices".
 * The matrix is classified on the host and the cheapest exact sweep is
 * chosen (Sec. II: skip multiplications by one and zero; Sec. III-B: a
 * conditional phase shift touches only a quarter of the vector):
 *   identity          -> nothing enqueued;
 *   diagonal, one entry != 1 -> multiply only the indices carrying it;
 *   diagonal          -> one elementwise multiply pass;
 *   monomial (one nonzero per row and column) -> move amplitudes, multiply
 *                        only where the entry is not exactly 1 (moves of
 *                        permutation gates are bit-exact);
 *   otherwise         -> dense group sweep.
 * Errors: QS_EINVAL for k out of range, duplicate or out-of-range targets,
 * controls overlapping targets, ctrl_vals outside ctrl_mask, NULL pointers. */
int qs_apply_gate(qs_handle h, int k, const int *targets, const double *matrix,
                  uint64_t ctrl_mask, uint64_t ctrl_vals);

/* Apply a sequence of already fused dense blocks in order: block b acts on
 * k_per_block[b] targets taken consecutively from targets_concat with its
 * matrix taken consecutively from matrices_concat (same layout as
 * qs_apply_gate, no controls). Equivalent to n_blocks qs_apply_gate calls. */
int qs_apply_fused(qs_handle h, int n_blocks, const int *k_per_block,
                   const int *targets_concat, const double *matrices_concat);

/* ---------------------------------------------------------------------- */
/* Circuits, fusion planning and compiled programs                         */
/* ---------------------------------------------------------------------- */

/* A gate list in circuit order (same per-gate layout as qs_apply_gate).
 * ctrl_mask / ctrl_vals may be NULL (no controls). */
typedef struct qs_circuit {
    int n_gates;
    const int *k;              /* [n_gates] */
    const int *targets;        /* concatenated, sum(k) entries */
    const double *matrices;    /* concatenated, sum(2^(2k+1)) doubles */
    const uint64_t *ctrl_mask; /* [n_gates] or NULL */
    const uint64_t *ctrl_vals; /* [n_gates] or NULL */
} qs_circuit;

/* Host-only greedy fusion plan: gates are grouped into blocks acting on at
 * most max_k distinct qubits (targets and controls together); a gate joins
 * the open block only if it commutes past every gate skipped so far (no
 * shared qubit), so applying the blocks in order equals applying the gates
 * in order. Outputs (caller-allocated): *n_blocks; block_of_gate[n_gates];
 * block_k[n_gates] (qubit count of each block, first *n_blocks used);
 * block_qubits[n_gates * QS_MAX_K] (ascending qubits of block b at
 * b*QS_MAX_K). A gate wider than max_k forms a block of its own. Blocks
 * with several qubits at or above 20 (for a complex128 state their rows are
 * 16 MiB or more apart, which the memory serves slowly) sweep more slowly,
 * so a second plan is made in which a gate does not join a block that would
 * then hold two such qubits (a block's first gate may bring more), and the
 * plan with the lower estimated sweep time is returned. qs_compile does the
 * same at the state's row size (qubit 21 for complex64). Runs without a
 * GPU. */
int qs_plan_fusion(const qs_circuit *c, int n_qubits, int max_k, int *n_blocks,
                   int *block_of_gate, int *block_k, int *block_qubits);

/* Plan (as qs_plan_fusion) and compose on the GPU, in FP64, the matrix of
 * every block: the ordered product of the block's gates embedded in the
 * block's 2^k space. Blocks whose gates are all diagonal are kept diagonal.
 * The program holds device copies of everything it needs and can be run on
 * any handle of the same qubit count, any number of times. */
int qs_compile(qs_handle h, const qs_circuit *c, int max_k, qs_program *out);

/* Number of blocks and, if block_k != NULL, their widths; amp_moves_per_run:
 * the amplitude reads plus writes one run must make. A dense block reads and
 * writes all 2^n amplitudes; a diagonal block only those whose entry is not
 * exactly one (a conditional phase shift changes only the amplitudes that
 * carry its phase, Sec. III-B), and a block whose diagonal is all ones
 * nothing. A program has no dtype of its own, so multiply by the amplitude
 * size of the handle it runs on (16 B complex128, 8 B complex64) for the
 * algorithmic HBM bytes. When a diagonal block has a target inside a
 * 128-byte line the kernel rewrites whole lines, so it moves more than this
 * count. */
int qs_program_info(qs_program p, int *n_blocks, int *block_k, double *amp_moves_per_run);

/* How block b runs (Sec. II sweep vs Sec. III-B's touched-only phases):
 * *kind = QS_BLOCK_DENSE (one sweep of the whole state), QS_BLOCK_DIAGONAL
 * (only the target patterns whose entry is not one are swept: one phase
 * launch for a single such entry, else one launch per distinct pattern of
 * the targets above the 128-byte line, or one elementwise pass when those
 * launches would touch more than half the state) or QS_BLOCK_IDENTITY
 * (nothing is launched). *changed_fraction: the fraction of amplitudes the
 * block changes (1 for dense blocks). Either output may be NULL.
 * QS_EINVAL for a NULL program or b outside [0, n_blocks). */
enum qs_block_kind { QS_BLOCK_DENSE = 0, QS_BLOCK_DIAGONAL = 1, QS_BLOCK_IDENTITY = 2 };
int qs_program_block_kind(qs_program p, int b, int *kind, double *changed_fraction);

/* Copy the composed FP64 matrix of block b (2^(2k+1) doubles) and its
 * ascending qubit list (k ints) to the host. */
int qs_program_block(qs_program p, int b, double *matrix_out, int *qubits_out);

/* Enqueue one run of the program on the handle. */
int qs_run_program(qs_handle h, qs_program p);

/* Enqueue blocks [b0, b1) of the program, in order (0 <= b0 <= b1 <=
 * n_blocks, else QS_EINVAL): running consecutive ranges equals one run.
 * Lets a caller put events between blocks to time each launch. */
int qs_run_program_range(qs_handle h, qs_program p, int b0, int b1);

int qs_program_free(qs_program p);

/* Compile with max_k, run once, free. */
int qs_apply_circuit(qs_handle h, const qs_circuit *c, int max_k);

/* ---------------------------------------------------------------------- */
/* Emulation: QFT as an FFT (Sec. III-B)                                   */
/* ---------------------------------------------------------------------- */

/* Replace the field of m qubits [q_lo, q_lo+m) by its QFT:
 *   alpha_l -> 2^(-m/2) sum_k alpha_k exp(+2 pi i k l / 2^m),
 * with the other index bits as spectators and the output in natural order;
 * inverse != 0 uses exp(-2 pi i k l / 2^m). Requires 1 <= m and
 * q_lo + m <= n. The result is the gate-level circuit's (Hadamards,
 * conditional phase shifts and the final SWAPs) up to rounding. */
int qs_emulate_qft(qs_handle h, int q_lo, int m, int inverse);

/* ---------------------------------------------------------------------- */
/* Emulation: arithmetic as a permutation of basis states (Sec. III-A)     */
/* ---------------------------------------------------------------------- */

enum qs_perm_kind { QS_PERM_MODMUL = 0, QS_PERM_TABLE = 1 };

typedef struct qs_perm {
    int kind;
    /* QS_PERM_MODMUL: |c>|x> -> |c>|a^c x mod N> for x < N, x >= N fixed.
     * x is the w-bit field at work_lo, c the c-bit field at ctrl_lo (c may
     * be 0: plain x -> a x mod N). Requires 2 <= N <= 2^w, N < 2^32,
     * gcd(a, N) = 1, disjoint fields inside the state. */
    int work_lo, w, ctrl_lo, c;
    uint64_t a, N;
    /* QS_PERM_TABLE: the nbits-wide field at lo moves from value f to
     * dest[f] (dest: 2^nbits entries, a permutation of 0..2^nbits-1,
     * nbits <= 24). */
    int lo, nbits;
    const uint64_t *dest;
} qs_perm;

/* Apply the permutation; amplitudes move bit-exactly. Out of place through
 * a library scratch state of the same size (allocated on first use); a
 * borrowed state buffer is refreshed from it, a library-owned one is
 * swapped with it (see qs_info). QS_EINVAL if a table is not a permutation
 * or gcd(a, N) != 1. */
int qs_emulate_permutation(qs_handle h, const qs_perm *p);

/* Integer multiplication and division into a third register (Sec. III-A):
 * a, b and c are the m-bit fields of the basis index at a_lo, b_lo and c_lo
 * (least significant bit first).
 *
 * QS_ARITH_MUL: (a, b, c) -> (a, b, c + a*b mod 2^m). With c = 0 this is the
 *   paper's (a, b, 0) -> (a, b, ab), the product cut to the m bits of c.
 * QS_ARITH_DIV: with c = 0, (a, b, 0) -> (a mod b, b, a div b); a divisor
 *   b = 0 gives (a, 0, 2^m - 1). For c != 0 the map is that of the
 *   restoring-division network (repeated subtraction and shift): with
 *   Y = a + 2^m c, for i = m-1 down to 0 the (m+1)-bit window W of Y at bit
 *   i becomes W - b mod 2^(m+1); if its top bit is then set, b is added back
 *   to its low m bits mod 2^m; the top bit is flipped. The result is a + 2^m c
 *   of the output.
 *
 * Both are permutations of basis states: amplitudes move bit-exactly, out of
 * place through the scratch state as in qs_emulate_permutation. Requires
 * m >= 1 and three disjoint fields inside the state; otherwise QS_EINVAL and
 * the state is unchanged. */
enum qs_arith_kind { QS_ARITH_MUL = 0, QS_ARITH_DIV = 1 };
int qs_emulate_arith(qs_handle h, int kind, int a_lo, int b_lo, int c_lo, int m);

/* ---------------------------------------------------------------------- */
/* Measurement quantities (Sec. III-D, Sec. II)                            */
/* ---------------------------------------------------------------------- */

/* sum_i |alpha_i|^2, accumulated in FP64. */
int qs_norm2(qs_handle h, double *out);

/* <psi|P|psi> for the Pauli string with X on x_mask, Y on y_mask, Z on
 * z_mask (disjoint masks), accumulated in FP64. */
int qs_expectation(qs_handle h, uint64_t x_mask, uint64_t y_mask, uint64_t z_mask,
                   double *out_re, double *out_im);

/* Measure m qubits (1 <= m <= 20, distinct): computes the marginal
 * probabilities p[o] (bit r of o = qubit qubits[r]); for each of `shots`
 * caller-supplied uniforms u in [0,1) returns the smallest o whose running
 * sum of p exceeds u * sum(p). probs_or_null receives p (2^m doubles) if
 * not NULL. collapse != 0 (requires shots >= 1) projects the state onto the
 * first shot's outcome and renormalises. */
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): qs_expectation without
 * any allocation or synchronisation. The result, <P> as (re, im) FP64, is
 * written to device_out (device memory, 2 doubles, 8-byte aligned) on the
 * handle's stream; the caller reads it after the stream. The per-block
 * partial sums live in a library-static device array of 4096 doubles
 * (32 KiB) per GPU, resolved once per device on the first call and kept
 * until the process ends; every reduction fits it (at most 2048 blocks of
 * two partials), a larger request would fail with QS_EUNSUPPORTED. Calls that
 * overlap on one GPU (two streams, or two threads) race on that array:
 * serialise them. Arguments are checked as in qs_expectation; QS_EINVAL for
 * a NULL device_out. */
int qs_expectation_noalloc(qs_handle h, uint64_t x_mask, uint64_t y_mask, uint64_t z_mask,
                           double *device_out);

int qs_measure(qs_handle h, int m, const int *qubits, int shots, const double *uniforms,
               uint64_t *outcomes, double *probs_or_null, int collapse);

/* ---------------------------------------------------------------------- */
/* Batches: many independent complex64 circuits in one persistent launch  */
/* ---------------------------------------------------------------------- */

/* Segment kinds. Every segment carries its gate-level form; QFT and modmul
 * segments also carry the subroutine description the emulator uses instead
 * (Sec. III: an emulator owes the caller the final state, not the gates). */
enum qs_seg_kind { QS_SEG_GATES = 0, QS_SEG_QFT = 1, QS_SEG_MODMUL = 2 };

/* Per-segment plan options: fuse the gate-level form into blocks of at most
 * 2, 4 or 6 qubits, or run the emulated subroutine (QFT as an FFT,
 * modmul as a basis-state permutation; not valid for QS_SEG_GATES). */
enum qs_plan_option { QS_PLAN_K2 = 0, QS_PLAN_K4 = 1, QS_PLAN_K6 = 2, QS_PLAN_EMULATE = 3 };

/* Features per segment returned by qs_batch_features. */
#define QS_N_FEATURES 24

typedef struct qs_segment {
    int kind;
    qs_circuit gates;      /* gate-level form (all kinds) */
    int q_lo, m, inverse;  /* QS_SEG_QFT: field and direction, as qs_emulate_qft */
    qs_perm perm;          /* QS_SEG_MODMUL: kind QS_PERM_MODMUL, as qs_emulate_permutation;
                              the gate form must agree with it on the states it meets */
} qs_segment;

typedef struct qs_batch_circuit {
    int n_qubits;          /* 2 .. 26 */
    int n_segments;
    const qs_segment *segments;
} qs_batch_circuit;

typedef struct qs_batch_t *qs_batch;

/* Copy the circuits (every circuit starts from |0...0>, complex64) and
 * allocate their states on the current device. Gate lists shared by
 * several segments (same array pointers) are stored once. */
int qs_batch_create(int n_circuits, const qs_batch_circuit *circuits, void *hip_stream,
                    qs_batch *out);

/* Total segment count (segments are numbered circuit by circuit, in order)
 * and total state bytes. */
int qs_batch_info(qs_batch b, int *n_segments, double *state_bytes);

/* Per segment (any pointer may be NULL): kind, owning circuit, qubits. */
int qs_batch_segment_info(qs_batch b, int *kind, int *circuit, int *n_qubits);

/* QS_N_FEATURES floats per segment describing it for the cost model: size,
 * kind, gate statistics, fused block counts at k = 2, 4, 6, LDS residency,
 * estimated bytes and flops. */
int qs_batch_features(qs_batch b, float *features);

/* Choose one qs_plan_option per segment: fuses (host plan, FP64 GPU
 * composition, cached per gate list and k) and builds the op lists. */
int qs_batch_set_plan(qs_batch b, const int *options);

/* Run every circuit in one persistent launch (as many workgroups as are
 * co-resident). A circuit of at most 13 qubits runs on one workgroup with
 * its state in LDS; a larger one is swept in HBM by a gang of workgroups
 * that meet at a cross-workgroup barrier between ops. Gangs are sized from
 * the plan's cost estimate: just large enough that no circuit outlasts a
 * quarter of the average work per workgroup (at most a quarter of the
 * grid, at least 2^12 amplitudes per member). wall_ms: launch time
 * (HIP events); seg_us (per segment, optional): device time of each segment
 * from the in-kernel real-time counter (0 for a segment with no ops, such as
 * an empty gate list); norms / z0 (per circuit, optional):
 * sum |a|^2 and <Z_0>, FP64 accumulated, summed over gang members in a
 * fixed order. Returns QS_EDEVICE if a gang barrier waited more than 5 s
 * (the kernel then gives up and drains; the states are invalid). */
int qs_batch_run(qs_batch b, double *wall_ms, double *seg_us, double *norms, double *z0);

/* Schedule of the last qs_batch_run, one entry per ticket (a circuit of at
 * most 13 qubits has one ticket, a gang one per member), in queue order:
 * start and end time in microseconds from the earliest start, owning
 * circuit, gang member, and the workgroup that ran it. Writes at most
 * `capacity` entries (any array may be NULL) and the ticket count to
 * *n_tickets. */
int qs_batch_trace(qs_batch b, int capacity, int *n_tickets, double *start_us, double *end_us,
                   int *circuit, int *member, int *workgroup);

/* Copy circuit c's final state (2^n complex64) to the host. */
int qs_batch_get_state(qs_batch b, int circuit, void *host_dst);

int qs_batch_free(qs_batch b);

/* ---------------------------------------------------------------------- */
/* Learned cost model and plan choice                                      */
/* ---------------------------------------------------------------------- */

/* A 24 -> 64 -> 64 -> 4 perceptron (ReLU, FP32) predicting the log device
 * time of a segment under each qs_plan_option. Parameters, 6020 floats:
 * W1[24][64], b1[64], W2[64][64], b2[64], W3[64][4], b3[4], row-major with
 * y = relu(relu(x W1 + b1) W2 + b2) W3 + b3. Inputs are standardised as
 * (x - mean) * inv_std before W1. Forward, backward and Adam run in the
 * library's kernels on the model's stream. */
#define QS_MLP_PARAMS 6020
typedef struct qs_mlp_t *qs_mlp;

/* params == NULL: He-initialised weights from `seed`, zero biases. */
int qs_mlp_create(const float *params, uint64_t seed, void *hip_stream, qs_mlp *out);
int qs_mlp_get_params(qs_mlp m, float *params);
int qs_mlp_set_norm(qs_mlp m, const float *mean, const float *inv_std);
/* Range of the raw features over the training rows (QS_N_FEATURES floats
 * each, lo <= hi, finite; a bound of +-3e38 turns the check off for that
 * feature). A segment with a feature more than 5% of its range outside it is
 * planned by the heuristic under QS_POLICY_LEARNED. lo = hi = NULL clears
 * the range (no check). QS_EINVAL for one NULL bound or a bad range. */
int qs_mlp_set_range(qs_mlp m, const float *lo, const float *hi);
/* Segment counts of the last qs_batch_choose(QS_POLICY_LEARNED) with this
 * model, counts[4]: planned by the model, fallen back for a feature outside
 * the range, for a non-finite prediction, and for a predicted gain below the
 * margin. */
int qs_mlp_choose_stats(qs_mlp m, int *counts);
/* y[n][4] for x[n][24] (host arrays). */
int qs_mlp_forward(qs_mlp m, int n, const float *x, float *y);
/* Loss sum(mask (y - t)^2) / sum(mask) and its gradient (6020 floats). */
int qs_mlp_loss_grad(qs_mlp m, int n, const float *x, const float *t, const float *mask,
                     float *loss, float *grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the gradient of the
 * last qs_mlp_loss_grad / training minibatch. */
int qs_mlp_adam_step(qs_mlp m, float lr);
/* Mini-batch Adam over `epochs` shuffled passes; final_loss on all rows. */
int qs_mlp_train(qs_mlp m, int n, const float *x, const float *t, const float *mask, int epochs,
                 int batch, float lr, uint64_t seed, float *final_loss);
int qs_mlp_free(qs_mlp m);

/* Plan choice for every segment of a batch:
 *   QS_POLICY_FIXED_K2/K4/K6: fuse gate lists at k, emulate subroutines;
 *   QS_POLICY_HEURISTIC: arithmetic emulated (Sec. III-A, IV-B); QFT
 *     emulated when Eq. (1) (one device, no exchange) beats Eq. (2); gate
 *     lists fused at the width with the lowest roofline estimate;
 *   QS_POLICY_LEARNED: the option with the smallest predicted time, unless
 *     the heuristic's rules (above; Eqs. (1), (2)) are the fallback for the
 *     segment: a feature outside the model's training range
 *     (qs_mlp_set_range), a non-finite prediction, or a predicted gain over
 *     the heuristic's own option below 5% (0.05 in natural-log time). Only
 *     the plan differs between policies: every option gives the same state
 *     up to rounding. */
enum qs_policy { QS_POLICY_HEURISTIC = 0, QS_POLICY_LEARNED = 1, QS_POLICY_FIXED_K2 = 2,
                 QS_POLICY_FIXED_K4 = 3, QS_POLICY_FIXED_K6 = 4 };
int qs_batch_choose(qs_batch b, int policy, qs_mlp model, int *options);

/* ---------------------------------------------------------------------- */
/* Dense unitaries and the controlled powers of phase estimation          */
/* ---------------------------------------------------------------------- */

/* Sec. III-C: b-bit phase estimation needs U^1, U^2, ..., U^(2^(b-1)); a
 * simulator runs the G gates of U 2^b - 1 times, an emulator builds the
 * dense matrix of U once and squares it. */
typedef struct qs_unitary_t *qs_unitary;

/* Build the dense 2^m x 2^m complex128 matrix of the gate list c, which must
 * act on qubits [0, m) only (1 <= m <= 15): the identity is swept as a
 * 2m-qubit work state by the fused program of c (max_k as qs_compile), so
 * column j becomes U e_j. Device memory: 16 * 4^m bytes (twice that once
 * squared). Synchronous on hip_stream. */
int qs_unitary_build(const qs_circuit *c, int m, int max_k, void *hip_stream, qs_unitary *out);
int qs_unitary_info(qs_unitary u, int *m);
/* U <- U U (FP64 complex GEMM from the BLAS library), on the build stream. */
int qs_unitary_square(qs_unitary u);
/* Copy U to the host: 2^m x 2^m complex128, row-major, (re, im) interleaved
 * like gate matrices (U[r][c] maps basis state c to r). */
int qs_unitary_get(qs_unitary u, double *host_dst);
/* Apply U to qubits [0, m) of the state where qubit ctrl (m <= ctrl < n) is
 * 1: one strided-batched GEMM over the state viewed as a 2^m x 2^(n-m)
 * column-major matrix, FP64 for complex128 states, FP32 (U rounded once)
 * for complex64. Writes the second buffer and swaps (a borrowed buffer is
 * refreshed by a device copy). */
int qs_apply_controlled_unitary(qs_handle h, qs_unitary u, int ctrl);
int qs_unitary_free(qs_unitary u);
/* The controlled powers of QPE by repeated squaring: for j = 0 .. b-1,
 * U^(2^j) controlled by qubit ctrl_lo + j (the register [ctrl_lo,
 * ctrl_lo + b) must lie above qubit m - 1). The Hadamards on the control
 * register and the inverse QFT (qs_emulate_qft with inverse = 1) are the
 * caller's. */
int qs_emulate_qpe_powers(qs_handle h, const qs_circuit *c, int m, int ctrl_lo, int b, int max_k);

/* The crossover precision of Table 2 (host only, no GPU): the smallest
 * b in [1, bmax] for which a simulator's 2^b - 1 applications of U
 * (t_apply each) cost at least the emulator's build plus its per-bit
 * squarings (per_bit != 0: t_build + b t_op) or its one eigendecomposition
 * (per_bit == 0: t_build + t_op). This rule reproduces both crossover rows
 * of Table 2 from its timing rows. *out_bits = 0 if no b up to bmax
 * qualifies. QS_EINVAL for a NULL output, a time that is negative or not
 * finite, or bmax outside [1, 1000]. */
int qs_qpe_crossover_bits(double t_apply, double t_build, double t_op, int per_bit, int bmax, int *out_bits);

/* The eigensolver route of Sec. III-C: U = V diag(e^(i theta)) V^dagger,
 * after which every controlled power costs the same. The library's
 * eigensolver is Hermitian (rocSOLVER zheevd; zheev, QR iteration, as a
 * retry when zheevd reports failure or its result leaves a non-finite
 * residual, which it has done on highly degenerate input), so it is given
 * H = (U + U^dagger)/2 + beta (U - U^dagger)/(2i), beta = 0.4011..., which
 * has U's eigenvectors. H's eigenvalues cos(theta) + beta sin(theta)
 * confuse mirror images about atan(beta): a run of three or more (nearly)
 * equal eigenvalues of H (a phase with a multiplicity plus its mirror image)
 * spans an invariant subspace of U on which K = (B - B^dagger)/(2i),
 * B = V^dagger U V restricted to the run, has eigenvalues sin(theta) that
 * separate the two phases; K is diagonalised by the library's own cyclic
 * Jacobi kernel (one workgroup, runs of up to 96) and the run's columns of
 * V rotated by its eigenvectors. Each pair of neighbouring eigenvectors is
 * then rotated by the exact eigenvectors of its 2 x 2 block of V^dagger U V
 * (even pairs, then odd pairs). theta_k is the argument of the final
 * diagonal, in (-pi, pi]. The result is checked: the largest off-diagonal
 * magnitude of V^dagger U V must not exceed 1e-10 (U's 2-norm is 1);
 * otherwise QS_EUNSUPPORTED, no decomposition is kept, and the squaring
 * route (qs_emulate_qpe_powers) still applies. Device memory: three more
 * 2^m x 2^m matrices during the call, V kept. Synchronous; QS_EDEVICE if
 * an eigensolver does not converge. */
int qs_unitary_eig(qs_unitary u);
/* The largest off-diagonal magnitude of V^dagger U V measured by the last
 * qs_unitary_eig (also after it failed the check). QS_EINVAL for NULL
 * arguments or before any qs_unitary_eig. */
int qs_unitary_eig_residual(qs_unitary u, double *offdiag);
/* Copy the eigenphases (2^m doubles) and/or V (2^m x 2^m complex128,
 * row-major as qs_unitary_get; column k belongs to theta_k); either pointer
 * may be NULL. QS_EINVAL before qs_unitary_eig. */
int qs_unitary_eig_get(qs_unitary u, double *host_theta, double *host_v);
/* All b controlled powers at once: the amplitudes whose control register
 * (qubits [ctrl_lo, ctrl_lo + b), above qubit m - 1) holds c get
 * U^c = V diag(e^(i c theta)) V^dagger on qubits [0, m): two GEMMs over the
 * state viewed as a 2^m x 2^(n-m) matrix (FP64, or FP32 with V rounded once
 * for complex64 states) around one elementwise phase computed in FP64. The
 * same result as qs_emulate_qpe_powers up to rounding. Uses the scratch
 * state; the result is written back in place. */
int qs_apply_qpe_eig(qs_handle h, qs_unitary u, int ctrl_lo, int b);

/* ---------------------------------------------------------------------- */
/* Launch-parameter table (filled by an autotuner, read by the dispatchers) */
/* ---------------------------------------------------------------------- */

/* Parameters. Every value is an int; 0 restores the built-in default.
 *   QS_TUNE_SWEEP_PATH (dtype, k, class, n bucket): kernel for an
 *     uncontrolled dense k-qubit block: 1 thread per group (registers),
 *     2 wave tiles staged through LDS (needs n >= 6 + k; k <= 5 for
 *     complex128), 3 FP32 matrix cores (complex64, k = 5 or 6, n >= 12),
 *     4 workgroup tiles with the output rows split over the waves (k >= 5,
 *     n >= 6 + k), 5 workgroup-shared 1024-amplitude tiles with one load
 *     per lane per tile row group (2 <= k <= 4, n >= 10). A path that does
 *     not apply to a block falls back to the default rule (matrix cores for
 *     complex64 k = 5 and 6, workgroup tiles for complex128 blocks of 5 or 6 qubits,
 *     shared 1024-amplitude tiles for complex128 blocks of 2 to 4 qubits on
 *     20 or more qubits, LDS below the line size, registers otherwise). Every path computes the same products; only the
 *     summation order of the FP32/FP64 dot products may differ.
 *   QS_TUNE_SWEEP_WG_PER_CU (dtype, k, class, n bucket): cap of the dense
 *     sweep grid in workgroups per compute unit (grid-stride beyond it);
 *     path 5 ignores it (one workgroup per tile).
 *   QS_TUNE_FFT_DIGIT (dtype, -, -, n bucket): largest FFT digit (bits per
 *     pass), 2..10.
 *   QS_TUNE_FFT_LDS_KB (dtype, -, -, n bucket): LDS tile budget of an FFT
 *     pass, 8..160 KiB (default 80: two workgroups per CU).
 *   QS_TUNE_MFMA_WG_PER_CU (complex64, k = 5 or 6, -, n bucket): persistent grid
 *     of the matrix-core sweep in workgroups per compute unit, 1..16 (the
 *     pair-layout kernels cap it at the number that fit; default: that
 *     number, 4 for the real-form kernel).
 *   QS_TUNE_BATCH_GANG_SHARE (-, -, -, -): a batch circuit's gang is sized
 *     so its time per member is below 1/value of the average work per
 *     workgroup, 1..256.
 *   QS_TUNE_BATCH_BARRIER_AMPS (-, -, -, -): cost of a gang barrier, in
 *     amplitude-op units, used to order the batch queue.
 *   QS_TUNE_FFT_KERNEL (dtype, -, -, n bucket): FFT pass kernel. Passes
 *     with a 10-bit digit: 0 or 4 persistent workgroups holding a register
 *     tile of 128-byte rows and prefetching the next one (default), 3 one
 *     workgroup per register tile, 5 persistent register tiles with eight
 *     values per thread (1024-thread workgroups). Other passes, and every
 *     pass under 1 or 2: an LDS tile per workgroup (1), or persistent
 *     workgroups streaming LDS tiles (2). The register-tile kernels ignore
 *     the cache-policy option.
 *   QS_TUNE_SWEEP_NT (dtype, k, class, n bucket): cache policy of the
 *     register and LDS-staged dense sweeps: bit 0 nontemporal (streaming)
 *     stores, bit 1 nontemporal loads; 0 plain accesses.
 *   QS_TUNE_FFT_NT (dtype, -, -, n bucket): the same for the FFT passes.
 *   QS_TUNE_MODMUL_KERNEL (dtype, -, -, -): controlled modular
 *     multiplication with the work register at qubit 0: 0 or 5 the tiled
 *     gather with 64 x 128 tiles in 1024-thread workgroups (default), 4
 *     with 64 x 64 tiles, 3 with 64 x 32, 2 with 64 x 16 (512 or 256
 *     threads), 1 the plain per-amplitude gather.
 *   QS_TUNE_MFMA_KERNEL (complex64, k = 5 or 6, -, n bucket): matrix-core
 *     sweep kernel: 0 or 5 the three-product form (Re Y = Mr Xr - Mi Xi,
 *     Im Y = (Mr + Mi)(Xr + Xi) - Mr Xr - Mi Xi: 3/4 of the matrix-core
 *     work; default; 16-byte accesses of two neighbouring amplitudes unless
 *     qubit 0 is a block qubit), 6 the same with 8-byte accesses, 3 the
 *     real block form in the same pair layout (tile
 *     staged once as (re, im) pairs, four workgroups per compute unit,
 *     next tile loaded after the outputs are staged), 2 the same with the
 *     next tile prefetched during the k loop (three workgroups per compute
 *     unit), 4 the same loading each tile when it starts, 1 the real-form
 *     layout (two 32 KiB buffers, two workgroups per compute unit; 6-qubit
 *     blocks only, 5-qubit blocks take the default). Variants 2, 3 and 4 give identical results; the others sum
 *     in other orders, and the three-product form rounds differently (its
 *     imaginary part is a difference of products).
 *   QS_TUNE_GEMM_LIB (-, -, -, -): complex products of the dense-unitary
 *     route (squaring, controlled powers, the eigensolver route's
 *     products): 0 the library's own matrix-core kernel, 1 rocBLAS (a
 *     baseline for timing).
 * Index dimensions: dtype QS_C64/QS_C128; k 0..QS_MAX_K; class
 * QS_TCLS_* of the lowest target; n bucket 0 (n < 22), 1 (22..27),
 * 2 (n >= 28). Dimensions a parameter ignores are read at index 0.
 * qs_tune_set accepts -1 in any index as "all". The table is process-wide
 * and not synchronised: set it before launching work from other threads. */
enum qs_tune_param { QS_TUNE_SWEEP_PATH = 0, QS_TUNE_SWEEP_WG_PER_CU = 1, QS_TUNE_FFT_DIGIT = 2,
                     QS_TUNE_FFT_LDS_KB = 3, QS_TUNE_MFMA_WG_PER_CU = 4,
                     QS_TUNE_BATCH_GANG_SHARE = 5, QS_TUNE_BATCH_BARRIER_AMPS = 6,
                     QS_TUNE_FFT_KERNEL = 7, QS_TUNE_SWEEP_NT = 8, QS_TUNE_FFT_NT = 9,
                     QS_TUNE_GEMM_LIB = 10, QS_TUNE_MODMUL_KERNEL = 11, QS_TUNE_MFMA_KERNEL = 12,
                     QS_TUNE_COUNT = 13 };
/* Target classes: lowest target inside a 128-byte line, inside a wave's
 * 64 consecutive amplitudes, or above bit 5. */
enum qs_tune_class { QS_TCLS_SUBLINE = 0, QS_TCLS_SUBWAVE = 1, QS_TCLS_HIGH = 2 };
int qs_tune_set(int param, int dtype, int k, int cls, int nbucket, int value);
int qs_tune_get(int param, int dtype, int k, int cls, int nbucket, int *value);
int qs_tune_reset(void);
/* The class and n bucket the dispatchers use for a block. */
int qs_tune_classify(int dtype, int n_qubits, int k, const int *targets, int *cls, int *nbucket);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
