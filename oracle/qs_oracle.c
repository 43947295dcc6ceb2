/*
 * CPU FP64 oracle for the state-vector path of "High Performance Emulation
 * of Quantum Circuits" (Haener, Steiger, Smelyanskiy, Troyer).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct
 * reference that the GPU library is checked against. It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * links or calls it. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.
 *
 * Conventions (Sec. II): a state of n qubits is 2^n complex amplitudes
 * alpha_i. Qubit q is bit q of the index i (qubit 0 = least significant
 * bit; the paper's Kronecker example lists qubit 0 as the most significant
 * factor, which is the relabelling q -> n-1-q). Amplitudes are stored as
 * C99 double complex.
 *
 * A gate on k targets t[0..k-1] is a 2^k x 2^k matrix M (row-major); bit m
 * of its local index is the bit of qubit t[m]. It acts only on indices i with
 * (i & ctrl_mask) == ctrl_vals.
 *
 * Every routine here is the plain definition: no fusion, no structure
 * shortcut, no blocking. Loops over disjoint groups may run under OpenMP.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_OK 0
#define OR_EINVAL 1

/* ---------------------------------------------------------------------- */
/* Table 1 gate constants, written out from the table.                     */
/* ---------------------------------------------------------------------- */
/* Number of host threads the OpenMP loops below use (a timing control for
 * the CPU baseline; results do not depend on it). Returns the count in
 * effect. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

void or_table1(int which, double theta, double *out /* 2^k x 2^k interleaved */)
{
    /* which: 0 X, 1 Y, 2 Z, 3 H, 4 S, 5 T, 6 Rz(theta), 7 CNOT, 8 CR(theta) */
    cplx m[16];
    int dim = which >= 7 ? 4 : 2;
    for (int i = 0; i < 16; ++i) m[i] = 0;
    const double r = 1.0 / sqrt(2.0);
    switch (which) {
    case 0: m[1] = 1; m[2] = 1; break;
    case 1: m[1] = -I; m[2] = I; break;
    case 2: m[0] = 1; m[3] = -1; break;
    case 3: m[0] = r; m[1] = r; m[2] = r; m[3] = -r; break;
    case 4: m[0] = 1; m[3] = I; break;
    case 5: m[0] = 1; m[3] = cexp(I * M_PI / 4.0); break;
    case 6: m[0] = cexp(-I * theta / 2.0); m[3] = cexp(I * theta / 2.0); break;
    case 7: m[0] = 1; m[5] = 1; m[11] = 1; m[14] = 1; break;
    case 8: m[0] = 1; m[5] = 1; m[10] = 1; m[15] = cexp(I * theta); break;
    default: return;
    }
    for (int i = 0; i < dim * dim; ++i) {
        out[2 * i] = creal(m[i]);
        out[2 * i + 1] = cimag(m[i]);
    }
}

/* ---------------------------------------------------------------------- */
/* One gate as a sparse mat-vec (Sec. II): the 2^n x 2^n operator is the   */
/* Kronecker product of M with identities; applied group by group.         */
/* ---------------------------------------------------------------------- */
int or_apply_gate(cplx *psi, int n, int k, const int *t, const double *mat,
                  uint64_t ctrl_mask, uint64_t ctrl_vals)
{
    if (k < 1 || k > 12 || n < k || n > 40) return OR_EINVAL;
    uint64_t tmask = 0;
    for (int m = 0; m < k; ++m) {
        if (t[m] < 0 || t[m] >= n || (tmask >> t[m]) & 1) return OR_EINVAL;
        tmask |= 1ull << t[m];
    }
    if (ctrl_mask & tmask) return OR_EINVAL;
    if (ctrl_vals & ~ctrl_mask) return OR_EINVAL;
    const int dim = 1 << k;
    const cplx *M = (const cplx *)mat;
    const uint64_t N = 1ull << n;
    /* offset of local index j inside a group */
    uint64_t *off = malloc(sizeof(uint64_t) * dim);
    for (int j = 0; j < dim; ++j) {
        uint64_t o = 0;
        for (int m = 0; m < k; ++m)
            if ((j >> m) & 1) o |= 1ull << t[m];
        off[j] = o;
    }
#pragma omp parallel
    {
        cplx *v = malloc(sizeof(cplx) * dim);
#pragma omp for schedule(static)
        for (int64_t base = 0; base < (int64_t)N; ++base) {
            if (((uint64_t)base & tmask) != 0) continue;
            if (((uint64_t)base & ctrl_mask) != ctrl_vals) continue;
            for (int j = 0; j < dim; ++j) v[j] = psi[base | off[j]];
            for (int j = 0; j < dim; ++j) {
                cplx acc = 0;
                for (int l = 0; l < dim; ++l) acc += M[(size_t)j * dim + l] * v[l];
                psi[base | off[j]] = acc;
            }
        }
        free(v);
    }
    free(off);
    return OR_OK;
}

/* A circuit is its gates applied one at a time, in order. */
int or_apply_circuit(cplx *psi, int n, int n_gates, const int *ks,
                     const int *targets, const double *mats,
                     const uint64_t *ctrl_masks, const uint64_t *ctrl_vals)
{
    size_t toff = 0, moff = 0;
    for (int g = 0; g < n_gates; ++g) {
        int rc = or_apply_gate(psi, n, ks[g], targets + toff, mats + moff,
                               ctrl_masks ? ctrl_masks[g] : 0,
                               ctrl_vals ? ctrl_vals[g] : 0);
        if (rc) return rc;
        toff += ks[g];
        moff += 2ull << (2 * ks[g]);
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* QFT (Sec. III-B): alpha_l -> 2^(-m/2) sum_k alpha_k exp(+2 pi i k l/2^m) */
/* on the m-qubit field [q_lo, q_lo+m) of the index; the other bits of the */
/* index are spectators. inverse != 0 takes the complex conjugate kernel.  */
/* ---------------------------------------------------------------------- */
static cplx unit_root(uint64_t num, int m, int sign)
{
    /* exp(sign * 2 pi i num / 2^m) with num reduced exactly mod 2^m */
    uint64_t r = num & ((1ull << m) - 1);
    double ang = 2.0 * M_PI * ((double)r / (double)(1ull << m));
    return cos(ang) + (double)sign * I * sin(ang);
}

/* Direct O(2^(n+m)) transform; psi_out must not alias psi_in. */
int or_qft_direct(const cplx *in, cplx *out, int n, int q_lo, int m, int inverse)
{
    if (m < 1 || q_lo < 0 || q_lo + m > n) return OR_EINVAL;
    const uint64_t N = 1ull << n, M = 1ull << m;
    const uint64_t fmask = (M - 1) << q_lo;
    const double scale = 1.0 / sqrt((double)M);
    const int sign = inverse ? -1 : 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)N; ++i) {
        uint64_t l = ((uint64_t)i >> q_lo) & (M - 1);
        uint64_t rest = (uint64_t)i & ~fmask;
        cplx acc = 0;
        for (uint64_t kk = 0; kk < M; ++kk)
            acc += in[rest | (kk << q_lo)] * unit_root(kk * l, m, sign);
        out[i] = acc * scale;
    }
    return OR_OK;
}

/* One output amplitude of the same transform, for spot checks at sizes
 * where the full transform is out of reach. */
int or_qft_sample(const cplx *in, int n, int q_lo, int m, int inverse,
                  uint64_t i, double *out2)
{
    if (m < 1 || q_lo < 0 || q_lo + m > n || i >> n) return OR_EINVAL;
    const uint64_t M = 1ull << m;
    const uint64_t l = (i >> q_lo) & (M - 1);
    const uint64_t rest = i & ~((M - 1) << q_lo);
    const int sign = inverse ? -1 : 1;
    double re = 0.0, im = 0.0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (int64_t kk = 0; kk < (int64_t)M; ++kk) {
        cplx p = in[rest | ((uint64_t)kk << q_lo)] * unit_root((uint64_t)kk * l, m, sign);
        re += creal(p);
        im += cimag(p);
    }
    out2[0] = re / sqrt((double)M);
    out2[1] = im / sqrt((double)M);
    return OR_OK;
}

/* Gate-level QFT (Sec. III-B): n Hadamards and n(n-1)/2 conditional phase
 * shifts CR(2 pi / 2^(d+1)) for qubit distance d, then the SWAPs that put
 * the output in natural order. */
int or_qft_gates(cplx *psi, int n, int q_lo, int m, int inverse)
{
    if (m < 1 || q_lo < 0 || q_lo + m > n) return OR_EINVAL;
    double h[8], crm[32], sw[32];
    or_table1(3, 0.0, h);
    memset(sw, 0, sizeof sw);
    sw[2 * 0] = 1; sw[2 * 6] = 1; sw[2 * 9] = 1; sw[2 * 15] = 1;
    const int sign = inverse ? -1 : 1;
    if (!inverse) {
        for (int t = m - 1; t >= 0; --t) {
            int tq = q_lo + t;
            or_apply_gate(psi, n, 1, &tq, h, 0, 0);
            for (int c = t - 1; c >= 0; --c) {
                int tg[2] = {q_lo + t, q_lo + c};
                or_table1(8, sign * 2.0 * M_PI / (double)(1ull << (t - c + 1)), crm);
                or_apply_gate(psi, n, 2, tg, crm, 0, 0);
            }
        }
        for (int q = 0; q < m / 2; ++q) {
            int tg[2] = {q_lo + q, q_lo + m - 1 - q};
            or_apply_gate(psi, n, 2, tg, sw, 0, 0);
        }
    } else {
        /* adjoint: the same gates in reverse order with conjugated phases */
        for (int q = m / 2 - 1; q >= 0; --q) {
            int tg[2] = {q_lo + q, q_lo + m - 1 - q};
            or_apply_gate(psi, n, 2, tg, sw, 0, 0);
        }
        for (int t = 0; t < m; ++t) {
            for (int c = 0; c <= t - 1; ++c) {
                int tg[2] = {q_lo + t, q_lo + c};
                or_table1(8, sign * 2.0 * M_PI / (double)(1ull << (t - c + 1)), crm);
                or_apply_gate(psi, n, 2, tg, crm, 0, 0);
            }
            int tq = q_lo + t;
            or_apply_gate(psi, n, 1, &tq, h, 0, 0);
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Arithmetic as a permutation of basis states (Sec. III-A).               */
/* ---------------------------------------------------------------------- */
static uint64_t powmod_u64(uint64_t a, uint64_t e, uint64_t N)
{
    /* square-and-multiply; N < 2^32 so every product fits in 64 bits */
    uint64_t r = 1 % N, b = a % N;
    while (e) {
        if (e & 1) r = (r * b) % N;
        b = (b * b) % N;
        e >>= 1;
    }
    return r;
}

/* |c>|x> -> |c>|a^c x mod N> with c the c-bit field at ctrl_lo and x the
 * w-bit field at work_lo; x >= N is left in place. out must not alias in.
 * Returns OR_EINVAL if the map is not a bijection (some destination hit
 * twice), which cannot happen for gcd(a, N) == 1. */
int or_modmul(const cplx *in, cplx *out, int n, int work_lo, int w,
              int ctrl_lo, int c, uint64_t a, uint64_t N)
{
    if (w < 1 || c < 0 || work_lo < 0 || ctrl_lo < 0 || work_lo + w > n ||
        ctrl_lo + c > n || N < 2 || N > (1ull << w) || N >= (1ull << 32))
        return OR_EINVAL;
    if (c > 0 && !(ctrl_lo >= work_lo + w || ctrl_lo + c <= work_lo)) return OR_EINVAL;
    const uint64_t NN = 1ull << n;
    const uint64_t wmask = ((1ull << w) - 1) << work_lo;
    uint64_t *A = malloc(sizeof(uint64_t) << c);
    for (uint64_t cc = 0; cc < (1ull << c); ++cc) A[cc] = powmod_u64(a, cc, N);
    unsigned char *hit = calloc(NN, 1);
    int bad = 0;
    for (uint64_t i = 0; i < NN; ++i) {
        uint64_t cc = c ? (i >> ctrl_lo) & ((1ull << c) - 1) : 0;
        uint64_t x = (i >> work_lo) & ((1ull << w) - 1);
        uint64_t xp = x < N ? (A[cc] * x) % N : x;
        uint64_t j = (i & ~wmask) | (xp << work_lo);
        if (hit[j]) bad = 1;
        hit[j] = 1;
        out[j] = in[i];
    }
    free(hit);
    free(A);
    return bad ? OR_EINVAL : OR_OK;
}

/* Generic permutation of the nbits-wide field at lo: field value f moves to
 * dest[f]. out must not alias in. */
int or_table_perm(const cplx *in, cplx *out, int n, int lo, int nbits,
                  const uint64_t *dest)
{
    if (nbits < 1 || lo < 0 || lo + nbits > n) return OR_EINVAL;
    const uint64_t NN = 1ull << n, F = 1ull << nbits;
    const uint64_t fmask = (F - 1) << lo;
    for (uint64_t i = 0; i < NN; ++i) {
        uint64_t f = (i >> lo) & (F - 1);
        if (dest[f] >= F) return OR_EINVAL;
        out[(i & ~fmask) | (dest[f] << lo)] = in[i];
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Measurement quantities read directly off the state (Sec. III-D).        */
/* ---------------------------------------------------------------------- */
double or_norm2(const cplx *psi, int n)
{
    double s = 0.0;
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < N; ++i) s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    return s;
}

/* <psi| P |psi> for the Pauli string with X on x_mask, Y on y_mask and Z on
 * z_mask (disjoint masks). Each Pauli factor is applied to |i> literally:
 * X|b> = |1-b>, Y|b> = i(-1)^b |1-b>, Z|b> = (-1)^b |b>. */
int or_expectation(const cplx *psi, int n, uint64_t xm, uint64_t ym, uint64_t zm,
                   double *out2)
{
    if ((xm & ym) || (xm & zm) || (ym & zm)) return OR_EINVAL;
    if (n < 64 && ((xm | ym | zm) >> n)) return OR_EINVAL;
    const int64_t N = (int64_t)1 << n;
    double re = 0.0, im = 0.0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        /* P|i> = coef |j> */
        uint64_t j = (uint64_t)i;
        cplx coef = 1;
        for (int q = 0; q < n; ++q) {
            int b = (int)(((uint64_t)i >> q) & 1);
            if ((xm >> q) & 1) { j ^= 1ull << q; }
            else if ((ym >> q) & 1) { j ^= 1ull << q; coef *= (b ? -I : I); }
            else if ((zm >> q) & 1) { if (b) coef = -coef; }
        }
        cplx term = conj(psi[j]) * coef * psi[i];
        re += creal(term);
        im += cimag(term);
    }
    out2[0] = re;
    out2[1] = im;
    return OR_OK;
}

/* Marginal probabilities p[o] over the listed qubits: bit r of o is the bit
 * of qubits[r]. */
int or_marginals(const cplx *psi, int n, int m, const int *qubits, double *p)
{
    if (m < 1 || m > n || m > 30) return OR_EINVAL;
    uint64_t seen = 0;
    for (int r = 0; r < m; ++r) {
        if (qubits[r] < 0 || qubits[r] >= n || (seen >> qubits[r]) & 1) return OR_EINVAL;
        seen |= 1ull << qubits[r];
    }
    memset(p, 0, sizeof(double) << m);
    const uint64_t N = 1ull << n;
    for (uint64_t i = 0; i < N; ++i) {
        uint64_t o = 0;
        for (int r = 0; r < m; ++r) o |= ((i >> qubits[r]) & 1) << r;
        p[o] += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    }
    return OR_OK;
}

/* Outcome for a uniform u: the smallest o whose running sum of p exceeds
 * u times the total (outcomes drawn with probability |alpha|^2, Sec. II). */
int or_sample(const double *p, int m, int shots, const double *uniforms, uint64_t *outcomes)
{
    const uint64_t M = 1ull << m;
    double total = 0.0;
    for (uint64_t o = 0; o < M; ++o) total += p[o];
    for (int s = 0; s < shots; ++s) {
        double target = uniforms[s] * total, run = 0.0;
        uint64_t pick = M - 1;
        for (uint64_t o = 0; o < M; ++o) {
            run += p[o];
            if (run > target) { pick = o; break; }
        }
        outcomes[s] = pick;
    }
    return OR_OK;
}

/* Collapse onto outcome o of the listed qubits: other amplitudes are set to
 * zero, the rest rescaled by 1/sqrt(p_o). */
int or_collapse(cplx *psi, int n, int m, const int *qubits, uint64_t o, double p_o)
{
    if (p_o <= 0.0) return OR_EINVAL;
    const uint64_t N = 1ull << n;
    const double s = 1.0 / sqrt(p_o);
    for (uint64_t i = 0; i < N; ++i) {
        uint64_t oi = 0;
        for (int r = 0; r < m; ++r) oi |= ((i >> qubits[r]) & 1) << r;
        psi[i] = (oi == o) ? psi[i] * s : 0.0;
    }
    return OR_OK;
}
