"""CPU FP64 oracle for the state-vector path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module. It shares no code with the GPU library: the C routines in
``qs_oracle.c`` are loaded from ``liboracle.so`` (built with gcc), and the
NumPy functions below are written from the paper's definitions.

Contents
--------
* ctypes wrappers of the C oracle (gate-by-gate simulation, Sec. II; QFT,
  Sec. III-B; arithmetic permutations, Sec. III-A; measurement, Sec. III-D).
* ``full_matrix``: brute-force 2^n x 2^n operator of one gate built from a
  Kronecker product and a qubit permutation, for n <= 8.
* ``block_matrix``: the product of embedded gates on a small qubit set (what a
  fused block must equal).
* ``MLP``: FP64 NumPy forward/backward/Adam of the 24-64-64-4 cost model,
  with central finite differences.
* Cost models of Sec. III-B (Eqs. 1 and 2) and the Table 2 crossover rule.
* Per-index forms for spot checks at sizes the full simulation cannot
  reach: ``modmul_source`` and ``layer_amplitudes``.
* ``qpe_powers``: the controlled powers of phase estimation applied gate by
  gate, 2^j runs of U per control qubit (Sec. III-C).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build_oracle  # noqa: WPS433
            build_oracle.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = C.c_int
        L.or_table1.argtypes = [C.c_int, C.c_double, P]
        L.or_apply_gate.argtypes = [P, C.c_int, C.c_int, P, P, C.c_uint64, C.c_uint64]
        L.or_apply_circuit.argtypes = [P, C.c_int, C.c_int, P, P, P, P, P]
        L.or_qft_direct.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_qft_sample.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, P]
        L.or_qft_gates.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_modmul.argtypes = [P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                C.c_uint64, C.c_uint64]
        L.or_table_perm.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P]
        L.or_norm2.argtypes = [P, C.c_int]
        L.or_norm2.restype = C.c_double
        L.or_expectation.argtypes = [P, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, P]
        L.or_marginals.argtypes = [P, C.c_int, C.c_int, P, P]
        L.or_sample.argtypes = [P, C.c_int, C.c_int, P, P]
        L.or_collapse.argtypes = [P, C.c_int, C.c_int, P, C.c_uint64, C.c_double]
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c128(psi):
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return psi


def _nq(psi):
    n = int(psi.size).bit_length() - 1
    assert psi.size == 1 << n
    return n


class OracleError(RuntimeError):
    pass


def _chk(rc):
    if rc != 0:
        raise OracleError("oracle rejected its arguments (rc=%d)" % rc)


def set_threads(n: int) -> int:
    """Host threads of the C oracle's loops (0 keeps the current count);
    returns the count in effect."""
    return int(lib().or_set_threads(int(n)))


# ---------------------------------------------------------------------------
# Table 1 and single gates
# ---------------------------------------------------------------------------
TABLE1 = {"X": 0, "Y": 1, "Z": 2, "H": 3, "S": 4, "T": 5, "RZ": 6, "CNOT": 7, "CR": 8}


def table1(name: str, theta: float = 0.0) -> np.ndarray:
    idx = TABLE1[name]
    dim = 4 if idx >= 7 else 2
    out = np.zeros(dim * dim, dtype=np.complex128)
    lib().or_table1(idx, theta, _p(out))
    return out.reshape(dim, dim)


def apply_gate(psi, targets, matrix, ctrl_mask=0, ctrl_vals=0):
    """Apply one gate in place (plain group-by-group mat-vec, Sec. II)."""
    psi = _c128(psi)
    t = np.ascontiguousarray(targets, dtype=np.int32)
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    _chk(lib().or_apply_gate(_p(psi), _nq(psi), len(t), _p(t), _p(m),
                             int(ctrl_mask), int(ctrl_vals)))
    return psi


def apply_circuit(psi, gates):
    """Apply a gate list one gate at a time, in order; returns the state."""
    psi = _c128(psi).copy()
    if not gates:
        return psi
    ks = np.array([len(g.targets) for g in gates], dtype=np.int32)
    tg = np.array([t for g in gates for t in g.targets], dtype=np.int32)
    mats = np.concatenate([np.ascontiguousarray(g.matrix, dtype=np.complex128).reshape(-1)
                           for g in gates])
    cm = np.array([g.ctrl_mask for g in gates], dtype=np.uint64)
    cv = np.array([g.ctrl_vals for g in gates], dtype=np.uint64)
    _chk(lib().or_apply_circuit(_p(psi), _nq(psi), len(gates), _p(ks), _p(tg), _p(mats),
                                _p(cm), _p(cv)))
    return psi


# ---------------------------------------------------------------------------
# QFT (Sec. III-B)
# ---------------------------------------------------------------------------
def qft_direct(psi, q_lo=0, m=None, inverse=False):
    psi = _c128(psi)
    n = _nq(psi)
    m = n - q_lo if m is None else m
    out = np.empty_like(psi)
    _chk(lib().or_qft_direct(_p(psi), _p(out), n, q_lo, m, int(bool(inverse))))
    return out


def qft_sample(psi, idx, q_lo=0, m=None, inverse=False):
    psi = _c128(psi)
    n = _nq(psi)
    m = n - q_lo if m is None else m
    out = np.zeros(2)
    _chk(lib().or_qft_sample(_p(psi), n, q_lo, m, int(bool(inverse)), int(idx), _p(out)))
    return complex(out[0], out[1])


def qft_gates(psi, q_lo=0, m=None, inverse=False):
    psi = _c128(psi).copy()
    n = _nq(psi)
    m = n - q_lo if m is None else m
    _chk(lib().or_qft_gates(_p(psi), n, q_lo, m, int(bool(inverse))))
    return psi


# ---------------------------------------------------------------------------
# Arithmetic permutations (Sec. III-A)
# ---------------------------------------------------------------------------
def modmul(psi, work_lo, w, ctrl_lo, c, a, N):
    psi = _c128(psi)
    out = np.zeros_like(psi)
    _chk(lib().or_modmul(_p(psi), _p(out), _nq(psi), work_lo, w, ctrl_lo, c, int(a), int(N)))
    return out


def modmul_source(idx, work_lo, w, ctrl_lo, c, a, N):
    """Per-index form of the controlled modular multiplication (Sec. III-A):
    for each output index i, the input index whose amplitude lands there.
    With x' the work-register value of i and c_val its control value,
    x' < N came from x = a^(-c_val) x' mod N; x' >= N is fixed. Python
    integers, one index at a time."""
    out = []
    wm = (1 << w) - 1
    for i in (int(v) for v in idx):
        xp = (i >> work_lo) & wm
        cv = (i >> ctrl_lo) & ((1 << c) - 1) if c else 0
        if xp < N:
            x = (pow(int(a), -cv, int(N)) * xp) % N
            i = (i & ~(wm << work_lo)) | (x << work_lo)
        out.append(i)
    return np.array(out, dtype=np.uint64)


ARITH_MUL, ARITH_DIV = 0, 1


def _field(idx, lo, m):
    return (idx >> np.uint64(lo)) & np.uint64((1 << m) - 1)


def arith_dest(idx, kind, a_lo, b_lo, c_lo, m):
    """Where each basis index goes under the emulated integer multiplication
    or division of Sec. III-A, for three m-bit registers a, b, c.

    Multiplication: (a, b, c) -> (a, b, c + a*b mod 2^m). With c = 0 this is
    the map (a, b, 0) -> (a, b, ab), the product cut to the m bits of c.

    Division: with c = 0 the map (a, b, 0) -> (a mod b, b, a div b) of the
    paper, computed here by integer division; b = 0 (undefined there) gives
    (a, 0, 2^m - 1), as the reversible restoring division below does. The
    paper fixes no action for c != 0; we take that of the restoring-division
    network that a simulator runs (repeated subtraction and shift): with
    Y = a + 2^m c, for i = m-1 down to 0 the (m+1)-bit window W of Y at bit i
    becomes W - b mod 2^(m+1); if its top bit is then set, b is added back
    to its low m bits mod 2^m; the top bit is flipped. The top bits left
    behind are the quotient bits."""
    idx = np.asarray(idx, dtype=np.uint64)
    M0 = np.uint64((1 << m) - 1)
    a, b, c = _field(idx, a_lo, m), _field(idx, b_lo, m), _field(idx, c_lo, m)
    if kind == ARITH_MUL:
        a2, c2 = a, (c + a * b) & M0
    elif kind == ARITH_DIV:
        a2, c2 = a.copy(), c.copy()
        clean = c == 0
        nz = clean & (b != 0)
        a2[nz] = a[nz] % b[nz]
        c2[nz] = a[nz] // b[nz]
        c2[clean & (b == 0)] = M0
        # c != 0: step through the network's arithmetic
        d = ~clean
        Y = a[d] | (c[d] << np.uint64(m))
        bd = b[d]
        M1 = np.uint64((1 << (m + 1)) - 1)
        top = np.uint64(1 << m)
        for i in range(m - 1, -1, -1):
            sh = np.uint64(i)
            W = (Y >> sh) & M1
            W = (W - bd) & M1
            s = W >> np.uint64(m)
            W = (W & top) | (((W & M0) + s * bd) & M0)
            W = W ^ top
            Y = (Y & ~(M1 << sh)) | (W << sh)
        a2[d] = Y & M0
        c2[d] = Y >> np.uint64(m)
    else:
        raise ValueError("unknown arithmetic kind")
    keep = ~((M0 << np.uint64(a_lo)) | (M0 << np.uint64(c_lo)))
    return (idx & keep) | (a2 << np.uint64(a_lo)) | (c2 << np.uint64(c_lo))


def arith(psi, kind, a_lo, b_lo, c_lo, m):
    """The whole state after the emulated multiplication or division: the
    amplitude at index i moves to arith_dest(i)."""
    psi = np.asarray(psi)
    dest = arith_dest(np.arange(psi.size, dtype=np.uint64), kind, a_lo, b_lo, c_lo, m)
    out = np.zeros_like(psi)
    out[dest.astype(np.int64)] = psi
    return out


def layer_amplitudes(one_qubit, cz_pairs, idx):
    """Amplitudes, at the given basis indices, of one random layer applied
    to |0...0>: single-qubit gates U_q on every qubit (a product state whose
    qubit-q factor is the first column of U_q, Sec. II) followed by CZ on
    disjoint pairs (each contributes -1 when both of its bits are 1)."""
    cols = [np.asarray(u, dtype=np.complex128)[:, 0] for u in one_qubit]
    out = np.empty(len(idx), dtype=np.complex128)
    for j, i in enumerate(int(v) for v in idx):
        amp = 1.0 + 0.0j
        for q, col in enumerate(cols):
            amp *= col[(i >> q) & 1]
        for qa, qb in cz_pairs:
            if (i >> qa) & 1 and (i >> qb) & 1:
                amp = -amp
        out[j] = amp
    return out


def table_perm(psi, lo, nbits, dest):
    psi = _c128(psi)
    out = np.zeros_like(psi)
    d = np.ascontiguousarray(dest, dtype=np.uint64)
    _chk(lib().or_table_perm(_p(psi), _p(out), _nq(psi), lo, nbits, _p(d)))
    return out


# ---------------------------------------------------------------------------
# Measurement (Sec. III-D)
# ---------------------------------------------------------------------------
def norm2(psi):
    psi = _c128(psi)
    return lib().or_norm2(_p(psi), _nq(psi))


def expectation(psi, x_mask=0, y_mask=0, z_mask=0):
    psi = _c128(psi)
    out = np.zeros(2)
    _chk(lib().or_expectation(_p(psi), _nq(psi), int(x_mask), int(y_mask), int(z_mask), _p(out)))
    return complex(out[0], out[1])


def marginals(psi, qubits):
    psi = _c128(psi)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    p = np.zeros(1 << len(q))
    _chk(lib().or_marginals(_p(psi), _nq(psi), len(q), _p(q), _p(p)))
    return p


def sample(p, uniforms):
    p = np.ascontiguousarray(p, dtype=np.float64)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    m = int(p.size).bit_length() - 1
    out = np.zeros(u.size, dtype=np.uint64)
    _chk(lib().or_sample(_p(p), m, u.size, _p(u), _p(out)))
    return out


def collapse(psi, qubits, outcome, p_outcome):
    psi = _c128(psi).copy()
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    _chk(lib().or_collapse(_p(psi), _nq(psi), len(q), _p(q), int(outcome), float(p_outcome)))
    return psi


# ---------------------------------------------------------------------------
# Brute force (n <= 8): the full operator of a gate from a Kronecker product
# ---------------------------------------------------------------------------
def full_matrix(n, targets, matrix, ctrl_mask=0, ctrl_vals=0):
    """2^n x 2^n operator: the (k+c)-qubit matrix (identity outside the block
    selected by the control values) is placed on the lowest qubits with
    kron(I, M), then conjugated by the permutation matrix that moves each
    listed qubit to its position."""
    targets = list(targets)
    ctrls = [q for q in range(n) if (ctrl_mask >> q) & 1]
    k, c = len(targets), len(ctrls)
    Mk = np.asarray(matrix, dtype=np.complex128)
    dimk = 1 << k
    # (k+c)-qubit matrix: low k local bits = targets, next c bits = controls
    big = np.eye(dimk << c, dtype=np.complex128)
    sel = 0
    for r, q in enumerate(ctrls):
        if (ctrl_vals >> q) & 1:
            sel |= 1 << r
    big[sel * dimk:(sel + 1) * dimk, sel * dimk:(sel + 1) * dimk] = Mk
    order = targets + ctrls + [q for q in range(n) if q not in targets and q not in ctrls]
    U0 = np.kron(np.eye(1 << (n - k - c)), big)
    # P maps basis |i> (original labels) to |i'> where bit r of i' = bit order[r] of i
    N = 1 << n
    perm = np.zeros(N, dtype=np.int64)
    for i in range(N):
        ip = 0
        for r, q in enumerate(order):
            ip |= ((i >> q) & 1) << r
        perm[i] = ip
    P = np.zeros((N, N))
    P[perm, np.arange(N)] = 1.0
    return P.T @ U0 @ P


def block_matrix(k, gates_local):
    """Product (last gate leftmost) of the embedded matrices of gates whose
    targets/controls are given in a k-qubit local numbering."""
    U = np.eye(1 << k, dtype=np.complex128)
    for g in gates_local:
        U = full_matrix(k, g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals) @ U
    return U


def qpe_powers(psi, gates, ctrl_lo, b):
    """The controlled powers of phase estimation as a simulator applies them
    (Sec. III-C): for j = 0 .. b-1 the gate list of U runs 2^j times, every
    gate controlled by qubit ctrl_lo + j."""
    from types import SimpleNamespace
    psi = _c128(psi).copy()
    for j in range(b):
        c = 1 << (ctrl_lo + j)
        cg = [SimpleNamespace(targets=tuple(g.targets), matrix=g.matrix, ctrl_mask=int(g.ctrl_mask) | c,
                              ctrl_vals=int(g.ctrl_vals) | c) for g in gates]
        for _ in range(1 << j):
            psi = apply_circuit(psi, cg)
    return psi


def qpe_eig_powers(psi, gates, m, ctrl_lo, b):
    """The same controlled powers by the eigensolver route of Sec. III-C:
    U = V diag(e^(i theta)) V^(-1) from numpy.linalg.eig of U's dense matrix
    (block_matrix); the slice of psi whose control register (qubits
    ctrl_lo .. ctrl_lo+b-1) holds c gets V diag(e^(i c theta)) V^(-1). The
    target register is qubits 0 .. m-1."""
    psi = _c128(psi).copy()
    n = _nq(psi)
    U = block_matrix(m, gates)
    w, V = np.linalg.eig(U)
    Vi = np.linalg.inv(V)
    theta = np.angle(w)
    X = psi.reshape(-1, 1 << m).T                    # column j: target amplitudes of the other bits j
    cols = np.arange(X.shape[1])
    c = (cols >> (ctrl_lo - m)) & ((1 << b) - 1)
    Y = Vi @ X
    Y *= np.exp(1j * np.outer(theta, c))
    out = (V @ Y).T.reshape(-1)
    assert out.size == 1 << n
    return out


def dft_numpy(psi, q_lo=0, m=None, inverse=False):
    """Independent library check of the QFT formula: ifft with orthonormal
    scaling has the +2 pi i sign of Sec. III-B; fft is its inverse."""
    psi = np.asarray(psi, dtype=np.complex128)
    n = _nq(psi)
    m = n - q_lo if m is None else m
    shaped = psi.reshape(1 << (n - q_lo - m), 1 << m, 1 << q_lo)
    f = np.fft.fft if inverse else np.fft.ifft
    return f(shaped, axis=1, norm="ortho").reshape(-1)


# ---------------------------------------------------------------------------
# Cost models of Sec. III-B and the QPE crossover of Table 2
# ---------------------------------------------------------------------------
def t_fft(n, eff, flops_peak, b_net, P=1):
    """Eq. (1): 5 N n / (Eff * FLOPS) + 3 * 16 N / B_net (no exchange for P = 1)."""
    N = 2.0 ** n
    comm = 3.0 * 16.0 * N / b_net if P > 1 else 0.0
    return 5.0 * N * n / (eff * flops_peak) + comm


def t_qft(n, b_mem, b_net, P=1):
    """Eq. (2): 4 N n^2 / B_mem + log2(P) * 16 N / B_net."""
    N = 2.0 ** n
    return 4.0 * N * n * n / b_mem + (np.log2(P) * 16.0 * N / b_net if P > 1 else 0.0)


def qpe_crossover(t_apply, t_build, t_op, repeated_squaring=True, bmax=200):
    """Smallest precision b (bits) at which emulated QPE is no slower than
    simulating it: simulation applies U 2^b - 1 times (Sec. III-C); emulation
    builds U once and then either squares it b times or runs one
    eigendecomposition."""
    for b in range(1, bmax):
        sim = (2.0 ** b - 1.0) * t_apply
        emu = t_build + (b * t_op if repeated_squaring else t_op)
        if sim >= emu:
            return b
    return None


# ---------------------------------------------------------------------------
# The 24-64-64-4 cost model in FP64 (reference for the GPU kernels)
# ---------------------------------------------------------------------------
class MLP:
    """y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, row-major (x @ W).

    Loss: masked mean squared error, sum(mask * (y - t)^2) / sum(mask)."""

    SHAPES = [(24, 64), (64,), (64, 64), (64,), (64, 4), (4,)]

    def __init__(self, params):
        self.p = [np.asarray(a, dtype=np.float64).copy() for a in params]

    @staticmethod
    def init(seed):
        rng = np.random.default_rng(seed)
        ps = []
        for s in MLP.SHAPES:
            if len(s) == 2:
                ps.append(rng.standard_normal(s) * np.sqrt(2.0 / s[0]))
            else:
                ps.append(np.zeros(s))
        return ps

    def forward(self, X):
        W1, b1, W2, b2, W3, b3 = self.p
        a1 = X @ W1 + b1
        h1 = np.maximum(a1, 0.0)
        a2 = h1 @ W2 + b2
        h2 = np.maximum(a2, 0.0)
        y = h2 @ W3 + b3
        return y, (X, a1, h1, a2, h2)

    def loss(self, X, T, mask):
        y, _ = self.forward(X)
        return float(np.sum(mask * (y - T) ** 2) / np.sum(mask))

    def grads(self, X, T, mask):
        W1, b1, W2, b2, W3, b3 = self.p
        y, (X, a1, h1, a2, h2) = self.forward(X)
        dy = 2.0 * mask * (y - T) / np.sum(mask)
        gW3 = h2.T @ dy
        gb3 = dy.sum(0)
        dh2 = dy @ W3.T
        da2 = dh2 * (a2 > 0)
        gW2 = h1.T @ da2
        gb2 = da2.sum(0)
        dh1 = da2 @ W2.T
        da1 = dh1 * (a1 > 0)
        gW1 = X.T @ da1
        gb1 = da1.sum(0)
        return [gW1, gb1, gW2, gb2, gW3, gb3]

    def fd_grads(self, X, T, mask, h=1e-6, entries=None):
        """Central finite differences on selected (param, flat index) pairs."""
        out = []
        for pi, fi in entries:
            old = self.p[pi].flat[fi]
            self.p[pi].flat[fi] = old + h
            lp = self.loss(X, T, mask)
            self.p[pi].flat[fi] = old - h
            lm = self.loss(X, T, mask)
            self.p[pi].flat[fi] = old
            out.append((lp - lm) / (2.0 * h))
        return np.array(out)

    @staticmethod
    def adam(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        """One Adam step (Kingma and Ba) in place; t counts from 1."""
        for p, g, mm, vv in zip(params, grads, m, v):
            mm *= b1
            mm += (1.0 - b1) * g
            vv *= b2
            vv += (1.0 - b2) * g * g
            mh = mm / (1.0 - b1 ** t)
            vh = vv / (1.0 - b2 ** t)
            p -= lr * mh / (np.sqrt(vh) + eps)
