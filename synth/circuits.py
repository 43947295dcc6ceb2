"""Seeded generators for circuits, initial states and arithmetic parameters.

Conventions shared by every consumer of these inputs:

* Amplitude ``i`` of an n-qubit state is basis state ``i``; qubit ``q`` is bit
  ``q`` of ``i`` (qubit 0 is the least significant bit). The paper's Kronecker
  example in Sec. II writes qubit 0 as the most significant factor; relabelling
  ``q -> n-1-q`` maps one convention onto the other.
* A gate acting on ``k`` targets carries a ``2^k x 2^k`` complex matrix ``M``
  whose local index ``j`` has bit ``m`` equal to the bit of ``targets[m]``;
  the gate maps ``out_j = sum_l M[j, l] in_l`` on every group of ``2^k``
  amplitudes that agree outside the targets. ``ctrl_mask``/``ctrl_vals``
  restrict the gate to indices with ``i & ctrl_mask == ctrl_vals``.
* Two-qubit gates from Table 1 (CNOT, CR) list the control as the more
  significant local bit, so such a gate is given as ``targets=(t, c)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import gcd, pi

import numpy as np

# Seeds of the five workloads: seed = SEED_BASE + workload index.
SEED_BASE = 160406460

# ---------------------------------------------------------------------------
# Gate constants used to *build* input circuits (Table 1).
# ---------------------------------------------------------------------------
_S2 = 1.0 / np.sqrt(2.0)
MAT_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
MAT_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
MAT_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
MAT_H = np.array([[_S2, _S2], [_S2, -_S2]], dtype=np.complex128)
MAT_S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
MAT_T = np.array([[1, 0], [0, np.exp(1j * pi / 4)]], dtype=np.complex128)
MAT_CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                    dtype=np.complex128)
MAT_SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                    dtype=np.complex128)
MAT_CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)


def mat_rz(theta: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)])


def mat_cr(theta: float) -> np.ndarray:
    return np.diag([1, 1, 1, np.exp(1j * theta)]).astype(np.complex128)


@dataclass
class Gate:
    targets: tuple
    matrix: np.ndarray
    ctrl_mask: int = 0
    ctrl_vals: int = 0
    name: str = ""

    @property
    def k(self) -> int:
        return len(self.targets)

    def qubits(self) -> set:
        qs = set(self.targets)
        m, q = self.ctrl_mask, 0
        while m:
            if m & 1:
                qs.add(q)
            m >>= 1
            q += 1
        return qs

    def dagger(self) -> "Gate":
        return Gate(self.targets, self.matrix.conj().T.copy(), self.ctrl_mask,
                    self.ctrl_vals, self.name + "^+")


def inverse_circuit(gates):
    return [g.dagger() for g in reversed(gates)]


# ---------------------------------------------------------------------------
# Named gates
# ---------------------------------------------------------------------------
def g1(mat, q, name=""):
    return Gate((int(q),), np.asarray(mat, dtype=np.complex128), name=name)


def cnot(c, t):
    return Gate((int(t), int(c)), MAT_CNOT.copy(), name="CNOT")


def cz(a, b):
    return Gate((int(a), int(b)), MAT_CZ.copy(), name="CZ")


def cr(c, t, theta):
    return Gate((int(t), int(c)), mat_cr(theta), name="CR")


def swap(a, b):
    return Gate((int(a), int(b)), MAT_SWAP.copy(), name="SWAP")


def mcx(controls, t):
    """X on ``t`` controlled on every qubit in ``controls`` being 1."""
    mask = 0
    for c in controls:
        mask |= 1 << int(c)
    return Gate((int(t),), MAT_X.copy(), mask, mask, name="C%dX" % len(controls))


# ---------------------------------------------------------------------------
# Random-layer family
# ---------------------------------------------------------------------------
def haar_2x2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 2x2 unitary: QR of a complex Ginibre matrix with the
    columns rephased by the phases of diag(R) (Mezzadri's recipe)."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) * _S2
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def random_layer_circuit(n: int, depth: int, seed: int):
    """Depth-``depth`` circuit; each layer is a Haar 2x2 on every qubit in
    order 0..n-1, then CZ on n//2 disjoint pairs (perm[2j], perm[2j+1])."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(depth):
        for q in range(n):
            gates.append(g1(haar_2x2(rng), q, "U"))
        perm = rng.permutation(n)
        for j in range(n // 2):
            gates.append(cz(perm[2 * j], perm[2 * j + 1]))
    return gates


# ---------------------------------------------------------------------------
# Structured circuits
# ---------------------------------------------------------------------------
def qft_circuit(m: int, q_lo: int = 0, inverse: bool = False, swaps: bool = True):
    """Gate-level QFT on qubits [q_lo, q_lo+m): for t = m-1 .. 0, H on t and
    then CR(2*pi/2^(t-c+1)) controlled by c = t-1 .. 0; finally SWAPs that
    reverse the register. The inverse is the adjoint sequence."""
    gates = []
    for t in range(m - 1, -1, -1):
        gates.append(g1(MAT_H, q_lo + t, "H"))
        for c in range(t - 1, -1, -1):
            gates.append(cr(q_lo + c, q_lo + t, 2.0 * pi / float(1 << (t - c + 1))))
    if swaps:
        for q in range(m // 2):
            gates.append(swap(q_lo + q, q_lo + m - 1 - q))
    return inverse_circuit(gates) if inverse else gates


def mat_rx(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def tfim_trotter_step(m: int, J: float = 1.0, hx: float = 0.7, dt: float = 0.1):
    """One first-order Trotter step of the 1D transverse-field Ising model on
    qubits 0..m-1 (open chain): Rx(2 hx dt) on every qubit, then for each
    neighbouring pair (q, q+1) the ZZ rotation exp(-i J dt Z Z) written as
    CNOT(q -> q+1), Rz(2 J dt) on q+1, CNOT(q -> q+1). That is m + 3(m-1) =
    4m - 3 gates, the gate count of the phase-estimation example of Table 2
    (the paper gives only the model and the count; this decomposition is
    ours)."""
    gates = [Gate((q,), mat_rx(2 * hx * dt), name="Rx") for q in range(m)]
    for q in range(m - 1):
        gates.append(Gate((q + 1, q), MAT_CNOT.copy(), name="CNOT"))
        gates.append(Gate((q + 1,), mat_rz(2 * J * dt), name="Rz"))
        gates.append(Gate((q + 1, q), MAT_CNOT.copy(), name="CNOT"))
    return gates


def ghz_circuit(n: int):
    """The entangling operation of Sec. IV-E: H on the first qubit, then a
    CNOT from it onto every other qubit."""
    return [g1(MAT_H, 0, "H")] + [cnot(0, j) for j in range(1, n)]


# ---------------------------------------------------------------------------
# States
# ---------------------------------------------------------------------------
def normal_state(n: int, seed: int) -> np.ndarray:
    """Re, Im i.i.d. N(0,1) from PCG64(seed), normalised in FP64."""
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi /= np.sqrt(np.vdot(psi, psi).real)
    return psi


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def modmul_input_state(w: int, c: int, seed: int, extra_low: int = 0) -> np.ndarray:
    """Control register (c qubits, above the work register) in uniform
    superposition, work register (w qubits) in a seeded normal state with
    distinct amplitudes; ``extra_low`` clean qubits below the work register.
    Index layout: [ctrl | work | extra]."""
    phi = normal_state(w, seed)
    amp = np.repeat(phi[None, :], 1 << c, axis=0) / np.sqrt(float(1 << c))
    flat = amp.reshape(-1)
    if extra_low:
        out = np.zeros(flat.size << extra_low, dtype=np.complex128)
        out[:: 1 << extra_low] = flat
        return out
    return flat


# ---------------------------------------------------------------------------
# Modular multiplication parameters and the reduced-width Toffoli network
# ---------------------------------------------------------------------------
def modmul_params(w: int, seed: int):
    """Odd modulus N in [2^(w-1)+1, 2^w-1] and a multiplier a in [2, N-1]
    coprime to N, both drawn from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    lo, hi = (1 << (w - 1)) + 1, (1 << w) - 1
    while True:
        N = int(rng.integers(lo, hi + 1))
        if N % 2 == 1:
            break
    while True:
        a = int(rng.integers(2, N))
        if gcd(a, N) == 1:
            break
    return a, N


@dataclass
class ModmulLayout:
    """Qubit layout of the gate-level controlled modular multiplier.

    x register (w qubits), accumulator (w+1 qubits), constant register
    (w+1 qubits), one carry ancilla, one flag ancilla and c control qubits.
    """
    w: int
    c: int
    x: list = field(default_factory=list)
    acc: list = field(default_factory=list)
    kreg: list = field(default_factory=list)
    carry: int = 0
    flag: int = 0
    ctrl: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return 3 * self.w + 4 + self.c

    @staticmethod
    def make(w: int, c: int) -> "ModmulLayout":
        L = ModmulLayout(w, c)
        q = 0
        L.x = list(range(q, q + w)); q += w
        L.acc = list(range(q, q + w + 1)); q += w + 1
        L.kreg = list(range(q, q + w + 1)); q += w + 1
        L.carry = q; q += 1
        L.flag = q; q += 1
        L.ctrl = list(range(q, q + c)); q += c
        assert q == L.n
        return L


def _maj(a, b, c):
    # Cuccaro MAJ block on (carry-in a, b, c): CNOT(c->b), CNOT(c->a), Toffoli(a,b->c)
    return [cnot(c, b), cnot(c, a), mcx((a, b), c)]


def _uma(a, b, c):
    # Cuccaro UMA block: Toffoli(a,b->c), CNOT(c->a), CNOT(a->b)
    return [mcx((a, b), c), cnot(c, a), cnot(a, b)]


def cuccaro_add(areg, breg, carry):
    """b <- a + b (mod 2^len) with one clean carry ancilla, ripple-carry
    adder built from MAJ/UMA blocks (the adder used by Sec. III-A)."""
    nb = len(areg)
    assert len(breg) == nb
    gates = []
    cin = carry
    for i in range(nb):
        gates += _maj(cin, breg[i], areg[i])
        cin = areg[i]
    for i in range(nb - 1, -1, -1):
        prev = carry if i == 0 else areg[i - 1]
        gates += _uma(prev, breg[i], areg[i])
    return gates


def _load_const(kreg, value, controls):
    gates = []
    for i, q in enumerate(kreg):
        if (value >> i) & 1:
            gates.append(mcx(controls, q) if controls else g1(MAT_X, q, "X"))
    return gates


def _add_const(L, value, controls, subtract=False):
    """acc <- acc +/- value (mod 2^(w+1)), the constant is loaded into the
    constant register under ``controls`` and unloaded afterwards."""
    load = _load_const(L.kreg, value, controls)
    add = cuccaro_add(L.kreg, L.acc, L.carry)
    if subtract:
        add = inverse_circuit(add)
    return load + add + load


def _modadd_const(L, K, N, controls):
    """acc <- (acc + K) mod N for acc < N, applied when all ``controls`` are 1.
    Add K, subtract N, copy the sign bit to the flag, add N back under the
    flag, subtract K, clear the flag from the sign bit, add K."""
    sign = L.acc[-1]
    g = []
    g += _add_const(L, K, controls)
    g += _add_const(L, N, [], subtract=True)
    g.append(cnot(sign, L.flag))
    g += _add_const(L, N, [L.flag])
    g += _add_const(L, K, controls, subtract=True)
    g.append(g1(MAT_X, sign, "X"))
    g.append(cnot(sign, L.flag))
    g.append(g1(MAT_X, sign, "X"))
    g += _add_const(L, K, controls)
    return g


def _mul_into_acc(L, a, N, ctrl):
    """acc <- acc + a*x mod N under control ``ctrl`` (shift-and-add)."""
    g = []
    for i in range(L.w):
        g += _modadd_const(L, (a * (1 << i)) % N, N, [ctrl, L.x[i]])
    return g


def modmul_gate_circuit(w: int, c: int, a: int, N: int):
    """Gate-level |ctrl>|x> -> |ctrl>|a^ctrl * x mod N> for x < N, built only
    from X, CNOT and Toffoli gates: for each control bit j, multiply-add
    a^(2^j) into the clean accumulator, controlled-swap x and acc, then run
    the inverse of the multiply-add by a^(-2^j). Ancillas return to 0."""
    L = ModmulLayout.make(w, c)
    gates = []
    for j in range(c):
        aj = pow(a, 1 << j, N)
        aj_inv = pow(aj, -1, N)
        cj = L.ctrl[j]
        gates += _mul_into_acc(L, aj, N, cj)
        for i in range(w):
            gates += [cnot(L.acc[i], L.x[i]), mcx((cj, L.x[i]), L.acc[i]),
                      cnot(L.acc[i], L.x[i])]
        gates += inverse_circuit(_mul_into_acc(L, aj_inv, N, cj))
    return gates, L


_MODMUL_CACHE = {}


def modmul_gate_circuit_on(x, acc, kreg, carry, flag, ctrl, a, N):
    """The same Toffoli network as modmul_gate_circuit on explicit qubit
    lists (x: w qubits, acc/kreg: w+1 qubits, ctrl: c qubits). Identical
    requests return the same (shared, read-only) gate list."""
    key = (tuple(x), tuple(acc), tuple(kreg), int(carry), int(flag), tuple(ctrl), int(a), int(N))
    hit = _MODMUL_CACHE.get(key)
    if hit is None:
        hit = _modmul_gates_on(x, acc, kreg, carry, flag, ctrl, a, N)
        _MODMUL_CACHE[key] = hit
    return hit


def _modmul_gates_on(x, acc, kreg, carry, flag, ctrl, a, N):
    w, c = len(x), len(ctrl)
    L = ModmulLayout(w, c, list(x), list(acc), list(kreg), int(carry), int(flag), list(ctrl))
    gates = []
    for j in range(c):
        aj = pow(a, 1 << j, N)
        aj_inv = pow(aj, -1, N)
        cj = L.ctrl[j]
        gates += _mul_into_acc(L, aj, N, cj)
        for i in range(w):
            gates += [cnot(L.acc[i], L.x[i]), mcx((cj, L.x[i]), L.acc[i]),
                      cnot(L.acc[i], L.x[i])]
        gates += inverse_circuit(_mul_into_acc(L, aj_inv, N, cj))
    return gates


def cuccaro_add_carry_out(areg, breg, carry, top):
    """b <- a + b over len+1 bits: the ripple-carry adder of cuccaro_add
    with its final carry XORed into ``top`` (the sum's bit len)."""
    nb = len(areg)
    assert len(breg) == nb
    gates = []
    cin = carry
    for i in range(nb):
        gates += _maj(cin, breg[i], areg[i])
        cin = areg[i]
    gates.append(cnot(areg[nb - 1], top))
    for i in range(nb - 1, -1, -1):
        prev = carry if i == 0 else areg[i - 1]
        gates += _uma(prev, breg[i], areg[i])
    return gates


def controlled(gates, ctrl):
    """Every gate of the list with one more control qubit."""
    bit = 1 << int(ctrl)
    return [Gate(g.targets, g.matrix, g.ctrl_mask | bit, g.ctrl_vals | bit, name="c" + g.name)
            for g in gates]


def mul_gate_circuit_on(aq, bq, cq, anc):
    """Gate-level c <- c + a*b mod 2^m (Sec. III-A: repeated addition and
    shift): for each bit i of b, the low m-i bits of a are added into bits
    i..m-1 of c by a Cuccaro adder controlled on b_i. One clean ancilla."""
    m = len(aq)
    gates = []
    for i in range(m):
        gates += controlled(cuccaro_add(list(aq[:m - i]), list(cq[i:]), anc), bq[i])
    return gates


def div_gate_circuit_on(aq, bq, cq, anc):
    """Gate-level restoring division (Sec. III-A: repeated subtraction and
    shift), (a, b, 0) -> (a mod b, b, a div b). Y = a + 2^m c is one 2m-qubit
    register; for i = m-1 down to 0 the (m+1)-qubit window of Y at bit i
    has b subtracted (the Cuccaro adder run backwards, carry into the
    window's top qubit), gets b added back to its low m qubits when its top
    qubit shows a borrow, and its top qubit is flipped into the quotient
    bit. One clean ancilla."""
    m = len(aq)
    Y = list(aq) + list(cq)
    gates = []
    for i in range(m - 1, -1, -1):
        low, top = Y[i:i + m], Y[i + m]
        gates += inverse_circuit(cuccaro_add_carry_out(list(bq), low, anc, top))
        gates += controlled(cuccaro_add(list(bq), low, anc), top)
        gates.append(g1(MAT_X, top, "X"))
    return gates


def arith_layout(m):
    """Registers of the multiplication/division workload as the index is
    written in Sec. III-A, a first and most significant: c on qubits 0..m-1,
    b on m..2m-1, a on 2m..3m-1. The gate-level networks add one ancilla,
    qubit 3m. Returns (a qubits, b qubits, c qubits, ancilla)."""
    return list(range(2 * m, 3 * m)), list(range(m, 2 * m)), list(range(m)), 3 * m


def arith_input_state(m, seed, extra=0):
    """a and b in a seeded normal superposition, c = 0, in the layout of
    arith_layout, on 3m + extra qubits (extra ancillas clean)."""
    ab = normal_state(2 * m, seed).reshape(1 << m, 1 << m)       # [a][b]
    psi = np.zeros((1 << extra, 1 << m, 1 << m, 1 << m), dtype=np.complex128)   # [anc][a][b][c]
    psi[0, :, :, 0] = ab
    return psi.reshape(-1)


def random_layer_on(qubits, rng):
    """One random layer restricted to `qubits`: a Haar 2x2 on each (in the
    listed order), then CZ on disjoint pairs of a random permutation."""
    nq = len(qubits)
    z = (rng.standard_normal((nq, 2, 2)) + 1j * rng.standard_normal((nq, 2, 2))) * _S2
    qm, rm = np.linalg.qr(z)
    d = np.diagonal(rm, axis1=1, axis2=2)
    us = qm * (d / np.abs(d))[:, None, :]
    gates = [Gate((int(q),), us[i], name="U") for i, q in enumerate(qubits)]
    perm = rng.permutation(nq)
    for j in range(len(qubits) // 2):
        gates.append(cz(qubits[perm[2 * j]], qubits[perm[2 * j + 1]]))
    return gates


# Segment kinds of the batched workload
SEG_LAYER, SEG_QFT, SEG_MODMUL = 0, 1, 2


@dataclass
class Segment:
    kind: int
    gates: list                 # gate-level form (always present)
    q_lo: int = 0               # QFT field
    m: int = 0
    inverse: bool = False
    modmul: tuple = ()          # (work_lo, w, ctrl_lo, c, a, N)


@dataclass
class BatchCircuit:
    n: int
    segments: list


def batch_mix(count: int, seed: int, n_range=(10, 22), d_range=(10, 60),
              p_qft=0.1, p_modmul=0.1):
    """Uneven batch of independent circuits: n ~ U{n_range}, depth ~
    U{d_range} slots; each slot is a random layer (on the data qubits), a
    QFT on a random contiguous range of m >= 3 data qubits, or a controlled
    modular multiplication.

    A circuit with n >= 16 that draws any modmul slot reserves its top
    qubits for arithmetic: a w-qubit work register x (w = 3 from n >= 20,
    else 2), a 2-qubit control register and 2w+4 clean ancillas, so that a
    gate-level Toffoli form exists. A preparation segment sets x = 1 and puts
    the control register in uniform superposition; only modmul slots touch
    these qubits afterwards, so x < N always holds and the gate-level and
    emulated forms agree exactly (the modular exponentiation structure of
    Shor's algorithm, Sec. III). Smaller circuits turn modmul slots into
    random layers."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        depth = int(rng.integers(d_range[0], d_range[1] + 1))
        kinds = rng.choice(3, size=depth, p=[1 - p_qft - p_modmul, p_qft, p_modmul])
        use_mm = n >= 16 and bool((kinds == SEG_MODMUL).any())
        w, c = (3 if n >= 20 else 2), 2
        n_data = n - (3 * w + c + 4) if use_mm else n
        data = list(range(n_data))
        xq = list(range(n_data, n_data + w))
        cq = list(range(n_data + w, n_data + w + c))
        anc = list(range(n_data + w + c, n))
        segs = []
        if use_mm:
            prep = [g1(MAT_X, xq[0], "X")] + [g1(MAT_H, q, "H") for q in cq]
            segs.append(Segment(SEG_LAYER, prep))
        for kd in kinds:
            if kd == SEG_MODMUL and not use_mm:
                kd = SEG_LAYER
            if kd == SEG_LAYER:
                segs.append(Segment(SEG_LAYER, random_layer_on(data, rng)))
            elif kd == SEG_QFT:
                m = int(rng.integers(3, n_data + 1))
                q_lo = int(rng.integers(0, n_data - m + 1))
                inv = bool(rng.integers(0, 2))
                segs.append(Segment(SEG_QFT, qft_circuit(m, q_lo, inverse=inv), q_lo, m, inv))
            else:
                a, N = modmul_params(w, int(rng.integers(0, 2 ** 31)))
                acc, kreg = anc[0:w + 1], anc[w + 1:2 * w + 2]
                carry, flag = anc[2 * w + 2], anc[2 * w + 3]
                g = modmul_gate_circuit_on(xq, acc, kreg, carry, flag, cq, a, N)
                segs.append(Segment(SEG_MODMUL, g, modmul=(xq[0], w, cq[0], c, a, N)))
        out.append(BatchCircuit(n, segs))
    return out


# ---------------------------------------------------------------------------
# Flat packing of gate lists for C interfaces
# ---------------------------------------------------------------------------
def pack(gates):
    """Flatten a gate list into (k[], targets_concat[], matrices_concat[],
    ctrl_mask[], ctrl_vals[]); matrices row-major, (re, im) interleaved."""
    ks = np.array([g.k for g in gates], dtype=np.int32)
    tg = np.array([t for g in gates for t in g.targets], dtype=np.int32)
    mats = np.concatenate([np.ascontiguousarray(g.matrix, dtype=np.complex128)
                           .reshape(-1).view(np.float64) for g in gates]) \
        if gates else np.zeros(0)
    cm = np.array([g.ctrl_mask for g in gates], dtype=np.uint64)
    cv = np.array([g.ctrl_vals for g in gates], dtype=np.uint64)
    return ks, tg, np.ascontiguousarray(mats, dtype=np.float64), cm, cv
