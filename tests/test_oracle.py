"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every oracle routine is checked here against something other than itself:
values printed in the paper (tests/golden/, each file cites its table or
section), closed forms, invariants, an independent library (numpy.fft) or a
brute-force construction of the full operator. These run without a GPU.
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(path):
    out, cur, rows = {}, None, []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        if len(parts) == 2 and parts[1].isdigit():
            cur, rows = parts[0], []
            out[cur] = (int(parts[1]), rows)
            continue
        rows.append([complex(*map(float, e.split(","))) for e in parts])
    return {k: np.array(r) for k, (d, r) in out.items()}


# ---------------------------------------------------------------------------
# Table 1 and the Kronecker example of Sec. II
# ---------------------------------------------------------------------------
def test_table1_constants(O):
    gold = _read_blocks(os.path.join(GOLD, "table1_gates.txt"))
    for name, ref in gold.items():
        got = O.table1(name, 0.7)
        assert np.abs(got - ref).max() < 1e-15, name


def test_kron_example_relabelled(O):
    """X on the paper's qubit 0 of n=2 is X on our qubit 1 (q -> n-1-q)."""
    ref = np.loadtxt(os.path.join(GOLD, "kron_example.txt"))
    U = np.zeros((4, 4), dtype=complex)
    for col in range(4):
        e = np.zeros(4, dtype=complex)
        e[col] = 1
        U[:, col] = O.apply_gate(e, [1], O.table1("X"))
    assert np.array_equal(U.real, ref) and not U.imag.any()


def test_full_matrix_is_textbook_kron(O):
    """The brute-force builder reduces to m_{n-1} (x) ... (x) m_0 for
    one-qubit gates (Sec. II's construction with LSB = qubit 0)."""
    rng = np.random.default_rng(1)
    n = 4
    for q in range(n):
        g = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        K = np.array([[1.0]])
        for j in range(n - 1, -1, -1):
            K = np.kron(K, g if j == q else np.eye(2))
        assert np.abs(O.full_matrix(n, [q], g) - K).max() < 1e-15


# ---------------------------------------------------------------------------
# Gate application (Sec. II) against the brute-force operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_apply_gate_vs_bruteforce(O, k):
    rng = np.random.default_rng(10 + k)
    n = 7
    for trial in range(6):
        qs = rng.permutation(n)
        targets = [int(q) for q in qs[:k]]
        nctrl = int(rng.integers(0, 3)) if k < 4 else int(rng.integers(0, 2))
        ctrls = [int(q) for q in qs[k:k + nctrl]]
        cm = sum(1 << q for q in ctrls)
        cv = sum((int(rng.integers(0, 2)) << q) for q in ctrls)
        M = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        got = O.apply_gate(psi.copy(), targets, M, cm, cv)
        ref = O.full_matrix(n, targets, M, cm, cv) @ psi
        assert np.abs(got - ref).max() < 1e-12


def test_apply_gate_rejects_bad_args(O):
    psi = np.zeros(8, dtype=complex)
    with pytest.raises(O.OracleError):
        O.apply_gate(psi, [0, 0], np.eye(4))
    with pytest.raises(O.OracleError):
        O.apply_gate(psi, [3], np.eye(2))
    with pytest.raises(O.OracleError):
        O.apply_gate(psi, [0], np.eye(2), ctrl_mask=1, ctrl_vals=1)


def test_norm_and_inverse_roundtrip(O, S):
    n = 10
    gates = S.random_layer_circuit(n, 6, seed=5)
    psi0 = S.normal_state(n, 6)
    psi = O.apply_circuit(psi0, gates)
    assert abs(O.norm2(psi) - 1.0) < 1e-14
    back = O.apply_circuit(psi, S.inverse_circuit(gates))
    assert np.abs(back - psi0).max() < 1e-13


def test_bell_and_ghz_closed_form(O, S):
    bell = O.apply_circuit(S.zero_state(2), [S.g1(S.MAT_H, 0), S.cnot(0, 1)])
    ref = np.zeros(4, dtype=complex)
    ref[0] = ref[3] = 1 / math.sqrt(2)
    assert np.abs(bell - ref).max() < 1e-15
    for n in (3, 6, 9):
        ghz = O.apply_circuit(S.zero_state(n), S.ghz_circuit(n))
        ref = np.zeros(1 << n, dtype=complex)
        ref[0] = ref[-1] = 1 / math.sqrt(2)
        assert np.abs(ghz - ref).max() < 1e-15


def test_random_circuit_porter_thomas(O, S):
    """Deep random circuits approach Porter-Thomas statistics:
    N * sum |a|^4 -> 2 (weak statistical sanity)."""
    n = 12
    psi = O.apply_circuit(S.zero_state(n), S.random_layer_circuit(n, 20, seed=S.SEED_BASE))
    ipr = (1 << n) * np.sum(np.abs(psi) ** 4)
    assert 1.8 < ipr < 2.2


# ---------------------------------------------------------------------------
# QFT (Sec. III-B)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,q_lo,m", [(1, 0, 1), (4, 0, 4), (7, 0, 7), (8, 2, 4), (9, 5, 4), (6, 0, 3)])
def test_qft_direct_vs_numpy(O, S, n, q_lo, m):
    x = S.normal_state(n, 100 + n)
    for inv in (False, True):
        got = O.qft_direct(x, q_lo, m, inv)
        assert np.abs(got - O.dft_numpy(x, q_lo, m, inv)).max() < 1e-13


def test_qft_basis_states_closed_form(O):
    n = 6
    N = 1 << n
    for j in (0, 1, 5, 37, 63):
        e = np.zeros(N, dtype=complex)
        e[j] = 1
        ref = np.exp(2j * np.pi * j * np.arange(N) / N) / math.sqrt(N)
        assert np.abs(O.qft_direct(e) - ref).max() < 1e-14


@pytest.mark.parametrize("n,q_lo,m", [(5, 0, 5), (8, 0, 8), (8, 3, 4), (10, 1, 6)])
def test_qft_gate_level_equals_transform(O, S, n, q_lo, m):
    x = S.normal_state(n, 7 + n)
    for inv in (False, True):
        g = O.qft_gates(x, q_lo, m, inv)
        assert np.abs(g - O.qft_direct(x, q_lo, m, inv)).max() < 1e-12


def test_qft_gate_list_and_roundtrip(O, S):
    n = 7
    x = S.normal_state(n, 77)
    y = O.apply_circuit(x, S.qft_circuit(n))
    assert np.abs(y - O.dft_numpy(x)).max() < 1e-12
    # without SWAPs the output sits at bit-reversed indices
    z = O.apply_circuit(x, S.qft_circuit(n, swaps=False))
    rev = [int(format(i, "0%db" % n)[::-1], 2) for i in range(1 << n)]
    assert np.abs(z[rev] - y).max() < 1e-12
    back = O.qft_direct(y, inverse=True)
    assert np.abs(back - x).max() < 1e-13


def test_qft_sample_matches_full(O, S):
    n = 9
    x = S.normal_state(n, 9)
    full = O.qft_direct(x, 1, 7)
    for i in (0, 3, 77, 300, 511):
        assert abs(O.qft_sample(x, i, 1, 7) - full[i]) < 1e-14


# ---------------------------------------------------------------------------
# Arithmetic permutations (Sec. III-A)
# ---------------------------------------------------------------------------
def _modmul_python(psi, n, work_lo, w, ctrl_lo, c, a, N):
    out = np.zeros_like(psi)
    for i in range(1 << n):
        cc = (i >> ctrl_lo) & ((1 << c) - 1)
        x = (i >> work_lo) & ((1 << w) - 1)
        xp = (pow(a, cc, N) * x) % N if x < N else x
        j = (i & ~(((1 << w) - 1) << work_lo)) | (xp << work_lo)
        out[j] = psi[i]
    return out


@pytest.mark.parametrize("w,c,work_lo,ctrl_lo,n", [(5, 3, 0, 5, 8), (4, 2, 2, 7, 10), (6, 2, 3, 0, 9)])
def test_modmul_vs_python_pow(O, S, w, c, work_lo, ctrl_lo, n):
    a, N = S.modmul_params(w, seed=w * 31 + c)
    psi = S.normal_state(n, 123)
    got = O.modmul(psi, work_lo, w, ctrl_lo, c, a, N)
    ref = _modmul_python(psi, n, work_lo, w, ctrl_lo, c, a, N)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_modmul_invariants(O, S):
    w, c = 7, 3
    a, N = S.modmul_params(w, seed=3)
    n = w + c
    psi = S.normal_state(n, 4)
    out = O.modmul(psi, 0, w, w, c, a, N)
    # control value 0 multiplies by a^0 = 1: identity on that block
    assert np.array_equal(out[: 1 << w], psi[: 1 << w])
    # x >= N stays in place for every control value
    for cc in range(1 << c):
        blk = slice(cc << w, (cc + 1) << w)
        assert np.array_equal(out[blk][N:], psi[blk][N:])
    # bijection: the multiset of amplitudes is unchanged
    assert np.array_equal(np.sort(out.view(np.float64)), np.sort(psi.view(np.float64)))


def test_modmul_rejects_even_overlap(O):
    psi = np.zeros(1 << 6, dtype=complex)
    with pytest.raises(O.OracleError):
        O.modmul(psi, 0, 4, 2, 2, 3, 11)  # overlapping fields


@pytest.mark.parametrize("w,c,seed", [(3, 2, 1), (4, 1, 7)])
def test_gate_level_modmul_bit_exact(O, S, w, c, seed):
    """The Toffoli/CNOT/X network (Cuccaro adders, Sec. III-A) and the
    permutation agree bit for bit on x < N; ancillas return to 0."""
    a, N = S.modmul_params(w, seed)
    gates, L = S.modmul_gate_circuit(w, c, a, N)
    for g in gates:  # only X, CNOT and Toffoli (X with up to two controls)
        assert g.name.replace("^+", "") in {"X", "CNOT", "C1X", "C2X"}
        assert set(np.unique(g.matrix)) <= {0, 1}
    rng = np.random.default_rng(seed)
    psi = np.zeros(1 << L.n, dtype=complex)
    for cc in range(1 << c):
        for x in range(N):
            psi[x | (cc << L.ctrl[0])] = rng.standard_normal() + 1j * rng.standard_normal()
    got = O.apply_circuit(psi, gates)
    ref = O.modmul(psi, 0, w, L.ctrl[0], c, a, N)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_table_perm_bit_reversal_equals_swap_network(O, S):
    """A field permutation given as a table (Sec. III-A: any classical
    bijection on basis states) must equal the same map built from gates. The
    bit reversal of an m-bit field is the SWAP network (q, m-1-q) run by the
    gate simulator; both are moves, so they agree bit for bit."""
    for (n, lo, nb, seed) in [(7, 2, 3, 1), (8, 0, 8, 2), (9, 3, 5, 3), (6, 1, 4, 4)]:
        dest = np.array([int(format(f, "0%db" % nb)[::-1], 2) for f in range(1 << nb)],
                        dtype=np.uint64)
        psi = S.normal_state(n, seed)
        got = O.table_perm(psi, lo, nb, dest)
        gates = [S.swap(lo + q, lo + nb - 1 - q) for q in range(nb // 2)]
        ref = O.apply_circuit(psi, gates)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_table_perm_increment_equals_cnot_ladder(O, S):
    """x -> x + 1 mod 2^m on a field, as a table, against the textbook
    multi-controlled-X incrementer (flip bit j when all lower bits are 1,
    highest bit first)."""
    for (n, lo, nb, seed) in [(7, 2, 4, 5), (6, 0, 6, 6)]:
        dest = np.array([(f + 1) % (1 << nb) for f in range(1 << nb)], dtype=np.uint64)
        psi = S.normal_state(n, seed)
        got = O.table_perm(psi, lo, nb, dest)
        gates = [S.mcx([lo + q for q in range(j)], lo + j) for j in range(nb - 1, -1, -1)]
        ref = O.apply_circuit(psi, gates)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_table_perm_modmul_table_equals_modmul(O, S):
    """The controlled modular multiplication written as a table over the
    joint (work, control) field, with a^c mod N from Python's pow, must place
    every amplitude where the modmul oracle does (itself pinned against the
    Cuccaro network), bit for bit."""
    for (w, c, lo, n, seed) in [(5, 2, 1, 9, 7), (4, 3, 0, 8, 8), (6, 0, 2, 9, 9)]:
        a, N = S.modmul_params(w, seed)
        nb = w + c
        dest = np.zeros(1 << nb, dtype=np.uint64)
        for f in range(1 << nb):
            cc, x = f >> w, f & ((1 << w) - 1)
            xp = (pow(a, cc, N) * x) % N if x < N else x
            dest[f] = (cc << w) | xp
        psi = S.normal_state(n, seed)
        got = O.table_perm(psi, lo, nb, dest)
        ref = O.modmul(psi, lo, w, lo + w, c, a, N)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


# ---------------------------------------------------------------------------
# Measurement (Sec. III-D)
# ---------------------------------------------------------------------------
_PAULI = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]),
          "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.diag([1, -1])}


def _pauli_full(n, xm, ym, zm):
    K = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        p = "X" if (xm >> q) & 1 else "Y" if (ym >> q) & 1 else "Z" if (zm >> q) & 1 else "I"
        K = np.kron(K, _PAULI[p])
    return K


def test_expectation_vs_kron_paulis(O, S):
    n = 5
    rng = np.random.default_rng(2)
    psi = S.normal_state(n, 2)
    for _ in range(12):
        lab = rng.integers(0, 4, n)
        xm = sum(1 << q for q in range(n) if lab[q] == 1)
        ym = sum(1 << q for q in range(n) if lab[q] == 2)
        zm = sum(1 << q for q in range(n) if lab[q] == 3)
        ref = np.vdot(psi, _pauli_full(n, xm, ym, zm) @ psi)
        got = O.expectation(psi, xm, ym, zm)
        assert abs(got - ref) < 1e-14 and abs(got.imag) < 1e-14


def test_expectation_closed_forms(O, S):
    n = 6
    assert O.expectation(S.zero_state(n), z_mask=1) == 1.0
    ghz = O.apply_circuit(S.zero_state(n), S.ghz_circuit(n))
    assert abs(O.expectation(ghz, z_mask=1)) < 1e-15
    assert abs(O.expectation(ghz, z_mask=3) - 1) < 1e-15
    assert abs(O.expectation(ghz, x_mask=(1 << n) - 1) - 1) < 1e-14
    rng = np.random.default_rng(9)
    U = S.haar_2x2(rng)
    psi = O.apply_circuit(S.zero_state(1), [S.g1(U, 0)])
    assert abs(O.expectation(psi, z_mask=1) - (abs(U[0, 0]) ** 2 - abs(U[1, 0]) ** 2)) < 1e-15


def test_marginals_and_sampling(O, S):
    n = 7
    ghz = O.apply_circuit(S.zero_state(n), S.ghz_circuit(n))
    p = O.marginals(ghz, [0])
    assert np.abs(p - 0.5).max() < 1e-15
    psi = S.normal_state(n, 5)
    qs = [5, 1, 3]
    p = O.marginals(psi, qs)
    ref = np.zeros(8)
    prob = np.abs(psi) ** 2
    for i in range(1 << n):
        ref[((i >> 5) & 1) | (((i >> 1) & 1) << 1) | (((i >> 3) & 1) << 2)] += prob[i]
    assert np.abs(p - ref).max() < 1e-15
    u = np.array([0.0, 0.3, 0.999999])
    o1, o2 = O.sample(p, u), O.sample(p, u)
    assert np.array_equal(o1, o2)
    cdf = np.cumsum(p) / p.sum()
    for uu, o in zip(u, o1):
        assert cdf[o] > uu and (o == 0 or cdf[o - 1] <= uu)


def test_sampling_chi_square(O, S):
    n = 4
    psi = S.normal_state(n, 11)
    p = O.marginals(psi, list(range(n)))
    u = np.random.default_rng(12).random(100000)
    cnt = np.bincount(O.sample(p, u).astype(np.int64), minlength=16)
    exp = p * u.size
    chi2 = np.sum((cnt - exp) ** 2 / exp)
    assert chi2 < 45.0  # 15 dof, p ~ 1e-4


def test_collapse(O, S):
    n = 6
    psi = S.normal_state(n, 8)
    qs = [2, 4]
    p = O.marginals(psi, qs)
    out = O.collapse(psi, qs, 2, p[2])
    assert abs(O.norm2(out) - 1) < 1e-14
    for i in range(1 << n):
        o = ((i >> 2) & 1) | (((i >> 4) & 1) << 1)
        assert (out[i] == 0) if o != 2 else abs(out[i] - psi[i] / math.sqrt(p[2])) < 1e-15


# ---------------------------------------------------------------------------
# Cost models of Sec. III-B and Table 2
# ---------------------------------------------------------------------------
def _table2():
    rows = np.loadtxt(os.path.join(GOLD, "table2_qpe.txt"))
    return rows


def test_table2_gate_count_is_4n_minus_3():
    t = _table2()
    assert np.array_equal(t[:, 1], 4 * t[:, 0] - 3)


def test_table2_crossover_rows_reproduced(O):
    for n, G, ta, tb, tg, te, xs, xe in _table2():
        assert O.qpe_crossover(ta, tb, tg, True) == int(xs), n
        assert O.qpe_crossover(ta, tb, te, False) == int(xe), n


def test_eq1_eq2_single_node_ratio(O):
    """With B_net terms absent (P = 1), Eq. (2) / Eq. (1) = 4 n F / (5 B);
    the Sec. IV-C numbers (n = 28, F = 20 GFLOP/s, B = 40 GB/s) give 11.2."""
    n, F, B = 28, 20e9, 40e9
    r = O.t_qft(n, B, 1.0) / O.t_fft(n, 1.0, F, 1.0)
    assert abs(r - 4 * n * F / (5 * B)) < 1e-12 and abs(r - 11.2) < 1e-12
    # the communication terms scale as stated: 3 exchanges vs log2(P)
    n, P = 30, 8
    d_fft = O.t_fft(n, 1.0, F, 1e9, P) - O.t_fft(n, 1.0, F, 1e9, 1)
    d_qft = O.t_qft(n, B, 1e9, P) - O.t_qft(n, B, 1e9, 1)
    assert abs(d_qft / d_fft - math.log2(P) / 3) < 1e-12


# ---------------------------------------------------------------------------
# MLP cost model (FP64 reference for the GPU kernels)
# ---------------------------------------------------------------------------
def test_mlp_param_count_and_fd_gradients(O):
    ps = O.MLP.init(3)
    assert sum(p.size for p in ps) == 6020
    # make biases nonzero so every gradient path is exercised
    rng = np.random.default_rng(4)
    ps = [p + 0.1 * rng.standard_normal(p.shape) for p in ps]
    net = O.MLP(ps)
    X = rng.standard_normal((37, 24))
    T = rng.standard_normal((37, 4))
    mask = (rng.random((37, 4)) < 0.8).astype(float)
    g = net.grads(X, T, mask)
    entries = [(pi, int(fi)) for pi in range(6) for fi in rng.integers(0, ps[pi].size, 6)]
    fd = net.fd_grads(X, T, mask, 1e-6, entries)
    an = np.array([g[pi].flat[fi] for pi, fi in entries])
    assert np.abs(fd - an).max() < 1e-6 * max(1.0, np.abs(an).max())


def test_adam_first_step_is_signed_lr():
    """Adam's first bias-corrected step moves every parameter by lr*sign(g)
    (up to eps)."""
    from oracle.oracle import MLP
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    MLP.adam(p, g, m, v, 1, lr=0.01)
    assert np.abs(p[0] - (np.array([1.0, -2.0, 3.0]) - 0.01 * np.sign(g[0]))).max() < 1e-7


def test_adam_constant_gradient_closed_form():
    """With the same gradient g at every step, bias correction makes the
    corrected moments exactly g and g^2 at every t, so step t moves each
    parameter by lr*g/(|g|+eps): after t steps p = p0 - t*lr*g/(|g|+eps).
    A wrong bias-correction exponent fails from t = 2 on."""
    from oracle.oracle import MLP
    p0 = np.array([0.3, -1.0, 2.0, 0.0])
    g = np.array([0.25, -3.0, 1e-4, 7.0])
    p, m, v = [p0.copy()], [np.zeros(4)], [np.zeros(4)]
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        MLP.adam(p, [g], m, v, t, lr=lr, eps=eps)
        assert np.abs(p[0] - (p0 - t * lr * g / (np.abs(g) + eps))).max() < 1e-13
        assert np.abs(m[0] - (1 - 0.9 ** t) * g).max() < 1e-14
        assert np.abs(v[0] - (1 - 0.999 ** t) * g * g).max() < 1e-12


def test_adam_alternating_gradient_closed_form():
    """Gradients g_s = (-1)^s g: the first moment is a geometric series,
    m_t = (1-b1) g (-1)^t (1-(-b1)^t)/(1+b1), while v_t = (1-b2^t) g^2 as for a
    constant gradient. Step t then moves p by -lr*mh/(sqrt(vh)+eps) with
    mh = m_t/(1-b1^t), vh = g^2."""
    from oracle.oracle import MLP
    b1, b2, lr, eps = 0.9, 0.999, 0.02, 1e-8
    p0 = np.array([1.0, -0.5, 0.25])
    g = np.array([0.5, -2.0, 3.0])
    p, m, v = [p0.copy()], [np.zeros(3)], [np.zeros(3)]
    want = p0.copy()
    for t in range(1, 6):
        gt = ((-1) ** t) * g
        MLP.adam(p, [gt], m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        mt = (1 - b1) * g * ((-1) ** t) * (1 - (-b1) ** t) / (1 + b1)
        mh = mt / (1 - b1 ** t)
        want = want - lr * mh / (np.abs(g) + eps)
        assert np.abs(m[0] - mt).max() < 1e-14
        assert np.abs(p[0] - want).max() < 1e-12


# ---------------------------------------------------------------------------
# Per-index forms used for full-size spot checks
# ---------------------------------------------------------------------------
def test_modmul_source_matches_the_permutation(O, S):
    for (w, c, work_lo, ctrl_lo, n, seed) in [(5, 3, 0, 5, 9, 1), (4, 0, 2, 0, 7, 2), (3, 2, 4, 0, 8, 3)]:
        a, N = S.modmul_params(w, seed)
        psi = S.normal_state(n, seed)
        out = O.modmul(psi, work_lo, w, ctrl_lo, c, a, N)
        src = O.modmul_source(np.arange(1 << n), work_lo, w, ctrl_lo, c, a, N)
        assert np.array_equal(out, psi[src.astype(np.int64)])
        assert np.array_equal(np.sort(src), np.arange(1 << n, dtype=np.uint64))   # a bijection


def test_layer_amplitudes_match_gate_by_gate_simulation(O, S):
    rng = np.random.default_rng(12)
    n = 9
    gates = S.random_layer_on(list(range(n)), rng)
    ones = [g.matrix for g in gates if g.k == 1]
    pairs = [tuple(g.targets) for g in gates if g.k == 2]
    assert len(ones) == n and len(pairs) == n // 2
    assert [g.targets[0] for g in gates if g.k == 1] == list(range(n))
    psi = O.apply_circuit(S.zero_state(n), gates)
    idx = np.arange(1 << n)
    assert np.abs(O.layer_amplitudes(ones, pairs, idx) - psi).max() < 1e-13


# ---------------------------------------------------------------------------
# Phase estimation: the gate-level controlled powers (Sec. III-C)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("b,k", [(3, 5), (4, 11), (5, 1)])
def test_qpe_powers_phase_kickback_closed_form(O, S, b, k):
    """U = diag(1, exp(2 pi i k / 2^b)) on an eigen qubit |1>: H on the b
    control qubits, the controlled powers, then the inverse QFT leave the
    control register exactly in |k>."""
    phase = np.diag([1.0, np.exp(2j * np.pi * k / 2 ** b)])
    gates = [S.Gate((0,), phase)]
    n = 1 + b
    psi = S.zero_state(n)
    psi = O.apply_circuit(psi, [S.g1(S.MAT_X, 0)] + [S.g1(S.MAT_H, 1 + j) for j in range(b)])
    psi = O.qpe_powers(psi, gates, 1, b)
    psi = O.qft_direct(psi, 1, b, inverse=True)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[(k << 1) | 1] = 1.0
    assert np.abs(psi - want).max() < 1e-12


def test_qpe_powers_equal_dense_matrix_powers(O, S):
    rng = np.random.default_rng(21)
    m, b = 3, 3
    gates = [S.Gate((q,), S.haar_2x2(rng)) for q in range(m)] + [S.cnot(0, 2), S.cz(1, 2)]
    U = O.block_matrix(m, gates)
    n = m + b
    psi0 = S.normal_state(n, 4)
    ref = psi0.copy()
    for j in range(b):
        V = np.linalg.matrix_power(U, 2 ** j)
        ref = O.full_matrix(n, list(range(m)), V, 1 << (m + j), 1 << (m + j)) @ ref
    assert np.abs(O.qpe_powers(psi0, gates, m, b) - ref).max() < 1e-12


def test_tfim_step_has_4m_minus_3_gates_and_is_unitary(O, S):
    for m in (2, 5, 8):
        g = S.tfim_trotter_step(m)
        assert len(g) == 4 * m - 3
    U = O.block_matrix(5, S.tfim_trotter_step(5))
    assert np.abs(U.conj().T @ U - np.eye(32)).max() < 1e-12


def test_library_crossover_rule_matches_the_oracle_on_table2(O):
    from paper_1604_06460_amd import qs as Q
    for n, G, ta, tb, tg, te, xs, xe in _table2():
        assert Q.qpe_crossover_bits(ta, tb, tg, True) == O.qpe_crossover(ta, tb, tg, True) == int(xs)
        assert Q.qpe_crossover_bits(ta, tb, te, False) == O.qpe_crossover(ta, tb, te, False) == int(xe)


# ---------------------------------------------------------------------------
# Integer multiplication and division into a third register (Sec. III-A)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_arith_on_a_clean_c_register_is_product_and_divmod(O, m):
    """Every (a, b, 0): multiplication leaves a*b mod 2^m in c; division
    leaves a mod b in a and a div b in c (Python integer arithmetic), and
    a divisor of 0 gives (a, 0, 2^m - 1)."""
    M = 1 << m
    a, b = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    a, b = a.ravel().astype(np.uint64), b.ravel().astype(np.uint64)
    idx = a | (b << np.uint64(m))
    got = O.arith_dest(idx, O.ARITH_MUL, 0, m, 2 * m, m)
    want = [int(x) | (int(y) << m) | (((int(x) * int(y)) % M) << (2 * m)) for x, y in zip(a, b)]
    assert got.tolist() == want
    got = O.arith_dest(idx, O.ARITH_DIV, 0, m, 2 * m, m)
    want = []
    for x, y in zip(a.tolist(), b.tolist()):
        q, r = divmod(x, y) if y else (M - 1, x)
        want.append(r | (y << m) | (q << (2 * m)))
    assert got.tolist() == want


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("m,lo", [(3, (0, 3, 6)), (4, (8, 0, 4)), (3, (6, 0, 3))])
def test_arith_is_a_bijection_that_keeps_b(O, kind, m, lo):
    n = 3 * m
    idx = np.arange(1 << n, dtype=np.uint64)
    d = O.arith_dest(idx, kind, *lo, m)
    assert np.unique(d).size == idx.size
    bm = np.uint64(((1 << m) - 1) << lo[1])
    assert np.array_equal(d & bm, idx & bm)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", [0, 1])
def test_arith_equals_the_cuccaro_networks_on_every_input(O, S, m, kind):
    """The repeated-addition and repeated-subtraction Toffoli networks of
    Sec. III-A (synth: Cuccaro adders, one ancilla) run by the oracle's gate
    simulator on a random state over all 3m register qubits, c != 0 included,
    equal the permutation exactly."""
    aq, bq, cq, anc = S.arith_layout(m)
    psi = np.zeros(1 << (3 * m + 1), dtype=np.complex128)
    psi[:1 << (3 * m)] = S.normal_state(3 * m, 30 + m)
    for qa, qb, qc in ((aq, bq, cq), (cq, aq, bq)):
        net = (S.mul_gate_circuit_on if kind == 0 else S.div_gate_circuit_on)(qa, qb, qc, anc)
        assert all(len(g.targets) <= 2 for g in net)
        ref = O.apply_circuit(psi, net)
        assert np.array_equal(O.arith(psi, kind, qa[0], qb[0], qc[0], m), ref)


def test_arith_gate_counts(S):
    """Multiplication: sum over bits of b of a (m-i)-bit adder, 6 gates per
    bit: 3m(m+1). Division: per quotient bit a subtraction with carry-out
    (6m+1), a controlled addition (6m) and one X: m(12m+2)."""
    for m in (2, 5, 7):
        aq, bq, cq, anc = S.arith_layout(m)
        assert len(S.mul_gate_circuit_on(aq, bq, cq, anc)) == 3 * m * (m + 1)
        assert len(S.div_gate_circuit_on(aq, bq, cq, anc)) == m * (12 * m + 2)


@pytest.mark.parametrize("m,b,n", [(2, 3, 5), (3, 3, 7), (3, 2, 8)])
def test_qpe_eig_route_equals_gate_level_powers(O, S, m, b, n):
    """The eigensolver route (numpy.linalg.eig of the dense U) gives the
    same state as running the gate list 2^j times per control qubit, also
    with a spectator qubit above the control register."""
    rng = np.random.default_rng(40 + m)
    gates = [S.Gate((q,), S.haar_2x2(rng)) for q in range(m)] + [S.cnot(0, m - 1), S.cz(0, 1)]
    psi = S.normal_state(n, 6 + m)
    ref = O.qpe_powers(psi, gates, m, b)
    assert np.abs(O.qpe_eig_powers(psi, gates, m, m, b) - ref).max() < 1e-12


def test_qpe_eig_route_phase_kickback(O, S):
    """A diagonal U with eigenphase 2 pi k / 2^b on |1..1>: after the powers
    the control register of the eigenstate holds e^(2 pi i k c / 2^b)."""
    m, b, k = 2, 4, 5
    th = 2 * np.pi * k / 2 ** b
    gates = [S.Gate((1, 0), np.diag([1, 1, 1, np.exp(1j * th)]))]
    psi = np.zeros(1 << (m + b), dtype=np.complex128)
    psi[3 + 4 * np.arange(1 << b)] = 2 ** (-b / 2)
    out = O.qpe_eig_powers(psi, gates, m, m, b)
    c = np.arange(1 << b)
    assert np.abs(out[3 + 4 * c] - np.exp(1j * th * c) * 2 ** (-b / 2)).max() < 1e-13
