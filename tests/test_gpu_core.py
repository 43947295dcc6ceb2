"""GPU parity of the gate sweeps, fused programs, reductions, measurement and
permutation emulation against the CPU oracle, through the C ABI.

Tolerances: max abs error <= 1e-10 for complex128 states and <= 1e-5 for
complex64 states against the FP64 oracle on normalised states; index
permutations are compared bit for bit.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {1: 1e-10, 0: 1e-5}


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def _rand_unitary(rng, k):
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diagonal(r) / np.abs(np.diagonal(r)))[None, :]


def _state(Q, S, n, dtype, seed):
    st = Q.State(n, dtype)
    psi = S.normal_state(n, seed)
    st.set(psi)
    # the oracle starts from exactly what the GPU holds: the input rounded
    # to the state's precision on the host
    return st, psi.astype(st.np_dtype).astype(np.complex128)


def _err(a, b):
    return float(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128)).max())


# ---------------------------------------------------------------------------
# Single gates: every width, target class and dtype, with and without controls
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_dense_gate_vs_oracle(Q, O, S, dtype, k):
    rng = np.random.default_rng(100 + k + 10 * dtype)
    n = 13
    cases = [list(range(k)),                                # all low
             list(range(n - k, n)),                         # all high
             [int(q) for q in rng.permutation(n)[:k]],      # mixed, unsorted
             [int(q) for q in rng.permutation(n)[:k]]]
    for ci, targets in enumerate(cases):
        st, psi = _state(Q, S, n, dtype, 7 + ci)
        U = _rand_unitary(rng, k)
        cm = cv = 0
        if ci == 3 and k < 6:
            free = [q for q in range(n) if q not in targets]
            cm = (1 << free[0]) | (1 << free[-1])
            cv = 1 << free[-1]
        st.apply_gate(targets, U, cm, cv)
        ref = O.apply_gate(psi.copy(), targets, U, cm, cv)
        assert _err(st.get(), ref) < TOL[dtype], (targets, cm)


@pytest.mark.parametrize("dtype", [1, 0])
def test_every_target_position_k1(Q, O, S, dtype):
    rng = np.random.default_rng(5)
    for n in (2, 7, 16):
        st, psi = _state(Q, S, n, dtype, n)
        for t in range(n):
            U = _rand_unitary(rng, 1)
            st.apply_gate([t], U)
            psi = O.apply_gate(psi, [t], U)
        assert _err(st.get(), psi) < TOL[dtype]


@pytest.mark.parametrize("dtype", [1, 0])
def test_structured_gates(Q, O, S, dtype):
    """Phase (CR, CZ, T), diagonal (Rz, fused diag) and monomial (X, Y,
    CNOT, SWAP, Toffoli) gates take their specialised sweeps."""
    n = 12
    st, psi = _state(Q, S, n, dtype, 3)
    gates = [S.cr(2, 9, 0.37), S.cz(0, 11), S.g1(O.table1("T"), 5), S.g1(S.mat_rz(1.1), 1),
             S.Gate((3, 7, 8), np.diag(np.exp(1j * np.arange(8) * 0.3))),
             S.g1(S.MAT_X, 0), S.g1(S.MAT_Y, 10), S.cnot(4, 0), S.swap(1, 11), S.mcx((2, 6), 3),
             S.Gate((5,), S.MAT_X, 1 << 9, 0), S.cr(0, 1, -2.0)]
    for g in gates:
        st.apply_gate(g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
        psi = O.apply_gate(psi, g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
    assert _err(st.get(), psi) < TOL[dtype]


@pytest.mark.parametrize("dtype", [1, 0])
def test_permutation_gates_bit_exact(Q, O, S, dtype):
    n = 14
    st, psi = _state(Q, S, n, dtype, 11)
    gates = [S.g1(S.MAT_X, 0), S.cnot(13, 2), S.swap(0, 12), S.mcx((1, 5), 9), S.mcx((7,), 0),
             S.Gate((3, 4), S.MAT_SWAP, 1 << 10, 1 << 10)]
    for g in gates:
        st.apply_gate(g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
        psi = O.apply_gate(psi, g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
    got = st.get()
    ref = psi.astype(got.dtype)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


def test_identity_gate_is_noop(Q, S):
    st, psi = _state(Q, S, 9, 1, 1)
    st.apply_gate([3, 4], np.eye(4))
    assert np.array_equal(st.get(), psi)


def test_bell_ghz_and_entangling_op(Q, S):
    for n in (2, 5, 20):
        st = Q.State(n, 1)
        st.apply_gates(S.ghz_circuit(n))
        a = st.amplitudes([0, (1 << n) - 1, 1, 1 << (n - 1)])
        assert abs(a[0] - 2 ** -0.5) < 1e-15 and abs(a[1] - 2 ** -0.5) < 1e-15
        assert a[2] == 0 and a[3] == 0
        assert abs(st.norm2() - 1) < 1e-14


def test_errors_leave_state_unchanged(Q, S):
    st, psi = _state(Q, S, 8, 1, 4)
    bad = [([0, 0], np.eye(4), 0, 0), ([8], np.eye(2), 0, 0), ([1], np.eye(2), 2, 2),
           ([1], np.eye(2), 1, 2), ([1], np.full((2, 2), np.nan), 0, 0)]
    for t, m, cm, cv in bad:
        with pytest.raises(Q.QSError) as e:
            st.apply_gate(t, m, cm, cv)
        assert e.value.status == Q.QS_EINVAL
    with pytest.raises(Q.QSError):
        st.emulate_modmul(0, 4, 4, 2, 3, 9)       # gcd(3, 9) != 1
    with pytest.raises(Q.QSError):
        st.emulate_modmul(0, 4, 2, 2, 2, 11)      # overlapping registers
    with pytest.raises(Q.QSError):
        st.emulate_table(0, 2, [0, 0, 1, 2])      # not a permutation
    with pytest.raises(Q.QSError):
        st.measure([0, 0], [0.5])
    with pytest.raises(Q.QSError):
        st.measure([0], [1.0])
    assert np.array_equal(st.get(), psi)


# ---------------------------------------------------------------------------
# Fused programs: planner + FP64 composer + sweeps vs unfused oracle
# ---------------------------------------------------------------------------
def test_composer_blocks_vs_kron_product(Q, O, S):
    n = 10
    gates = S.random_layer_circuit(n, 5, seed=21)
    st = Q.State(n, 1)
    for max_k in (2, 4, 6):
        prog = st.compile(gates, max_k)
        bog, blocks = Q.plan_fusion(gates, n, max_k)
        nb, ks, _ = prog.info()
        assert nb == len(blocks)
        for b in range(nb):
            M, qs = prog.block(b)
            assert list(qs) == [int(q) for q in blocks[b]]
            loc = {int(q): i for i, q in enumerate(qs)}
            gl = [S.Gate(tuple(loc[t] for t in gates[g].targets), gates[g].matrix)
                  for g in range(len(gates)) if bog[g] == b]
            ref = O.block_matrix(len(qs), gl)
            assert np.abs(M - ref).max() < 1e-13


@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("max_k", [1, 2, 4, 6])
def test_fused_random_circuit_vs_oracle(Q, O, S, dtype, max_k):
    """The 16-qubit depth-20 random circuit, start |0...0>, plus <Z_0>."""
    n, depth = 16, 20
    gates = S.random_layer_circuit(n, depth, seed=S.SEED_BASE + 0)
    ref = O.apply_circuit(S.zero_state(n), gates)
    st = Q.State(n, dtype)
    prog = st.compile(gates, max_k)
    st.run(prog)
    assert _err(st.get(), ref) < TOL[dtype]
    z0 = st.expectation(z_mask=1)
    assert abs(z0 - O.expectation(ref, z_mask=1)) < TOL[dtype]


def test_fused_circuit_with_controls_and_wide_gates(Q, O, S):
    n = 11
    rng = np.random.default_rng(8)
    gates = []
    for _ in range(60):
        kind = rng.integers(0, 4)
        qs = [int(q) for q in rng.permutation(n)[:4]]
        if kind == 0:
            gates.append(S.Gate((qs[0],), _rand_unitary(rng, 1), 1 << qs[1], 0))
        elif kind == 1:
            gates.append(S.mcx((qs[0], qs[1]), qs[2]))
        elif kind == 2:
            gates.append(S.Gate(tuple(qs[:3]), _rand_unitary(rng, 3)))
        else:
            gates.append(S.cr(qs[0], qs[1], float(rng.random())))
    psi0 = S.normal_state(n, 3)
    ref = O.apply_circuit(psi0, gates)
    for max_k in (3, 5):
        st = Q.State(n, 1)
        st.set(psi0)
        st.apply_circuit(gates, max_k)
        assert _err(st.get(), ref) < 1e-10


def test_apply_fused_equals_gates(Q, O, S):
    rng = np.random.default_rng(2)
    n = 12
    blocks = [([int(q) for q in rng.permutation(n)[:k]], _rand_unitary(rng, k)) for k in (1, 4, 2, 3, 4)]
    st, psi = _state(Q, S, n, 1, 5)
    st.apply_fused(blocks)
    for t, m in blocks:
        psi = O.apply_gate(psi, t, m)
    assert _err(st.get(), psi) < 1e-10


def test_sweeps_are_deterministic(Q, S):
    n = 18
    gates = S.random_layer_circuit(n, 4, seed=9)
    outs = []
    for _ in range(2):
        st = Q.State(n, 1)
        st.apply_circuit(gates, 4)
        outs.append(st.get())
    assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))


# ---------------------------------------------------------------------------
# Reductions and measurement (Sec. III-D)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [1, 0])
def test_norm_and_pauli_expectations(Q, O, S, dtype):
    n = 15
    st, psi = _state(Q, S, n, dtype, 13)
    assert abs(st.norm2() - O.norm2(psi)) < 1e-12
    rng = np.random.default_rng(3)
    for _ in range(10):
        lab = rng.integers(0, 4, n)
        xm = sum(1 << q for q in range(n) if lab[q] == 1)
        ym = sum(1 << q for q in range(n) if lab[q] == 2)
        zm = sum(1 << q for q in range(n) if lab[q] == 3)
        got = st.expectation(xm, ym, zm)
        ref = O.expectation(psi, xm, ym, zm)
        assert abs(got - ref) < 1e-12


def test_expectation_closed_forms(Q, S):
    n = 9
    st = Q.State(n, 1)
    assert st.expectation(z_mask=1) == 1.0
    st.apply_gates(S.ghz_circuit(n))
    assert abs(st.expectation(z_mask=1)) < 1e-15
    assert abs(st.expectation(z_mask=0b11) - 1) < 1e-15
    assert abs(st.expectation(x_mask=(1 << n) - 1) - 1) < 1e-14


@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("qubits", [[0], [3, 1, 9], list(range(12)), [15, 2, 7, 0, 11, 4, 13, 5, 1, 14, 6, 8, 10]])
def test_measure_marginals_sampling_collapse(Q, O, S, dtype, qubits):
    n = 16
    st, psi = _state(Q, S, n, dtype, 17)
    p_ref = O.marginals(psi, qubits)
    u = np.random.default_rng(4).random(64)
    out, p = st.measure(qubits, u, collapse=False)
    assert np.abs(p - p_ref).max() < 1e-12
    ref_out = O.sample(p_ref, u)
    cdf = np.cumsum(p_ref) / p_ref.sum()
    for uu, a, b in zip(u, out, ref_out):
        if a != b:  # only allowed when u sits on a CDF boundary
            assert abs(cdf[min(a, b)] - uu) < 1e-12
    out, p = st.measure(qubits, u[:1], collapse=True)
    ref = O.collapse(psi, qubits, int(out[0]), p_ref[int(out[0])])
    assert _err(st.get(), ref) < TOL[dtype]


def test_measure_deterministic_given_uniforms(Q, S):
    st, _ = _state(Q, S, 12, 1, 1)
    u = np.linspace(0, 0.999, 33)
    a, _ = st.measure([0, 5, 7], u)
    b, _ = st.measure([0, 5, 7], u)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Arithmetic as a permutation (Sec. III-A)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("w,c,work_lo,ctrl_lo,n,seed", [
    (12, 4, 0, 12, 16, 1), (10, 3, 4, 14, 18, 2), (9, 0, 3, 0, 14, 3), (8, 5, 6, 0, 15, 4)])
def test_modmul_bit_exact(Q, O, S, dtype, w, c, work_lo, ctrl_lo, n, seed):
    a, N = S.modmul_params(w, seed)
    st, psi = _state(Q, S, n, dtype, seed)
    st.emulate_modmul(work_lo, w, ctrl_lo, c, a, N)
    ref = O.modmul(psi, work_lo, w, ctrl_lo, c, a, N).astype(st.np_dtype)
    got = st.get()
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("w,c,ctrl_lo,n,a,N", [
    (15, 3, 15, 19, None, None),        # seeded a, N just above 2^14
    (16, 4, 17, 21, 2, 65521),          # a = 2: small powers give short gaps (plain blocks) next to tiled ones
    (16, 2, 16, 19, 65520, 65521),      # a = N - 1: gaps of 1 and N - 1 in every block
    (17, 5, 18, 24, 3, 131071),         # spectator qubits between and above the registers
    (20, 1, 20, 22, None, None)])
def test_modmul_tiled_gather_bit_exact(Q, O, S, dtype, w, c, ctrl_lo, n, a, N):
    """The tiled gather (work register at qubit 0, three-gap rows per
    control value; default 64 x 128 tiles) against the oracle and against
    the plain per-amplitude gather and the narrower tiles, bit for bit; multipliers whose rows degenerate
    fall back to the plain gather per control block."""
    if a is None:
        a, N = S.modmul_params(w, 1000 + w)
    st, psi = _state(Q, S, n, dtype, 17 + n)
    st.emulate_modmul(0, w, ctrl_lo, c, a, N)
    got = st.get()
    ref = O.modmul(psi, 0, w, ctrl_lo, c, a, N).astype(st.np_dtype)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
    try:
        for kern in (1, 2, 3, 4):   # plain gather, 64 x 16, 64 x 32 and 64 x 64 tiles
            Q.tune_set(Q.QS_TUNE_MODMUL_KERNEL, kern)
            st.set(psi)
            st.emulate_modmul(0, w, ctrl_lo, c, a, N)
            other = st.get()
            assert np.array_equal(got.view(np.uint8), other.view(np.uint8)), kern
    finally:
        Q.tune_set(Q.QS_TUNE_MODMUL_KERNEL, 0)
    st.free()


def test_table_permutation_bit_exact(Q, O, S):
    n, lo, nb = 13, 3, 7
    dest = np.random.default_rng(6).permutation(1 << nb).astype(np.uint64)
    st, psi = _state(Q, S, n, 1, 2)
    st.emulate_table(lo, nb, dest)
    ref = O.table_perm(psi, lo, nb, dest)
    assert np.array_equal(st.get().view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("w,c,seed", [(3, 2, 1), (4, 2, 5)])
def test_gate_level_modmul_on_gpu_bit_exact(Q, O, S, w, c, seed):
    """The Toffoli/CNOT/X network applied by the GPU gate sweeps equals the
    emulated permutation bit for bit on x < N (ancillas back to 0)."""
    a, N = S.modmul_params(w, seed)
    gates, L = S.modmul_gate_circuit(w, c, a, N)
    rng = np.random.default_rng(seed)
    psi = np.zeros(1 << L.n, dtype=complex)
    for cc in range(1 << c):
        for x in range(N):
            psi[x | (cc << L.ctrl[0])] = rng.standard_normal() + 1j * rng.standard_normal()
    g = Q.State(L.n, 1)
    g.set(psi)
    g.apply_gates(gates)
    e = Q.State(L.n, 1)
    e.set(psi)
    e.emulate_modmul(0, w, L.ctrl[0], c, a, N)
    ref = O.modmul(psi, 0, w, L.ctrl[0], c, a, N)
    assert np.array_equal(g.get().view(np.uint8), ref.view(np.uint8))
    assert np.array_equal(e.get().view(np.uint8), ref.view(np.uint8))


def test_borrowed_torch_buffer_and_stream(Q, O, S):
    """A torch tensor's memory and torch's current stream serve as the state;
    an out-of-place permutation refreshes the borrowed buffer."""
    import torch
    n = 14
    psi = S.normal_state(n, 31)
    t = torch.from_numpy(psi.copy()).to("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = Q.State(n, Q.QS_C128, device_buf=t.data_ptr(), stream=stream)
    g = S.random_layer_circuit(n, 3, seed=4)
    st.apply_circuit(g, 4)
    a, N = S.modmul_params(10, 7)
    st.emulate_modmul(0, 10, 10, 4, a, N)
    st.sync()
    ref = O.modmul(O.apply_circuit(psi, g), 0, 10, 10, 4, a, N)
    got = t.cpu().numpy()
    assert np.abs(got - ref).max() < 1e-10
    assert st.info()[2] == t.data_ptr()
    st.free()
    # the freed handle did not free torch's memory
    assert np.abs(t.cpu().numpy() - ref).max() < 1e-10


def test_handles_after_out_of_place_ops_free_cleanly(Q, S):
    for _ in range(3):
        st = Q.State(12, 1)
        st.emulate_modmul(0, 6, 6, 3, 5, 63 - 2)
        st.emulate_table(0, 3, [1, 2, 3, 4, 5, 6, 7, 0])
        st.free()
    st = Q.State(12, 1)
    st.apply_gate([0], S.MAT_H)
    assert abs(st.norm2() - 1) < 1e-14


@pytest.mark.parametrize("dtype", [1, 0])
def test_load_device_streaming_copy_and_fallbacks(Q, S, dtype):
    """qs_load_device copies with the library's 16-byte streaming kernel when
    both buffers are 16-byte aligned and falls back to the runtime copy
    otherwise (a complex64 source one amplitude, 8 bytes, into a tensor):
    both paths move the amplitudes bit for bit, from 2 to 2^21 amplitudes
    (at 2^21 the copy's 1024-thread blocks number 2048 (complex128) or 1024
    (complex64), enough for the chunked XCD order); an overlapping source is
    rejected."""
    import torch
    tdt = torch.complex128 if dtype == 1 else torch.complex64
    for n in (1, 2, 7, 17, 21):
        x = torch.randn((1 << n) + 1, dtype=tdt, device="cuda")
        ref = x.cpu().numpy()
        for off in (0, 1):                                 # aligned, then one amplitude in
            st = Q.State(n, dtype)
            st.load_device(x.data_ptr() + off * x.element_size())
            got = st.get()
            assert np.array_equal(got.view(np.uint8), ref[off:off + (1 << n)].view(np.uint8)), (n, off)
            st.free()
    st = Q.State(4, dtype)
    _, _, p = st.info()
    with pytest.raises(Q.QSError):
        st.load_device(p)
    st.free()


@pytest.mark.parametrize("dtype", [1, 0])
def test_structured_gates_inside_a_cache_line(Q, O, S, dtype):
    """Phase gates whose pinned bits lie inside a 128-byte line take the
    whole-line form (every amplitude of the touched lines read and written
    back), and permutation gates with targets there move only what they
    touch: same result as the oracle, permutations bit for bit."""
    n = 12
    psi = S.normal_state(n, 77)
    th = 0.7
    cases = [
        S.cr(0, 1, th), S.cr(1, 2, th), S.cr(2, 3, th), S.cr(0, 11, th), S.cr(3, 1, th),
        S.Gate((0,), np.diag([1, np.exp(1j * th)])),                            # phase on qubit 0
        S.Gate((5,), np.diag([1, np.exp(1j * th)]), 0b11, 0b01),                 # controls 0 (=1), 1 (=0)
        S.Gate((2,), np.diag([np.exp(1j * th), 1]), 1 << 9, 1 << 9),             # phase on |0> of qubit 2
    ]
    perms = [S.swap(0, 11), S.swap(1, 2), S.swap(3, 9), S.cnot(0, 7), S.cnot(7, 1), S.mcx((3, 8), 0)]
    for g, is_perm in [(g, False) for g in cases] + [(g, True) for g in perms]:
        st = Q.State(n, dtype)
        st.set(psi)
        before = st.get()
        st.apply_gate(g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
        ref = O.apply_gate(before.astype(np.complex128), g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
        got = st.get()
        if is_perm:
            assert np.array_equal(got.view(np.uint8), ref.astype(got.dtype).view(np.uint8)), g.name
        else:
            assert np.abs(got - ref).max() < (1e-13 if dtype == 1 else 2e-6), g.name
        st.free()
