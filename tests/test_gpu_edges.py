"""Degenerate and boundary cases of every entry point against the oracle:
the smallest states, empty circuits, a one-qubit QFT at the top of the
register, identity and full-range modular multiplications, a measurement of
every qubit, and batches with empty or minimal circuits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 2e-6, 1: 1e-13}
TOL_FFT = {0: 1e-5, 1: 1e-12}   # the parity bars hold for the FFT passes too


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


@pytest.mark.parametrize("dtype", [1, 0])
def test_one_qubit_state(Q, O, S, dtype):
    st = Q.State(1, dtype)
    st.apply_gate([0], S.MAT_H)
    ref = O.apply_gate(S.zero_state(1), [0], S.MAT_H)
    assert np.abs(st.get() - ref).max() < TOL[dtype]
    st.set_zero()
    st.emulate_qft(0, 1)                       # a one-qubit QFT is a Hadamard
    assert np.abs(st.get() - ref).max() < TOL[dtype]
    out, p = st.measure([0], [0.7])
    assert out[0] == 1 and np.abs(p - 0.5).max() < TOL[dtype]
    st.free()


@pytest.mark.parametrize("dtype", [1, 0])
def test_two_qubit_state_dense_and_fused(Q, O, S, dtype):
    rng = np.random.default_rng(3)
    gates = [S.Gate((0,), S.haar_2x2(rng)), S.Gate((1, 0), S.MAT_CNOT), S.Gate((1,), S.haar_2x2(rng))]
    ref = O.apply_circuit(S.zero_state(2), gates)
    for max_k in (1, 2):
        st = Q.State(2, dtype)
        st.apply_circuit(gates, max_k)
        assert np.abs(st.get() - ref).max() < TOL[dtype], max_k
        st.free()


@pytest.mark.parametrize("dtype", [1, 0])
def test_empty_circuit_and_empty_program(Q, S, dtype):
    psi = S.normal_state(10, 4)
    st = Q.State(10, dtype)
    st.set(psi)
    before = st.get()
    st.apply_circuit([], 4)
    prog = st.compile([], 4)
    nb, ks, moves = prog.info()
    assert nb == 0 and moves == 0
    st.run(prog)
    prog.free()
    assert np.array_equal(st.get().view(np.uint8), before.view(np.uint8))
    st.free()


@pytest.mark.parametrize("dtype", [1, 0])
def test_top_qubit_qft_and_full_register_qft(Q, O, S, dtype):
    n = 12
    psi = S.normal_state(n, 6)
    for q_lo, m in ((n - 1, 1), (0, n), (n - 2, 2)):
        st = Q.State(n, dtype)
        st.set(psi)
        st.emulate_qft(q_lo, m)
        ref = O.qft_direct(psi, q_lo, m)
        assert np.abs(st.get() - ref).max() < TOL_FFT[dtype], (q_lo, m)
        st.emulate_qft(q_lo, m, inverse=True)
        assert np.abs(st.get() - psi).max() < TOL_FFT[dtype], (q_lo, m)
        st.free()


@pytest.mark.parametrize("dtype", [1, 0])
def test_modmul_identity_and_full_range_modulus(Q, O, S, dtype):
    n = 12
    psi = S.normal_state(n, 8)
    st = Q.State(n, dtype)
    st.set(psi)
    before = st.get()
    st.emulate_modmul(0, 6, 6, 3, 1, 61)           # a = 1: every power is 1
    assert np.array_equal(st.get().view(np.uint8), before.view(np.uint8))
    st.emulate_modmul(0, 6, 6, 3, 5, 64)           # N = 2^w: no fixed work values
    ref = O.modmul(before.astype(np.complex128), 0, 6, 6, 3, 5, 64).astype(before.dtype)
    assert np.array_equal(st.get().view(np.uint8), ref.view(np.uint8))
    st.emulate_modmul(3, 1, 0, 0, 1, 2)            # one-qubit work register, N = 2, no control
    assert np.array_equal(st.get().view(np.uint8), ref.view(np.uint8))
    st.free()


@pytest.mark.parametrize("dtype", [1, 0])
def test_measure_every_qubit(Q, O, S, dtype):
    n = 11
    psi = S.normal_state(n, 10)
    st = Q.State(n, dtype)
    st.set(psi)
    qubits = list(range(n))
    u = np.random.default_rng(2).random(64)
    out, p = st.measure(qubits, u)
    ref = O.marginals(psi, qubits)
    assert np.abs(p - ref).max() < TOL[dtype]
    assert np.abs(p - np.abs(psi) ** 2).max() < TOL[dtype]
    st.free()


def test_batch_with_empty_and_minimal_circuits(Q, O, S):
    rng = np.random.default_rng(4)
    circuits = [
        S.BatchCircuit(5, []),                                                 # no segments
        S.BatchCircuit(2, [S.Segment(S.SEG_LAYER, [S.Gate((0,), S.haar_2x2(rng))])]),
        S.BatchCircuit(2, [S.Segment(S.SEG_QFT, S.qft_circuit(2, 0), 0, 2, False)]),
        S.BatchCircuit(7, [S.Segment(S.SEG_LAYER, [])]),                       # empty gate list
        S.BatchCircuit(15, [S.Segment(S.SEG_LAYER, S.random_layer_on(list(range(15)), rng))]),
    ]
    b = Q.Batch(circuits)
    kinds, _, _ = b.segment_info()
    for rule in (0, 1, 2):
        opts = np.array([rule if k == 0 else 3 for k in kinds], dtype=np.int32)
        b.set_plan(opts)
        _, _, norms, _ = b.run()
        for c, circ in enumerate(circuits):
            psi = S.zero_state(circ.n)
            for s in circ.segments:
                psi = O.qft_direct(psi, s.q_lo, s.m, s.inverse) if s.kind == S.SEG_QFT else O.apply_circuit(psi, s.gates)
            assert np.abs(b.state(c).astype(np.complex128) - psi).max() < 2e-6, (rule, c)
            assert abs(norms[c] - 1) < 1e-5
    b.free()
