"""FP32 states with FP64 accumulation: 6-qubit fused blocks on the matrix
cores (complex64) against the FP64 oracle.

The 32-qubit depth-40 workload is checked on its 22-qubit twin (same
generator and seed) amplitude by amplitude, and at full size through
properties that hold at any size (norm accumulated in FP64, circuit followed
by its inverse returns |0...0>)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def test_twin_22q_k6_complex64_vs_fp64_oracle(Q, O, S):
    n, depth = 22, 40
    gates = S.random_layer_circuit(n, depth, seed=S.SEED_BASE + 3)
    ref = O.apply_circuit(S.zero_state(n), gates)
    st = Q.State(n, Q.QS_C64)
    prog = st.compile(gates, 6)
    nb, ks, _ = prog.info()
    assert max(ks) == 6
    st.run(prog)
    got = st.get().astype(np.complex128)
    err = np.abs(got - ref)
    rel_l2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    fid = abs(np.vdot(ref, got)) ** 2 / (np.vdot(got, got).real)
    print("twin 22q k=6 c64: blocks=%d max_abs=%.3e rel_l2=%.3e fidelity=%.12f" % (nb, err.max(), rel_l2, fid))
    assert err.max() < 1e-5
    assert rel_l2 < 1e-4 and fid > 1 - 1e-7
    assert abs(st.norm2() - 1.0) < 1e-5
    z = st.expectation(z_mask=1).real
    assert abs(z - O.expectation(ref, z_mask=1).real) < 1e-5


def test_mfma_block_every_target_class(Q, O, S):
    """6- and 5-qubit blocks on complex64 take the matrix-core path for low,
    high and mixed targets."""
    rng = np.random.default_rng(12)
    n = 16
    for targets in ([0, 1, 2, 3, 4, 5], [10, 11, 12, 13, 14, 15], [0, 7, 3, 15, 9, 1],
                    [6, 2, 13, 8, 11, 4], [0, 1, 2, 3, 4], [11, 12, 13, 14, 15], [0, 7, 3, 15, 9],
                    [6, 2, 13, 8, 11]):
        d = 1 << len(targets)
        z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        U = np.linalg.qr(z)[0]
        st = Q.State(n, Q.QS_C64)
        st.set(S.normal_state(n, 5))
        psi = st.get().astype(np.complex128)
        st.apply_gate(targets, U)
        ref = O.apply_gate(psi, targets, U)
        assert np.abs(st.get() - ref).max() < 1e-5, targets


def test_32q_k6_complex64_norm_and_roundtrip(Q, S):
    """Full size: 32 qubits complex64, depth-40 random circuit fused into
    6-qubit blocks; norm stays 1 (FP64 accumulation) and the inverse
    circuit returns |0...0> to FP32 accuracy."""
    n, depth = 32, 40
    gates = S.random_layer_circuit(n, depth, seed=S.SEED_BASE + 3)
    st = Q.State(n, Q.QS_C64)
    prog = st.compile(gates, 6)
    st.run(prog)
    nrm = st.norm2()
    assert abs(nrm - 1.0) < 1e-5
    inv = st.compile(S.inverse_circuit(gates), 6)
    st.run(inv)
    a0 = st.amplitudes([0, 1, (1 << n) - 1, 12345678])
    print("32-qubit round trip: |a0 - 1| = %.3e, max other = %.3e" % (abs(a0[0] - 1.0), np.abs(a0[1:]).max()))
    assert abs(a0[0] - 1.0) < 1e-5
    assert np.abs(a0[1:]).max() < 1e-5
    st.free()
