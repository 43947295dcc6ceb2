"""GPU parity of the emulated QFT (Sec. III-B) against the oracle.

Small and mid sizes compare every amplitude with the oracle's direct
transform or numpy's ifft(norm="ortho"); the 30-qubit workload is checked
on sampled outputs (closed form for basis states, the oracle's per-output
sum for the seeded normal state)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {1: 1e-10, 0: 1e-5}


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def _err(a, b):
    return float(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128)).max())


@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("n,q_lo,m", [
    (1, 0, 1), (3, 0, 3), (6, 2, 3), (10, 0, 10), (12, 1, 9),       # one pass
    (11, 0, 11), (14, 0, 14), (16, 3, 12), (17, 0, 13),              # two passes
    (21, 0, 21), (22, 1, 21), (22, 0, 22)])                          # three passes
def test_qft_vs_oracle(Q, O, S, dtype, n, q_lo, m):
    psi = S.normal_state(n, 1000 + n + m)
    for inverse in (False, True):
        st = Q.State(n, dtype)
        st.set(psi)
        x = st.get().astype(np.complex128)
        st.emulate_qft(q_lo, m, inverse)
        ref = O.qft_direct(x, q_lo, m, inverse) if n <= 12 else O.dft_numpy(x, q_lo, m, inverse)
        assert _err(st.get(), ref) < TOL[dtype], (n, q_lo, m, inverse)


def test_numpy_and_oracle_agree_where_both_run(O, S):
    x = S.normal_state(12, 5)
    assert _err(O.qft_direct(x, 2, 9), O.dft_numpy(x, 2, 9)) < 1e-13


@pytest.mark.parametrize("dtype", [1, 0])
def test_qft_roundtrip_and_norm(Q, S, dtype):
    n = 23
    psi = S.normal_state(n, 3)
    st = Q.State(n, dtype)
    st.set(psi)
    x = st.get().astype(np.complex128)
    st.emulate_qft(0, n)
    assert abs(st.norm2() - 1) < (1e-12 if dtype else 1e-5)
    st.emulate_qft(0, n, inverse=True)
    assert _err(st.get(), x) < TOL[dtype]


def test_gate_level_qft_on_gpu_equals_emulated(Q, O, S):
    """The gate-level circuit (Hadamards, conditional phase shifts, SWAPs)
    run through the GPU gate sweeps equals the emulated transform."""
    for n, q_lo, m in ((14, 0, 14), (15, 2, 11)):
        psi = S.normal_state(n, 8)
        g = Q.State(n, 1)
        g.set(psi)
        g.apply_gates(S.qft_circuit(m, q_lo))
        e = Q.State(n, 1)
        e.set(psi)
        e.emulate_qft(q_lo, m)
        assert _err(g.get(), e.get()) < 1e-10
        assert _err(e.get(), O.dft_numpy(psi, q_lo, m)) < 1e-10


def test_qft_on_borrowed_buffer(Q, O, S):
    import torch
    n = 18
    psi = S.normal_state(n, 12)
    t = torch.from_numpy(psi.copy()).to("cuda")
    st = Q.State(n, Q.QS_C128, device_buf=t.data_ptr(),
                 stream=torch.cuda.current_stream().cuda_stream)
    st.emulate_qft(0, n)
    st.sync()
    assert _err(t.cpu().numpy(), O.dft_numpy(psi)) < 1e-10
    assert st.info()[2] == t.data_ptr()


def test_qft_invalid_fields_rejected(Q):
    st = Q.State(8, 1)
    for q_lo, m in ((0, 0), (0, 9), (5, 4), (-1, 3)):
        with pytest.raises(Q.QSError):
            st.emulate_qft(q_lo, m)


def test_qft_30q_basis_states_closed_form(Q):
    """QFT|j> = 2^(-n/2) sum_l exp(2 pi i j l / 2^n) |l> at the full size."""
    n = 30
    N = 1 << n
    st = Q.State(n, 1)
    rng = np.random.default_rng(4)
    idx = np.concatenate([[0, 1, N - 1, 1 << 29], rng.integers(0, N, 60)]).astype(np.uint64)
    for j in (0, 1, 123456789, N - 1):
        st.set_zero()
        st.apply_gates([])  # no-op
        if j:
            # |j> from |0> with X gates on the set bits
            for q in range(n):
                if (j >> q) & 1:
                    st.apply_gate([q], np.array([[0, 1], [1, 0]]))
        st.emulate_qft(0, n)
        got = st.amplitudes(idx)
        ref = np.exp(2j * np.pi * ((j * idx.astype(object)) % N).astype(np.float64) / N) / np.sqrt(N)
        assert _err(got, ref) < 1e-12
    st.free()


def test_qft_30q_seeded_state_sampled_vs_oracle(Q, O, S):
    """The 30-qubit workload: seeded normal amplitudes, emulated QFT,
    outputs sampled and recomputed one by one by the oracle."""
    n = 30
    psi = S.normal_state(n, S.SEED_BASE + 1)
    st = Q.State(n, 1)
    st.set(psi)
    st.emulate_qft(0, n)
    idx = np.array([0, 1, 777777, (1 << 30) - 1], dtype=np.uint64)
    got = st.amplitudes(idx)
    for i, g in zip(idx, got):
        assert abs(g - O.qft_sample(psi, int(i))) < 1e-10
    assert abs(st.norm2() - 1) < 1e-12
