"""Fused diagonal blocks sweep only what they change (Sec. III-B: a
conditional phase shift reads and writes only the amplitudes carrying its
phase). Each block class is run against the oracle's gate-by-gate result:
one changed entry (phase kernel), several changed patterns above the line
(one pinned launch each), patterns with targets inside a 128-byte line
(whole lines rewritten), an all-ones block (nothing launched) and a block
whose every entry changes (one elementwise pass). The program's reported
changed fraction is checked against the block's diagonal counted on the
host, and running a program in block ranges equals one run."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-10}


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def _rz3(S):
    return S.Gate((2, 6, 9), np.diag(np.exp(1j * (0.3 + 0.17 * np.arange(8)))))


def _cases(S):
    # (gates, max_k, expected changed fraction of the single block)
    return [
        ([S.cz(9, 12)], 2, 1 / 4),
        ([S.cz(4, 7), S.cz(10, 13)], 4, 6 / 16),
        ([S.cz(0, 5), S.cz(1, 5)], 3, 2 / 8),
        ([S.cz(2, 7), S.cz(3, 7)], 3, 2 / 8),
        ([S.cz(2, 3), S.cz(2, 3)], 2, 0.0),
        ([_rz3(S)], 3, 1.0),
        ([S.cr(6, 8, 0.41), S.g1(S.MAT_T, 8)], 2, 2 / 4),
        ([S.cr(0, 1, -1.3), S.cz(1, 2)], 3, 3 / 8),
    ]


@pytest.mark.parametrize("dtype", [1, 0])
def test_diagonal_block_classes_vs_oracle(Q, O, S, dtype):
    n = 14
    psi0 = S.normal_state(n, 31)
    for gates, max_k, frac in _cases(S):
        st = Q.State(n, dtype)
        st.set(psi0)
        prog = st.compile(gates, max_k)
        nb, ks, moves = prog.info()
        assert nb == 1, [g.targets for g in gates]
        kind, f = prog.block_kind(0)
        want_kind = Q.QS_BLOCK_IDENTITY if frac == 0 else Q.QS_BLOCK_DIAGONAL
        assert kind == want_kind and f == frac, ([g.targets for g in gates], kind, f)
        assert moves == frac * 2 * (1 << n)
        st.run(prog)
        ref = O.apply_circuit(psi0, gates)
        err = np.abs(st.get().astype(np.complex128) - ref).max()
        assert err < TOL[dtype], ([g.targets for g in gates], err)
        prog.free()
        st.free()


@pytest.mark.parametrize("dtype", [1, 0])
def test_dense_blocks_report_full_sweeps_and_ranges_equal_one_run(Q, O, S, dtype):
    n = 13
    gates = S.random_layer_circuit(n, 4, seed=S.SEED_BASE + 77)
    psi0 = S.normal_state(n, 32)
    st = Q.State(n, dtype)
    st.set(psi0)
    prog = st.compile(gates, 4)
    nb, ks, moves = prog.info()
    kinds = [prog.block_kind(b) for b in range(nb)]
    assert moves == sum(f for _, f in kinds) * 2 * (1 << n)
    for kind, f in kinds:
        if kind == Q.QS_BLOCK_DENSE:
            assert f == 1.0
    cut = nb // 3
    st.run_range(prog, 0, cut)
    st.run_range(prog, cut, cut)
    st.run_range(prog, cut, nb)
    a = st.get()
    st.set(psi0)
    st.run(prog)
    b = st.get()
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    ref = O.apply_circuit(psi0, gates)
    assert np.abs(b.astype(np.complex128) - ref).max() < TOL[dtype]
    with pytest.raises(Q.QSError):
        st.run_range(prog, 0, nb + 1)
    with pytest.raises(Q.QSError):
        st.run_range(prog, 2, 1)
    prog.free()
    st.free()
