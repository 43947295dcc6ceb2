"""Every launch choice the autotuner can make gives the oracle's result:
each dense sweep path for every width and target class, grid caps that
force grid-stride loops, every FFT digit/LDS budget, the matrix-core grid,
and batch gang sizing (states bit-identical across gang settings)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture
def Q():
    from paper_1604_06460_amd import qs
    qs.tune_reset()
    yield qs
    qs.tune_reset()
    if os.path.exists(qs.TUNED_FILE):
        qs.load_tuning()


def _unitary(k, rng):
    d = 1 << k
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _targets(cls, k, n, dtype, Q):
    lb = 3 if dtype == Q.QS_C128 else 4
    lo = {Q.QS_TCLS_SUBLINE: 0, Q.QS_TCLS_SUBWAVE: lb, Q.QS_TCLS_HIGH: 6}[cls]
    return sorted([lo] + [n - 1 - 2 * i for i in range(k - 1)])


TOL = {0: 1e-5, 1: 1e-12}   # complex64 / complex128, max abs error on a normalised state


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_every_sweep_path_matches_oracle(Q, O, S, dtype, k):
    n = 16
    rng = np.random.default_rng(100 + 10 * k + dtype)
    psi0 = S.normal_state(n, 7 + k)
    for cls in (Q.QS_TCLS_SUBLINE, Q.QS_TCLS_SUBWAVE, Q.QS_TCLS_HIGH):
        t = _targets(cls, k, n, dtype, Q)
        assert Q.tune_classify(dtype, n, t)[0] == cls
        m = _unitary(k, rng)
        ref = O.apply_gate(psi0.copy(), t, m)
        for path in (1, 2, 3, 4, 5):
            for cap, nt in ((0, 0), (1, 3)):   # cap 1: one workgroup per CU, grid-stride; nt 3: streaming
                Q.tune_set(Q.QS_TUNE_SWEEP_PATH, path, dtype, k, cls, -1)
                Q.tune_set(Q.QS_TUNE_SWEEP_WG_PER_CU, cap, dtype, k, cls, -1)
                Q.tune_set(Q.QS_TUNE_SWEEP_NT, nt, dtype, k, cls, -1)
                st = Q.State(n, dtype)
                st.set(psi0)
                st.apply_gate(t, m)
                got = st.get().astype(np.complex128)
                st.free()
                assert np.abs(got - ref).max() < TOL[dtype], (dtype, k, cls, path, cap, nt)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k", [2, 3, 4])
def test_shared_tile_sweep_matches_oracle(Q, O, S, dtype, k):
    """The workgroup-shared 1024-amplitude tile (path 5, the complex128
    default for 2 to 4 qubits on 20 or more qubits) at 22 qubits, where its
    4096 workgroups take the chunked XCD order, and at 19 (512 tiles).
    Targets inside a cache line, inside a wave, above it and at or above
    qubit 20, given in arbitrary order, with both cache policies. At 10
    qubits, the smallest state the path takes, the tile is the whole state
    and the grid one workgroup."""
    rng = np.random.default_rng(300 + 10 * k + dtype)
    sets = {22: [[3, 0, 21, 9], [0, 1, 2, 3], [5, 6, 7, 8], [21, 20, 19, 12], [4, 13, 2, 17]],
            19: [[18, 0, 7, 2], [6, 9, 13, 17]],
            10: [[9, 0, 5, 3], [6, 7, 8, 9]]}
    for n, ts in sets.items():
        psi0 = S.normal_state(n, 40 + n + k)
        for t in ts:
            t = t[:k]
            m = _unitary(k, rng)
            ref = O.apply_gate(psi0.copy(), t, m)
            for nt in (0, 3):
                cls = Q.tune_classify(dtype, n, t)[0]
                Q.tune_set(Q.QS_TUNE_SWEEP_PATH, 5, dtype, k, cls, -1)
                Q.tune_set(Q.QS_TUNE_SWEEP_NT, nt, dtype, k, cls, -1)
                st = Q.State(n, dtype)
                st.set(psi0)
                st.apply_gate(t, m)
                got = st.get().astype(np.complex128)
                st.free()
                assert np.abs(got - ref).max() < TOL[dtype], (dtype, k, n, t, nt)


@pytest.mark.parametrize("dtype", [0, 1])
def test_every_fft_shape_matches_oracle(Q, O, S, dtype):
    n = 15
    psi0 = S.normal_state(n, 21)
    for q_lo, m in ((0, 15), (2, 11)):
        ref = O.dft_numpy(psi0, q_lo, m, False)
        for digit in (2, 4, 7, 10):
            for kb, nt in ((8, 0), (64, 3), (160, 1)):
                Q.tune_set(Q.QS_TUNE_FFT_DIGIT, digit, dtype)
                Q.tune_set(Q.QS_TUNE_FFT_LDS_KB, kb, dtype)
                Q.tune_set(Q.QS_TUNE_FFT_NT, nt, dtype)
                st = Q.State(n, dtype)
                st.set(psi0)
                st.emulate_qft(q_lo, m)
                got = st.get().astype(np.complex128)
                st.free()
                assert np.abs(got - ref).max() < TOL[dtype], (dtype, q_lo, m, digit, kb)


@pytest.mark.parametrize("dtype", [0, 1])
def test_every_fft_kernel_matches_oracle(Q, O, S, dtype):
    """Every pass kernel the FFT option selects, on fields with 10-bit
    digits (the register-tile kernels) and without: forward and inverse,
    spectator qubits below and above the field, single and final passes."""
    cases = ((20, 0, 20, False), (20, 0, 20, True), (22, 5, 10, False), (22, 2, 20, True),
             (21, 0, 20, False), (21, 1, 10, True), (20, 3, 17, False))
    for n, q_lo, m, inv in cases:
        psi0 = S.normal_state(n, 40 + n + q_lo)
        ref = O.dft_numpy(psi0, q_lo, m, inv)
        for kern in (1, 2, 3, 4, 5):
            Q.tune_set(Q.QS_TUNE_FFT_KERNEL, kern, dtype)
            st = Q.State(n, dtype)
            st.set(psi0)
            st.emulate_qft(q_lo, m, inverse=inv)
            got = st.get().astype(np.complex128)
            st.free()
            err = float(np.abs(got - ref).max())
            assert err < TOL[dtype], (dtype, kern, n, q_lo, m, inv, err)


def test_mfma_grid_sizes_match_oracle(Q, O, S):
    n = 18
    rng = np.random.default_rng(5)
    psi0 = S.normal_state(n, 3)
    t = [0, 3, 6, 9, 12, 17]
    m = _unitary(6, rng)
    ref = O.apply_gate(psi0.copy(), t, m)
    for w in (1, 3, 8, 16):
        Q.tune_set(Q.QS_TUNE_MFMA_WG_PER_CU, w)
        st = Q.State(n, Q.QS_C64)
        st.set(psi0)
        st.apply_gate(t, m)
        got = st.get().astype(np.complex128)
        st.free()
        assert np.abs(got - ref).max() < TOL[0], w


def test_every_mfma_kernel_matches_oracle(Q, O, S):
    """Every matrix-core sweep variant (the two LDS layouts, with and
    without register prefetch, the three-product form) against the
    oracle, for 6- and 5-qubit
    blocks with targets below, above and across bit 6, given in ascending
    and in scrambled order."""
    n = 16
    rng = np.random.default_rng(23)
    psi0 = S.normal_state(n, 8)
    cases = ([0, 1, 2, 3, 4, 5], [5, 3, 0, 1, 4, 2], [10, 11, 12, 13, 14, 15], [15, 6, 9, 12, 7, 10],
             [0, 7, 3, 15, 9, 1], [6, 2, 13, 8, 11, 4], [5, 6, 7, 8, 9, 10], [1, 4, 6, 8, 9, 14],
             [0, 1, 2, 3, 4], [4, 2, 0, 1, 3], [10, 11, 12, 13, 14], [2, 7, 12, 6, 1], [5, 6, 7, 8, 9],
             [3, 9, 0, 15, 5], [6, 15, 8, 12, 10])
    mats = [_unitary(len(t), rng) for t in cases]
    refs = [O.apply_gate(psi0.copy(), t, m) for t, m in zip(cases, mats)]
    try:
        for kern in (1, 2, 3, 4, 5, 6):
            Q.tune_set(Q.QS_TUNE_MFMA_KERNEL, kern)
            for t, m, ref in zip(cases, mats, refs):
                st = Q.State(n, Q.QS_C64)
                st.set(psi0)
                st.apply_gate(t, m)
                got = st.get().astype(np.complex128)
                st.free()
                err = float(np.abs(got - ref).max())
                assert err < TOL[0], (kern, t, err)
    finally:
        Q.tune_set(Q.QS_TUNE_MFMA_KERNEL, 0)


def test_mfma_kernels_on_one_and_two_tiles(Q, O, S):
    """The smallest states the matrix-core path takes: 12 qubits (one
    4096-amplitude tile, a grid of one workgroup) and 13 qubits (two
    tiles), for 5- and 6-qubit blocks whose targets fill the tile or leave
    it the fewest free bits, in every kernel variant."""
    rng = np.random.default_rng(29)
    cases = [(12, [6, 7, 8, 9, 10, 11]), (12, [0, 11, 5, 6, 2, 9]), (12, [0, 1, 2, 3, 4, 5]),
             (12, [7, 8, 9, 10, 11]), (12, [4, 0, 11, 3, 1]), (13, [12, 6, 7, 8, 9, 10]),
             (13, [0, 1, 2, 3, 4]), (13, [12, 11, 10, 9, 8])]
    try:
        for n, t in cases:
            psi0 = S.normal_state(n, 3 + n)
            m = _unitary(len(t), rng)
            ref = O.apply_gate(psi0.copy(), t, m)
            for kern in (1, 2, 3, 4, 5, 6):
                Q.tune_set(Q.QS_TUNE_MFMA_KERNEL, kern)
                st = Q.State(n, Q.QS_C64)
                st.set(psi0)
                st.apply_gate(t, m)
                got = st.get().astype(np.complex128)
                st.free()
                err = float(np.abs(got - ref).max())
                assert err < TOL[0], (n, t, kern, err)
    finally:
        Q.tune_set(Q.QS_TUNE_MFMA_KERNEL, 0)


def test_batch_gang_settings_give_identical_states(Q, S):
    circuits = S.batch_mix(24, 91, n_range=(12, 19), d_range=(3, 6), p_qft=0.3, p_modmul=0.3)
    b = Q.Batch(circuits)
    opts = Q.choose(b, Q.QS_POLICY_FIXED_K4)
    ref = None
    for share, bar in ((1, 1), (4, 4096), (64, 1 << 20), (256, 16)):
        Q.tune_set(Q.QS_TUNE_BATCH_GANG_SHARE, share)
        Q.tune_set(Q.QS_TUNE_BATCH_BARRIER_AMPS, bar)
        b.set_plan(opts)
        _, _, norms, _ = b.run()
        states = [b.state(c) for c in range(len(circuits))]
        tr = b.trace()
        assert len(tr["circuit"]) >= len(circuits)
        assert (tr["end_us"] >= tr["start_us"]).all()
        if ref is None:
            ref = states
        for c in range(len(circuits)):
            assert np.array_equal(states[c].view(np.uint8), ref[c].view(np.uint8)), (share, bar, c)
        assert np.abs(norms - 1).max() < 1e-5
    b.free()
