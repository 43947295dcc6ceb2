"""Parity at the benchmark's full size, in the launch configuration bench.py
times: 30-qubit states, circuits compiled into k = 4 blocks with the tuned
launch table in effect, the 20-bit-work / 8-bit-control modmul. The oracle
cannot simulate 2^30 amplitudes gate by gate in a test, so sampled outputs
are checked against its per-index forms, and whole-state properties (norm,
an inverse circuit returning |0...0>) that hold at any size."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 30


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def _sample(n, count, seed):
    idx = np.random.default_rng(seed).integers(0, 1 << n, count).astype(np.uint64)
    idx[:3] = [0, (1 << n) - 1, 1 << (n - 1)]
    return idx


@pytest.mark.parametrize("dtype", [1, 0])
def test_30q_random_layer_fused_k4_sampled_vs_oracle(Q, O, S, dtype):
    rng = np.random.default_rng(S.SEED_BASE + 11)
    gates = S.random_layer_on(list(range(N)), rng)
    ones = [g.matrix for g in gates if g.k == 1]
    pairs = [tuple(g.targets) for g in gates if g.k == 2]
    st = Q.State(N, dtype)
    prog = st.compile(gates, 4)
    st.run(prog)
    prog.free()
    idx = _sample(N, 512, 5)
    got = st.amplitudes(idx).astype(np.complex128)
    ref = O.layer_amplitudes(ones, pairs, idx)
    scale = np.abs(ref).max()
    tol = 1e-10 if dtype == 1 else 1e-5
    assert np.abs(got - ref).max() < tol * scale
    assert abs(st.norm2() - 1) < (1e-12 if dtype == 1 else 1e-5)
    # marginals of 8 qubits: CZ only changes signs, so they factor
    qubits = [0, 3, 7, 11, 16, 22, 27, 29]
    _, p = st.measure(qubits, [0.5])
    p_ref = np.ones(1)
    for q in qubits:          # outcome bit r = qubit qubits[r]: later qubits are more significant
        pq = np.abs(ones[q][:, 0]) ** 2
        p_ref = np.concatenate([p_ref * pq[0], p_ref * pq[1]])
    assert np.abs(p - p_ref).max() < (1e-12 if dtype == 1 else 1e-5)
    st.free()


def test_30q_bench_circuit_then_inverse_returns_to_zero(Q, S):
    """The benchmark's depth-30 circuit, compiled at k = 4, followed by its
    inverse (reversed gates, conjugate transposes): |0...0> again."""
    gates = S.random_layer_circuit(N, 30, S.SEED_BASE + 1)
    inv = [dataclasses.replace(g, matrix=np.ascontiguousarray(g.matrix.conj().T)) for g in reversed(gates)]
    st = Q.State(N, Q.QS_C128)
    for gl in (gates, inv):
        prog = st.compile(gl, 4)
        nb, ks, moves = prog.info()
        kinds = [prog.block_kind(b) for b in range(nb)]
        assert nb > 100 and max(ks) <= 4
        # dense blocks move the whole state, diagonal (CZ-only) blocks only
        # the amplitudes whose sign flips
        assert moves == sum(f for _, f in kinds) * 2.0 * 2 ** N <= nb * 2.0 * 2 ** N
        if gl is gates:       # the last layer's CZs form diagonal blocks
            assert moves < nb * 2.0 * 2 ** N
        assert all(f == 1.0 for k, f in kinds if k == Q.QS_BLOCK_DENSE)
        st.run(prog)
        prog.free()
    a = st.amplitudes(_sample(N, 64, 9))
    assert abs(a[0] - 1) < 1e-10
    assert np.abs(a[1:]).max() < 1e-10
    assert abs(st.norm2() - 1) < 1e-10
    st.free()


def test_30q_modmul_sampled_bit_exact(Q, O, S):
    """The benchmark's permutation (work qubits 0..19, control 20..27) on a
    resident seeded state: every sampled output is exactly the input
    amplitude at the oracle's source index."""
    import torch
    a, Nmod = S.modmul_params(20, S.SEED_BASE + 1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(S.SEED_BASE + 1)
    x = torch.randn(1 << N, dtype=torch.complex128, device="cuda", generator=gen)
    st = Q.State(N, Q.QS_C128)
    st.load_device(x.data_ptr())
    st.emulate_modmul(0, 20, 20, 8, a, Nmod)
    idx = _sample(N, 4096, 13)
    src = O.modmul_source(idx, 0, 20, 20, 8, a, Nmod)
    want = x[torch.from_numpy(src.astype(np.int64)).to("cuda")].cpu().numpy()
    got = st.amplitudes(idx)
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))
    st.free()
    del x
    torch.cuda.empty_cache()


def test_28q_modmul_configuration_full_state_bit_exact(Q, O, S):
    """The 28-qubit arithmetic workload: control register (qubits 20..27) in
    uniform superposition, seeded normal 20-qubit work register, an odd
    20-bit modulus. All 2^28 outputs against the oracle, bit for bit."""
    a, Nmod = S.modmul_params(20, S.SEED_BASE + 2)
    w = S.normal_state(20, S.SEED_BASE + 2)
    psi = np.tile(w, 256) / 16.0                      # H on each control qubit: amplitude 1/16
    st = Q.State(28, Q.QS_C128)
    st.set(psi)
    st.emulate_modmul(0, 20, 20, 8, a, Nmod)
    got = st.get()
    st.free()
    ref = O.modmul(psi, 0, 20, 20, 8, a, Nmod)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("targets", [[26, 3, 17, 31, 0, 9], [12, 13, 14, 15, 16, 17], [5, 4, 3, 2, 1, 0],
                                     [31, 2, 20, 7, 11], [0, 1, 2, 3, 4]])
def test_32q_matrix_core_block_sampled_vs_oracle(Q, O, S, targets):
    """The 32-qubit complex64 matrix-core sweep (64-bit tile indices, the
    tuned kernel and grid that bench.py's 32-qubit circuit runs) on a
    random state: sampled outputs against the oracle applied to each
    sample's group of 2^k input amplitudes, read from the state before the
    block."""
    import torch
    n, k = 32, len(targets)
    rng = np.random.default_rng(S.SEED_BASE + 37 + k)
    z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    U = np.linalg.qr(z)[0]
    gen = torch.Generator(device="cuda").manual_seed(1604 + sum(targets))
    x = torch.randn(2 << n, generator=gen, dtype=torch.float32, device="cuda")
    x.mul_(2.0 ** (-(n + 1) / 2))
    st = Q.State(n, Q.QS_C64)
    st.load_device(x.data_ptr())
    st.sync()
    del x
    torch.cuda.empty_cache()
    out_idx = _sample(n, 192, 40 + k)
    tmask = sum(1 << t for t in targets)
    local = np.arange(1 << k, dtype=np.uint64)
    offs = np.zeros(1 << k, dtype=np.uint64)
    for i, t in enumerate(targets):
        offs |= ((local >> np.uint64(i)) & np.uint64(1)) << np.uint64(t)
    base = out_idx & ~np.uint64(tmask)
    groups = base[:, None] | offs[None, :]
    inputs = st.amplitudes(groups.reshape(-1)).astype(np.complex128).reshape(len(out_idx), 1 << k)
    st.apply_gate(targets, U)
    got = st.amplitudes(out_idx).astype(np.complex128)
    st.free()
    torch.cuda.empty_cache()
    ref = np.empty(len(out_idx), dtype=np.complex128)
    for s in range(len(out_idx)):
        i_out = sum(((int(out_idx[s]) >> t) & 1) << i for i, t in enumerate(targets))
        ref[s] = O.apply_gate(inputs[s].copy(), list(range(k)), U)[i_out]
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() < 1e-5 * scale, (targets, np.abs(got - ref).max(), scale)
