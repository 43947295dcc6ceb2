"""GPU parity of the batched persistent launch against the oracle.

Every plan (fusion width per segment, emulated or gate-level subroutines)
must give the same states: within 1e-5 of the FP64 oracle for these
complex64 circuits, and bit-identical between the gate-level and emulated
forms of a modular multiplication (both only move amplitudes)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def oracle_circuit(O, S, c):
    psi = S.zero_state(c.n)
    for s in c.segments:
        if s.kind == S.SEG_QFT:
            psi = O.qft_direct(psi, s.q_lo, s.m, s.inverse) if c.n <= 12 else \
                O.dft_numpy(psi, s.q_lo, s.m, s.inverse)
        elif s.kind == S.SEG_MODMUL:
            psi = O.modmul(psi, *s.modmul)
        else:
            psi = O.apply_circuit(psi, s.gates)
    return psi


@pytest.fixture(scope="module")
def small_batch(S):
    # sizes on both sides of the LDS-resident limit, all segment kinds
    b = S.batch_mix(20, 77, n_range=(10, 18), d_range=(3, 8), p_qft=0.3, p_modmul=0.3)
    b += S.batch_mix(4, 78, n_range=(16, 19), d_range=(4, 6), p_qft=0.2, p_modmul=0.6)
    return b


@pytest.fixture(scope="module")
def refs(O, S, small_batch):
    return [oracle_circuit(O, S, c) for c in small_batch]


def _options(kinds, rule, rng=None):
    out = np.zeros(len(kinds), dtype=np.int32)
    for i, k in enumerate(kinds):
        if rule == "random":
            out[i] = rng.integers(0, 3 if k == 0 else 4)
        elif rule == "emulate":
            out[i] = 1 if k == 0 else 3
        else:
            out[i] = rule
    return out


@pytest.mark.parametrize("rule", [0, 1, 2, "emulate", "random"])
def test_batch_plans_match_oracle(Q, S, small_batch, refs, rule):
    b = Q.Batch(small_batch)
    kinds, circ, nq = b.segment_info()
    assert set(kinds) == {0, 1, 2}
    opts = _options(kinds, rule, np.random.default_rng(5))
    b.set_plan(opts)
    ms, seg_us, norms, z0 = b.run()
    assert ms > 0 and (seg_us > 0).all()
    for c, ref in enumerate(refs):
        got = b.state(c).astype(np.complex128)
        assert np.abs(got - ref).max() < 1e-5, (rule, c, small_batch[c].n)
        assert abs(norms[c] - 1) < 1e-5
        zr = float(np.sum(np.abs(ref) ** 2 * (1 - 2 * (np.arange(ref.size) & 1))))
        assert abs(z0[c] - zr) < 1e-5
    b.free()


@pytest.mark.parametrize("fuse", [1, 2])
def test_modmul_gate_level_and_emulated_bit_identical(Q, S, small_batch, fuse):
    """Fused at k = 4 or 6, a gate-level modular multiplication's blocks are
    monomials (moves and phases), which stay on the exact ALU op also in
    circuits whose other dense blocks run on the matrix cores."""
    b = Q.Batch(small_batch)
    kinds, _, nq = b.segment_info()
    assert (kinds == 2).any() and (nq[kinds == 2] >= 14).any()
    base = _options(kinds, fuse)       # every segment fused at k = 4 (1) or 6 (2)
    emu = base.copy()
    emu[kinds == 2] = 3                # modmul emulated
    b.set_plan(base)
    b.run()
    s_gate = [b.state(c) for c in range(len(small_batch))]
    b.set_plan(emu)
    b.run()
    for c in range(len(small_batch)):
        assert np.array_equal(b.state(c).view(np.uint8), s_gate[c].view(np.uint8)), c
    b.free()


def test_batch_rejects_bad_plans(Q, S, small_batch):
    b = Q.Batch(small_batch[:3])
    kinds, _, _ = b.segment_info()
    with pytest.raises(Q.QSError):
        b.set_plan(np.full(len(kinds), 3, dtype=np.int32))   # emulate a plain gate list
    with pytest.raises(Q.QSError):
        b.set_plan(np.full(len(kinds), 7, dtype=np.int32))
    with pytest.raises(Q.QSError):
        b.run()                                              # no plan yet
    b.free()


def test_batch_features_shape_and_content(Q, S, small_batch):
    b = Q.Batch(small_batch)
    f = b.features()
    kinds, circ, nq = b.segment_info()
    assert f.shape == (b.n_segments, Q.QS_N_FEATURES)
    assert np.array_equal(f[:, 0], nq.astype(np.float32))
    assert np.array_equal(f[np.arange(len(kinds)), 3 + kinds], np.ones(len(kinds), dtype=np.float32))
    assert np.array_equal(f[:, 3:6].sum(1), np.ones(len(kinds), dtype=np.float32))
    assert (f[:, 17] >= f[:, 18]).all() and (f[:, 18] >= f[:, 19]).all()   # fewer blocks at larger k
    b.free()


def test_gangs_on_large_circuits_match_oracle(Q, O, S):
    """20-22 qubit circuits swept by gangs of 64-128 workgroups (one gang may
    be the whole grid when the batch is this small)."""
    circuits = S.batch_mix(3, 79, n_range=(20, 22), d_range=(3, 5), p_qft=0.3, p_modmul=0.3)
    b = Q.Batch(circuits)
    kinds, _, _ = b.segment_info()
    b.set_plan(_options(kinds, "random", np.random.default_rng(9)))
    _, _, norms, z0 = b.run()
    for c, circ in enumerate(circuits):
        ref = oracle_circuit(O, S, circ)
        got = b.state(c).astype(np.complex128)
        assert np.abs(got - ref).max() < 1e-5, (c, circ.n)
        assert abs(norms[c] - 1) < 1e-5
    b.free()


def test_batch_runs_are_bit_reproducible(Q, S, small_batch):
    """Gang members split every op over disjoint amplitudes and the norm
    partials are summed in member order, so two runs agree bit for bit."""
    b = Q.Batch(small_batch)
    kinds, _, _ = b.segment_info()
    b.set_plan(_options(kinds, 1))
    _, _, n1, z1 = b.run()
    s1 = [b.state(c) for c in range(len(small_batch))]
    _, _, n2, z2 = b.run()
    assert np.array_equal(n1, n2) and np.array_equal(z1, z2)
    for c in range(len(small_batch)):
        assert np.array_equal(b.state(c).view(np.uint8), s1[c].view(np.uint8)), c
    b.free()
