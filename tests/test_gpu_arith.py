"""Integer multiplication and division into a third register (Sec. III-A):
the emulated permutation against the oracle, bit for bit, and against the
gate-level Toffoli networks (Cuccaro adders) that a simulator runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MUL, DIV = 0, 1


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def _emulate(st, kind, lo, m):
    (st.emulate_mul if kind == MUL else st.emulate_div)(*lo, m)


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint8)


# (m, (a_lo, b_lo, c_lo), n): register orders, spectator qubits below, between
# and above the registers; m = 7 and 8 with c above bit 3 take the LDS-tiled
# multiplication kernel (a tile of 2^(m+3) complex128 or 2^(m+4) complex64);
# a above c with b above bit 3 takes the b-major output order of division.
CASES = [
    (1, (0, 1, 2), 3),
    (2, (4, 2, 0), 6),
    (3, (0, 3, 6), 9),
    (3, (2, 8, 5), 12),
    (4, (0, 4, 8), 12),
    (5, (5, 10, 0), 16),
    (4, (9, 4, 0), 14),
    (6, (12, 6, 0), 18),
    (6, (0, 6, 12), 18),
    (7, (0, 7, 14), 21),
    (7, (1, 9, 16), 23),
    (8, (0, 8, 16), 24),
]


@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("kind", [MUL, DIV])
@pytest.mark.parametrize("m,lo,n", CASES)
def test_emulated_arith_vs_oracle_bit_exact(Q, O, S, dtype, kind, m, lo, n):
    """A seeded normal state over all n qubits (so c != 0 too): every output
    amplitude is the input amplitude the oracle's map sends there."""
    st = Q.State(n, dtype)
    st.set(S.normal_state(n, 40 + m + n))
    before = st.get()
    _emulate(st, kind, lo, m)
    ref = O.arith(before, kind, *lo, m)
    assert np.array_equal(_bits(st.get()), _bits(ref))
    st.free()


@pytest.mark.parametrize("kind", [MUL, DIV])
@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_gate_level_network_equals_emulation(Q, S, kind, m):
    """The Cuccaro multiplier / restoring divider applied gate by gate on
    3m + 1 qubits equals the emulated permutation on the same state bit for
    bit (every gate is an X with controls: amplitudes only move); the
    network compiled into fused 4-qubit blocks agrees to rounding."""
    aq, bq, cq, anc = S.arith_layout(m)
    net = (S.mul_gate_circuit_on if kind == MUL else S.div_gate_circuit_on)(aq, bq, cq, anc)
    psi = S.arith_input_state(m, 50 + m, extra=1)
    sim = Q.State(3 * m + 1, Q.QS_C128)
    sim.set(psi)
    sim.apply_gates(net)
    emu = Q.State(3 * m + 1, Q.QS_C128)
    emu.set(psi)
    _emulate(emu, kind, (aq[0], bq[0], cq[0]), m)
    assert np.array_equal(_bits(sim.get()), _bits(emu.get()))
    fused = Q.State(3 * m + 1, Q.QS_C128)
    fused.set(psi)
    fused.apply_circuit(net, 4)
    assert np.abs(fused.get() - emu.get()).max() < 1e-12
    for s in (sim, emu, fused):
        s.free()


def test_division_reads_quotient_and_remainder(Q, S):
    """A basis state (a, b, 0): the output is the basis state
    (a mod b, b, a div b)."""
    m = 6
    st = Q.State(3 * m, Q.QS_C64)
    for a, b in ((45, 7), (63, 1), (5, 9), (0, 3), (17, 0)):
        psi = np.zeros(1 << (3 * m), dtype=np.complex64)
        psi[a | (b << m)] = 1
        st.set(psi)
        st.emulate_div(0, m, 2 * m, m)
        out = st.get()
        q, r = divmod(a, b) if b else ((1 << m) - 1, a)
        assert out[r | (b << m) | (q << (2 * m))] == 1 and np.count_nonzero(out) == 1
    st.free()


@pytest.mark.parametrize("lo", [(20, 10, 0), (0, 10, 20)])
@pytest.mark.parametrize("kind", [MUL, DIV])
def test_30q_arith_sampled_bit_exact(Q, O, S, kind, lo):
    """The benchmark's size: three 10-bit registers of a 30-qubit complex128
    state drawn on the GPU (c != 0 too), in the benchmark's layout (c on the
    low qubits: the plain gather for both maps) and with c on top (the
    LDS-tiled multiplication). For 4096 sampled inputs i the output at the
    oracle's destination of i is the input amplitude, bit for bit; the norm
    is unchanged."""
    import torch
    n, m = 30, 10
    gen = torch.Generator(device="cuda")
    gen.manual_seed(S.SEED_BASE + 3)
    x = torch.randn(1 << n, dtype=torch.complex128, device="cuda", generator=gen)
    st = Q.State(n, Q.QS_C128)
    st.load_device(x.data_ptr())
    n0 = st.norm2()
    _emulate(st, kind, lo, m)
    idx = np.random.default_rng(17).integers(0, 1 << n, 4096).astype(np.uint64)
    idx[:4] = [0, (1 << n) - 1, (1 << (2 * m)) - 1, 5 | (3 << m)]
    dest = O.arith_dest(idx, kind, *lo, m)
    want = x[torch.from_numpy(idx.astype(np.int64)).to("cuda")].cpu().numpy()
    assert np.array_equal(_bits(st.amplitudes(dest)), _bits(want))
    assert abs(st.norm2() - n0) < 1e-9 * n0
    st.free()
    del x
    torch.cuda.empty_cache()


def test_arith_rejects_bad_registers_and_leaves_the_state(Q, S):
    st = Q.State(9, Q.QS_C128)
    st.set(S.normal_state(9, 3))
    before = st.get()
    for args in ((0, 3, 6, 4), (0, 2, 6, 3), (0, 3, 7, 3), (-1, 3, 6, 3), (0, 3, 6, 0)):
        with pytest.raises(Q.QSError):
            st.emulate_mul(*args)
    assert Q.lib().qs_emulate_arith(st.handle, 2, 0, 3, 6, 3) == Q.QS_EINVAL
    assert np.array_equal(_bits(st.get()), _bits(before))
    st.free()
