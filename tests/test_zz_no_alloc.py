"""The allocation-free Pauli expectation against qs_expectation, through
the C ABI: two calls in a row on one GPU (sharing the static scratch), the
second on a smaller state, for Z-only, X/Y and mixed Pauli strings."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-10}


def test_noalloc_expectation_matches_expectation(O, S):
    import torch
    from paper_1604_06460_amd import qs as Q
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    # (n, dtype, x, y, z): the second case of each dtype is smaller than the first
    cases = [(20, 1, 0b101, 0b1000, 0b10010), (11, 1, 0, 0, 0b1),
             (18, 0, 0b1, 0b110, 0), (9, 0, 0b100000000, 0, 0b1011)]
    for n, dtype, xm, ym, zm in cases:
        psi = S.normal_state(n, 90 + n)
        st = Q.State(n, dtype)
        st.set(psi)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        st.expectation_noalloc(out.data_ptr(), xm, ym, zm)
        st.sync()
        got = out.cpu().numpy()
        ref = st.expectation(xm, ym, zm)
        assert abs(got[0] - ref.real) <= TOL[dtype] and abs(got[1] - ref.imag) <= TOL[dtype], (n, got, ref)
        want = O.expectation(psi, xm, ym, zm)
        assert abs(complex(got[0], got[1]) - want) < TOL[dtype], (n, got, want)
        with pytest.raises(Q.QSError):
            st.expectation_noalloc(None, xm, ym, zm)
        with pytest.raises(Q.QSError):
            st.expectation_noalloc(out.data_ptr(), 1, 1, 0)
        st.free()
