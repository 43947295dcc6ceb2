"""CPU-only checks of the C ABI: the library loads, exports every entry point
include/*.h declares, rejects bad arguments on the host, and its fusion
planner (host logic) produces valid plans. No GPU call is made here."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(qs_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def test_header_declares_the_named_entry_points():
    names = set(_declared())
    for n in ("qs_alloc", "qs_apply_gate", "qs_apply_fused", "qs_emulate_qft",
              "qs_emulate_permutation", "qs_expectation", "qs_measure"):
        assert n in names


def test_library_exports_every_declared_symbol(Q):
    lib = Q.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_validation_without_gpu(Q):
    L = Q.lib()
    assert L.qs_apply_gate(None, 1, None, None, 0, 0) == Q.QS_EINVAL
    assert "handle" in Q.last_error()
    assert L.qs_emulate_qft(None, 0, 1, 0) == Q.QS_EINVAL
    assert L.qs_emulate_arith(None, 0, 0, 1, 2, 1) == Q.QS_EINVAL
    assert L.qs_norm2(None, None) == Q.QS_EINVAL
    h = C.c_void_p()
    assert L.qs_alloc(0, 1, None, None, C.byref(h)) == Q.QS_EINVAL
    assert L.qs_alloc(35, 1, None, None, C.byref(h)) == Q.QS_EINVAL
    assert L.qs_alloc(4, 7, None, None, C.byref(h)) == Q.QS_EINVAL
    assert L.qs_version() >= 10000


def _check_plan(gates, n, max_k, bog, blocks):
    assert len(bog) == len(gates)
    assert all(0 <= b < len(blocks) for b in bog)
    for b, qs in enumerate(blocks):
        members = [g for g in range(len(gates)) if bog[g] == b]
        assert members, "empty block"
        used = set().union(*[gates[g].qubits() for g in members])
        assert used == set(int(q) for q in qs)
        if len(members) > 1:
            assert len(qs) <= max_k
    # gates sharing a qubit keep their order across blocks
    for g2 in range(len(gates)):
        for g1 in range(g2):
            if gates[g1].qubits() & gates[g2].qubits():
                assert bog[g1] <= bog[g2]


@pytest.mark.parametrize("max_k", [1, 2, 3, 4, 6])
def test_fusion_plan_is_valid(Q, S, max_k):
    n = 12
    gates = S.random_layer_circuit(n, 8, seed=3) + S.qft_circuit(6, 3) + [S.mcx((0, 1), 2)]
    bog, blocks = Q.plan_fusion(gates, n, max_k)
    _check_plan(gates, n, max_k, bog, blocks)
    if max_k >= 2:
        assert len(blocks) < len(gates)


def test_fusion_plan_wide_gate_stands_alone(Q, S):
    gates = [S.g1(S.MAT_H, 0), S.Gate((0, 1, 2), np.eye(8)), S.g1(S.MAT_H, 1)]
    bog, blocks = Q.plan_fusion(gates, 4, 2)
    _check_plan(gates, 4, 2, bog, blocks)
    assert len(blocks) == 3


def test_fusion_block_count_for_the_30_qubit_circuit(Q, S):
    """The depth-30, 30-qubit random circuit (1350 gates) fuses into a few
    hundred 4-qubit blocks."""
    gates = S.random_layer_circuit(30, 30, seed=S.SEED_BASE + 1)
    bog, blocks = Q.plan_fusion(gates, 30, 4)
    assert len(gates) == 1350
    assert 150 <= len(blocks) <= 450
    assert max(len(b) for b in blocks) <= 4


def test_planner_rejects_bad_input(Q, S):
    with pytest.raises(Q.QSError):
        Q.plan_fusion([S.g1(S.MAT_H, 5)], 4, 2)
    with pytest.raises(Q.QSError):
        Q.plan_fusion([S.g1(S.MAT_H, 0)], 4, 7)


# ---------------------------------------------------------------------------
# Launch-parameter table (host only)
# ---------------------------------------------------------------------------
@pytest.fixture
def clean_tune(Q):
    Q.tune_reset()
    yield Q
    Q.tune_reset()
    if os.path.exists(Q.TUNED_FILE):
        Q.load_tuning()


def test_tune_table_set_get_and_wildcards(clean_tune):
    Q = clean_tune
    assert Q.tune_get(Q.QS_TUNE_SWEEP_PATH, Q.QS_C128, 4, 0, 2) == 0
    Q.tune_set(Q.QS_TUNE_SWEEP_PATH, 2, Q.QS_C128, 4, Q.QS_TCLS_SUBWAVE, 2)
    assert Q.tune_get(Q.QS_TUNE_SWEEP_PATH, Q.QS_C128, 4, Q.QS_TCLS_SUBWAVE, 2) == 2
    assert Q.tune_get(Q.QS_TUNE_SWEEP_PATH, Q.QS_C128, 4, Q.QS_TCLS_SUBWAVE, 1) == 0
    assert Q.tune_get(Q.QS_TUNE_SWEEP_PATH, Q.QS_C64, 4, Q.QS_TCLS_SUBWAVE, 2) == 0
    Q.tune_set(Q.QS_TUNE_FFT_DIGIT, 8)                      # every index
    for dt in (Q.QS_C64, Q.QS_C128):
        for nb in range(3):
            assert Q.tune_get(Q.QS_TUNE_FFT_DIGIT, dt, 0, 0, nb) == 8
    Q.tune_reset()
    assert Q.tune_get(Q.QS_TUNE_FFT_DIGIT, Q.QS_C64, 0, 0, 0) == 0


@pytest.mark.parametrize("args", [
    (99, -1, -1, -1, -1, 1),                   # unknown parameter
    (0, 7, -1, -1, -1, 1),                     # dtype
    (0, -1, 9, -1, -1, 1),                     # k
    (0, -1, -1, 3, -1, 1),                     # class
    (0, -1, -1, -1, 3, 1),                     # n bucket
    (0, -1, -1, -1, -1, 6),                    # path value
    (2, -1, -1, -1, -1, 11),                   # FFT digit
    (3, -1, -1, -1, -1, 200),                  # FFT LDS KiB
    (4, -1, -1, -1, -1, 17),                   # MFMA WG/CU
])
def test_tune_set_rejects_bad_arguments(clean_tune, args):
    Q = clean_tune
    with pytest.raises(Q.QSError):
        Q.tune_set(args[0], args[5], *args[1:5])
    assert Q.tune_get(Q.QS_TUNE_SWEEP_PATH, Q.QS_C64, 1, 0, 0) == 0


def test_tune_classes_and_buckets(Q):
    # lowest target inside a 128-byte line (8 c128 / 16 c64 amplitudes),
    # inside 64 amplitudes, or above
    assert Q.tune_classify(Q.QS_C128, 30, [2, 9]) == (Q.QS_TCLS_SUBLINE, 2)
    assert Q.tune_classify(Q.QS_C128, 30, [3, 9]) == (Q.QS_TCLS_SUBWAVE, 2)
    assert Q.tune_classify(Q.QS_C64, 25, [3, 9]) == (Q.QS_TCLS_SUBLINE, 1)
    assert Q.tune_classify(Q.QS_C64, 21, [4, 5]) == (Q.QS_TCLS_SUBWAVE, 0)
    assert Q.tune_classify(Q.QS_C64, 28, [6, 29]) == (Q.QS_TCLS_HIGH, 2)


def test_committed_tuning_table_is_valid(clean_tune):
    Q = clean_tune
    if not os.path.exists(Q.TUNED_FILE):
        pytest.skip("no tuned table committed")
    assert Q.load_tuning() > 0
