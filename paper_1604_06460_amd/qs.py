"""Thin ctypes binding of libqs (include/qs.h): argument marshalling only.

Every operation on a state runs in the library's HIP kernels. There is no
fallback: if libqs.so has not been built, importing this module raises.
torch is imported first so that the library binds to the same HIP runtime
instance torch already loaded (both carry the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # share torch's HIP runtime when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libqs.so is not built: run `python -m paper_1604_06460_amd.build` "
                      "(or __graft_entry__.build()) first")

_L = C.CDLL(LIB_PATH)

QS_C64, QS_C128 = 0, 1
QS_OK, QS_EINVAL, QS_ENOMEM, QS_EDEVICE, QS_EUNSUPPORTED, QS_ENOTUNITARY = range(6)
QS_MAX_K = 6
QS_PERM_MODMUL, QS_PERM_TABLE = 0, 1

_P = C.c_void_p
_I = C.c_int
_U64 = C.c_uint64
_D = C.c_double


class Circuit(C.Structure):
    _fields_ = [("n_gates", _I), ("k", _P), ("targets", _P), ("matrices", _P),
                ("ctrl_mask", _P), ("ctrl_vals", _P)]


class Perm(C.Structure):
    _fields_ = [("kind", _I), ("work_lo", _I), ("w", _I), ("ctrl_lo", _I), ("c", _I),
                ("a", _U64), ("N", _U64), ("lo", _I), ("nbits", _I), ("dest", _P)]


def _sig(name, args, res=_I):
    f = getattr(_L, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("qs_last_error", [], C.c_char_p)
_sig("qs_version", [])
_sig("qs_alloc", [_I, _I, _P, _P, C.POINTER(_P)])
_sig("qs_free", [_P])
_sig("qs_info", [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(_P)])
_sig("qs_set_zero", [_P])
_sig("qs_get_state", [_P, _P])
_sig("qs_set_state", [_P, _P])
_sig("qs_sync", [_P])
_sig("qs_get_amplitudes", [_P, _I, _P, _P])
_sig("qs_load_device", [_P, _P])
_sig("qs_apply_gate", [_P, _I, _P, _P, _U64, _U64])
_sig("qs_apply_fused", [_P, _I, _P, _P, _P])
_sig("qs_plan_fusion", [C.POINTER(Circuit), _I, _I, C.POINTER(_I), _P, _P, _P])
_sig("qs_compile", [_P, C.POINTER(Circuit), _I, C.POINTER(_P)])
_sig("qs_program_info", [_P, C.POINTER(_I), _P, C.POINTER(_D)])
_sig("qs_program_block", [_P, _I, _P, _P])
_sig("qs_run_program", [_P, _P])
_sig("qs_program_free", [_P])
_sig("qs_apply_circuit", [_P, C.POINTER(Circuit), _I])
_sig("qs_emulate_qft", [_P, _I, _I, _I])
_sig("qs_emulate_permutation", [_P, C.POINTER(Perm)])
_sig("qs_norm2", [_P, C.POINTER(_D)])
_sig("qs_expectation", [_P, _U64, _U64, _U64, C.POINTER(_D), C.POINTER(_D)])
_sig("qs_measure", [_P, _I, _P, _I, _P, _P, _P, _I])


class QSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("qs status %d: %s" % (status, msg))
        self.status = status


def _chk(rc):
    if rc != QS_OK:
        raise QSError(rc, _L.qs_last_error().decode(errors="replace"))


def _ptr(a):
    return a.ctypes.data_as(_P) if a is not None else None


def lib():
    return _L


def last_error() -> str:
    return _L.qs_last_error().decode(errors="replace")


# ---------------------------------------------------------------------------
# Circuits
# ---------------------------------------------------------------------------
class PackedCircuit:
    """Keeps the flat arrays of a gate list alive next to their C view."""

    def __init__(self, gates):
        ks = np.array([len(g.targets) for g in gates], dtype=np.int32)
        tg = np.array([t for g in gates for t in g.targets], dtype=np.int32)
        mats = (np.concatenate([np.ascontiguousarray(g.matrix, dtype=np.complex128).reshape(-1)
                                for g in gates]).view(np.float64)
                if gates else np.zeros(2))
        cm = np.array([g.ctrl_mask for g in gates], dtype=np.uint64)
        cv = np.array([g.ctrl_vals for g in gates], dtype=np.uint64)
        self._keep = (ks, tg, np.ascontiguousarray(mats), cm, cv)
        self.c = Circuit(len(gates), _ptr(ks), _ptr(tg), _ptr(self._keep[2]), _ptr(cm), _ptr(cv))
        self.n_gates = len(gates)


def plan_fusion(gates, n_qubits, max_k):
    """Host-only fusion plan: (block_of_gate, [qubits of each block])."""
    pc = PackedCircuit(gates)
    ng = max(1, pc.n_gates)
    nb = _I(0)
    bog = np.zeros(ng, dtype=np.int32)
    bk = np.zeros(ng, dtype=np.int32)
    bq = np.zeros(ng * QS_MAX_K, dtype=np.int32)
    _chk(_L.qs_plan_fusion(C.byref(pc.c), n_qubits, max_k, C.byref(nb), _ptr(bog), _ptr(bk), _ptr(bq)))
    blocks = [list(bq[b * QS_MAX_K: b * QS_MAX_K + bk[b]]) for b in range(nb.value)]
    return bog[:pc.n_gates].copy(), blocks


class Program:
    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self):
        nb = _I(0)
        by = _D(0)
        _chk(_L.qs_program_info(self._h, C.byref(nb), None, C.byref(by)))
        ks = np.zeros(max(1, nb.value), dtype=np.int32)
        _chk(_L.qs_program_info(self._h, None, _ptr(ks), None))
        return nb.value, ks[:nb.value].copy(), by.value

    def block(self, b):
        nb, ks, _ = self.info()
        k = int(ks[b])
        m = np.zeros(2 << (2 * k), dtype=np.float64)
        q = np.zeros(k, dtype=np.int32)
        _chk(_L.qs_program_block(self._h, b, _ptr(m), _ptr(q)))
        return m.view(np.complex128).reshape(1 << k, 1 << k), q

    def free(self):
        if self._h:
            _L.qs_program_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# State handle
# ---------------------------------------------------------------------------
class State:
    """An n-qubit state on the current HIP device (QS_C128 or QS_C64)."""

    def __init__(self, n, dtype=QS_C128, device_buf=None, stream=None):
        h = _P()
        _chk(_L.qs_alloc(int(n), int(dtype), device_buf, stream, C.byref(h)))
        self._h = h
        self.n = int(n)
        self.dtype = int(dtype)

    @property
    def handle(self):
        return self._h

    @property
    def np_dtype(self):
        return np.complex128 if self.dtype == QS_C128 else np.complex64

    def free(self):
        if self._h:
            _chk(_L.qs_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        n, dt, p = _I(), _I(), _P()
        _chk(_L.qs_info(self._h, C.byref(n), C.byref(dt), C.byref(p)))
        return n.value, dt.value, p.value

    def set_zero(self):
        _chk(_L.qs_set_zero(self._h))

    def get(self):
        out = np.empty(1 << self.n, dtype=self.np_dtype)
        _chk(_L.qs_get_state(self._h, _ptr(out)))
        return out

    def set(self, psi):
        a = np.ascontiguousarray(psi, dtype=self.np_dtype)
        if a.size != 1 << self.n:
            raise ValueError("state must have 2^n entries")
        _chk(_L.qs_set_state(self._h, _ptr(a)))

    def load_device(self, device_ptr):
        _chk(_L.qs_load_device(self._h, device_ptr))

    def amplitudes(self, indices):
        idx = np.ascontiguousarray(indices, dtype=np.uint64)
        out = np.empty(idx.size, dtype=self.np_dtype)
        _chk(_L.qs_get_amplitudes(self._h, int(idx.size), _ptr(idx), _ptr(out)))
        return out

    def sync(self):
        _chk(_L.qs_sync(self._h))

    def apply_gate(self, targets, matrix, ctrl_mask=0, ctrl_vals=0):
        t = np.ascontiguousarray(targets, dtype=np.int32)
        m = np.ascontiguousarray(matrix, dtype=np.complex128).view(np.float64)
        _chk(_L.qs_apply_gate(self._h, int(t.size), _ptr(t), _ptr(m), int(ctrl_mask), int(ctrl_vals)))

    def apply_fused(self, blocks):
        """blocks: list of (targets, matrix)."""
        ks = np.array([len(t) for t, _ in blocks], dtype=np.int32)
        tg = np.array([q for t, _ in blocks for q in t], dtype=np.int32)
        ms = np.concatenate([np.ascontiguousarray(m, dtype=np.complex128).reshape(-1)
                             for _, m in blocks]).view(np.float64)
        _chk(_L.qs_apply_fused(self._h, len(blocks), _ptr(ks), _ptr(tg), _ptr(ms)))

    def apply_gates(self, gates):
        for g in gates:
            self.apply_gate(g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)

    def compile(self, gates, max_k):
        pc = PackedCircuit(gates)
        p = _P()
        _chk(_L.qs_compile(self._h, C.byref(pc.c), int(max_k), C.byref(p)))
        return Program(p)

    def run(self, program):
        _chk(_L.qs_run_program(self._h, program.handle))

    def apply_circuit(self, gates, max_k):
        pc = PackedCircuit(gates)
        _chk(_L.qs_apply_circuit(self._h, C.byref(pc.c), int(max_k)))

    def emulate_qft(self, q_lo=0, m=None, inverse=False):
        m = self.n - q_lo if m is None else m
        _chk(_L.qs_emulate_qft(self._h, int(q_lo), int(m), int(bool(inverse))))

    def emulate_modmul(self, work_lo, w, ctrl_lo, c, a, N):
        p = Perm(QS_PERM_MODMUL, int(work_lo), int(w), int(ctrl_lo), int(c), int(a), int(N), 0, 0, None)
        _chk(_L.qs_emulate_permutation(self._h, C.byref(p)))

    def emulate_table(self, lo, nbits, dest):
        d = np.ascontiguousarray(dest, dtype=np.uint64)
        p = Perm(QS_PERM_TABLE, 0, 0, 0, 0, 0, 0, int(lo), int(nbits), _ptr(d))
        _chk(_L.qs_emulate_permutation(self._h, C.byref(p)))

    def norm2(self):
        out = _D()
        _chk(_L.qs_norm2(self._h, C.byref(out)))
        return out.value

    def expectation(self, x_mask=0, y_mask=0, z_mask=0):
        re, im = _D(), _D()
        _chk(_L.qs_expectation(self._h, int(x_mask), int(y_mask), int(z_mask), C.byref(re), C.byref(im)))
        return complex(re.value, im.value)

    def measure(self, qubits, uniforms=(), collapse=False, want_probs=True):
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        outc = np.zeros(max(1, u.size), dtype=np.uint64)
        probs = np.zeros(1 << q.size) if want_probs else None
        _chk(_L.qs_measure(self._h, int(q.size), _ptr(q), int(u.size), _ptr(u) if u.size else None,
                           _ptr(outc), _ptr(probs), int(bool(collapse))))
        return outc[:u.size].copy(), probs
