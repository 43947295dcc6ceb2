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
QS_ARITH_MUL, QS_ARITH_DIV = 0, 1
QS_BLOCK_DENSE, QS_BLOCK_DIAGONAL, QS_BLOCK_IDENTITY = 0, 1, 2

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


class Segment(C.Structure):
    _fields_ = [("kind", _I), ("gates", Circuit), ("q_lo", _I), ("m", _I), ("inverse", _I),
                ("perm", Perm)]


class BatchCircuit(C.Structure):
    _fields_ = [("n_qubits", _I), ("n_segments", _I), ("segments", _P)]


QS_SEG_GATES, QS_SEG_QFT, QS_SEG_MODMUL = 0, 1, 2
QS_PLAN_K2, QS_PLAN_K4, QS_PLAN_K6, QS_PLAN_EMULATE = 0, 1, 2, 3
QS_N_FEATURES = 24


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
_sig("qs_run_program_range", [_P, _P, _I, _I])
_sig("qs_qpe_crossover_bits", [_D, _D, _D, _I, _I, C.POINTER(_I)])
_sig("qs_unitary_eig_residual", [_P, C.POINTER(_D)])
_sig("qs_mlp_set_range", [_P, _P, _P])
_sig("qs_expectation_noalloc", [_P, _U64, _U64, _U64, _P])
_sig("qs_mlp_choose_stats", [_P, _P])
_sig("qs_program_block_kind", [_P, _I, C.POINTER(_I), C.POINTER(_D)])
_sig("qs_program_free", [_P])
_sig("qs_apply_circuit", [_P, C.POINTER(Circuit), _I])
_sig("qs_emulate_qft", [_P, _I, _I, _I])
_sig("qs_emulate_permutation", [_P, C.POINTER(Perm)])
_sig("qs_emulate_arith", [_P, _I, _I, _I, _I, _I])
_sig("qs_norm2", [_P, C.POINTER(_D)])
_sig("qs_expectation", [_P, _U64, _U64, _U64, C.POINTER(_D), C.POINTER(_D)])
_sig("qs_measure", [_P, _I, _P, _I, _P, _P, _P, _I])
_sig("qs_batch_create", [_I, _P, _P, C.POINTER(_P)])
_sig("qs_batch_info", [_P, C.POINTER(_I), C.POINTER(_D)])
_sig("qs_batch_segment_info", [_P, _P, _P, _P])
_sig("qs_batch_features", [_P, _P])
_sig("qs_batch_set_plan", [_P, _P])
_sig("qs_batch_run", [_P, C.POINTER(_D), _P, _P, _P])
_sig("qs_batch_get_state", [_P, _I, _P])
_sig("qs_batch_trace", [_P, _I, C.POINTER(_I), _P, _P, _P, _P, _P])
_sig("qs_batch_free", [_P])
_sig("qs_mlp_create", [_P, _U64, _P, C.POINTER(_P)])
_sig("qs_mlp_get_params", [_P, _P])
_sig("qs_mlp_set_norm", [_P, _P, _P])
_sig("qs_mlp_forward", [_P, _I, _P, _P])
_sig("qs_mlp_loss_grad", [_P, _I, _P, _P, _P, C.POINTER(C.c_float), _P])
_sig("qs_mlp_adam_step", [_P, C.c_float])
_sig("qs_mlp_train", [_P, _I, _P, _P, _P, _I, _I, C.c_float, _U64, C.POINTER(C.c_float)])
_sig("qs_mlp_free", [_P])
_sig("qs_batch_choose", [_P, _I, _P, _P])

QS_MLP_PARAMS = 6020
QS_POLICY_HEURISTIC, QS_POLICY_LEARNED, QS_POLICY_FIXED_K2, QS_POLICY_FIXED_K4, QS_POLICY_FIXED_K6 = range(5)


class Mlp:
    """The 24-64-64-4 cost model; every computation runs in libqs kernels."""

    def __init__(self, params=None, seed=0, stream=None):
        h = _P()
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        _chk(_L.qs_mlp_create(_ptr(p), int(seed), stream, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def params(self):
        out = np.zeros(QS_MLP_PARAMS, dtype=np.float32)
        _chk(_L.qs_mlp_get_params(self._h, _ptr(out)))
        return out

    def set_norm(self, mean, inv_std):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(inv_std, dtype=np.float32)
        _chk(_L.qs_mlp_set_norm(self._h, _ptr(m), _ptr(s)))

    def set_range(self, lo, hi):
        """Training range of the raw features (None, None: no range check)."""
        if lo is None and hi is None:
            _chk(_L.qs_mlp_set_range(self._h, None, None))
            return
        a = np.ascontiguousarray(lo, dtype=np.float32)
        b = np.ascontiguousarray(hi, dtype=np.float32)
        _chk(_L.qs_mlp_set_range(self._h, _ptr(a), _ptr(b)))

    def choose_stats(self):
        """Segments of the last learned choice: learned, out of range,
        non-finite prediction, gain below the margin."""
        out = np.zeros(4, dtype=np.int32)
        _chk(_L.qs_mlp_choose_stats(self._h, _ptr(out)))
        return dict(zip(("learned", "fallback_range", "fallback_nonfinite", "fallback_margin"),
                        (int(v) for v in out)))

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros((x.shape[0], 4), dtype=np.float32)
        _chk(_L.qs_mlp_forward(self._h, x.shape[0], _ptr(x), _ptr(y)))
        return y

    def loss_grad(self, x, t, mask):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        mk = np.ascontiguousarray(mask, dtype=np.float32)
        g = np.zeros(QS_MLP_PARAMS, dtype=np.float32)
        loss = C.c_float()
        _chk(_L.qs_mlp_loss_grad(self._h, x.shape[0], _ptr(x), _ptr(t), _ptr(mk), C.byref(loss), _ptr(g)))
        return loss.value, g

    def adam_step(self, lr):
        _chk(_L.qs_mlp_adam_step(self._h, float(lr)))

    def train(self, x, t, mask, epochs, batch, lr, seed=0):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        mk = np.ascontiguousarray(mask, dtype=np.float32)
        loss = C.c_float()
        _chk(_L.qs_mlp_train(self._h, x.shape[0], _ptr(x), _ptr(t), _ptr(mk), int(epochs), int(batch),
                             float(lr), int(seed), C.byref(loss)))
        return loss.value

    def free(self):
        if self._h:
            _L.qs_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def choose(batch, policy, model=None):
    """Per-segment plan options for a Batch under a policy."""
    out = np.zeros(batch.n_segments, dtype=np.int32)
    _chk(_L.qs_batch_choose(batch._h, int(policy), model.handle if model is not None else None, _ptr(out)))
    return out


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
        """(block count, block widths, amplitude reads + writes per run)."""
        nb = _I(0)
        by = _D(0)
        _chk(_L.qs_program_info(self._h, C.byref(nb), None, C.byref(by)))
        ks = np.zeros(max(1, nb.value), dtype=np.int32)
        _chk(_L.qs_program_info(self._h, None, _ptr(ks), None))
        return nb.value, ks[:nb.value].copy(), by.value

    def block_kind(self, b):
        """(QS_BLOCK_* kind, fraction of amplitudes block b changes)."""
        kind, frac = _I(0), _D(0)
        _chk(_L.qs_program_block_kind(self._h, int(b), C.byref(kind), C.byref(frac)))
        return kind.value, frac.value

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

    def run_range(self, program, b0, b1):
        _chk(_L.qs_run_program_range(self._h, program.handle, int(b0), int(b1)))

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

    def emulate_mul(self, a_lo, b_lo, c_lo, m):
        """(a, b, c) -> (a, b, c + a*b mod 2^m) on three m-bit registers."""
        _chk(_L.qs_emulate_arith(self._h, QS_ARITH_MUL, int(a_lo), int(b_lo), int(c_lo), int(m)))

    def emulate_div(self, a_lo, b_lo, c_lo, m):
        """(a, b, 0) -> (a mod b, b, a div b) on three m-bit registers."""
        _chk(_L.qs_emulate_arith(self._h, QS_ARITH_DIV, int(a_lo), int(b_lo), int(c_lo), int(m)))

    def norm2(self):
        out = _D()
        _chk(_L.qs_norm2(self._h, C.byref(out)))
        return out.value

    def expectation_noalloc(self, device_out, x_mask=0, y_mask=0, z_mask=0):
        """qs_expectation_noalloc: (re, im) written to device_out (a device
        pointer to 2 doubles) on the state's stream; nothing is allocated."""
        _chk(_L.qs_expectation_noalloc(self._h, int(x_mask), int(y_mask), int(z_mask), device_out))

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


# ---------------------------------------------------------------------------
# Batches of independent complex64 circuits (one persistent launch)
# ---------------------------------------------------------------------------
class Batch:
    """circuits: objects with .n and .segments; each segment has .kind,
    .gates (gate list), and for QFT segments .q_lo/.m/.inverse, for modmul
    segments .modmul = (work_lo, w, ctrl_lo, c, a, N). Gate lists that are
    the same Python object are passed once."""

    def __init__(self, circuits, stream=None):
        packed = {}
        self._keep = []
        seg_arrays = []
        cs = (BatchCircuit * len(circuits))()
        for ci, c in enumerate(circuits):
            segs = (Segment * len(c.segments))()
            for si, s in enumerate(c.segments):
                key = id(s.gates)
                if key not in packed:
                    packed[key] = (PackedCircuit(s.gates), s.gates)
                pc = packed[key][0]
                segs[si].kind = int(s.kind)
                segs[si].gates = pc.c
                if s.kind == QS_SEG_QFT:
                    segs[si].q_lo, segs[si].m, segs[si].inverse = int(s.q_lo), int(s.m), int(bool(s.inverse))
                elif s.kind == QS_SEG_MODMUL:
                    wl, w, cl, cc, a, N = s.modmul
                    segs[si].perm = Perm(QS_PERM_MODMUL, int(wl), int(w), int(cl), int(cc), int(a), int(N), 0, 0, None)
            seg_arrays.append(segs)
            cs[ci].n_qubits = int(c.n)
            cs[ci].n_segments = len(c.segments)
            cs[ci].segments = C.cast(segs, _P)
        h = _P()
        _chk(_L.qs_batch_create(len(circuits), C.cast(cs, _P), stream, C.byref(h)))
        self._h = h
        self.n_circuits = len(circuits)
        self.ns = [int(c.n) for c in circuits]
        # the library copied everything it needs
        del packed, seg_arrays
        nseg, sb = _I(), _D()
        _chk(_L.qs_batch_info(h, C.byref(nseg), C.byref(sb)))
        self.n_segments = nseg.value
        self.state_bytes = sb.value

    def segment_info(self):
        kind = np.zeros(self.n_segments, dtype=np.int32)
        circ = np.zeros(self.n_segments, dtype=np.int32)
        nq = np.zeros(self.n_segments, dtype=np.int32)
        _chk(_L.qs_batch_segment_info(self._h, _ptr(kind), _ptr(circ), _ptr(nq)))
        return kind, circ, nq

    def features(self):
        f = np.zeros((self.n_segments, QS_N_FEATURES), dtype=np.float32)
        _chk(_L.qs_batch_features(self._h, _ptr(f)))
        return f

    def set_plan(self, options):
        o = np.ascontiguousarray(options, dtype=np.int32)
        if o.size != self.n_segments:
            raise ValueError("one option per segment")
        _chk(_L.qs_batch_set_plan(self._h, _ptr(o)))

    def run(self):
        ms = _D()
        seg = np.zeros(self.n_segments, dtype=np.float64)
        norms = np.zeros(self.n_circuits, dtype=np.float64)
        z0 = np.zeros(self.n_circuits, dtype=np.float64)
        _chk(_L.qs_batch_run(self._h, C.byref(ms), _ptr(seg), _ptr(norms), _ptr(z0)))
        return ms.value, seg, norms, z0

    def trace(self):
        """Schedule of the last run, one row per ticket in queue order:
        dict of start_us, end_us, circuit, member, workgroup arrays."""
        cnt = _I()
        _chk(_L.qs_batch_trace(self._h, 0, C.byref(cnt), None, None, None, None, None))
        n = cnt.value
        out = {"start_us": np.zeros(n), "end_us": np.zeros(n), "circuit": np.zeros(n, dtype=np.int32),
               "member": np.zeros(n, dtype=np.int32), "workgroup": np.zeros(n, dtype=np.int32)}
        _chk(_L.qs_batch_trace(self._h, n, C.byref(cnt), _ptr(out["start_us"]), _ptr(out["end_us"]),
                               _ptr(out["circuit"]), _ptr(out["member"]), _ptr(out["workgroup"])))
        return out

    def state(self, c):
        out = np.empty(1 << self.ns[c], dtype=np.complex64)
        _chk(_L.qs_batch_get_state(self._h, int(c), _ptr(out)))
        return out

    def free(self):
        if self._h:
            _L.qs_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Launch-parameter table
# ---------------------------------------------------------------------------
_sig("qs_tune_set", [_I, _I, _I, _I, _I, _I])
_sig("qs_tune_get", [_I, _I, _I, _I, _I, C.POINTER(_I)])
_sig("qs_tune_reset", [])
_sig("qs_tune_classify", [_I, _I, _I, _P, C.POINTER(_I), C.POINTER(_I)])

(QS_TUNE_SWEEP_PATH, QS_TUNE_SWEEP_WG_PER_CU, QS_TUNE_FFT_DIGIT, QS_TUNE_FFT_LDS_KB,
 QS_TUNE_MFMA_WG_PER_CU, QS_TUNE_BATCH_GANG_SHARE, QS_TUNE_BATCH_BARRIER_AMPS, QS_TUNE_FFT_KERNEL,
 QS_TUNE_SWEEP_NT, QS_TUNE_FFT_NT, QS_TUNE_GEMM_LIB, QS_TUNE_MODMUL_KERNEL, QS_TUNE_MFMA_KERNEL) = range(13)
QS_TCLS_SUBLINE, QS_TCLS_SUBWAVE, QS_TCLS_HIGH = range(3)
TUNE_PARAMS = {"sweep_path": QS_TUNE_SWEEP_PATH, "sweep_wg_per_cu": QS_TUNE_SWEEP_WG_PER_CU,
               "fft_digit": QS_TUNE_FFT_DIGIT, "fft_lds_kb": QS_TUNE_FFT_LDS_KB,
               "mfma_wg_per_cu": QS_TUNE_MFMA_WG_PER_CU, "batch_gang_share": QS_TUNE_BATCH_GANG_SHARE,
               "batch_barrier_amps": QS_TUNE_BATCH_BARRIER_AMPS, "fft_kernel": QS_TUNE_FFT_KERNEL,
               "sweep_nt": QS_TUNE_SWEEP_NT, "fft_nt": QS_TUNE_FFT_NT, "gemm_lib": QS_TUNE_GEMM_LIB,
               "modmul_kernel": QS_TUNE_MODMUL_KERNEL, "mfma_kernel": QS_TUNE_MFMA_KERNEL}
TUNED_FILE = os.path.join(_HERE, "tuned", "gfx950.json")


def tune_set(param, value, dtype=-1, k=-1, cls=-1, nbucket=-1):
    _chk(_L.qs_tune_set(int(param), int(dtype), int(k), int(cls), int(nbucket), int(value)))


def tune_get(param, dtype=QS_C64, k=0, cls=0, nbucket=0):
    v = _I()
    _chk(_L.qs_tune_get(int(param), int(dtype), int(k), int(cls), int(nbucket), C.byref(v)))
    return v.value


def tune_reset():
    _chk(_L.qs_tune_reset())


def tune_classify(dtype, n_qubits, targets):
    t = np.ascontiguousarray(targets, dtype=np.int32)
    cls, nb = _I(), _I()
    _chk(_L.qs_tune_classify(int(dtype), int(n_qubits), int(t.size), _ptr(t), C.byref(cls), C.byref(nb)))
    return cls.value, nb.value


def load_tuning(path=TUNED_FILE):
    """Apply a tuning table written by autotune.save (entries of param name,
    index fields with -1 for "all", and value). Returns the entry count."""
    import json
    with open(path) as f:
        doc = json.load(f)
    for e in doc["entries"]:
        tune_set(TUNE_PARAMS[e["param"]], e["value"], e.get("dtype", -1), e.get("k", -1),
                 e.get("cls", -1), e.get("nbucket", -1))
    return len(doc["entries"])


if os.path.exists(TUNED_FILE):
    load_tuning(TUNED_FILE)


# ---------------------------------------------------------------------------
# Dense unitaries and the controlled powers of phase estimation
# ---------------------------------------------------------------------------
_sig("qs_unitary_build", [C.POINTER(Circuit), _I, _I, _P, C.POINTER(_P)])
_sig("qs_unitary_info", [_P, C.POINTER(_I)])
_sig("qs_unitary_square", [_P])
_sig("qs_unitary_get", [_P, _P])
_sig("qs_apply_controlled_unitary", [_P, _P, _I])
_sig("qs_unitary_free", [_P])
_sig("qs_emulate_qpe_powers", [_P, C.POINTER(Circuit), _I, _I, _I, _I])
_sig("qs_unitary_eig", [_P])
_sig("qs_unitary_eig_get", [_P, _P, _P])
_sig("qs_apply_qpe_eig", [_P, _P, _I, _I])


class Unitary:
    """Dense 2^m x 2^m matrix of a gate list on qubits [0, m), on the device."""

    def __init__(self, gates, m, max_k=4, stream=None):
        pc = PackedCircuit(gates)
        h = _P()
        _chk(_L.qs_unitary_build(C.byref(pc.c), int(m), int(max_k), stream, C.byref(h)))
        self._h = h
        self.m = int(m)

    def square(self):
        _chk(_L.qs_unitary_square(self._h))

    def get(self):
        d = 1 << self.m
        out = np.empty((d, d), dtype=np.complex128)
        _chk(_L.qs_unitary_get(self._h, _ptr(out)))
        return out

    def apply_controlled(self, state, ctrl):
        _chk(_L.qs_apply_controlled_unitary(state.handle, self._h, int(ctrl)))

    def eig(self):
        """Eigendecomposition U = V diag(e^(i theta)) V^dagger on the device."""
        _chk(_L.qs_unitary_eig(self._h))

    def eig_residual(self):
        """Max off-diagonal magnitude of V^dagger U V from the last eig()."""
        out = _D(0)
        _chk(_L.qs_unitary_eig_residual(self._h, C.byref(out)))
        return out.value

    def eig_get(self):
        """(theta, V): eigenphases and eigenvectors (columns) on the host."""
        d = 1 << self.m
        th = np.empty(d)
        v = np.empty((d, d), dtype=np.complex128)
        _chk(_L.qs_unitary_eig_get(self._h, _ptr(th), _ptr(v)))
        return th, v

    def apply_qpe_eig(self, state, ctrl_lo, b):
        """Every controlled power U^c at once (c = control register value)."""
        _chk(_L.qs_apply_qpe_eig(state.handle, self._h, int(ctrl_lo), int(b)))

    def free(self):
        if self._h:
            _L.qs_unitary_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def emulate_qpe_powers(state, gates, m, ctrl_lo, b, max_k=4):
    """U^(2^j) controlled by qubit ctrl_lo + j for j < b, by repeated squaring."""
    pc = PackedCircuit(gates)
    _chk(_L.qs_emulate_qpe_powers(state.handle, C.byref(pc.c), int(m), int(ctrl_lo), int(b), int(max_k)))


def qpe_crossover_bits(t_apply, t_build, t_op, per_bit=True, bmax=200):
    """qs_qpe_crossover_bits (Table 2's rule); None if no b <= bmax."""
    out = _I(0)
    _chk(_L.qs_qpe_crossover_bits(float(t_apply), float(t_build), float(t_op), int(bool(per_bit)),
                                  int(bmax), C.byref(out)))
    return out.value or None
