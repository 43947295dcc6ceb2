"""Autotuner for the launch-parameter table of libqs.

    python -m paper_1604_06460_amd.autotune [--quick] [--out FILE] [--no-batch]

Times candidate launch parameters on the current device and writes the JSON
table that the binding applies at import (qs.TUNED_FILE):

  * dense sweep path (registers / LDS-staged wave tiles / matrix cores /
    workgroup tiles with rows split over waves / shared 1024-amplitude
    tiles), its cache policy and the grid cap in workgroups per CU, per
    (dtype, k, class of the lowest target, n bucket); each path is timed
    with plain and with streaming accesses and keeps its better time;
  * FFT digit width and LDS tile budget per (dtype, n bucket);
  * persistent grid of the matrix-core sweep (complex64, k = 6);
  * batch gang sizing and barrier cost.

Every candidate is timed with HIP events on the state's stream around
repeated applications of the public entry points (median of `reps` timed
launches after a warm-up). A candidate replaces the built-in default only
when it is faster by more than `margin`, so timing noise does not flip
choices. All candidates compute the same result (they differ in launch
shape and summation order only); the GPU tests check every path against
the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import qs as Q

BUCKET_N = {Q.QS_C128: (20, 26, 30), Q.QS_C64: (20, 26, 30)}
# The cache policy changes only how lines are allocated, so its timings
# repeat closely (well under 1 % between runs) and a smaller margin than
# for launch shapes is enough to keep noise from flipping it.
NT_MARGIN = 0.01
DT_NAME = {Q.QS_C64: "c64", Q.QS_C128: "c128"}


def random_unitary(k, rng):
    """Haar-like 2^k x 2^k unitary (QR of a complex Gaussian matrix)."""
    d = 1 << k
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def class_targets(cls, k, n, dtype):
    """Two representative target sets whose lowest target is in class cls
    (tight low block and a spread one)."""
    lb = 3 if dtype == Q.QS_C128 else 4
    lo = {Q.QS_TCLS_SUBLINE: 0, Q.QS_TCLS_SUBWAVE: lb, Q.QS_TCLS_HIGH: 6}[cls]
    tight = list(range(lo, lo + k))
    spread = [lo] + [n - 1 - 3 * i for i in range(k - 1)]
    out = [tight]
    if len(set(spread)) == k and min(spread) == lo:
        out.append(sorted(spread))
    return out


class _Timer:
    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream

    def ms(self, fn, reps):
        torch = self.torch
        fn()
        self.stream.synchronize()
        out = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(self.stream)
            fn()
            e1.record(self.stream)
            e1.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))


def _pick(times, default_key, margin):
    """Best candidate, or the default unless the best beats it by margin."""
    best = min(times, key=times.get)
    if default_key in times and times[best] > (1.0 - margin) * times[default_key]:
        return default_key
    return best


def tune_sweep(timer, dtype, n, nb, reps, margin, log, rng):
    entries = []
    st = Q.State(n, dtype, stream=timer.stream.cuda_stream)
    for k in range(1, Q.QS_MAX_K + 1):
        if n < 6 + k:
            continue
        mat = random_unitary(k, rng)
        for cls in (Q.QS_TCLS_SUBLINE, Q.QS_TCLS_SUBWAVE, Q.QS_TCLS_HIGH):
            sets = class_targets(cls, k, n, dtype)
            paths = [1, 2] + ([3] if dtype == Q.QS_C64 and k >= 5 else []) + ([4] if k >= 5 else []) + \
                ([5] if 2 <= k <= 4 else [])
            if dtype == Q.QS_C128 and k == 6:
                paths = [1, 4]

            def run_sets():
                for t in sets:
                    st.apply_gate(t, mat)

            # each path is timed with plain and with streaming loads and
            # stores and keeps its better time: paths differ in how much the
            # cache policy is worth to them
            times = {}
            for p in paths + [0]:
                Q.tune_set(Q.QS_TUNE_SWEEP_PATH, p, dtype, k, cls, nb)
                tt = []
                for ntv in (0, 3):
                    Q.tune_set(Q.QS_TUNE_SWEEP_NT, ntv, dtype, k, cls, nb)
                    tt.append(timer.ms(run_sets, reps))
                times[p] = min(tt)
            Q.tune_set(Q.QS_TUNE_SWEEP_NT, 0, dtype, k, cls, nb)
            path = _pick(times, 0, margin)
            Q.tune_set(Q.QS_TUNE_SWEEP_PATH, path, dtype, k, cls, nb)
            entries.append({"param": "sweep_path", "dtype": dtype, "k": k, "cls": cls, "nbucket": nb,
                            "value": int(path), "ms": {str(a): round(b, 4) for a, b in times.items()}})
            # grid cap for the chosen path (the matrix-core path has its own,
            # the shared-tile path launches one workgroup per tile)
            tile_default = dtype == Q.QS_C128 and 2 <= k <= 4 and n >= 20
            gtimes = {}
            if path in (1, 2, 4) or (path == 0 and k <= 4 and not tile_default):
                for g in (0, 8, 32, 128):
                    Q.tune_set(Q.QS_TUNE_SWEEP_WG_PER_CU, g, dtype, k, cls, nb)
                    gtimes[g] = timer.ms(run_sets, reps)
                g = _pick(gtimes, 0, margin)
                Q.tune_set(Q.QS_TUNE_SWEEP_WG_PER_CU, g, dtype, k, cls, nb)
                entries.append({"param": "sweep_wg_per_cu", "dtype": dtype, "k": k, "cls": cls,
                                "nbucket": nb, "value": int(g),
                                "ms": {str(a): round(b, 4) for a, b in gtimes.items()}})
            # cache policy of the register, LDS-staged and shared-tile paths
            ntimes = {}
            if path in (1, 2, 5) or (path == 0 and k <= 4):
                for ntv in (0, 1, 2, 3):
                    Q.tune_set(Q.QS_TUNE_SWEEP_NT, ntv, dtype, k, cls, nb)
                    ntimes[ntv] = timer.ms(run_sets, reps)
                ntv = _pick(ntimes, 0, NT_MARGIN)
                Q.tune_set(Q.QS_TUNE_SWEEP_NT, ntv, dtype, k, cls, nb)
                entries.append({"param": "sweep_nt", "dtype": dtype, "k": k, "cls": cls, "nbucket": nb,
                                "value": int(ntv), "ms": {str(a): round(b, 4) for a, b in ntimes.items()}})
            log("sweep %s n=%d k=%d cls=%d: path %s %s grid %s nt %s" %
                (DT_NAME[dtype], n, k, cls, path, {a: round(b, 3) for a, b in times.items()},
                 {a: round(b, 3) for a, b in gtimes.items()}, {a: round(b, 3) for a, b in ntimes.items()}))
    st.free()
    return entries


def tune_fft(timer, dtype, n, nb, reps, margin, log):
    st = Q.State(n, dtype, stream=timer.stream.cuda_stream)
    times = {}
    # LDS-tile kernels over digit widths and tile budgets; the register-tile
    # kernels (10-bit digits, their own LDS use) once each
    cands = [(kern, digit, kb) for kern in (1, 2) for digit in (7, 8, 9, 10) for kb in (40, 80, 160)]
    cands += [(kern, 10, 80) for kern in (3, 4, 5)]
    for kern, digit, kb in cands:
        Q.tune_set(Q.QS_TUNE_FFT_KERNEL, kern, dtype, 0, 0, nb)
        Q.tune_set(Q.QS_TUNE_FFT_DIGIT, digit, dtype, 0, 0, nb)
        Q.tune_set(Q.QS_TUNE_FFT_LDS_KB, kb, dtype, 0, 0, nb)
        times[(kern, digit, kb)] = timer.ms(lambda: st.emulate_qft(0, n), reps)
    st.free()
    dflt = (4, 10, 80)
    best = _pick(times, dflt, margin)
    vals = best if best != dflt else (0, 0, 0)
    Q.tune_set(Q.QS_TUNE_FFT_KERNEL, vals[0], dtype, 0, 0, nb)
    Q.tune_set(Q.QS_TUNE_FFT_DIGIT, vals[1], dtype, 0, 0, nb)
    Q.tune_set(Q.QS_TUNE_FFT_LDS_KB, vals[2], dtype, 0, 0, nb)
    st = Q.State(n, dtype, stream=timer.stream.cuda_stream)
    ntimes = {}
    for ntv in (0, 1, 2, 3):
        Q.tune_set(Q.QS_TUNE_FFT_NT, ntv, dtype, 0, 0, nb)
        ntimes[ntv] = timer.ms(lambda: st.emulate_qft(0, n), reps)
    st.free()
    ntv = _pick(ntimes, 0, NT_MARGIN)
    Q.tune_set(Q.QS_TUNE_FFT_NT, ntv, dtype, 0, 0, nb)
    log("fft %s n=%d: best kernel %d digit %d lds %d KiB (%.3f ms; default %.3f ms); nt %d %s" %
        (DT_NAME[dtype], n, best[0], best[1], best[2], times[best], times[dflt], ntv,
         {a: round(b, 3) for a, b in ntimes.items()}))
    ms = {"%d/%d/%d" % a: round(b, 4) for a, b in times.items()}
    return [{"param": "fft_kernel", "dtype": dtype, "k": 0, "cls": 0, "nbucket": nb, "value": vals[0], "ms": ms},
            {"param": "fft_digit", "dtype": dtype, "k": 0, "cls": 0, "nbucket": nb, "value": vals[1]},
            {"param": "fft_lds_kb", "dtype": dtype, "k": 0, "cls": 0, "nbucket": nb, "value": vals[2]},
            {"param": "fft_nt", "dtype": dtype, "k": 0, "cls": 0, "nbucket": nb, "value": int(ntv),
             "ms": {str(a): round(b, 4) for a, b in ntimes.items()}}]


def tune_mfma(timer, n, nb, reps, margin, log, rng):
    st = Q.State(n, Q.QS_C64, stream=timer.stream.cuda_stream)
    mat = random_unitary(6, rng)
    sets = [[0, 1, 2, 3, 4, 5], [0, 7, 9, 13, 17, n - 1], [8, 9, 10, 11, 12, 13]]

    def run_sets():
        for t in sets:
            st.apply_gate(t, mat)

    # kernel first (each at its own default grid), then the grid for it
    ktimes = {}
    for kern in (5, 6, 3, 2, 4, 1):
        Q.tune_set(Q.QS_TUNE_MFMA_KERNEL, kern, Q.QS_C64, 6, 0, nb)
        ktimes[kern] = timer.ms(run_sets, reps)
    kbest = _pick(ktimes, 5, margin)
    Q.tune_set(Q.QS_TUNE_MFMA_KERNEL, kbest, Q.QS_C64, 6, 0, nb)
    times = {}
    for w in (1, 2, 3, 4, 6, 8):
        Q.tune_set(Q.QS_TUNE_MFMA_WG_PER_CU, w, Q.QS_C64, 6, 0, nb)
        times[w] = timer.ms(run_sets, reps)
    st.free()
    best = _pick(times, 4, margin)
    Q.tune_set(Q.QS_TUNE_MFMA_WG_PER_CU, best, Q.QS_C64, 6, 0, nb)
    log("mfma n=%d: kernel %d %s, %d WG/CU %s" % (n, kbest, {a: round(b, 3) for a, b in ktimes.items()}, best,
                                                 {a: round(b, 3) for a, b in times.items()}))
    return [{"param": "mfma_kernel", "dtype": Q.QS_C64, "k": 6, "cls": 0, "nbucket": nb, "value": int(kbest),
             "ms": {str(a): round(b, 4) for a, b in ktimes.items()}},
            {"param": "mfma_wg_per_cu", "dtype": Q.QS_C64, "k": 6, "cls": 0, "nbucket": nb, "value": int(best),
             "ms": {str(a): round(b, 4) for a, b in times.items()}}]


def tune_batch(circuits, reps, margin, log):
    b = Q.Batch(circuits)
    opts = Q.choose(b, Q.QS_POLICY_HEURISTIC)
    times = {}
    for share in (2, 4, 8, 16, 32):
        for bar in (1024, 4096, 16384):
            Q.tune_set(Q.QS_TUNE_BATCH_GANG_SHARE, share)
            Q.tune_set(Q.QS_TUNE_BATCH_BARRIER_AMPS, bar)
            b.set_plan(opts)
            b.run()
            times[(share, bar)] = float(np.median([b.run()[0] for _ in range(reps)]))
    b.free()
    best = _pick(times, (4, 4096), margin)
    Q.tune_set(Q.QS_TUNE_BATCH_GANG_SHARE, best[0])
    Q.tune_set(Q.QS_TUNE_BATCH_BARRIER_AMPS, best[1])
    log("batch (%d circuits): share %d barrier %d (%.2f ms; default %.2f ms)" %
        (len(circuits), best[0], best[1], times[best], times[(4, 4096)]))
    ms = {"%d/%d" % a: round(v, 3) for a, v in times.items()}
    return [{"param": "batch_gang_share", "value": int(best[0]), "ms": ms},
            {"param": "batch_barrier_amps", "value": int(best[1])}]


def autotune(quick=False, batch=True, reps=5, margin=0.03, log=print, seed=0):
    """Run every tuner on the current device; returns the table document.
    The table starts from the built-in defaults (it is reset first)."""
    import torch
    rng = np.random.default_rng(seed)
    Q.tune_reset()
    stream = torch.cuda.Stream()          # default priority
    timer = _Timer(stream)
    entries = []
    t0 = time.time()
    for dtype in (Q.QS_C128, Q.QS_C64):
        ns = BUCKET_N[dtype][-1:] if quick else BUCKET_N[dtype]
        for n in ns:
            nb = Q.tune_classify(dtype, n, [0])[1]
            entries += tune_sweep(timer, dtype, n, nb, reps, margin, log, rng)
            entries += tune_fft(timer, dtype, n, nb, max(3, reps // 2), margin, log)
            if dtype == Q.QS_C64:
                entries += tune_mfma(timer, n, nb, reps, margin, log, rng)
            torch.cuda.empty_cache()
    if batch:
        from synth import circuits as S
        circuits = S.batch_mix(256 if quick else 1024, S.SEED_BASE * 1000 + 900000)
        entries += tune_batch(circuits, 3, margin, log)
    props = torch.cuda.get_device_properties(0)
    return {"device": getattr(props, "gcnArchName", "gfx950"), "name": props.name,
            "tuned_s": round(time.time() - t0, 1), "margin": margin, "reps": reps, "entries": entries}


def save(doc, path=Q.TUNED_FILE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="largest n bucket only, smaller batch")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=Q.TUNED_FILE)
    a = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    doc = autotune(quick=a.quick, batch=not a.no_batch, reps=a.reps, log=log)
    save(doc, a.out)
    log("wrote %d entries to %s" % (len(doc["entries"]), a.out))


if __name__ == "__main__":
    main()
