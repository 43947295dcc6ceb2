#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline]

Workload (30 qubits, complex128, inputs resident in HBM):
  * a depth-30 random circuit (Haar 2x2 on every qubit, then CZ on 15
    disjoint pairs, per layer; 1350 gates) from |0...0>, planned and composed
    in FP64 into k=4 blocks and applied as dense sweeps, then <Z_0> and the
    norm;
  * the full 30-qubit QFT on a seeded normal state, gate-level (30 H, 435
    conditional phase shifts, 15 SWAPs) and then undone by the emulated
    inverse QFT (in-place multi-pass FFT);
  * controlled modular multiplication emulated as a permutation (20-bit
    work register, 8-bit control register);
  * marginals and sampling on the 8 control qubits.
One step runs all of it. `value` is the algorithmic HBM bytes the step
moves divided by the step time. The JSON line also carries the roofline of
the dominant kernel (the k=4 dense sweep) timed with HIP events on the
library's stream, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
N_QUBITS = 30
DEPTH = 30
MAX_K = 4


def qft_gate_bytes(n, amp):
    """Algorithmic bytes of the gate-level QFT: H reads+writes every
    amplitude, a conditional phase shift a quarter of them, a SWAP half."""
    N = float(1 << n)
    n_cr = n * (n - 1) // 2
    return n * 2 * amp * N + n_cr * 2 * amp * N / 4 + (n // 2) * 2 * amp * N / 2


T_START = time.perf_counter()


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench %6.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per launch of the dense sweep from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (scaled by a plain copy of known size), or
    None if the sweep source changed since the counters were taken."""
    import hashlib
    rec = os.path.join(ROOT, "profiles", "dense_sweep_c128_30q_pmc.json")
    src = os.path.join(ROOT, "paper_1604_06460_amd", "csrc", "sweep.hip")
    try:
        d = json.load(open(rec))
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return d["traffic_bytes_per_launch"] if h == d.get("sweep_hip_sha256_prefix") else None


def host_info():
    """CPU model and RAM of the host the oracle runs on."""
    model, ram = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) * 1024 / 2 ** 30, 1)
                break
    except OSError:
        pass
    return model, ram


def cpu_baseline(n, gates, budget_s=12.0, budget_1t_s=10.0):
    """The CPU oracle (plain gate-by-gate FP64 simulator) applying the first
    gates of the same circuit to |0...0>; stops after ~budget_s seconds.
    Run once with every host thread OpenMP gives it and once with one."""
    from oracle import oracle as O

    def run(budget):
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1.0
        done = 0
        t0 = time.perf_counter()
        while done < len(gates) and (done < 2 or time.perf_counter() - t0 < budget):
            g = gates[done]
            O.apply_gate(psi, g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
            done += 1
        dt = time.perf_counter() - t0
        del psi
        return done, dt, done * 2 * 16 * float(1 << n) / dt / 1e9

    cores = O.set_threads(0)
    done, dt, gbs = run(budget_s)
    O.set_threads(1)
    done1, dt1, gbs1 = run(budget_1t_s)
    O.set_threads(cores)
    model, ram = host_info()
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": "first %d gates (unfused, one sweep each) of the depth-%d %d-qubit circuit "
                      "from |0...0>, complex128, %.1f s on %d threads" % (done, DEPTH, n, dt, cores),
            "single_thread": {"value": round(gbs1, 3), "unit": "GB/s", "cores": 1,
                              "sample": "first %d gates of the same circuit, %.1f s" % (done1, dt1)},
            "cpu_model": model, "ram_gib": ram, "host_logical_cpus": os.cpu_count()}


def config0_gate_level(Q, S):
    """16 qubits, complex128, |0...0>, depth-20 random circuit applied gate
    by gate (480 gates), then <Z_0>: wall time per circuit, host launches
    included (synchronised before and after). The same circuit fused into
    blocks of up to 4 qubits is timed too. The final state and <Z_0> are
    compared with the oracle."""
    from oracle import oracle as O
    n, depth = 16, 20
    gates = S.random_layer_circuit(n, depth, seed=S.SEED_BASE)
    st = Q.State(n, Q.QS_C128)

    def gate_level():
        st.set_zero()
        st.apply_gates(gates)
        return st.expectation(z_mask=1).real

    def fused():
        st.set_zero()
        prog = st.compile(gates, 4)
        st.run(prog)
        z = st.expectation(z_mask=1).real
        prog.free()
        return z

    out = {"n_qubits": n, "depth": depth, "gates": len(gates), "dtype": "c128"}
    for name, fn in (("gate_level", gate_level), ("fused_k4", fused)):
        fn()
        st.sync()
        ts = []
        for _ in range(20):
            t0 = time.perf_counter()
            z = fn()
            ts.append((time.perf_counter() - t0) * 1e3)
        out[name + "_ms_per_circuit"] = round(float(np.median(ts)), 4)
        out[name + "_z0"] = z
    ref = O.apply_circuit(S.zero_state(n), gates)
    gate_level()
    out["max_abs_err_vs_oracle"] = float(np.abs(st.get() - ref).max())
    out["z0_oracle"] = float(O.expectation(ref, z_mask=1).real)
    st.free()
    log("c0 16q gate-level: %.3f ms per circuit, fused %.3f ms"
        % (out["gate_level_ms_per_circuit"], out["fused_k4_ms_per_circuit"]))
    return out


def config2_modmul28(Q, S):
    """28-qubit complex128 state: 20-bit work register (qubits 0..19) in a
    seeded normal state with distinct amplitudes, 8-bit control register
    (qubits 20..27) in uniform superposition; |c>|x> -> |c>|a^c x mod N>
    emulated as an index permutation. Timed with HIP events on the state's
    stream; 4096 sampled outputs are checked bit for bit against the
    oracle's per-index source map."""
    import torch
    from oracle import oracle as O
    n, w, c = 28, 20, 8
    a, N = S.modmul_params(w, S.SEED_BASE + 2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(S.SEED_BASE + 2)
        v = torch.randn(1 << w, dtype=torch.complex128, device="cuda", generator=gen)
        v /= torch.linalg.vector_norm(v) * (2.0 ** (c / 2))
        x = v.repeat(1 << c)
    stream.synchronize()
    st = Q.State(n, Q.QS_C128, stream=stream.cuda_stream)
    st.load_device(x.data_ptr())
    st.sync()
    st.emulate_modmul(0, w, w, c, a, N)          # warm: scratch buffer, code objects
    st.load_device(x.data_ptr())
    reps = 10
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    evs[0].record(stream)
    for r in range(reps):
        st.emulate_modmul(0, w, w, c, a, N)
        evs[r + 1].record(stream)
    stream.synchronize()
    ms = [evs[r].elapsed_time(evs[r + 1]) for r in range(reps)]
    avg = float(np.mean(ms))
    # check one application to the resident input
    st.load_device(x.data_ptr())
    st.emulate_modmul(0, w, w, c, a, N)
    idx = np.random.default_rng(5).integers(0, 1 << n, 4096).astype(np.uint64)
    got = st.amplitudes(idx)
    src = O.modmul_source(idx, 0, w, w, c, a, N).astype(np.int64)
    ref = x[torch.from_numpy(src).to("cuda")].cpu().numpy()
    exact = bool(np.array_equal(got.view(np.uint64), ref.view(np.uint64)))
    st.free()
    del x, v
    torch.cuda.empty_cache()
    byts = 2 * 16 * float(1 << n)
    log("c2 28q modmul: %.3f ms (%.0f GB/s), sampled bit-exact %s" % (avg, byts / avg / 1e6, exact))
    return {"n_qubits": n, "work_bits": w, "ctrl_bits": c, "a": a, "N": N, "dtype": "c128",
            "avg_ms": round(avg, 4), "gbs": round(byts / (avg * 1e-3) / 1e9, 1),
            "frac_of_hbm_peak": round(byts / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_launch": byts, "samples_bit_exact": exact, "samples": int(idx.size)}


def config3_mfma32(Q, S):
    """32 qubits complex64, depth-40 random circuit fused into blocks of up
    to 6 qubits; 6- and 5-qubit blocks run on the FP32 matrix cores. The
    complex work is 512 N and 256 N flop per launch (8 flop per complex
    multiply-add); the three-product form executes 3/4 of it on the matrix
    cores. Per-block HIP events on the state's
    stream give the matrix-core kernel's average launch time; the norm is
    accumulated in FP64. The same generator at 22 qubits (the twin) runs on
    the GPU in complex64 and on the FP64 oracle for the error."""
    import torch
    from oracle import oracle as O
    n, depth, k = 32, 40, 6
    gates = S.random_layer_circuit(n, depth, seed=S.SEED_BASE + 3)
    stream = torch.cuda.Stream()
    st = Q.State(n, Q.QS_C64, stream=stream.cuda_stream)
    prog = st.compile(gates, k)
    nb, ks, moves = prog.info()
    kinds = [prog.block_kind(b)[0] for b in range(nb)]
    st.run(prog)                               # warm
    st.set_zero()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 1)]
    evs[0].record(stream)
    for b in range(nb):
        st.run_range(prog, b, b + 1)
        evs[b + 1].record(stream)
    stream.synchronize()
    ms = np.array([evs[b].elapsed_time(evs[b + 1]) for b in range(nb)])
    nrm = st.norm2()
    mfma = [b for b in range(nb) if ks[b] == 6 and kinds[b] == Q.QS_BLOCK_DENSE]
    mfma5 = [b for b in range(nb) if ks[b] == 5 and kinds[b] == Q.QS_BLOCK_DENSE]
    N = float(1 << n)
    t_mfma = float(np.mean(ms[mfma]))
    t_mfma5 = float(np.mean(ms[mfma5])) if mfma5 else 0.0
    flop = 512.0 * N
    tflops = flop / (t_mfma * 1e-3) / 1e12
    prog.free()
    st.free()
    torch.cuda.empty_cache()
    # 22-qubit twin against the FP64 oracle
    nt = 22
    tg = S.random_layer_circuit(nt, depth, seed=S.SEED_BASE + 3)
    tw = Q.State(nt, Q.QS_C64)
    tw.apply_circuit(tg, k)
    got = tw.get().astype(np.complex128)
    tw.free()
    ref = O.apply_circuit(S.zero_state(nt), tg)
    err = float(np.abs(got - ref).max())
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    fid = float(abs(np.vdot(ref, got)) ** 2)
    log("c3 32q c64 k=6: %d blocks (%d 6-qubit and %d 5-qubit on matrix cores), %.2f ms per 6-qubit launch "
        "(%.1f TFLOP/s), %.2f ms per 5-qubit launch, twin err %.2e" % (nb, len(mfma), len(mfma5), t_mfma, tflops,
                                                                       t_mfma5, err))
    return {"n_qubits": n, "depth": depth, "fusion_k": k, "dtype": "c64", "blocks": nb,
            "mfma_blocks": len(mfma), "circuit_ms": round(float(ms.sum()), 2),
            "mfma_avg_launch_ms": round(t_mfma, 4),
            "mfma5_blocks": len(mfma5), "mfma5_avg_launch_ms": round(t_mfma5, 4),
            "mfma5_tflops": round(256.0 * N / (t_mfma5 * 1e-3) / 1e12, 2) if mfma5 else None,
            "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 157.3, "unit": "TFLOP/s",
                         "frac": round(tflops / 157.3, 4), "flop_per_launch": flop,
                         "matrix_core_flop_per_launch": 0.75 * flop,
                         "matrix_core_tflops": round(0.75 * tflops, 2),
                         "hbm_gbs": round(2 * 8 * N / (t_mfma * 1e-3) / 1e9, 1),
                         "kernel": "k_dense_mfma_3m<u64,6> (v_mfma_f32_16x16x4f32, 6-qubit blocks, three real "
                                   "products per complex product)"},
            "norm_fp64": nrm,
            "twin": {"n_qubits": nt, "max_abs_err": err, "rel_l2": rel, "fidelity": fid}}


def batch_learned(Q, S):
    """4096 uneven circuits (n ~ U{10..22}, depth ~ U{10..60}; random
    layers, QFTs, modular multiplications) in one persistent launch per
    policy. The cost model is trained on in-kernel segment timings of a
    disjoint 512-circuit batch run under the plain policies and 12
    perturbations of them; every policy is timed on the 4096-circuit batch
    (median of 3 launches), and the learned plan's states are checked
    against the oracle on sampled circuits."""
    from oracle import oracle as O
    from paper_1604_06460_amd import learn
    t0 = time.perf_counter()
    train = Q.Batch(S.batch_mix(512, S.SEED_BASE * 1000 + 500000))
    log("training batch created: %d segments" % train.n_segments)
    X, T, mask = learn.collect(train, runs=12, seed=1, log=log)
    train.free()
    model, loss = learn.fit(X, T, mask, epochs=60)
    t_train = time.perf_counter() - t0
    log("cost model trained: %d rows, loss %.4f" % (X.shape[0], loss))
    circuits = S.batch_mix(4096, S.SEED_BASE + 4)
    log("4096-circuit batch generated")
    ev = Q.Batch(circuits)
    log("4096-circuit batch created: %d segments, %.1f GB of states" % (ev.n_segments, ev.state_bytes / 1e9))
    res, plans = learn.wall_times(ev, model, repeats=3, log=log)
    ratio, best = learn.learned_vs_plain(res)
    ev.set_plan(plans["learned"])
    ev.run()
    err = 0.0
    checked = 0
    for c in range(0, len(circuits), 97):
        if circuits[c].n <= 16:
            psi = S.zero_state(circuits[c].n)
            for s in circuits[c].segments:
                if s.kind == S.SEG_QFT:
                    psi = O.dft_numpy(psi, s.q_lo, s.m, s.inverse)
                elif s.kind == S.SEG_MODMUL:
                    psi = O.modmul(psi, *s.modmul)
                else:
                    psi = O.apply_circuit(psi, s.gates)
            err = max(err, float(np.abs(ev.state(c).astype(np.complex128) - psi).max()))
            checked += 1
    ev.free()
    model.free()
    return {"circuits": len(circuits), "segments": int(len(plans["learned"])),
            "wall_ms": {k: round(v, 2) for k, v in res.items()},
            "learned_vs_best_plain": round(ratio, 4), "best_plain": best,
            "circuits_per_s_learned": round(len(circuits) / (res["learned"] * 1e-3), 1),
            "train_rows": int(X.shape[0]), "train_loss": round(float(loss), 5),
            "train_s": round(t_train, 1),
            "max_abs_err_vs_oracle": err, "circuits_checked": checked}


def qpe_table(Q, S, ms=(8, 9, 10, 11, 12, 13, 14)):
    """Phase estimation of a 1D transverse-field Ising Trotter step (4m-3
    gates) on m qubits, the example of Table 2, timed on this GPU:
    applying controlled U once to an (m+1)-qubit state,
    building the dense U, one FP64 squaring, the eigendecomposition; the
    crossover precisions follow from the rule behind Table 2. Then one whole b-bit estimate both ways at
    m = 10, b = 10 (state of 20 qubits): the controlled powers simulated
    (2^b - 1 runs of U) against the emulated ones (squaring, and the
    eigensolver route), each followed by the emulated inverse QFT. Simulation runs U as a program fused into blocks of
    up to 4 qubits, the simulator's fastest form."""
    import torch
    out = {"unit": "ms", "rows": []}
    stream = torch.cuda.Stream()

    def timed(fn, reps=3):
        fn()
        stream.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    for m in ms:
        gates = S.tfim_trotter_step(m)
        ctl = [S.Gate(g.targets, g.matrix, g.ctrl_mask | (1 << m), g.ctrl_vals | (1 << m)) for g in gates]
        st = Q.State(m + 1, Q.QS_C128, stream=stream.cuda_stream)
        prog = st.compile(ctl, 4)
        t_apply = timed(lambda: st.run(prog))
        prog.free()
        st.free()
        t_build = timed(lambda: Q.Unitary(gates, m, 4, stream=stream.cuda_stream).free(), reps=2)
        u = Q.Unitary(gates, m, 4, stream=stream.cuda_stream)
        t_sq = timed(u.square, reps=2)
        Q.tune_set(Q.QS_TUNE_GEMM_LIB, 1)          # rocBLAS zgemm as the baseline
        t_sq_lib = timed(u.square, reps=2)
        Q.tune_set(Q.QS_TUNE_GEMM_LIB, 0)
        u.free()
        u = Q.Unitary(gates, m, 4, stream=stream.cuda_stream)
        eig_err = None
        try:
            t_eig = timed(u.eig, reps=1)
            resid = u.eig_residual()
        except Q.QSError as e:              # an unresolved mirror cluster
            t_eig, resid, eig_err = float("nan"), u.eig_residual(), str(e)
        u.free()
        torch.cuda.empty_cache()
        flop = 8.0 * float(1 << m) ** 3
        row = {"m": m, "gates": len(gates), "t_apply_ms": round(t_apply, 4),
               "t_build_ms": round(t_build, 4), "t_square_ms": round(t_sq, 4),
               "square_tflops": round(flop / (t_sq * 1e-3) / 1e12, 2),
               "square_frac_fp64_peak": round(flop / (t_sq * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
               "t_square_rocblas_ms": round(t_sq_lib, 4),
               "t_eig_ms": round(t_eig, 3), "eig_residual": resid,
               "crossover_bits_squaring": Q.qpe_crossover_bits(t_apply, t_build, t_sq, True),
               "crossover_bits_eig": (Q.qpe_crossover_bits(t_apply, t_build, t_eig, False)
                                      if eig_err is None else None)}
        if eig_err is not None:
            row["eig_error"] = eig_err
        out["rows"].append(row)
        log("qpe m=%d: apply %.3f ms, build %.3f ms, square %.3f ms (%.1f TFLOP/s; rocBLAS %.3f ms), eig %.1f ms"
            % (m, t_apply, t_build, t_sq, row["square_tflops"], t_sq_lib, t_eig))
    m, b = 10, 10
    gates = S.tfim_trotter_step(m)
    n = m + b
    psi = S.normal_state(m, 5)

    def run(emulate):
        st = Q.State(n, Q.QS_C128, stream=stream.cuda_stream)
        st.set(np.kron(np.ones(1 << b) / 2 ** (b / 2), psi))   # Hadamards on the control register
        t0 = time.perf_counter()
        if emulate == "eig":
            u = Q.Unitary(gates, m, 4, stream=stream.cuda_stream)
            u.eig()
            u.apply_qpe_eig(st, m, b)
            st.sync()
            u.free()
        elif emulate:
            Q.emulate_qpe_powers(st, gates, m, m, b)
        else:
            for j in range(b):
                c = 1 << (m + j)
                prog = st.compile([S.Gate(g.targets, g.matrix, c, c) for g in gates], 4)
                for _ in range(1 << j):
                    st.run(prog)
                prog.free()
        st.emulate_qft(m, b, inverse=True)
        st.sync()
        dt = (time.perf_counter() - t0) * 1e3
        probs = st.measure(list(range(m, n)))[1]
        st.free()
        return dt, probs

    run(False)                       # warm-up: library handles, code objects
    run(True)
    run("eig")
    t_gate, p_gate = run(False)
    t_emu, p_emu = run(True)
    t_eig, p_eig = run("eig")
    out["estimate"] = {"m": m, "b": b, "simulated_ms": round(t_gate, 2), "emulated_ms": round(t_emu, 2),
                       "emulated_eig_ms": round(t_eig, 2), "speedup": round(t_gate / t_emu, 1),
                       "max_abs_diff_phase_distribution": float(np.abs(p_gate - p_emu).max()),
                       "max_abs_diff_phase_distribution_eig": float(np.abs(p_gate - p_eig).max())}
    log("qpe estimate m=%d b=%d: simulated %.1f ms, emulated %.1f ms (squaring) / %.1f ms (eigensolver)"
        % (m, b, t_gate, t_emu, t_eig))
    return out


def arith_table(Q, S, ms=(4, 6, 8, 10)):
    """Integer multiplication and division of two m-bit registers into a
    third (Sec. III-A), n = 3m qubits, complex128, registers a, b, c from
    the most significant qubits down as the paper writes the index: the
    emulated permutation
    against the gate-level network a simulator runs on 3m + 1 qubits
    (Cuccaro adders, one ancilla), applied gate by gate and as a program
    fused into blocks of up to 4 qubits. a and b start in a seeded normal
    superposition, c = 0. Times from HIP events on the state's stream."""
    import torch
    stream = torch.cuda.Stream()

    def timed(fn, reps):
        fn()
        stream.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def input_state(n, m, seed):
        # a, b in a seeded normal superposition, c = 0, in the arith_layout
        # order: index = anc.a.b.c from the top
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        x = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
        v = torch.randn(1 << (2 * m), dtype=torch.complex128, device="cuda", generator=gen)
        M = 1 << m
        x.view(-1, M, M, M)[0, :, :, 0] = (v / torch.linalg.vector_norm(v)).view(M, M)
        st = Q.State(n, Q.QS_C128, stream=stream.cuda_stream)
        st.load_device(x.data_ptr())
        st.sync()
        del x, v
        return st

    rows = []
    for m in ms:
        row = {"m": m, "n_emulated": 3 * m, "n_simulated": 3 * m + 1}
        aq, bq, cq, anc = S.arith_layout(m)
        for kind, name, net_fn in ((0, "mul", S.mul_gate_circuit_on), (1, "div", S.div_gate_circuit_on)):
            net = net_fn(aq, bq, cq, anc)
            st = input_state(3 * m, m, S.SEED_BASE + 20 + m)
            op = st.emulate_mul if kind == 0 else st.emulate_div
            t_emu = timed(lambda: op(aq[0], bq[0], cq[0], m), 3)
            st.free()
            torch.cuda.empty_cache()
            st = input_state(3 * m + 1, m, S.SEED_BASE + 20 + m)
            reps = 1 if m >= 10 else 2
            t_gates = timed(lambda: st.apply_gates(net), reps)
            prog = st.compile(net, 4)
            blocks = prog.info()[0]
            t_fused = timed(lambda: st.run(prog), reps)
            prog.free()
            st.free()
            torch.cuda.empty_cache()
            t_sim = min(t_gates, t_fused)
            row[name] = {"gates": len(net), "fused_blocks": blocks, "emulated_ms": round(t_emu, 4),
                         "simulated_gate_by_gate_ms": round(t_gates, 3), "simulated_fused_ms": round(t_fused, 3),
                         "speedup": round(t_sim / t_emu, 1),
                         "emulated_gbs": round(2 * 16 * 2 ** (3 * m) / (t_emu * 1e-3) / 1e9, 1)}
            log("arith m=%d %s: emulated %.3f ms, gate by gate %.1f ms (%d gates), fused %.1f ms (%d blocks)"
                % (m, name, t_emu, t_gates, len(net), t_fused, blocks))
        rows.append(row)
    return {"unit": "ms", "dtype": "c128", "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--parts", default="all",
                    help="all | fused | batch | qpe | arith | configs (profiling runs: one part only)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched learned-vs-plain part")
    ap.add_argument("--no-qpe", action="store_true", help="skip the phase-estimation part")
    ap.add_argument("--no-arith", action="store_true", help="skip the multiplication/division part")
    ap.add_argument("--arith-ms", default="4,6,8,10", help="register widths m of the multiplication/division part")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 16-qubit gate-level, 28-qubit modmul and 32-qubit matrix-core parts")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the state-vector path is not sharded "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1604_06460_amd import qs as Q
    from synth import circuits as S

    torch.cuda.set_device(0)
    if args.parts == "batch":
        print(json.dumps({"parts": "batch", "batched_learned": batch_learned(Q, S)}), flush=True)
        return
    if args.parts == "qpe":
        print(json.dumps({"parts": "qpe", "phase_estimation": qpe_table(Q, S)}), flush=True)
        return
    if args.parts == "configs":
        print(json.dumps({"parts": "configs", "configs": {
            "c0_16q_gate_level": config0_gate_level(Q, S),
            "c2_28q_modmul": config2_modmul28(Q, S),
            "c3_32q_c64_k6_mfma": config3_mfma32(Q, S)}}), flush=True)
        return
    if args.parts == "arith":
        ms = tuple(int(v) for v in args.arith_ms.split(","))
        print(json.dumps({"parts": "arith", "arithmetic": arith_table(Q, S, ms)}), flush=True)
        return
    stream = torch.cuda.Stream()  # default priority
    n = N_QUBITS
    amp = 16
    N = float(1 << n)
    seed = S.SEED_BASE + 1
    gates = S.random_layer_circuit(n, DEPTH, seed)
    qft_g = S.qft_circuit(n)
    a_mod, N_mod = S.modmul_params(20, seed)
    uniforms = np.random.default_rng(seed).random(16)
    st = Q.State(n, Q.QS_C128, stream=stream.cuda_stream)

    # resident seeded normal input for the QFT part
    with torch.cuda.stream(stream):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        normal = torch.randn(1 << n, dtype=torch.complex128, device="cuda", generator=gen)
        normal /= torch.linalg.vector_norm(normal)
    stream.synchronize()

    # compile once to learn the blocks (the step compiles again): kinds,
    # widths and the bytes each block must move
    prog0 = st.compile(gates, MAX_K)
    n_blocks, block_k, amp_moves = prog0.info()
    block_kind = [prog0.block_kind(b) for b in range(n_blocks)]
    prog0.free()
    dense4 = [b for b in range(n_blocks) if block_kind[b][0] == Q.QS_BLOCK_DENSE and block_k[b] == 4]
    parts_all = args.parts == "all"

    ev = {}
    # the program split into maximal runs of consecutive blocks of one
    # class (dense 4-qubit sweeps or anything else); one event pair per
    # run, so the dense sweep's launch time is read without an event
    # between every two of its launches
    runs = []
    for b in range(n_blocks):
        cls = b in dense4
        if runs and runs[-1][2] == cls:
            runs[-1][1] = b + 1
        else:
            runs.append([b, b + 1, cls])
    run_ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(runs) + 1)]
    run_ms = []

    def mark(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        ev[name] = e

    def step():
        mark("t0")
        st.set_zero()
        mark("init")
        prog = st.compile(gates, MAX_K)
        mark("compile")
        run_ev[0].record(stream)
        for r, (b0, b1, _) in enumerate(runs):
            st.run_range(prog, b0, b1)
            run_ev[r + 1].record(stream)
        mark("fused")
        z0 = st.expectation(z_mask=1).real
        nrm = st.norm2()
        mark("reduce")
        if parts_all:
            st.load_device(normal.data_ptr())
            mark("load")
            for g in qft_g:
                st.apply_gate(g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
            mark("qft_gates")
            st.emulate_qft(0, n, inverse=True)
            mark("qft_emulated")
            st.emulate_modmul(0, 20, 20, 8, a_mod, N_mod)
            mark("modmul")
            st.measure(list(range(20, 28)), uniforms)
            mark("measure")
        prog.free()
        return z0, nrm

    log("setup done (%d fused blocks)" % n_blocks)
    for w in range(args.warmup):
        step()
        log("warmup step %d done" % (w + 1))
    torch.cuda.synchronize()
    part_ms = {}
    t0 = time.perf_counter()
    for k in range(args.steps):
        z0, nrm = step()
        stream.synchronize()
        log("timed step %d done" % (k + 1))
        names = list(ev.keys())
        for a, b in zip(names[:-1], names[1:]):
            part_ms.setdefault(b, []).append(ev[a].elapsed_time(ev[b]))
        run_ms.append([run_ev[r].elapsed_time(run_ev[r + 1]) for r in range(len(runs))])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    part_ms = {k: float(np.mean(v)) for k, v in part_ms.items()}

    bytes_part = {
        "init": amp * N,
        "fused": amp_moves * amp,
        "reduce": 2 * amp * N,
    }
    if parts_all:
        bytes_part.update({
            "load": 2 * amp * N,
            "qft_gates": qft_gate_bytes(n, amp),
            "qft_emulated": 3 * 2 * amp * N,
            "modmul": 2 * amp * N,
            "measure": amp * N,
        })
    total_bytes = sum(bytes_part.values())
    value = total_bytes / (ms_per_step * 1e-3) / 1e9

    # dominant kernel: the dense 4-qubit block sweep (k_dense_tile<double,4>,
    # the tuned complex128 path for 2- to 4-qubit blocks); each launch reads
    # and writes the whole state once. Its average launch time is the time
    # of the runs of such blocks over their launch count, in the timed steps.
    rms = np.array(run_ms)                        # steps x runs
    d4_runs = [r for r, (_, _, cls) in enumerate(runs) if cls]
    sweep_ms = float(rms[:, d4_runs].sum(axis=1).mean()) / len(dense4)
    achieved = 2 * amp * N / (sweep_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "kernel": "k_dense_tile<double,4>: dense 4-qubit fused-block sweep, complex128, "
                          "average over the %d such launches per step" % len(dense4),
                "avg_launch_ms": round(sweep_ms, 4), "bytes_per_launch": 2 * amp * N}
    kinds_count = {"dense": sum(1 for k, _ in block_kind if k == Q.QS_BLOCK_DENSE),
                   "diagonal": sum(1 for k, _ in block_kind if k == Q.QS_BLOCK_DIAGONAL),
                   "identity": sum(1 for k, _ in block_kind if k == Q.QS_BLOCK_IDENTITY)}
    diag_b = [b for b in range(n_blocks) if block_kind[b][0] == Q.QS_BLOCK_DIAGONAL]
    fused_detail = {"blocks": n_blocks, "kinds": kinds_count,
                    "dense_k4_launches": len(dense4),
                    "block_widths": {str(k): int(np.sum(np.asarray(block_k) == k)) for k in range(1, MAX_K + 1)},
                    "diagonal_blocks": [{"k": int(block_k[b]), "changed_fraction": block_kind[b][1]}
                                        for b in diag_b],
                    "other_blocks_ms": round(float(rms[:, [r for r in range(len(runs)) if r not in d4_runs]]
                                                   .sum(axis=1).mean()), 3),
                    "amp_moves_per_run": amp_moves}

    # at-scale consistency (untimed): gate-level QFT then emulated inverse
    # returns the input; sampled amplitudes compared with the resident input
    check = {}
    if parts_all:
        st.load_device(normal.data_ptr())
        for g in qft_g:
            st.apply_gate(g.targets, g.matrix, g.ctrl_mask, g.ctrl_vals)
        st.emulate_qft(0, n, inverse=True)
        idx = np.random.default_rng(1).integers(0, 1 << n, 256).astype(np.uint64)
        got = st.amplitudes(idx)
        ref = normal[torch.from_numpy(idx.astype(np.int64)).to("cuda")].cpu().numpy()
        check["qft_gate_vs_emulated_max_abs_err"] = float(np.abs(got - ref).max())
        check["z0_after_circuit"] = z0
        check["norm_after_circuit"] = nrm

    # plain device copy of the state: achievable-bandwidth reference
    mark("c0")
    for _ in range(3):
        st.load_device(normal.data_ptr())
    mark("c1")
    stream.synchronize()
    copy_gbs = 3 * 2 * amp * N / (ev["c0"].elapsed_time(ev["c1"]) * 1e-3) / 1e9

    st.free()
    del normal
    torch.cuda.empty_cache()
    batched = None
    if not args.no_batch and parts_all:
        batched = batch_learned(Q, S)
    qpe = None
    if not args.no_qpe and parts_all:
        qpe = qpe_table(Q, S)
    arith = None
    if not args.no_arith and parts_all:
        arith = arith_table(Q, S, tuple(int(v) for v in args.arith_ms.split(",")))
    configs = None
    if not args.no_configs and parts_all:
        configs = {"c0_16q_gate_level": config0_gate_level(Q, S),
                   "c2_28q_modmul": config2_modmul28(Q, S),
                   "c3_32q_c64_k6_mfma": config3_mfma32(Q, S)}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) starts")
        cpu = cpu_baseline(n, gates)
        log("cpu baseline done")

    out = {
        "metric": "HBM GB/s of gate sweeps at 30q; learned-vs-plain wall time at 1e-5 amp error",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "30-qubit complex128: depth-30 random circuit fused into k=4 blocks "
                               "(%d blocks) + gate-level QFT then emulated inverse QFT + modmul "
                               "permutation + reductions" % n_blocks,
                   "n_qubits": n, "depth": DEPTH, "fusion_k": MAX_K, "seed": seed,
                   "parts": args.parts},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fused_detail": fused_detail,
        "breakdown_ms": {k: round(v, 3) for k, v in part_ms.items()},
        "breakdown_gbs": {k: round(bytes_part[k] / (part_ms[k] * 1e-3) / 1e9, 1)
                          for k in bytes_part if k in part_ms and part_ms[k] > 0},
        "copy_ceiling_gbs": round(copy_gbs, 1),
        "check": check,
        "batched_learned": batched,
        "phase_estimation": qpe,
        "arithmetic": arith,
        "configs": configs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
