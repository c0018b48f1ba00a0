"""Benchmark of the state-vector hot path on one MI355X.

Workload: the 30-qubit random circuit -- 40 layers of a Haar-random 2x2 gate
on every qubit then CNOTs on alternating neighbour pairs (1200 + 580 gates),
complex128, from |0...0>.  One step = reset the state, queue the 1780 gates,
flush (fusion + LDS-tile passes), then the reductions: the squared norm, an
8-term Pauli-sum expectation value and 1000 samples.  Inputs are seeded and
synthetic; the state is resident in HBM for the whole run.

value = original gates x 2^30 amplitudes x steps / wall time of the timed
steps (amplitude-gate updates per second).  Also reported: the algorithmic
HBM bytes per step over its time (fraction of the 8 TB/s peak), the roofline
of the dominant kernel (the LDS-tile pass) from HIP events recorded by the
library around every launch, a complex64 (FP32) leg of the same circuit, a
per-gate FP64 leg, and the CPU oracle timed on a bounded sample.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
FP64_PEAK = 78.6e12        # MI355X FP64 (vector and matrix), flop/s

# Measured HBM traffic of the dominant kernel (k_tile_reg<double,4,8,*>: the
# instance with table ops, 132 of 141 launches in the profiled run, and the
# one without, the 9 passes that only move qubits back), from two rocprofv3
# --pmc runs of this script's main leg (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, mean over the tile dispatches).  The counters are scaled by what
# they read for the copy probe of the same runs (16 GiB read + 16 GiB
# written: FETCH_SIZE reads half the bytes, WRITE_SIZE all of them).  Valid
# only for the sources they were taken with: the digest below covers every
# file that shapes the kernel or its launches.
TRAFFIC = {"kernel": "k_tile_reg<double,4,8,*>", "fetch_kib": 8394362.6, "write_kib": 16785437.0,
           "fetch_scale": 2.0, "write_scale": 1.0, "digest": "8a514cddf6243155"}
TRAFFIC_SOURCES = ("paper_1612_08091_amd/csrc/kernels_tile.hip",
                   "paper_1612_08091_amd/csrc/lds_ops.hpp",
                   "paper_1612_08091_amd/csrc/device.hpp",
                   "paper_1612_08091_amd/csrc/tileprog.cpp",
                   "paper_1612_08091_amd/csrc/tileprog.hpp",
                   "paper_1612_08091_amd/csrc/planner.cpp",
                   "paper_1612_08091_amd/csrc/qsv_internal.hpp",
                   "paper_1612_08091_amd/build.py")


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel, or None when the counters
    were taken from other sources than the ones built here."""
    t = TRAFFIC
    if t["fetch_kib"] is None or t["digest"] != kernel_source_digest():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_hamiltonian(n: int):
    """4 Z-strings (one shared pass) + 4 terms with X/Y letters."""
    import workloads as W
    s = []
    for t in range(4):
        z = ["I"] * n
        for q in (t, 7 + t, 15 + t, 29 - t):
            z[q] = "Z"
        s.append("".join(z))
    for t in range(4):
        p = ["I"] * n
        p[2 * t] = "X"
        p[2 * t + 11] = "Y"
        p[27 - t] = "Z"
        s.append("".join(p))
    rng = np.random.default_rng(W.SEED_BASE + 1)
    return W.PauliSum.from_strings(s, rng.standard_normal(len(s)))


def run_leg(circ, ham, u, steps, warmup, dtype, mode, k_max, tile_bits, timing=True, reduce=True,
            reg_bits=0):
    import torch
    from paper_1612_08091_amd import qsv as Q
    n = circ.n
    sim = Q.Simulator(n_max=n, dtype=dtype, mode=mode, k_max=k_max, tile_bits=tile_bits,
                      timing=timing, reg_bits=reg_bits)
    sim.allocate(n)
    diag_ops = 0
    if mode == "tiled":
        # the lowering the flushes will run (host side): table ops present?
        sim.run(circ)
        try:
            diag_ops = sim.check_tile_programs(None)[1]["diag_ops"]
        except Exception:
            diag_ops = -1
        sim.reset()
    gates = [(np.ascontiguousarray(g.matrix), list(g.targets), list(g.controls))
             for g in circ.gates]
    out = {}

    def one_step():
        sim.reset()
        for m, t, c in gates:
            sim.apply(m, t, c)
        sim.flush()
        if reduce:
            out["norm2"] = sim.norm2()
            out["energy"] = sim.expectation(ham)
            out["samples"] = sim.sample(u)

    for w in range(warmup):
        one_step()
        sim.synchronize()
        log("  warmup step %d done" % w)
    torch.cuda.synchronize()
    sim.synchronize()
    sim.reset_stats()
    t0 = time.perf_counter()
    for k in range(steps):
        one_step()
        log("  step %d queued/done" % k)
    sim.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats()
    kt = sim.kernel_times() if timing else {}
    sim.close()
    wall = t1 - t0
    return {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "stats": st, "ktimes": kt,
            "norm2": out.get("norm2"), "energy": out.get("energy"), "diag_ops": diag_ops,
            "updates_per_step": len(circ.gates) * float(1 << n)}


def copy_bandwidth(gib: int = 16, reps: int = 5):
    """Achievable HBM bandwidth: the library's streaming copy kernel
    (qsv_copy_probe) over two gib-GiB device buffers, timed with events on
    the stream it runs on; read + write bytes per second."""
    import torch
    from paper_1612_08091_amd import qsv as Q
    a = torch.empty((gib << 30) // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    st = torch.cuda.current_stream()
    Q.copy_probe(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        Q.copy_probe(a, b)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a[:1 << 20], b[:1 << 20]))
    del a, b
    torch.cuda.empty_cache()
    return {"GBps": 2.0 * (gib << 30) / (ms * 1e-3) / 1e9, "ms": ms, "bytes_each_way": gib << 30,
            "copy_checked": ok}


def fp32_state_error(circ):
    """Normwise relative error of the complex64 state against the complex128
    state of the same circuit (both from the fused tile passes), over every
    amplitude: the two states sit in device buffers the simulators borrow."""
    import torch
    from paper_1612_08091_amd import qsv as Q
    n = circ.n
    b128 = torch.empty(2 << n, dtype=torch.float64, device="cuda")
    b64 = torch.empty(2 << n, dtype=torch.float32, device="cuda")
    for dt, buf in (("c128", b128), ("c64", b64)):
        sim = Q.Simulator(n_max=n, dtype=dt, mode="tiled", k_max=2, state=buf)
        sim.allocate(n)
        sim.run(circ)
        sim.flush()
        sim.synchronize()
        sim.close()
    torch.cuda.synchronize()
    num = 0.0
    den = 0.0
    step = 1 << 26
    for a in range(0, 2 << n, step):
        x = b128[a:a + step]
        d = b64[a:a + step].double() - x
        num += float(torch.dot(d, d))
        den += float(torch.dot(x, x))
    del b128, b64
    torch.cuda.empty_cache()
    return math.sqrt(num / den)


def _timed_circuit(sim, circ):
    import torch
    sim.reset()
    sim.run(circ)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.flush()
    sim.synchronize()
    return time.perf_counter() - t0


def form_precision(samples: int = 1 << 20):
    """32-qubit Haar + CZ brick circuit (1900 gates): complex64 state with fused
    passes versus the same circuit in complex128; the FP32 error is measured on
    a seeded sample of amplitudes (normwise relative error over the sample)."""
    import workloads as W
    from paper_1612_08091_amd import qsv as Q
    circ = W.config2()
    idx = np.sort(np.random.default_rng(W.SEED_BASE + 2).integers(0, 1 << 32, size=samples,
                                                                   dtype=np.uint64))
    out = {"workload": "config 2: 32-qubit Haar + CZ brick, 40 layers, 1900 gates"}
    amps = {}
    # complex64 with 2-qubit fusion (register tiles), complex64 with 5-qubit
    # fused unitaries on FP32 MFMA (LDS tiles), and the complex128 reference
    for key, dtype, k in (("c64", "c64", 2), ("c64_k5_mfma", "c64", 5), ("c128", "c128", 2)):
        sim = Q.Simulator(n_max=32, dtype=dtype, mode="tiled", k_max=k, timing=True)
        sim.allocate(32)
        _timed_circuit(sim, circ)                  # allocation + warm-up
        sim.reset_stats()
        t = _timed_circuit(sim, circ)
        st = sim.stats()
        tile_ms, tile_n, _ = sim.kernel_times()["tile"]
        amps[key] = sim.get_amplitudes(idx)
        out[key] = {"s_per_circuit": t,
                    "amp_gate_per_s": len(circ.gates) * float(1 << 32) / t,
                    "pct_hbm_peak": st["alg_bytes"] / t / HBM_PEAK,
                    "passes": st["passes"], "fused_ops": st["fused_ops"],
                    "tile_avg_ms": tile_ms / max(tile_n, 1),
                    "norm2_drift": abs(sim.norm2() - 1.0)}
        sim.close()
        log("  precision leg %s: %.3f s" % (key, t))
    ref = np.linalg.norm(amps["c128"])
    for key in ("c64", "c64_k5_mfma"):
        out[key]["fp32_rel_err_sampled"] = float(np.linalg.norm(amps[key] - amps["c128"]) / ref)
    out["samples"] = samples
    return out


def form_fusion_qft(n: int = 30):
    """Config 1 beside the main leg: the random circuit with fusion widths
    k = 3..5 (LDS tiles, MFMA for k >= 3), and the n-qubit QFT of a random
    basis state per gate and fused, checked against its closed form."""
    import workloads as W
    from paper_1612_08091_amd import qsv as Q
    out = {}
    circ = W.config1_random(n=n)
    for k in (3, 4, 5):
        sim = Q.Simulator(n_max=n, dtype="c128", mode="tiled", k_max=k, timing=True)
        sim.allocate(n)
        _timed_circuit(sim, circ)
        sim.reset_stats()
        t = _timed_circuit(sim, circ)
        st = sim.stats()
        tile_ms, tile_n, tile_b = sim.kernel_times()["tile"]
        out["random_k%d" % k] = {"s_per_circuit": t,
                                 "amp_gate_per_s": len(circ.gates) * float(1 << n) / t,
                                 "passes": st["passes"], "fused_ops": st["fused_ops"],
                                 "tile_GBps": tile_b / (tile_ms * 1e-3) / 1e9 if tile_ms else None}
        sim.close()
        log("  fusion k=%d: %.3f s" % (k, t))
    x, qft = W.config1_qft(n)
    prep = W.basis_prep(n, x)
    idx = np.random.default_rng(W.SEED_BASE + 1).integers(0, 1 << n, size=4096, dtype=np.uint64)
    ph = np.array([float((x * int(v)) % (1 << n)) for v in idx.astype(object)]) / (1 << n)
    want = np.exp(2j * np.pi * ph) / (2 ** (n / 2))
    for mode, k in (("pergate", 1), ("tiled", 2)):
        sim = Q.Simulator(n_max=n, dtype="c128", mode=mode, k_max=k, timing=True)
        sim.allocate(n)
        for rep in range(2):
            sim.reset()
            sim.run(prep)
            sim.flush()
            sim.synchronize()
            sim.reset_stats()
            sim.run(qft)
            t0 = time.perf_counter()
            sim.flush()
            sim.synchronize()
            t = time.perf_counter() - t0
        st = sim.stats()
        err = float(np.max(np.abs(sim.get_amplitudes(idx) - want)))
        out["qft_%s" % mode] = {"s_per_circuit": t,
                                "amp_gate_per_s": len(qft.gates) * float(1 << n) / t,
                                "pct_hbm_peak": st["alg_bytes"] / t / HBM_PEAK,
                                "passes_or_kernels": st["passes"] or st["kernels"],
                                "max_abs_err_vs_closed_form": err}
        sim.close()
        log("  qft %s: %.3f s" % (mode, t))
    return out


def form_simcomparison(n: int = 30):
    """The paper's own simulator benchmark circuit (Sec. 4.3.2): H on every
    qubit, a chain of controlled Rz, H on every qubit, at 30 qubits complex128,
    fused tile passes versus per gate.  The paper reports only a relative
    speed-up over its predecessor for this circuit, no absolute figure."""
    import workloads as W
    from paper_1612_08091_amd import qsv as Q
    circ = W.simcomparison(n, np.random.default_rng(W.SEED_BASE + 5))
    out = {"workload": "%d-qubit H-transform, %d-gate CRz chain, H-transform (%d gates), "
                       "complex128" % (n, n - 1, len(circ.gates))}
    for mode, k in (("tiled", 2), ("pergate", 1)):
        sim = Q.Simulator(n_max=n, dtype="c128", mode=mode, k_max=k, timing=True)
        sim.allocate(n)
        _timed_circuit(sim, circ)
        sim.reset_stats()
        t = _timed_circuit(sim, circ)
        st = sim.stats()
        out[mode] = {"s_per_circuit": t, "amp_gate_per_s": len(circ.gates) * float(1 << n) / t,
                     "pct_hbm_peak": st["alg_bytes"] / t / HBM_PEAK,
                     "passes_or_kernels": st["passes"] or st["kernels"]}
        sim.close()
        log("  simcomparison %s: %.3f s" % (mode, t))
    return out


def form_emulation(n: int = 30, w: int = 20):
    """Emulated math gates (Sec. 4.3.3) at 30 qubits complex128: AddConstant
    and Shor's controlled modular multiplication on a 20-bit register as one
    gather pass each, beside the gate-level AddConstant (QFT, phases, inverse
    QFT: the decomposition the paper gives) run through the fused tile path.
    The state is a product of seeded Haar 1-qubit states."""
    import torch
    import workloads as W
    from paper_1612_08091_amd import qsv as Q
    rng = np.random.default_rng(W.SEED_BASE + 6)
    reg = list(range(6, 6 + w))
    const, a, N = 123457, 5, 1048573
    add_tab = W.add_constant_table(w, const)
    mul_tab = W.mul_mod_table(w, a, N)
    prep = [W.haar_2x2(rng) for _ in range(n)]
    idx = rng.integers(0, 1 << n, 1024, dtype=np.uint64)
    sim = Q.Simulator(n_max=n, dtype="c128", mode="tiled", k_max=2, timing=True)
    sim.allocate(n)

    def prepare():
        sim.reset()
        for q in range(n):
            sim.apply(prep[q], [q])
        sim.flush()
        sim.synchronize()

    def timed(fn, reps=3):
        best = None
        for _ in range(reps):
            prepare()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            sim.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    sim.reset_stats()
    t_add = timed(lambda: sim.apply_math(reg, add_tab))
    emu = sim.get_amplitudes(idx)
    k_add = sim.kernel_times()["mono"]      # the gather kernels (HIP events)
    sim.reset_stats()
    t_mul = timed(lambda: sim.apply_math(reg, mul_tab, [0]))
    k_mul = sim.kernel_times()["mono"]
    adder = W.draper_add(n, const, reg)
    prepare()
    sim.run(adder)
    _, adder_passes = sim.plan()
    t_gates = timed(lambda: (sim.run(adder), sim.flush()), reps=2)
    gates = sim.get_amplitudes(idx)
    sim.close()
    log("  emulation: add %.4f s, mulmod %.4f s, gate-level adder %.3f s" % (t_add, t_mul, t_gates))
    return {"workload": "%d-qubit product state, complex128; %d-bit register" % (n, w),
            "add_constant_emulated": {
                "s": t_add, "kernel_ms": k_add[0] / max(k_add[1], 1),
                "kernel_GBps": k_add[2] / max(k_add[1], 1) / (k_add[0] / max(k_add[1], 1) * 1e-3) / 1e9,
                "kernel_pct_hbm_peak": k_add[2] / (k_add[0] * 1e-3) / HBM_PEAK},
            "mul_mod_N_controlled_emulated": {
                "s": t_mul, "kernel_ms": k_mul[0] / max(k_mul[1], 1),
                "kernel_GBps": k_mul[2] / max(k_mul[1], 1) / (k_mul[0] / max(k_mul[1], 1) * 1e-3) / 1e9,
                "kernel_pct_hbm_peak": k_mul[2] / (k_mul[0] * 1e-3) / HBM_PEAK},
            "add_constant_gate_level": {"s": t_gates, "gates": len(adder.gates),
                                        "passes": adder_passes},
            "emulation_speedup": t_gates / t_add,
            "max_abs_diff_emulated_vs_gates": float(np.max(np.abs(emu - gates)))}


def form_noise(n: int = 15, layers: int = 10):
    """Density matrix of a noisy 15-qubit brick circuit (Haar 1-qubit gates
    and CNOTs, each followed by depolarizing noise p = 1e-3 on its qubits and
    amplitude damping 1e-3 on CNOT targets): vec(rho) is a 30-qubit complex128
    vector; gates and channel superoperators run through the fused tile
    passes.  Reports the time per circuit, the passes, and the trace."""
    import torch
    import workloads as W
    from paper_1612_08091_amd import qsv as Q
    ev = W.noisy_brick(n, layers, 1e-3, np.random.default_rng(W.SEED_BASE + 7), gamma=1e-3)
    d = Q.DensityMatrix(n, dtype="c128", mode="tiled", k_max=2, timing=True)
    d.run(ev)
    _, npass = d.sim.plan()
    times = []
    for _ in range(2):
        d.sim.reset()
        d.run(ev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.flush()
        d.sim.synchronize()
        times.append(time.perf_counter() - t0)
    p = d.probabilities()
    kt = d.sim.kernel_times()
    d.close()
    t = min(times)
    gates = sum(1 for e in ev if e[0] == "gate")
    # the same circuit as stochastic trajectories on the 15-qubit state: every
    # channel is one reduction (its branch probabilities), a host draw and
    # the chosen branch queued as a gate
    s = Q.Simulator(n_max=n, dtype="c128", mode="tiled", k_max=2)
    s.allocate(n)
    urng = np.random.default_rng(W.SEED_BASE + 8)
    ttimes = []
    for _ in range(4):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in ev:
            if e[0] == "gate":
                s.apply(e[1], list(e[2]), list(e[3]))
            else:
                s.apply_kraus_sampled(e[1], list(e[2]), float(urng.uniform()))
        s.flush()
        s.synchronize()
        ttimes.append(time.perf_counter() - t0)
    s.close()
    tt = min(ttimes[1:])
    return {"workload": "%d-qubit noisy brick, %d layers: %d gates, %d channels; vec(rho) on %d "
                        "qubits, complex128" % (n, layers, gates, len(ev) - gates, 2 * n),
            "s_per_circuit": t, "passes": npass,
            "events_per_s": len(ev) / t,
            "tile_kernel_ms_avg": kt["tile"][0] / max(kt["tile"][1], 1),
            "trace_minus_one": float(p.sum() - 1.0),
            "trajectory": {"s_per_trajectory": tt, "channels_per_s": (len(ev) - gates) / tt}}


def form_batched(pergate_sample: int = 256):
    """Config 3: 4096 HEA circuits (8..20 qubits, depth 6) with 64-term Pauli
    sums, complex64, one persistent graph-captured launch per evaluation;
    beside it the same batch in complex128, and the plain FP64 per-gate path
    (one circuit at a time) on a seeded sample of circuits.  Accuracy: the
    largest |<H>_c64 - <H>_fp64| / sum|c| over the circuits."""
    import workloads as W
    from paper_1612_08091_amd import qsv as Q
    t0 = time.perf_counter()
    circuits, hams = W.config3()
    scale = np.array([float(np.sum(np.abs(h.coeff))) for h in hams])
    out = {"workload": "config 3: 4096 circuits, n ~ U{8..20}, 64-term <H> each"}
    vals = {}
    for dt in ("c64", "c128"):
        t1 = time.perf_counter()
        b = Q.Batch(circuits, hams, dtype=dt, autotune=True, use_graph=True)
        setup = time.perf_counter() - t1
        vals[dt] = np.array(b.run())
        times = []
        for _ in range(5):
            t1 = time.perf_counter()
            b.run()
            times.append(time.perf_counter() - t1)
        info = b.info()
        b.close()
        best = min(times)
        out[dt] = {"circuits_per_s": len(circuits) / best, "s_per_batch": best,
                   "device_ms": info["last_ms"], "tile_bits": info["tile_bits"],
                   "k_fuse": info["k_fuse"], "setup_s_incl_autotune": setup}
        # Global-memory bytes of the Pauli sums of the circuits above the LDS
        # limit: each chunk of 2^cl amplitudes is read once into LDS, and a
        # term whose highest X bit lies above the chunk reads the partner half
        # of the state (the pairs' other members); strings of Z letters and
        # pairs inside a chunk add nothing.  A lower bound on the batch's
        # traffic (the tile passes add 2 x state per pass), much of it served
        # by L2 and the last-level cache since a state is re-read per term.
        elem = 8 if dt == "c64" else 16
        mb = info["tile_bits"]
        cl = 12 if dt == "c64" else 11
        sweep = 0.0
        for c, h in zip(circuits, hams):
            if c.n <= mb:
                continue
            dim = float(1 << c.n)
            clc = min(cl, c.n)
            far = sum(1 for x in h.xmask if int(x) and int(x).bit_length() - 1 >= clc)
            sweep += dim * elem + far * dim / 2 * elem
        out[dt]["roofline"] = {
            "pauli_read_bytes": sweep,
            "pauli_read_GBps": sweep / (info["last_ms"] * 1e-3) / 1e9 if info["last_ms"] else None,
            "frac_of_hbm_peak": sweep / (info["last_ms"] * 1e-3) / HBM_PEAK if info["last_ms"] else None,
            "note": "Pauli-sum global reads only, over the whole batch time; the tile passes of "
                    "the large circuits add 2 x state per pass"}
        log("  batched %s: %.4f s per batch" % (dt, best))
    out["c64"]["max_abs_err_over_sum_abs_c_vs_c128_batch"] = float(
        np.max(np.abs(vals["c64"] - vals["c128"]) / scale))
    # the FP64 per-gate path, one circuit at a time, on a seeded sample
    pick = np.sort(np.random.default_rng(W.SEED_BASE + 3).choice(len(circuits), pergate_sample,
                                                                  replace=False))
    sims = {}
    ref = np.zeros(len(pick))
    t1 = time.perf_counter()
    for j, i in enumerate(pick):
        c = circuits[i]
        if c.n not in sims:
            sims[c.n] = Q.Simulator(n_max=c.n, dtype="c128", mode="pergate", k_max=1)
            sims[c.n].allocate(c.n)
        s = sims[c.n]
        s.reset()
        s.run(c)
        s.flush()
        ref[j] = s.expectation(hams[i])
    s_pg = time.perf_counter() - t1
    for s in sims.values():
        s.close()
    out["fp64_pergate_sample"] = {
        "circuits": int(len(pick)), "s": s_pg,
        "circuits_per_s": len(pick) / s_pg,
        "c64_batch_max_abs_err_over_sum_abs_c": float(np.max(np.abs(vals["c64"][pick] - ref)
                                                             / scale[pick])),
        "c128_batch_max_abs_err_over_sum_abs_c": float(np.max(np.abs(vals["c128"][pick] - ref)
                                                              / scale[pick]))}
    out["c64_speedup_vs_fp64_pergate"] = out["c64"]["circuits_per_s"] / (len(pick) / s_pg)
    out["total_s"] = time.perf_counter() - t0
    log("  batched per-gate FP64 sample: %.2f s for %d circuits" % (s_pg, len(pick)))
    return out


def form_adjoint():
    """Config 4: 24-qubit HEA (480 angles), 200-term Pauli sum: <H> and the full
    gradient by the adjoint method, complex128; the tiled reverse sweep beside
    the plain per-gate one, both checked against the stored oracle values
    (tests/golden/config4_adjoint.json: the energy and a seeded subset of the
    gradient, written by a script that calls only the oracle)."""
    import workloads as W
    from paper_1612_08091_amd import qsv as Q
    with open(os.path.join(ROOT, "tests", "golden", "config4_adjoint.json")) as f:
        gold = json.load(f)
    circ, ham = W.config4()
    scale = float(np.sum(np.abs(ham.coeff)))
    out = {"workload": "config 4: 24-qubit HEA, 480 angles, 200 Pauli terms"}
    for mode, k in (("tiled", 2), ("pergate", 1)):
        sim = Q.Simulator(n_max=24, dtype="c128", mode=mode, k_max=k)
        Q.adjoint_gradient(sim, circ, ham)
        times = []
        for _ in range(3):
            t1 = time.perf_counter()
            val, grad = Q.adjoint_gradient(sim, circ, ham)
            times.append(time.perf_counter() - t1)
        sim.close()
        got = np.asarray(grad)[gold["params"]]
        out[mode] = {"s_per_value_and_gradient": min(times), "energy": val,
                     "energy_abs_err_over_sum_abs_c": abs(val - gold["energy"]) / scale,
                     "grad_max_abs_err_over_sum_abs_c": float(
                         np.max(np.abs(got - np.asarray(gold["grad"]))) / scale),
                     "grad_norm": float(np.linalg.norm(grad))}
        log("  adjoint %s: %.3f s" % (mode, min(times)))
    out["tiled_speedup_vs_pergate"] = (out["pergate"]["s_per_value_and_gradient"]
                                       / out["tiled"]["s_per_value_and_gradient"])
    return out


def host_description():
    """Cores this process may use, the CPU model and the RAM of the host."""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        cores = min(cores, int(omp))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram_gib = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram_gib = int(line.split()[1]) / 2**20
                    break
    except OSError:
        pass
    return {"cores_usable": cores, "nproc": os.cpu_count(), "cpu_model": model,
            "ram_GiB": ram_gib}


def _oracle_circuit(circ, threads, psi=None, max_gates=None, budget_s=None):
    """Oracle run of the first gates of circ (all by default) on `threads`
    threads; returns (gates done, seconds)."""
    import oracle
    oracle.set_threads(threads)
    if psi is None:
        psi = oracle.zero_state(circ.n)
    done = 0
    t0 = time.perf_counter()
    for g in circ.gates:
        oracle.apply(psi, g.matrix, g.targets, g.controls)
        done += 1
        if max_gates is not None and done >= max_gates:
            break
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            break
    t = time.perf_counter() - t0
    oracle.set_threads(1)
    return done, t


def cpu_baseline(circ, budget_s=12.0):
    """The oracle (plain C, one gate at a time, complex128) on the host cores:
    a bounded sample of the 30-qubit circuit (its first gates, one thread and
    all cores, outer loop of each gate shared out), with the full circuit's
    time extrapolated from it, and two small configurations in full: the
    16-qubit 20-layer brick circuit and the 20-qubit twin of the 32-qubit
    Haar + CZ brick circuit."""
    import oracle
    import workloads as W
    host = host_description()
    cores = host["cores_usable"]
    n = circ.n
    psi = oracle.zero_state(n)
    g1, t1 = _oracle_circuit(circ, 1, psi=psi, max_gates=2, budget_s=budget_s)
    rate1 = g1 * float(1 << n) / t1
    gn, tn = _oracle_circuit(circ, cores, psi=psi, max_gates=60, budget_s=budget_s)
    raten = gn * float(1 << n) / tn
    del psi
    log("  cpu: 30q %d gates on 1 thread %.1f s, %d gates on %d threads %.1f s" % (g1, t1, gn, cores, tn))
    c0, _ = W.config0()
    d0a, s0a = _oracle_circuit(c0, 1)
    d0n, s0n = _oracle_circuit(c0, cores)
    c2 = W.config2(n=20)
    d2a, s2a = _oracle_circuit(c2, 1)
    d2n, s2n = _oracle_circuit(c2, cores)
    log("  cpu: config 0 %.2f s / %.2f s, 20q twin %.2f s / %.2f s" % (s0a, s0n, s2a, s2n))
    full = len(circ.gates) * float(1 << n)
    return {"value": raten, "unit": "amp*gate/s", "cores": cores, "kind": "oracle",
            "sample": "the first %d gates of the %d-qubit circuit (of %d), complex128, the "
                      "oracle's gate loop shared over %d threads (%.1f s); the full circuit "
                      "is extrapolated below" % (gn, n, len(circ.gates), cores, tn),
            "single_thread": {"value": rate1, "sample": "first %d gates, %.1f s" % (g1, t1)},
            "extrapolated_full_circuit_s": {"threads_%d" % cores: full / raten,
                                            "threads_1": full / rate1,
                                            "note": "extrapolation from the sample, not run"},
            "config0_16q_20layers_full": {"gates": d0a, "s_1_thread": s0a,
                                          "s_%d_threads" % cores: s0n},
            "config2_twin_20q_full": {"gates": d2a, "s_1_thread": s2a,
                                      "s_%d_threads" % cores: s2n},
            "host": host}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--qubits", type=int, default=30)
    ap.add_argument("--mode", default="tiled")
    ap.add_argument("--k-max", type=int, default=2)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"],
                    help="state type of the main leg (the workload's is complex128)")
    ap.add_argument("--reg-bits", type=int, default=0)
    ap.add_argument("--tile-bits", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-legs", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--fp32-k-max", type=int, default=2)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the 32-qubit precision, batched and adjoint forms")
    ap.add_argument("--only-form", default="",
                    choices=["", "adjoint", "batched", "precision", "fusion", "simcomparison",
                             "emulation", "noise"],
                    help="run just this form, print its JSON object and exit (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the state-vector path here runs on a single MI355X; "
              "a sharded multi-GPU state is not built (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.only_form:
        forms = {"adjoint": form_adjoint, "batched": form_batched, "precision": form_precision,
                 "fusion": lambda: form_fusion_qft(args.qubits),
                 "simcomparison": lambda: form_simcomparison(args.qubits),
                 "emulation": lambda: form_emulation(args.qubits),
                 "noise": form_noise}
        print(json.dumps({args.only_form: forms[args.only_form]()}))
        return

    n = args.qubits
    circ = W.config1_random(n=n)
    ham = step_hamiltonian(n)
    u = W.streams(1)[3].random(1000)
    log("bench: %d qubits, %d gates, mode=%s k_max=%d" % (n, len(circ.gates), args.mode, args.k_max))

    main_leg = run_leg(circ, ham, u, args.steps, args.warmup, args.dtype, args.mode, args.k_max,
                       args.tile_bits, reg_bits=args.reg_bits)
    log("main leg: %.2f ms/step" % main_leg["ms_per_step"])
    steps = args.steps
    value = main_leg["updates_per_step"] * steps / main_leg["wall_s"]
    st = main_leg["stats"]
    alg_bytes_step = st["alg_bytes"] / steps
    pct_hbm = alg_bytes_step / (main_leg["ms_per_step"] * 1e-3) / HBM_PEAK

    log("copy probe ...")
    copy = copy_bandwidth()
    log("copy probe: %.0f GB/s" % copy["GBps"])
    kt = main_leg["ktimes"]
    dom = "tile" if kt.get("tile", (0, 0, 0))[1] > 0 else "dense"
    ms, launches, kbytes = kt[dom]
    per_launch_bytes = kbytes / max(launches, 1)
    avg_ms = ms / max(launches, 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) if avg_ms > 0 else 0.0
    rname = "double" if args.dtype == "c128" else "float"
    default_cfg = (args.dtype == "c128" and args.mode == "tiled" and args.k_max == 2
                   and args.reg_bits in (0, 4) and args.tile_bits in (0, 12))
    if dom != "tile":
        kname = "k_dense<%s,1>" % rname
    elif args.k_max <= 2:
        # the real split leaves diagonal phases as table ops: passes with one
        # run the kernel instance with that case
        rb = args.reg_bits or 4
        tb = (args.tile_bits or 12) - rb
        # both instances: with table ops (most passes) and without (the
        # passes that only move qubits back to their own positions)
        kname = "k_tile_reg<%s,%d,%d,*>" % (rname, rb, tb)
    else:
        kname = "k_tile_lds<%s,k<=%d> (MFMA for k>=3)" % (rname, args.k_max)
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK,
                "traffic": measured_traffic() if default_cfg else None,
                "kernel": kname,
                "launches": launches, "avg_ms": avg_ms, "alg_bytes_per_launch": per_launch_bytes,
                "copy_GBps": copy["GBps"], "frac_of_copy": achieved / (copy["GBps"] * 1e9)}
    if dom == "tile" and avg_ms > 0:
        # the same launches against the vector-ALU peak (FP64, and FP32 with
        # packed math off, are both 78.6 TFLOP/s): the pass's arithmetic
        # intensity sits close to the FP64 ridge point
        fl = st["alg_flops"] / max(launches, 1)
        roofline["alu"] = {"achieved_TFLOPs": fl / (avg_ms * 1e-3) / 1e12,
                           "peak_TFLOPs": FP64_PEAK / 1e12,
                           "frac": fl / (avg_ms * 1e-3) / FP64_PEAK,
                           "alg_flops_per_launch": fl}

    extra = {}
    if not args.no_extra_legs:
        leg32 = run_leg(circ, ham, u, steps, 1, "c64", args.mode, args.fp32_k_max, 0)
        ms32, l32, b32 = leg32["ktimes"]["tile"]
        err32 = fp32_state_error(circ)
        log("fp32 state error: %.3g" % err32)
        extra["fp32_fused"] = {
            "value": leg32["updates_per_step"] * steps / leg32["wall_s"],
            "ms_per_step": leg32["ms_per_step"],
            "state_rel_err_vs_fp64_all_amplitudes": err32,
            "pct_hbm_peak": leg32["stats"]["alg_bytes"] / steps / (leg32["ms_per_step"] * 1e-3)
            / HBM_PEAK,
            "tile_kernel_GBps": (b32 / max(l32, 1)) / (ms32 / max(l32, 1) * 1e-3) / 1e9 if ms32 else None,
            "energy_abs_diff_vs_fp64": abs(leg32["energy"] - main_leg["energy"]),
            "speedup_vs_fp64_fused": main_leg["ms_per_step"] / leg32["ms_per_step"],
        }
        if ms32:
            # the FP32 tile kernel against both bounds: HBM (half the bytes
            # of FP64) and the vector ALU (FP32 issues at the FP64 rate here:
            # packed FP32 math is off)
            f32 = leg32["stats"]["alg_flops"] / max(l32, 1)
            t32 = ms32 / max(l32, 1) * 1e-3
            gbps = (b32 / max(l32, 1)) / t32
            extra["fp32_fused"]["roofline"] = {
                "hbm_frac": gbps / HBM_PEAK, "frac_of_copy": gbps / (copy["GBps"] * 1e9),
                "alu_TFLOPs": f32 / t32 / 1e12, "alu_frac": f32 / t32 / FP64_PEAK,
                "bound": "alu" if f32 / t32 / FP64_PEAK > gbps / (copy["GBps"] * 1e9) else "hbm"}
        log("fp32 leg: %.2f ms/step" % leg32["ms_per_step"])
        pg = run_leg(circ, ham, u, 1, 0, "c128", "pergate", 1, 0, reduce=False)
        d_ms, d_l, d_b = pg["ktimes"]["dense"]
        m_ms, m_l, m_b = pg["ktimes"]["mono"]
        extra["fp64_pergate"] = {
            "value": pg["updates_per_step"] / pg["wall_s"],
            "ms_per_step": pg["ms_per_step"],
            "dense_1q_GBps": d_b / (d_ms * 1e-3) / 1e9 if d_ms else None,
            "cnot_GBps": m_b / (m_ms * 1e-3) / 1e9 if m_ms else None,
            "dense_1q_frac_of_copy": d_b / (d_ms * 1e-3) / (copy["GBps"] * 1e9) if d_ms else None,
            "cnot_frac_of_copy": m_b / (m_ms * 1e-3) / (copy["GBps"] * 1e9) if m_ms else None,
            "pct_hbm_peak": pg["stats"]["alg_bytes"] / (pg["ms_per_step"] * 1e-3) / HBM_PEAK,
        }
        extra["fp64_fused_speedup_vs_fp64_pergate"] = pg["ms_per_step"] / main_leg["ms_per_step"]
        extra["fp32_fused"]["speedup_vs_fp64_pergate"] = pg["ms_per_step"] / leg32["ms_per_step"]
        log("per-gate leg: %.2f ms/step" % pg["ms_per_step"])
    if not args.no_forms:
        extra["fusion_and_qft_30q"] = form_fusion_qft(n)
        log("fusion / QFT form done")
        extra["paper_benchmark_circuit_30q"] = form_simcomparison(n)
        log("paper benchmark circuit form done")
        extra["precision_32q"] = form_precision()
        log("precision form done")
        extra["batched"] = form_batched()
        log("batched form done")
        extra["emulation_30q"] = form_emulation(n)
        log("emulation form done")
        extra["noise_density_matrix_15q"] = form_noise()
        log("noise form done")
        extra["adjoint_24q"] = form_adjoint()
        log("adjoint form done")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        cpu = cpu_baseline(circ, args.cpu_budget)

    line = {
        "metric": "amplitude*gate updates/s + % HBM peak, 30q random circuit; fp64 vs fused fp32",
        "value": value,
        "unit": "amp*gate/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": "%d-qubit random circuit, 40 layers of Haar 1q + CNOT brick "
                               "(%d gates), %s from |0..0>, then norm, 8-term <H>, "
                               "1000 samples" % (n, len(circ.gates),
                                                 "complex128" if args.dtype == "c128" else "complex64"),
                   "n_qubits": n, "gates": len(circ.gates), "mode": args.mode,
                   "k_max": args.k_max, "tile_bits": args.tile_bits or 12,
                   "reg_bits": args.reg_bits or 4},
        "pct_hbm_peak": pct_hbm,
        "alg_bytes_per_step": alg_bytes_step,
        "hbm_passes_per_step": st["passes"] / steps,
        "fused_ops_per_step": st["fused_ops"] / steps,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": extra,
        "check": {"norm2": main_leg["norm2"], "energy": main_leg["energy"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
