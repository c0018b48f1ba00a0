"""Host-side tests of libqsv: the library loads and exports every symbol of
include/qsv.h, arguments are validated before any device call, and the
fusion / pass planners (host C++) produce operation lists whose product is
the per-gate product (checked with the CPU oracle).  No GPU is needed: the
library materialises its device state lazily."""
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1612_08091_amd import qsv as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "qsv.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:qsv_status|const char \*)\s*(qsv_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(Q.lib, name), name
    assert Q.lib.qsv_version().decode().startswith("qsv")


def new_sim(n=6, **kw):
    s = Q.Simulator(n_max=kw.pop("n_max", 12), use_torch_stream=False, **kw)
    ids = s.allocate(n)
    return s, ids


def expect_status(code, fn, *args, **kw):
    with pytest.raises(Q.QsvError) as ei:
        fn(*args, **kw)
    assert ei.value.code == code, str(ei.value)


def test_create_validation():
    for kw in [dict(n_max=0), dict(n_max=40), dict(k_max=0), dict(k_max=6),
               dict(tile_bits=3), dict(tile_bits=20), dict(queue_limit=-1)]:
        expect_status(1, Q.Simulator, **dict(kw, use_torch_stream=False))
    opt = Q.Options()
    Q.lib.qsv_options_default(Q.ctypes.byref(opt))
    opt.dtype = 7
    h = Q.ctypes.c_void_p()
    assert Q.lib.qsv_create(Q.ctypes.byref(opt), Q.ctypes.byref(h)) == 1
    assert b"dtype" in Q.lib.qsv_last_error(None)


def test_apply_validation_keeps_handle_usable():
    s, ids = new_sim(4)
    expect_status(1, s.apply, W.H, [9])                   # unknown id
    expect_status(1, s.apply, W.X, [1], [1])              # target == control
    expect_status(1, s.apply, W.SWAP, [2, 2])             # repeated target
    expect_status(1, s.apply, np.eye(64), list(range(6))) # k > 5 (and > n)
    bad = W.H.copy()
    bad[0, 0] = np.nan
    expect_status(1, s.apply, bad, [0])                   # non-finite entry
    bad[0, 0] = np.inf
    expect_status(1, s.apply, bad, [0])
    s.apply(W.H, [0])                                     # still usable
    s.apply(W.X, [1], [0])
    ops, npass = s.plan()
    assert len(ops) >= 1


def test_apply_math_validation_before_any_device_work():
    s, ids = new_sim(6)
    add3 = W.add_constant_table(3, 3)
    expect_status(1, s.apply_math, [0, 1, 9], add3)                 # unknown id
    expect_status(1, s.apply_math, [0, 1, 1], add3)                 # repeated qubit
    expect_status(1, s.apply_math, [0, 1, 2], add3, [2])            # control in the register
    expect_status(1, s.apply_math, [0, 1, 2], np.array([0, 1, 2, 3, 4, 5, 6, 6]))  # not a bijection
    expect_status(1, s.apply_math, [0, 1, 2], np.array([0, 1, 2, 3, 4, 5, 6, 8]))  # value >= 2^w
    expect_status(1, s.apply_math, [0, 1, 2, 3, 4], W.add_constant_table(5, 1), [5, 0])  # w + c > n
    for w in (0, 27):                                               # width outside 1..26
        tab = np.zeros(4, dtype=np.uint32)
        q = np.arange(6, dtype=np.int32)
        assert Q.lib.qsv_apply_math(s._h, w, Q._ptr(q), Q._ptr(tab), 0, Q._ptr(q)) == 1
    # the pending queue is untouched by the rejected calls
    s.apply(W.H, [0])
    ops, npass = s.plan()
    assert len(ops) == 1


def test_math_table_packs_registers():
    # two registers (3 and 2 bits): (a, b) -> (a + b mod 8, b)
    tab = Q.math_table(lambda a, b: ((a + b) % 8, b), [3, 2])
    assert tab.shape == (32,)
    for a in range(8):
        for b in range(4):
            assert tab[a | (b << 3)] == ((a + b) % 8) | (b << 3)
    assert np.array_equal(np.sort(tab), np.arange(32))


def test_allocation_limits_and_ids():
    s = Q.Simulator(n_max=5, use_torch_stream=False)
    assert s.allocate(3) == [0, 1, 2]
    expect_status(2, s.allocate, 3)                       # exceeds n_max
    assert s.allocate(2) == [3, 4]
    # deallocating |0> qubits of an untouched state is bookkeeping only
    s.deallocate(1)
    assert s.qubits() == [0, 2, 3, 4]
    assert s.allocate(1) == [1]                           # lowest free id reused
    assert s.qubits() == [0, 2, 3, 4, 1]                  # takes the highest position
    expect_status(1, s.deallocate, 7)


def test_use_after_destroy():
    s, _ = new_sim(2)
    h = s._h
    s.close()
    code = Q.lib.qsv_flush(h)
    assert code == 5                                      # QSV_ESTATE
    assert Q.lib.qsv_destroy(h) == 5


def test_reductions_validate_before_device():
    s, ids = new_sim(3)
    expect_status(1, s.get_probability, [0, 0], [1, 1])   # repeated qubit
    expect_status(1, s.get_probability, [5], [1])         # unknown qubit
    expect_status(1, s.measure, [0], [1.0])               # u outside [0,1)
    expect_status(1, s.sample, [0.5, -0.1])
    expect_status(1, s.get_expectation, [1 << 9], [0], [1.0])   # term on unknown id
    expect_status(1, s.get_amplitudes, [8])               # index >= 2^n


def test_apply_diag_validation_and_plan():
    s, ids = new_sim(3)
    assert Q.lib.qsv_apply_diag(s._h, None, 1, Q._ptr(np.zeros(1, np.int32)), 0, None) == 1
    d = np.exp(1j * np.array([0.1, 0.2, 0.3, 0.4]))
    expect_status(1, s.apply_diag, d, [0, 0])            # repeated target
    expect_status(1, s.apply_diag, d, [0, 7])            # unknown id
    bad = d.copy()
    bad[2] = np.nan
    expect_status(1, s.apply_diag, bad, [0, 1])          # non-finite entry
    s.apply_diag(d, [2, 0], [1])                         # queued as the diagonal matrix
    ops, npass = s.plan()
    assert len(ops) == 1
    mat, targets, cmask = ops[0]
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    want = oracle.apply(psi.copy(), np.diag(d), [2, 0], [1])
    controls = [p for p in range(64) if (cmask >> p) & 1]
    got = oracle.apply(psi.copy(), mat, targets, controls)
    assert np.max(np.abs(got - want)) <= 1e-15


def test_sampled_channel_validates_before_device():
    s, ids = new_sim(3)
    ad = W.amplitude_damping(0.2)
    expect_status(1, s.apply_kraus_sampled, ad, [0], 1.0)          # u outside [0,1)
    expect_status(1, s.apply_kraus_sampled, ad, [0], -0.5)
    expect_status(1, s.apply_kraus_sampled, ad, [7], 0.5)          # unknown id
    two = [np.kron(a, b) for a in ad for b in ad]
    expect_status(1, s.apply_kraus_sampled, two, [1, 1], 0.5)      # repeated id
    three = [np.eye(8)]
    expect_status(1, s.apply_kraus_sampled, three, [0, 1, 2], 0.5)  # k > 2
    bad = [ad[0].copy(), ad[1].copy()]
    bad[1][0, 1] = np.nan
    expect_status(1, s.apply_kraus_sampled, bad, [0], 0.5)         # non-finite entry


# ----------------------------------------------------------- planner exactness
def planned_product(sim, n):
    ops, npass = sim.plan()
    psi = oracle.zero_state(n)
    psi[:] = 0
    return ops, npass


def apply_plan_with_oracle(ops, psi):
    for mat, targets, cmask in ops:
        controls = [p for p in range(64) if (cmask >> p) & 1]
        oracle.apply(psi, mat, targets, controls)
    return psi


def random_circuit(rng, n, count):
    c = W.Circuit(n)
    for _ in range(count):
        kind = rng.integers(0, 6)
        if kind == 0:
            k = int(rng.integers(1, 4))
            qs = rng.permutation(n)[:k].tolist()
            c.add(W.haar_unitary(1 << k, rng), qs)
        elif kind == 1:
            a, b = rng.permutation(n)[:2].tolist()
            c.add(W.X, (b,), (a,))
        elif kind == 2:
            a, b = rng.permutation(n)[:2].tolist()
            c.add(W.phase(float(rng.uniform(0, 6))), (b,), (a,))
        elif kind == 3:
            a, b = rng.permutation(n)[:2].tolist()
            c.add(W.SWAP, (a, b))
        elif kind == 4:
            qs = rng.permutation(n)[:3].tolist()
            c.add(W.haar_2x2(rng), qs[:1], qs[1:])
        else:
            q = int(rng.integers(0, n))
            c.add(W.rz(float(rng.uniform(0, 6))), (q,))
    return c


@pytest.mark.parametrize("mode,k_max,tile_bits", [
    ("pergate", 1, 0), ("fused", 2, 0), ("fused", 3, 0), ("fused", 4, 0), ("fused", 5, 0),
    ("tiled", 1, 6), ("tiled", 2, 6), ("tiled", 3, 7), ("tiled", 5, 8), ("tiled", 4, 0)])
def test_plan_equals_per_gate(rng, mode, k_max, tile_bits):
    n = 10
    for rep in range(3):
        circ = random_circuit(rng, n, 60)
        s = Q.Simulator(n_max=n, mode=mode, k_max=k_max, tile_bits=tile_bits,
                        use_torch_stream=False)
        s.allocate(n)
        s.run(circ)
        ops, npass = s.plan()
        want = oracle.run(circ)
        got = apply_plan_with_oracle(ops, oracle.zero_state(n))
        assert np.max(np.abs(got - want)) <= 1e-13
        assert len(ops) <= len(circ.gates)
        if mode == "fused":
            # a fused op spans at most k_max qubits, unless it is a single
            # original gate that was wider than k_max to begin with
            widest = max(len(g.targets) + len(g.controls) for g in circ.gates)
            assert all(len(t) + bin(cm).count("1") <= max(k_max, widest) for _, t, cm in ops)
        s.close()


def test_fusion_reduces_passes_on_brick_circuit():
    circ = W.random_brick(20, 6, np.random.default_rng(3), "cnot")
    counts = {}
    for mode, k in [("pergate", 1), ("fused", 2), ("fused", 5), ("tiled", 3)]:
        s = Q.Simulator(n_max=20, mode=mode, k_max=k, use_torch_stream=False)
        s.allocate(20)
        s.run(circ)
        ops, npass = s.plan()
        counts[(mode, k)] = npass
        s.close()
    assert counts[("pergate", 1)] == len(circ.gates)
    assert counts[("fused", 2)] < counts[("pergate", 1)]
    assert counts[("fused", 5)] < counts[("fused", 2)]
    assert counts[("tiled", 3)] < counts[("fused", 5)]


def test_canonical_forms_drop_identities_and_extract_controls():
    s, ids = new_sim(4, mode="pergate")
    cz_dense = np.diag([1, 1, 1, -1]).astype(complex)
    s.apply(cz_dense, [0, 1])          # CZ given as a 4x4 dense diagonal
    s.apply(np.eye(2), [2])            # identity: dropped
    cnot_dense = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], complex)
    s.apply(cnot_dense, [0, 1])        # control on bit 0 hidden in the matrix
    ops, _ = s.plan()
    assert len(ops) == 2
    (m0, t0, c0), (m1, t1, c1) = ops
    assert len(t0) == 1 and bin(c0).count("1") == 1
    assert len(t1) == 1 and c1 == 1 and t1 == [1]


# ----------------------------------------------------------------- bench.py
def test_bench_refuses_more_than_one_gpu():
    # the measured path runs on one GPU; the check comes before any GPU work
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_traffic_is_tied_to_the_kernel_sources():
    # bench.py reports measured HBM traffic only while the digest of the
    # kernel's sources is the one the counters were taken with
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    t = dict(b.TRAFFIC)
    got = b.measured_traffic()
    if t["digest"] == b.kernel_source_digest():
        assert got == 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])
    else:
        assert got is None
    b.TRAFFIC["digest"] = "0" * 16
    try:
        assert b.measured_traffic() is None
    finally:
        b.TRAFFIC.update(t)


def test_enomem_decided_on_the_host_before_allocating():
    """With a mem_limit the allocation decision needs no device: the first
    flush of a state larger than the limit fails with ENOMEM before any HIP
    call, and the queue and the register stay as they were."""
    s = Q.Simulator(n_max=20, mem_limit=1 << 20, use_torch_stream=False)
    ids = s.allocate(20)
    s.apply(W.H, [ids[0]])
    s.apply(W.X, [ids[1]], [ids[0]])
    with pytest.raises(Q.QsvError) as ei:
        s.flush()
    assert ei.value.code == 2
    assert "16777216 bytes" in str(ei.value) and "mem_limit" in str(ei.value)
    ops, _ = s.plan()
    assert len(ops) == 1        # the queue is kept (H and CNOT fuse into one op)
    with pytest.raises(Q.QsvError) as ei:
        s.flush()
    assert ei.value.code == 2
    s.close()
