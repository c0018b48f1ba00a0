"""Batched form on the GPU: many HEA circuits of uneven size, each with its
own Pauli sum, evaluated by one HIP-graph replay (circuits that fit in LDS
in one persistent launch, larger ones pass-major).

Bars: complex128 batches within 1e-12 * sum|c| of the oracle; complex64
batches within 1e-5 * sum|c| (the FP32 tolerance on reductions).  Graph
replays are checked against an eager (non-graph) run, with other device work
between the replays.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def small_batch(count, n_lo, n_hi, layers, terms, seed):
    rng = np.random.default_rng(seed)
    circuits, hams = [], []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        circuits.append(W.hea(n, layers, rng.uniform(0, 2 * math.pi, 2 * n * layers)))
        hams.append(W.random_pauli_dense(n, terms, rng))
    return circuits, hams


@pytest.mark.parametrize("dtype,tile_bits", [("c128", 10), ("c128", 8), ("c64", 12), ("c64", 9)])
def test_batch_matches_oracle(dtype, tile_bits):
    from paper_1612_08091_amd import qsv as Q
    # sizes on both sides of the LDS-resident limit
    circuits, hams = small_batch(40, 3, 14, 3, 16, seed=41 + tile_bits)
    b = Q.Batch(circuits, hams, dtype=dtype, autotune=False, tile_bits=tile_bits)
    got = b.run()
    want = np.array([oracle.energy(c, h) for c, h in zip(circuits, hams)])
    scale = np.array([np.sum(np.abs(h.coeff)) for h in hams])
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert np.all(np.abs(got - want) <= tol * scale), np.max(np.abs(got - want) / scale)
    b.close()


def test_batch_graph_replays_equal_eager():
    import torch
    from paper_1612_08091_amd import qsv as Q
    circuits, hams = small_batch(64, 4, 15, 4, 12, seed=43)
    eager = Q.Batch(circuits, hams, dtype="c64", autotune=False, tile_bits=11, use_graph=False)
    ref = eager.run()
    g = Q.Batch(circuits, hams, dtype="c64", autotune=False, tile_bits=11, use_graph=True)
    x = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        out = g.run()
        assert np.array_equal(out, ref), rep
        y = (x * 2.0 + 1.0).sum()     # unrelated device work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y)
    eager.close()
    g.close()


def test_batch_autotune_and_cache(tmp_path):
    from paper_1612_08091_amd import qsv as Q
    circuits, hams = small_batch(24, 6, 16, 2, 8, seed=44)
    cache = str(tmp_path / "tune.json")
    b = Q.Batch(circuits, hams, dtype="c64", autotune=True, tune_cache=cache)
    info = b.info()
    out1 = b.run()
    b.close()
    b2 = Q.Batch(circuits, hams, dtype="c64", autotune=True, tune_cache=cache)
    assert b2.info()["tile_bits"] == info["tile_bits"] and b2.info()["k_fuse"] == info["k_fuse"]
    want = np.array([oracle.energy(c, h) for c, h in zip(circuits, hams)])
    scale = np.array([np.sum(np.abs(h.coeff)) for h in hams])
    assert np.all(np.abs(b2.run() - want) <= 1e-5 * scale)
    assert np.all(np.abs(out1 - want) <= 1e-5 * scale)
    b2.close()


def test_config3_full_batch_against_single_circuit_fp64_and_oracle():
    """The benched batch itself: all 4096 circuits of config 3 (complex64,
    autotuned, graph-captured) against the non-batched FP64 path run circuit
    by circuit on the GPU, every <H> within 1e-5 * sum|c|; a seeded 64 of
    them also against the oracle."""
    from paper_1612_08091_amd import qsv as Q
    circuits, hams = W.config3()
    assert len(circuits) == 4096
    b = Q.Batch(circuits, hams, dtype="c64", autotune=True, use_graph=True)
    got = b.run()
    b.close()
    scale = np.array([np.sum(np.abs(h.coeff)) for h in hams])
    sims = {}
    ref = np.zeros(len(circuits))
    for i, (c, h) in enumerate(zip(circuits, hams)):
        if c.n not in sims:
            sims[c.n] = Q.Simulator(n_max=c.n, dtype="c128", mode="tiled", k_max=2)
            sims[c.n].allocate(c.n)
        s = sims[c.n]
        s.reset()
        s.run(c)
        s.flush()
        ref[i] = s.expectation(h)
    for s in sims.values():
        s.close()
    err = np.abs(got - ref) / scale
    assert np.all(err <= 1e-5), (int(np.argmax(err)), float(np.max(err)))
    pick = np.random.default_rng(45).choice(len(circuits), size=64, replace=False)
    oracle.set_threads(8)
    try:
        for i in pick:
            want = oracle.energy(circuits[i], hams[i])
            assert abs(ref[i] - want) <= 1e-12 * scale[i], i
            assert abs(got[i] - want) <= 1e-5 * scale[i], i
    finally:
        oracle.set_threads(1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_tiny_and_empty_circuits(dtype):
    from paper_1612_08091_amd import qsv as Q
    # 1- and 2-qubit circuits (some with no gates at all), and a batch that
    # holds a single circuit
    rng = np.random.default_rng(47)
    circuits, hams = [], []
    for i in range(12):
        n = 1 + i % 2
        c = W.Circuit(n)
        for _ in range(0 if i % 3 == 0 else 6):
            c.add(W.haar_2x2(rng), (int(rng.integers(0, n)),))
            if n == 2:
                c.add(W.X, (1,), (0,))
        circuits.append(c)
        hams.append(W.random_pauli_dense(n, 4, rng))
    tol = 1e-12 if dtype == "c128" else 1e-5
    for lo, hi in [(0, 12), (5, 6)]:
        b = Q.Batch(circuits[lo:hi], hams[lo:hi], dtype=dtype, autotune=False)
        got = b.run()
        want = np.array([oracle.energy(c, h) for c, h in zip(circuits[lo:hi], hams[lo:hi])])
        scale = np.array([np.sum(np.abs(h.coeff)) for h in hams[lo:hi]])
        assert np.all(np.abs(got - want) <= tol * scale), np.max(np.abs(got - want) / scale)
        b.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_pass_major_and_per_workgroup_paths(dtype):
    """Circuits whose state exceeds the LDS tile run pass-major by default
    (one launch per pass index over every such circuit's tiles, Pauli sums in
    chunks) or, with big_per_workgroup, each on one workgroup.  Both paths
    against the oracle, on a batch that mixes sizes on both sides of the tile
    (with circuits that have no gates at all on the big side), on a batch
    where every circuit is big and on a batch of one big circuit; a 16-qubit
    circuit spans several Pauli chunks."""
    from paper_1612_08091_amd import qsv as Q
    rng = np.random.default_rng(48)
    circuits, hams = small_batch(20, 4, 13, 2, 8, seed=49)
    for n in (10, 12, 16):
        circuits.append(W.Circuit(n))                    # no gates: |0...0>
        hams.append(W.random_pauli_dense(n, 6, rng))
    circuits.append(W.hea(16, 2, rng.uniform(0, 2 * math.pi, 64)))
    hams.append(W.random_pauli_dense(16, 10, rng))
    want = np.array([oracle.energy(c, h) for c, h in zip(circuits, hams)])
    scale = np.array([np.sum(np.abs(h.coeff)) for h in hams])
    tol = 1e-12 if dtype == "c128" else 1e-5
    big = [i for i, c in enumerate(circuits) if c.n > 9]
    cases = [list(range(len(circuits))), big, [big[-1]]]
    for sel in cases:
        outs = []
        for per_wg in (False, True):
            b = Q.Batch([circuits[i] for i in sel], [hams[i] for i in sel], dtype=dtype,
                        autotune=False, tile_bits=9, big_per_workgroup=per_wg)
            got = b.run()
            b.close()
            err = np.abs(got - want[sel]) / scale[sel]
            assert np.all(err <= tol), (per_wg, len(sel), float(np.max(err)))
            outs.append(got)
        assert np.all(np.abs(outs[0] - outs[1]) <= 2 * tol * scale[sel])
