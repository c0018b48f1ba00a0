"""The register-tile programs, checked on the CPU against the oracle.

The tiled flush lowers every pass to an instruction list for the
register-resident tile kernel: 1- and 2-qubit ops split into diagonal phases
times a real matrix where such a split exists, diagonal ops gathered into
tables, layout changes through LDS, every offset precomputed on the host.
``qsv_check_tile_programs`` runs those lists through the library's host model
of the kernel (thread by thread, with the kernel's LDS offsets and table
lookups, each bounds-checked), so the lowering is tested without a GPU.  The
expected states come from the oracle (one gate at a time in complex128).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

Q = None


def setup_module(module):
    global Q
    from paper_1612_08091_amd import qsv
    Q = qsv


def rand_state(n, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def run_check(circ, psi0, k_max=2, tile_bits=0, reg_bits=0):
    s = Q.Simulator(n_max=circ.n, mode="tiled", k_max=k_max, tile_bits=tile_bits,
                    reg_bits=reg_bits, use_torch_stream=False)
    s.allocate(circ.n)
    s.run(circ)
    got, info = s.check_tile_programs(psi0)
    s.close()
    want = oracle.run(circ, psi0)
    return got, want, info


def random_circuit(rng, n, count):
    """1- and 2-qubit gates of every kind the register kernel runs: Haar
    unitaries, real rotations, controlled gates (controls anywhere in the
    index), diagonal gates and permutations."""
    c = W.Circuit(n)
    for _ in range(count):
        kind = int(rng.integers(0, 9))
        q = rng.permutation(n)[:3].tolist()
        if kind == 0:
            c.add(W.haar_unitary(4, rng), q[:2])
        elif kind == 1:
            c.add(W.haar_2x2(rng), q[:1])
        elif kind == 2:
            c.add(W.ry(float(rng.uniform(0, 6))), q[:1])
        elif kind == 3:
            c.add(W.X, q[:1], q[1:2])
        elif kind == 4:
            c.add(W.phase(float(rng.uniform(0, 6))), q[:1], q[1:2])
        elif kind == 5:
            c.add(W.rz(float(rng.uniform(0, 6))), q[:1])
        elif kind == 6:
            c.add(W.haar_2x2(rng), q[:1], q[1:3])
        elif kind == 7:
            c.add(W.SWAP, q[:2])
        else:
            c.add(W.rx(float(rng.uniform(0, 6))), q[:1], q[1:2])
    return c


@pytest.mark.parametrize("n,tile_bits,reg_bits", [(12, 11, 3), (13, 12, 4), (14, 12, 4),
                                                  (15, 13, 5), (16, 13, 4), (16, 12, 4)])
def test_random_circuits(n, tile_bits, reg_bits):
    rng = np.random.default_rng(100 * n + tile_bits + reg_bits)
    circ = random_circuit(rng, n, 120)
    psi0 = rand_state(n, rng)
    got, want, info = run_check(circ, psi0, tile_bits=tile_bits, reg_bits=reg_bits)
    assert info["reg_passes"] == info["passes"] >= 1
    assert float(np.max(np.abs(got - want))) <= 1e-13


@pytest.mark.parametrize("n", [13, 16])
def test_brick_circuit_splits_into_real_ops(n):
    """The random brick circuit (Haar 1-qubit layers + CNOT brick): every
    fused block after the first layer is CNOT (U x V) = D_L M D_R with M real,
    and the phases of a layer gather into few tables."""
    circ = W.config1_random(n, layers=12)
    rng = np.random.default_rng(5)
    psi0 = rand_state(n, rng)
    got, want, info = run_check(circ, psi0)
    assert float(np.max(np.abs(got - want))) <= 1e-13
    fused = info["real_ops"]
    assert fused >= 0.9 * (12 * (n - 1) // 2)
    # each split op leaves two phase pieces; they share tables, so there are
    # fewer tables than split ops
    assert info["diag_ops"] < fused
    assert info["diag_merged"] >= fused // 2


def test_qft_controlled_phases_and_swaps():
    n = 14
    x = 0x2a5b
    circ = W.Circuit(n)
    for g in W.basis_prep(n, x).gates + W.qft(n).gates:
        circ.gates.append(g)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1.0
    got, want, info = run_check(circ, psi0)
    assert float(np.max(np.abs(got - want))) <= 1e-13
    y = np.arange(1 << n)
    closed = np.exp(2j * math.pi * ((x * y) % (1 << n)) / (1 << n)) / 2 ** (n / 2)
    assert float(np.max(np.abs(got - closed))) <= 1e-12


def test_controls_outside_the_tile():
    """Diagonal and dense ops whose controls lie outside every tile: the
    register kernel reads a table of ones (diagonal) or keeps the old value
    (dense) on the tiles that fail them."""
    n = 15
    rng = np.random.default_rng(9)
    c = W.Circuit(n)
    for _ in range(40):
        t = int(rng.integers(0, 6))
        ctl = int(rng.integers(12, n))
        c.add(W.haar_2x2(rng), (t,), (ctl,))
        c.add(W.phase(float(rng.uniform(0, 6))), (int(rng.integers(0, 12)),), (ctl,))
        c.add(W.rz(float(rng.uniform(0, 6))), (int(rng.integers(0, n)),))
    psi0 = rand_state(n, rng)
    got, want, info = run_check(c, psi0, tile_bits=12)
    assert float(np.max(np.abs(got - want))) <= 1e-13


def test_real_split_identities():
    """Plans that must not split: a layer of 1-qubit gates on both sides of a
    CNOT fuses into a block that is not real up to diagonal phases."""
    n = 12
    rng = np.random.default_rng(3)
    c = W.Circuit(n)
    for q in range(n):
        c.add(W.haar_2x2(rng), (q,))
    for q in range(0, n - 1, 2):
        c.add(W.X, (q + 1,), (q,))
    for q in range(n):
        c.add(W.haar_2x2(rng), (q,))
    psi0 = rand_state(n, rng)
    got, want, info = run_check(c, psi0, tile_bits=12)
    assert float(np.max(np.abs(got - want))) <= 1e-13


@pytest.mark.parametrize("n,layers", [(18, 20), (16, 40), (19, 20)])
def test_relabeling_plans_through_the_kernel_model(n, layers):
    """Passes that move their qubits to other positions inside the tile: the
    stores go to the new positions, the next passes find their qubits there,
    and trailing passes put every qubit back.  At 18 and 19 qubits the tile
    (12 bits) holds positions at and above the 2 MiB page bit (17), so the
    planner also caps how many of those a tile takes.  The 16- and 19-qubit
    plans hold passes without a workgroup remap whose threads store what
    other threads loaded: the host model rejects such a program unless it
    has the barrier before its stores."""
    circ = W.config1_random(n, layers=layers)
    rng = np.random.default_rng(21)
    psi0 = rand_state(n, rng)
    want = oracle.run(circ, psi0.copy())
    s = Q.Simulator(n_max=n, mode="tiled", k_max=2, use_torch_stream=False, relabel=True)
    s.allocate(n)
    s.run(circ)
    got, info = s.check_tile_programs(psi0)
    s.close()
    assert info["relabel_passes"] > 0
    assert float(np.max(np.abs(got - want))) <= 1e-13
    s = Q.Simulator(n_max=n, mode="tiled", k_max=2, use_torch_stream=False, relabel=False)
    s.allocate(n)
    s.run(circ)
    got0, info0 = s.check_tile_programs(psi0)
    s.close()
    assert info0["relabel_passes"] == 0
    assert float(np.max(np.abs(got0 - want))) <= 1e-13


@pytest.mark.parametrize("seed", [1, 2])
def test_relabeling_random_circuits(seed):
    """Every gate kind of the register kernel under relabeling plans (tile of
    11 bits on 15 qubits)."""
    n = 15
    rng = np.random.default_rng(700 + seed)
    circ = random_circuit(rng, n, 150)
    psi0 = rand_state(n, rng)
    got, want, info = run_check(circ, psi0, tile_bits=11, reg_bits=3)
    assert float(np.max(np.abs(got - want))) <= 1e-13


def plan_passes(circ, relabel, dtype="c128", k_max=2):
    s = Q.Simulator(n_max=circ.n, mode="tiled", k_max=k_max, use_torch_stream=False,
                    relabel=relabel, dtype=dtype)
    s.allocate(circ.n)
    s.run(circ)
    ops, npass = s.plan()
    s.close()
    return ops, npass


def test_relabeling_cuts_passes_of_the_30q_brick_circuit():
    """Host-side plan of the 30-qubit random brick circuit: with relabeling
    the three positions every tile holds carry qubits in use and tiles keep
    to few page positions, so fewer passes over the state (62 with fixed
    positions)."""
    circ = W.config1_random(n=30)
    _, fixed = plan_passes(circ, False)
    _, moved = plan_passes(circ, True)
    assert fixed == 62
    assert moved <= 45


def test_relabeling_plan_ops_in_qubit_order():
    """qsv_plan lists a relabeling plan's ops on their qubits' own
    positions: applied one after the other by the oracle they give the
    circuit's state."""
    n = 12
    rng = np.random.default_rng(33)
    circ = random_circuit(rng, n, 100)
    s = Q.Simulator(n_max=n, mode="tiled", k_max=2, tile_bits=8, reg_bits=0,
                    use_torch_stream=False, relabel=True)
    s.allocate(n)
    s.run(circ)
    ops, npass = s.plan()
    s.close()
    s = Q.Simulator(n_max=n, mode="tiled", k_max=2, tile_bits=8, use_torch_stream=False,
                    relabel=False)
    s.allocate(n)
    s.run(circ)
    assert npass < s.plan()[1]
    s.close()
    psi = oracle.zero_state(n)
    for mat, targets, cmask in ops:
        oracle.apply(psi, mat, targets, [p for p in range(64) if (cmask >> p) & 1])
    assert float(np.max(np.abs(psi - oracle.run(circ)))) <= 1e-13
