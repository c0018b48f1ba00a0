"""Density matrices (noise) on the GPU against the CPU oracle.

vec(rho) lives on 2n qubits and every gate (U on the row bits, conj(U) on
the column bits) and every Kraus channel (its superoperator on the row and
column bits) runs through the ordinary fusion and tile passes.  Bars: rho,
the probabilities and Tr(rho H) within 1e-12 (complex128) or 1e-5 (complex64)
of the oracle's density matrix; at 13 qubits (a 26-qubit vector), where the
oracle's matrices are too large, trace, Hermiticity and a pure-state check
against the state-vector path.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

Q = None


def setup_module(module):
    global Q
    from paper_1612_08091_amd import qsv
    Q = qsv


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode,k_max", [("tiled", 2), ("tiled", 4), ("pergate", 1), ("fused", 3)])
def test_noisy_brick_against_oracle(mode, k_max):
    n = 5
    rng = np.random.default_rng(50)
    ev = W.noisy_brick(n, 3, 0.02, rng, gamma=0.05)
    log("noisy brick", mode, k_max, len(ev), "events")
    d = Q.DensityMatrix(n, mode=mode, k_max=k_max, use_torch_stream=False)
    d.run(ev)
    rho = d.matrix()
    probs = d.probabilities()
    ham = W.random_pauli_dense(n, 16, np.random.default_rng(51))
    e = d.expectation(ham)
    d.close()
    want = oracle.dm_run(ev, n)
    assert np.max(np.abs(rho - want)) <= 1e-12
    assert np.max(np.abs(probs - np.real(np.diag(want)))) <= 1e-12
    assert abs(e - oracle.dm_expectation(want, ham)[0]) <= 1e-12 * np.sum(np.abs(ham.coeff))


def test_noisy_circuit_c64():
    n = 6
    rng = np.random.default_rng(52)
    ev = W.noisy_brick(n, 3, 0.01, rng, gamma=0.02)
    d = Q.DensityMatrix(n, dtype="c64", use_torch_stream=False)
    d.run(ev)
    rho = d.matrix().astype(np.complex128)
    probs = d.probabilities()
    d.close()
    want = oracle.dm_run(ev, n)
    assert np.linalg.norm(rho - want) / np.linalg.norm(want) <= 1e-5
    assert np.max(np.abs(probs - np.real(np.diag(want)))) <= 1e-5


def test_two_qubit_channels_and_controlled_gates():
    n = 5
    rng = np.random.default_rng(53)
    q, _ = np.linalg.qr(rng.standard_normal((12, 4)) + 1j * rng.standard_normal((12, 4)))
    kr = [np.ascontiguousarray(q[4 * j:4 * j + 4, :]) for j in range(3)]   # 2-qubit channel
    ev = [("gate", W.H, (0,), ()), ("gate", W.haar_unitary(4, rng), (1, 3), (0,)),
          ("kraus", kr, (3, 1)), ("gate", W.X, (4,), (1, 2)), ("kraus", W.dephasing(0.3), (4,)),
          ("gate", W.haar_2x2(rng), (2,), (4,)), ("kraus", kr, (0, 4))]
    d = Q.DensityMatrix(n, use_torch_stream=False)
    d.run(ev)
    rho = d.matrix()
    d.close()
    want = oracle.dm_run(ev, n)
    assert np.max(np.abs(rho - want)) <= 1e-12
    assert abs(np.trace(rho) - 1.0) <= 1e-12


def test_pure_state_13q_matches_state_vector():
    """Without noise, rho = |psi><psi| with psi from the state-vector path
    (sampled entries), and the trace stays 1 (26-qubit vector)."""
    n = 13
    rng = np.random.default_rng(54)
    circ = W.random_brick(n, 4, rng, "cnot")
    d = Q.DensityMatrix(n)
    for g in circ.gates:
        d.apply(g.matrix, g.targets, g.controls)
    d.flush()
    s = Q.Simulator(n_max=n)
    s.allocate(n)
    s.run(circ)
    psi = s.get_state()
    s.close()
    r = rng.integers(0, 1 << n, 2048, dtype=np.uint64)
    c = rng.integers(0, 1 << n, 2048, dtype=np.uint64)
    got = d.sim.get_amplitudes(r + (c << np.uint64(n)))
    want = psi[r.astype(np.int64)] * np.conj(psi[c.astype(np.int64)])
    assert np.max(np.abs(got - want)) <= 1e-12
    p = d.probabilities()
    assert abs(p.sum() - 1.0) <= 1e-12
    assert np.max(np.abs(p - np.abs(psi) ** 2)) <= 1e-12
    d.close()


def test_noisy_13q_trace_hermiticity_and_full_depolarization():
    n = 13
    rng = np.random.default_rng(55)
    d = Q.DensityMatrix(n)
    d.run(W.noisy_brick(n, 3, 0.01, rng, gamma=0.01))
    d.flush()
    p = d.probabilities()
    assert abs(p.sum() - 1.0) <= 1e-12 and p.min() >= -1e-15
    r = rng.integers(0, 1 << n, 2048, dtype=np.uint64)
    c = rng.integers(0, 1 << n, 2048, dtype=np.uint64)
    a = d.sim.get_amplitudes(r + (c << np.uint64(n)))
    b = d.sim.get_amplitudes(c + (r << np.uint64(n)))
    assert np.max(np.abs(a - np.conj(b))) <= 1e-13
    # depolarize qubit 0 completely: every Pauli term acting on it vanishes
    d.channel(W.depolarizing(1.0), [0])
    ham = W.PauliSum.from_strings(["X" + "I" * (n - 1), "Z" + "I" * (n - 1), "Y" + "Z" * (n - 1)],
                                  [1.0, 1.0, 1.0])
    assert abs(d.expectation(ham)) <= 1e-13
    d.close()
