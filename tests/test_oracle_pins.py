"""Pins of the CPU oracle against things other than itself.

Each function of ``oracle`` is checked against an independent route to the
same number: dense Kronecker-product operators (tests/brute.py), closed forms
(GHZ, W, QFT of a basis state, Draper addition, Grover's success probability),
library routines (numpy FFT, cumsum + searchsorted), invariants (norm, U^dag U,
Pauli purity) and the worked examples the paper prints (the 3-qubit Entangle
histogram of Sec. 4.3.1, teleportation and Grover of App. A).

Pinned: apply, run, probs, prob_bits, norm2, expectation, measure, sample,
dealloc, allocate, grad_param_shift, grad_fd, apply_math (emulated math gates:
closed forms of AddConstant and modular multiplication on basis states, the
QFT-phase-QFT^-1 construction of AddConstant through ``apply`` and through the
gate-level Draper adder, the X gate as the 1-bit table), dm_apply / dm_kraus /
dm_expectation (pure states against the state-vector oracle, closed forms of
the depolarizing, amplitude-damping and dephasing channels, trace
preservation, Kronecker-product operators from tests/brute.py), kraus_sample
(closed forms of the bit-flip and amplitude-damping branches, the branch
probabilities against dense operators, the probability-weighted branches
against the density-matrix channel, the tie rule at a running-sum boundary).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_gate(rng, n, kmax=3, cmax=2):
    k = int(rng.integers(1, kmax + 1))
    c = int(rng.integers(0, min(cmax, n - k) + 1))
    qs = rng.permutation(n)[: k + c].tolist()
    return W.haar_unitary(1 << k, rng), qs[:k], qs[k:]


def random_state(rng, n):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------- apply / run
@pytest.mark.parametrize("n", [1, 3, 5, 8])
def test_apply_matches_dense_operator(rng, n):
    for _ in range(25 if n < 8 else 10):
        u, t, c = random_gate(rng, n, kmax=min(3, n), cmax=2)
        psi = random_state(rng, n)
        want = brute.gate_operator(u, t, c, n) @ psi
        got = oracle.apply(psi.copy(), u, t, c)
        assert np.max(np.abs(got - want)) <= 1e-13


def test_apply_target_order_matters(rng):
    # bit j of the matrix index belongs to targets[j]: swapping the target list
    # must equal conjugating U by SWAP.
    n = 4
    u = W.haar_unitary(4, rng)
    psi = random_state(rng, n)
    a = oracle.apply(psi.copy(), u, [1, 3])
    b = oracle.apply(psi.copy(), W.SWAP @ u @ W.SWAP, [3, 1])
    assert np.max(np.abs(a - b)) <= 1e-14


def test_circuit_matches_dense_product(rng):
    circ = W.random_brick(6, 5, rng, "cnot")
    psi = oracle.run(circ)
    want = brute.circuit_operator(circ)[:, 0]
    assert np.max(np.abs(psi - want)) <= 1e-13


def test_config0_norm_preserved():
    circ, _ = W.config0()
    assert len(circ.gates) == 470 and circ.counts() == {"haar": 320, "cnot": 150}
    psi = oracle.run(circ)
    assert abs(oracle.norm2(psi) - 1.0) <= 1e-13 * len(circ.gates)


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [2, 3, 7, 12])
def test_ghz_closed_form(n):
    psi = oracle.run(W.ghz(n))
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) <= 1e-15


def test_entangle_histogram_golden():
    # Sec. 4.3.1: Entangle on 3 qubits; the noiseless outcome is 50 % all-zeros
    # and 50 % all-ones.
    with open(os.path.join(GOLDEN, "entangle_3q.json")) as f:
        gold = json.load(f)
    p = oracle.probs(oracle.run(W.ghz(3)))
    for idx, want in enumerate(gold["probabilities"]):
        assert abs(p[idx] - want) <= 1e-15


@pytest.mark.parametrize("n", [2, 5, 9])
def test_w_state_closed_form(n):
    psi = oracle.run(W.w_state(n))
    want = np.zeros(1 << n, dtype=np.complex128)
    for q in range(n):
        want[1 << q] = 1 / math.sqrt(n)
    assert np.max(np.abs(psi - want)) <= 1e-14


@pytest.mark.parametrize("n,x", [(3, 5), (6, 37), (10, 681)])
def test_qft_of_basis_state(n, x):
    psi = oracle.run(W.qft(n), oracle.basis_state(n, x))
    y = np.arange(1 << n)
    closed = np.exp(2j * math.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    e = np.zeros(1 << n)
    e[x] = 1.0
    fft = np.fft.ifft(e) * math.sqrt(1 << n)   # numpy's inverse DFT has the + sign
    assert np.max(np.abs(psi - closed)) <= 1e-13
    assert np.max(np.abs(psi - fft)) <= 1e-13


def test_qft_gate_counts():
    c = W.qft(30)
    assert c.counts() == {"h": 30, "cphase": 435, "swap": 15}


def test_qft_dagger_is_inverse(rng):
    n = 7
    psi = random_state(rng, n)
    out = oracle.run(W.qft(n, inverse=True), oracle.run(W.qft(n), psi.copy()))
    assert np.max(np.abs(out - psi)) <= 1e-13


@pytest.mark.parametrize("n,x,c", [(4, 3, 11), (6, 50, 27), (8, 200, 113)])
def test_draper_adder(n, x, c):
    # Sec. 3: QFT, phases from the bits of c, inverse QFT maps |x> to |x+c mod 2^n>.
    psi = oracle.run(W.draper_add(n, c), oracle.basis_state(n, x))
    p = oracle.probs(psi)
    assert abs(p[(x + c) % (1 << n)] - 1.0) <= 1e-12


def test_cnot_flip_identity(rng):
    # Sec. 4.3.1: a CNOT with control and target exchanged equals the original
    # conjugated by Hadamards on both qubits.
    n = 5
    psi = random_state(rng, n)
    a = oracle.apply(psi.copy(), W.X, [3], [1])
    b = psi.copy()
    for q in (1, 3):
        oracle.apply(b, W.H, [q])
    oracle.apply(b, W.X, [1], [3])
    for q in (1, 3):
        oracle.apply(b, W.H, [q])
    assert np.max(np.abs(a - b)) <= 1e-14


def test_unitary_then_dagger(rng):
    n = 6
    psi = random_state(rng, n)
    gates = [random_gate(rng, n) for _ in range(20)]
    x = psi.copy()
    for u, t, c in gates:
        oracle.apply(x, u, t, c)
    for u, t, c in reversed(gates):
        oracle.apply(x, u.conj().T, t, c)
    assert np.max(np.abs(x - psi)) <= 1e-13


@pytest.mark.parametrize("n", [3, 5, 7])
def test_grover_success_probability(n):
    # App. A.2 with e = 1010...101 (alternating, lowest bit 1).
    marked = sum(1 << q for q in range(0, n, 2))
    theta = math.asin(2 ** (-n / 2))
    for j in (1, 2, int(math.floor(math.pi * math.sqrt(2 ** n) / 4))):
        psi = oracle.run(W.grover(n, marked, j))
        p = oracle.prob_bits(psi, list(range(n)), [(marked >> q) & 1 for q in range(n)])
        assert abs(p - math.sin((2 * j + 1) * theta) ** 2) <= 1e-12


def test_simcomparison_fwht_closed_form(rng):
    # H-transform, CRz chain, H-transform: psi_y = 2^-n sum_x e^{i phi(x)} (-1)^{x.y}
    n = 6
    circ = W.simcomparison(n, np.random.default_rng(5))
    psi = oracle.run(circ)
    xs = np.arange(1 << n)
    phi = np.zeros(1 << n)
    for g in circ.gates:
        if g.name == "crz":
            c, t = g.controls[0], g.targets[0]
            ang = np.angle(g.matrix[1, 1]) * 2          # Rz(theta) = diag(e^{-i t/2}, e^{i t/2})
            on = ((xs >> c) & 1) == 1
            phi[on] += np.where(((xs[on] >> t) & 1) == 1, ang / 2, -ang / 2)
    amp = np.exp(1j * phi)
    sign = np.array([[(-1) ** bin(x & y).count("1") for x in xs] for y in xs])
    want = sign @ amp / (1 << n)
    assert np.max(np.abs(psi - want)) <= 1e-13


# -------------------------------------------------------- emulated math gates
def _reg_index(qubits, x, rest=0):
    i = rest
    for b, q in enumerate(qubits):
        if (x >> b) & 1:
            i |= 1 << q
    return i


def test_math_add_constant_on_basis_states():
    # AddConstant(c) | quint maps |x> to |x + c mod 2^w>, other qubits untouched
    n, reg, c = 7, [1, 4, 5, 2], 11
    tab = W.add_constant_table(len(reg), c)
    for x in range(16):
        for rest in (0, 1 << 0, (1 << 3) | (1 << 6)):
            psi = oracle.basis_state(n, _reg_index(reg, x, rest))
            oracle.apply_math(psi, tab, reg)
            want = oracle.basis_state(n, _reg_index(reg, (x + c) % 16, rest))
            assert np.array_equal(psi, want)


def test_math_add_constant_is_qft_phase_inverse_qft(rng):
    # the decomposition the paper gives for AddConstant: QFT on the register,
    # addition in the phases, inverse QFT (shift theorem of the DFT), here as
    # dense controlled gates through oracle.apply, on a random state
    n, reg, ctrl, c = 7, [0, 3, 5, 6], [2], 5
    N = 1 << len(reg)
    k = np.arange(N)
    F = np.exp(2j * np.pi * np.outer(k, k) / N) / math.sqrt(N)
    D = np.diag(np.exp(2j * np.pi * c * k / N))
    psi0 = random_state(rng, n)
    gates = psi0.copy()
    oracle.apply(gates, F, reg, ctrl)
    oracle.apply(gates, D, reg, ctrl)
    oracle.apply(gates, F.conj().T, reg, ctrl)
    emu = psi0.copy()
    oracle.apply_math(emu, W.add_constant_table(len(reg), c), reg, ctrl)
    assert np.max(np.abs(emu - gates)) <= 1e-13


def test_math_add_constant_matches_draper_circuit(rng):
    n, reg, c = 8, [6, 1, 3, 7, 4], 19
    psi0 = random_state(rng, n)
    emu = oracle.apply_math(psi0.copy(), W.add_constant_table(len(reg), c), reg)
    gate_level = oracle.run(W.draper_add(n, c, reg), psi0.copy())
    assert np.max(np.abs(emu - gate_level)) <= 1e-12


def test_math_modular_multiplication(rng):
    # x -> a x mod N on x < N (x itself above): a bijection when gcd(a, N) = 1;
    # multiplying by a and then by a^-1 mod N restores the state exactly
    w, N, a = 5, 21, 2
    ainv = pow(a, -1, N)
    tab, inv = W.mul_mod_table(w, a, N), W.mul_mod_table(w, ainv, N)
    n, reg, ctrl = 8, [7, 0, 2, 5, 3], [4]
    for x in range(1 << w):
        psi = oracle.basis_state(n, _reg_index(reg, x, 1 << 4))
        oracle.apply_math(psi, tab, reg, ctrl)
        want = (a * x) % N if x < N else x
        assert psi[_reg_index(reg, want, 1 << 4)] == 1.0
        off = oracle.basis_state(n, _reg_index(reg, x))     # control 0: unchanged
        assert np.array_equal(oracle.apply_math(off.copy(), tab, reg, ctrl), off)
    psi0 = random_state(rng, n)
    psi = oracle.apply_math(psi0.copy(), tab, reg, ctrl)
    oracle.apply_math(psi, inv, reg, ctrl)
    assert np.array_equal(psi, psi0)


def test_math_one_bit_table_is_x_gate(rng):
    n = 5
    psi0 = random_state(rng, n)
    a = oracle.apply_math(psi0.copy(), np.array([1, 0]), [3], [0, 4])
    b = oracle.apply(psi0.copy(), W.X, [3], [0, 4])
    assert np.array_equal(a, b)


def test_math_rejects_non_bijection():
    psi = oracle.zero_state(4)
    with pytest.raises(ValueError):
        oracle.apply_math(psi, np.array([0, 1, 1, 3]), [0, 2])
    with pytest.raises(ValueError):
        oracle.apply_math(psi, np.array([0, 1, 2, 4]), [0, 2])


# ------------------------------------------------------------ density matrices
def test_dm_pure_state_follows_state_vector(rng):
    # rho = |psi><psi| stays the projector of the state-vector oracle's state
    n = 5
    rho = oracle.dm_zero(n)
    psi = oracle.zero_state(n)
    for _ in range(25):
        u, t, c = random_gate(rng, n)
        oracle.dm_apply(rho, u, t, c)
        oracle.apply(psi, u, t, c)
    assert np.max(np.abs(rho - np.outer(psi, psi.conj()))) <= 1e-13
    ham = W.random_pauli_dense(n, 12, rng)
    re, im, terms = oracle.dm_expectation(rho, ham, return_terms=True)
    re2, im2, terms2 = oracle.expectation(psi, ham, return_terms=True)
    assert abs(re - re2) <= 1e-13 and np.max(np.abs(terms - terms2)) <= 1e-13


def test_dm_gate_matches_dense_operator(rng):
    n = 4
    a = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    rho = np.ascontiguousarray(a @ a.conj().T / np.trace(a @ a.conj().T))
    u, t, c = W.haar_unitary(4, rng), [3, 1], [0]
    G = brute.gate_operator(u, t, c, n)
    want = G @ rho @ G.conj().T
    got = oracle.dm_apply(rho.copy(), u, t, c)
    assert np.max(np.abs(got - want)) <= 1e-13


def test_dm_channel_closed_forms():
    # one qubit: depolarizing keeps (1-p) of rho and adds p I/2; amplitude
    # damping moves gamma of |1><1| to |0><0| and scales coherences by
    # sqrt(1-gamma); dephasing scales coherences by 1-p
    rho = np.array([[0.3, 0.2 - 0.1j], [0.2 + 0.1j, 0.7]], dtype=np.complex128)
    p, g = 0.3, 0.4
    dep = oracle.dm_kraus(rho.copy(), W.depolarizing(p), [0])
    assert np.max(np.abs(dep - ((1 - p) * rho + p * np.eye(2) / 2))) <= 1e-15
    ad = oracle.dm_kraus(rho.copy(), W.amplitude_damping(g), [0])
    want = np.array([[0.3 + g * 0.7, math.sqrt(1 - g) * rho[0, 1]],
                     [math.sqrt(1 - g) * rho[1, 0], (1 - g) * 0.7]])
    assert np.max(np.abs(ad - want)) <= 1e-15
    dp = oracle.dm_kraus(rho.copy(), W.dephasing(p), [0])
    want = rho.copy()
    want[0, 1] *= 1 - p
    want[1, 0] *= 1 - p
    assert np.max(np.abs(dp - want)) <= 1e-15


def test_dm_channel_on_a_register_and_trace(rng):
    # a channel on qubit 2 of a 4-qubit state equals I (x) K (x) I operators;
    # a random Kraus set (sum K^dag K = I) keeps the trace
    n = 4
    a = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    rho = np.ascontiguousarray(a @ a.conj().T / np.trace(a @ a.conj().T))
    ks = W.amplitude_damping(0.25)
    want = sum(brute.gate_operator(k, [2], [], n) @ rho @ brute.gate_operator(k, [2], [], n).conj().T
               for k in ks)
    got = oracle.dm_kraus(rho.copy(), ks, [2])
    assert np.max(np.abs(got - want)) <= 1e-13
    q, _ = np.linalg.qr(rng.standard_normal((8, 4)) + 1j * rng.standard_normal((8, 4)))
    kr = [q[2 * j:2 * j + 2, :2] for j in range(4)]          # stacked isometry: sum K^dag K = I
    kr = [np.ascontiguousarray(k) for k in kr]
    assert np.allclose(sum(k.conj().T @ k for k in kr), np.eye(2))
    out = oracle.dm_kraus(rho.copy(), kr, [1])
    assert abs(np.trace(out) - 1.0) <= 1e-14
    assert np.max(np.abs(out - out.conj().T)) <= 1e-15


def test_dm_fully_depolarized_expectations_vanish(rng):
    n = 3
    rho = oracle.dm_run(W.noisy_brick(n, 2, 0.05, rng), n)
    for q in range(n):
        oracle.dm_kraus(rho, W.depolarizing(1.0), [q])
    assert np.max(np.abs(rho - np.eye(8) / 8)) <= 1e-15
    ham = W.random_pauli_dense(n, 10, rng)
    re, im, terms = oracle.dm_expectation(rho, ham, return_terms=True)
    ident = (np.asarray(ham.xmask) == 0) & (np.asarray(ham.zmask) == 0)
    assert np.max(np.abs(terms[~ident])) <= 1e-15


# ------------------------------------------------- stochastic trajectories
def test_kraus_sample_bit_flip_closed_form(rng):
    # K0 = sqrt(1-p) I, K1 = sqrt(p) X: p_0 = 1 - p and p_1 = p for any unit
    # state; branch 0 leaves the state alone, branch 1 applies X
    n, q, p = 4, 2, 0.3
    ks = [math.sqrt(1 - p) * np.eye(2), math.sqrt(p) * np.array([[0, 1], [1, 0]])]
    psi = random_state(rng, n)
    a = psi.copy()
    j, pr = oracle.kraus_sample(a, ks, [q], 0.69)
    assert j == 0 and abs(pr[0] - (1 - p)) <= 1e-15 and abs(pr[1] - p) <= 1e-15
    assert np.max(np.abs(a - psi)) <= 1e-15
    b = psi.copy()
    j, _ = oracle.kraus_sample(b, ks, [q], 0.71)
    assert j == 1
    assert np.max(np.abs(b - brute.gate_operator(np.array([[0, 1], [1, 0]]), [q], [], n) @ psi)) <= 1e-15


def test_kraus_sample_boundary_takes_next_branch():
    # the branch is the first whose running sum EXCEEDS u * total: at u = 1/2
    # with p = (1/2, 1/2) that is branch 1
    ks = [math.sqrt(0.5) * np.eye(2), math.sqrt(0.5) * np.array([[0, 1], [1, 0]])]
    psi = np.array([1.0, 0.0], dtype=np.complex128)
    j, _ = oracle.kraus_sample(psi, ks, [0], 0.5)
    assert j == 1 and abs(psi[1] - 1.0) <= 1e-15


def test_kraus_sample_amplitude_damping_closed_form():
    # |1> on qubit 1 of |0 1 0>: p(decay) = gamma exactly, and the decayed
    # branch is |000>; the other branch stays |010>
    g = 0.35
    ks = W.amplitude_damping(g)
    psi = oracle.basis_state(3, 0b010)
    j, pr = oracle.kraus_sample(psi, ks, [1], 0.99)
    assert j == 1 and abs(pr[1] - g) <= 1e-15 and abs(pr[0] - (1 - g)) <= 1e-15
    assert abs(psi[0] - 1.0) <= 1e-15 and np.sum(np.abs(psi) ** 2) - 1 <= 1e-15
    psi = oracle.basis_state(3, 0b010)
    j, _ = oracle.kraus_sample(psi, ks, [1], 0.2)
    assert j == 0 and abs(abs(psi[0b010]) - 1.0) <= 1e-15


@pytest.mark.parametrize("targets", [[1], [3, 0]])
def test_kraus_sample_branches_average_to_channel(rng, targets):
    # sum_j p_j |psi_j><psi_j| over the branches equals the channel applied to
    # |psi><psi| (dm_kraus), and p_j = ||K_j psi||^2 with dense operators
    n = 4
    if len(targets) == 1:
        ks = W.amplitude_damping(0.3) + [0.0 * np.eye(2)]
    else:
        ks = [np.kron(a, b) for a in W.depolarizing(0.4) for b in W.dephasing(0.5)]
    psi = random_state(rng, n)
    want = oracle.dm_kraus(np.ascontiguousarray(np.outer(psi, psi.conj())), ks, targets)
    pd = [np.linalg.norm(brute.gate_operator(k, targets, [], n) @ psi) ** 2 for k in ks]
    _, pr = oracle.kraus_sample(psi.copy(), ks, targets, 0.0)
    assert np.max(np.abs(pr - pd)) <= 1e-14
    total = float(np.sum(pr))
    acc = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    run = 0.0
    for j, pj in enumerate(pr):
        if pj > 0:
            u = (run + pj / 2) / total
            a = psi.copy()
            jj, _ = oracle.kraus_sample(a, ks, targets, u)
            assert jj == j
            acc += pj * np.outer(a, a.conj())
        run += pj
    assert np.max(np.abs(acc - want)) <= 1e-14


# ------------------------------------------------------------ probabilities
def test_probs_and_prob_bits(rng):
    n = 7
    psi = random_state(rng, n)
    p = oracle.probs(psi)
    assert np.max(np.abs(p - np.abs(psi) ** 2)) <= 1e-16
    idx = np.arange(1 << n)
    for qs, bs in [([0], [1]), ([6, 2], [0, 1]), ([1, 3, 5], [1, 1, 0]), ([], [])]:
        mask = np.ones(1 << n, dtype=bool)
        for q, b in zip(qs, bs):
            mask &= ((idx >> q) & 1) == b
        assert abs(oracle.prob_bits(psi, qs, bs) - (np.abs(psi[mask]) ** 2).sum()) <= 1e-14


# ------------------------------------------------------------- expectation
def test_expectation_matches_dense(rng):
    n = 6
    psi = random_state(rng, n)
    ham = W.random_pauli_dense(n, 40, rng)
    re, im = oracle.expectation(psi, ham)
    dense = brute.hamiltonian_operator(ham, n)
    want = np.vdot(psi, dense @ psi)
    assert abs(re - want.real) <= 1e-12 and abs(im) <= 1e-12


def test_expectation_per_term_matches_dense(rng):
    n = 5
    psi = random_state(rng, n)
    ham = W.random_pauli_local(n, 30, 4, rng)
    _, _, terms = oracle.expectation(psi, ham, return_terms=True)
    for s, val in zip(ham.strings(n), terms):
        want = np.vdot(psi, brute.pauli_operator(s) @ psi)
        assert abs(val - want) <= 1e-13


def test_expectation_basis_states(rng):
    n = 8
    ham = W.random_pauli_dense(n, 50, rng)
    for x in (0, 1, 77, 255):
        psi = oracle.basis_state(n, x)
        _, _, terms = oracle.expectation(psi, ham, return_terms=True)
        for xm, zm, val in zip(ham.xmask.tolist(), ham.zmask.tolist(), terms):
            want = 0.0 if xm else (-1.0) ** bin(x & zm).count("1")
            assert abs(val - want) <= 1e-15


def test_expectation_ghz():
    n = 6
    psi = oracle.run(W.ghz(n))
    strings = ["X" * n, "ZZ" + "I" * (n - 2), "I" * 2 + "Z" + "I" * 2 + "Z", "Z" + "I" * (n - 1),
               "YY" + "X" * (n - 2)]
    ham = W.PauliSum.from_strings(strings, [1.0] * len(strings))
    _, _, terms = oracle.expectation(psi, ham, return_terms=True)
    # <X^n> = 1, <Z_i Z_j> = 1, <Z_0> = 0, <Y Y X..X> = -1 for GHZ.
    assert np.allclose(terms, [1, 1, 1, 0, -1], atol=1e-14)


def test_pauli_purity_identity(rng):
    # For a pure state, sum over all 4^n Pauli strings of <P>^2 equals 2^n.
    n = 4
    psi = random_state(rng, n)
    strings = []
    for code in range(4 ** n):
        strings.append("".join("IXYZ"[(code >> (2 * q)) & 3] for q in range(n)))
    ham = W.PauliSum.from_strings(strings, np.ones(len(strings)))
    _, _, terms = oracle.expectation(psi, ham, return_terms=True)
    assert np.max(np.abs(terms.imag)) <= 1e-14
    assert abs(np.sum(terms.real ** 2) - 2 ** n) <= 1e-12


# ---------------------------------------------------- measurement, sampling
def test_sample_matches_cumsum_searchsorted(rng):
    n = 10
    psi = random_state(rng, n)
    u = rng.random(5000)
    got = oracle.sample(psi, u)
    c = np.cumsum(np.abs(psi) ** 2)
    want = np.searchsorted(c, u * c[-1], side="right")
    assert np.array_equal(got, want.astype(np.uint64))


def test_sample_ghz_only_extremes(rng):
    n = 9
    out = oracle.sample(oracle.run(W.ghz(n)), rng.random(2000))
    assert set(out.tolist()) <= {0, (1 << n) - 1}
    assert 800 < int(np.sum(out == 0)) < 1200


def test_sample_edges():
    # u -> 1 must not run off the end: the last index with p > 0 is returned.
    psi = np.zeros(8, dtype=np.complex128)
    psi[2] = psi[5] = 1 / math.sqrt(2)
    out = oracle.sample(psi, np.array([0.0, 0.4999, 0.5, np.nextafter(1.0, 0)]))
    assert out.tolist() == [2, 2, 5, 5]


def test_sample_chi_square(rng):
    n = 5
    psi = random_state(rng, n)
    shots = 200000
    out = oracle.sample(psi, rng.random(shots))
    p = np.abs(psi) ** 2
    obs = np.bincount(out.astype(np.int64), minlength=1 << n)
    chi2 = np.sum((obs - shots * p) ** 2 / (shots * p))
    # 31 degrees of freedom: the 1e-6 tail lies near 80.
    assert chi2 < 80


def test_fair_coin():
    # Sec. 4: H then Measure is a fair random-number generator.
    u = np.random.default_rng(7).random(4000)
    ones = 0
    for x in u:
        psi = oracle.run(W.Circuit(1).add(W.H, (0,)))
        out, p0, p1 = oracle.measure(psi, 0, x)
        assert abs(p0 - 0.5) <= 1e-15 and abs(p1 - 0.5) <= 1e-15
        assert out == (0 if x < 0.5 else 1)
        ones += out
    assert 1800 < ones < 2200


def test_measure_collapse_and_repeat(rng):
    n = 6
    psi = random_state(rng, n)
    idx = np.arange(1 << n)
    p1 = float(np.sum(np.abs(psi[(idx >> 2) & 1 == 1]) ** 2))
    for u, want in [(0.0, 0), (np.nextafter(1.0, 0), 1)]:
        x = psi.copy()
        out, q0, q1 = oracle.measure(x, 2, u)
        assert out == want and abs(q1 - p1) <= 1e-14
        keep = ((idx >> 2) & 1) == out
        ref = np.where(keep, psi, 0) / math.sqrt(q1 if out else q0)
        assert np.max(np.abs(x - ref)) <= 1e-14
        # measuring again repeats the outcome whatever the uniform
        for u2 in (0.0, 0.5, 0.999):
            y = x.copy()
            assert oracle.measure(y, 2, u2)[0] == out


@pytest.mark.parametrize("branch", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_teleportation_all_branches(branch):
    # App. A.1: qubits b1 = 0, b2 = 1, psi = 2.  Bob's qubit b2 ends in the state
    # created on psi, for each of the four measurement outcomes (forced by u).
    u_create = W.haar_2x2(np.random.default_rng(99))
    st = np.zeros(8, dtype=np.complex128)
    st[0] = 1
    oracle.apply(st, W.H, [0])
    oracle.apply(st, W.X, [1], [0])
    oracle.apply(st, u_create, [2])
    oracle.apply(st, W.X, [0], [2])
    oracle.apply(st, W.H, [2])
    m_psi, m_b1 = branch
    u_psi = 0.0 if m_psi == 0 else np.nextafter(1.0, 0)
    u_b1 = 0.0 if m_b1 == 0 else np.nextafter(1.0, 0)
    assert oracle.measure(st, 2, u_psi)[0] == m_psi
    assert oracle.measure(st, 0, u_b1)[0] == m_b1
    if m_b1:
        oracle.apply(st, W.X, [1], [0])
    if m_psi:
        oracle.apply(st, W.Z, [1], [2])
    base = m_b1 * 1 + m_psi * 4
    bob = np.array([st[base], st[base + 2]])
    want = u_create @ np.array([1, 0])
    assert np.max(np.abs(bob - want)) <= 1e-14


# -------------------------------------------------------------- dealloc/alloc
def test_dealloc_classical_and_superposition(rng):
    n = 5
    psi = random_state(rng, 4)
    # put a |1> qubit at position 2 between random ones
    full = np.zeros(1 << n, dtype=np.complex128)
    t = psi.reshape(4, 4)              # [high 2 bits][low 2 bits]
    full.reshape(4, 2, 4)[:, 1, :] = t
    v, out = oracle.dealloc(full, 2, 1e-12)
    assert v == 1 and np.max(np.abs(out - psi)) == 0.0
    with pytest.raises(ValueError):
        oracle.dealloc(oracle.run(W.Circuit(2).add(W.H, (1,))), 1, 1e-12)


def test_allocate_extends_with_zero(rng):
    psi = random_state(rng, 3)
    out = oracle.allocate(psi, 2)
    assert out.size == 32 and np.array_equal(out[:8], psi) and not out[8:].any()


# ------------------------------------------------------------------ gradients
def test_grad_single_qubit_closed_form():
    # d<Z>/d theta of RY(theta)|0> = -sin(theta)
    ham = W.PauliSum.from_strings(["Z"], [1.0])
    for th in (0.3, 1.7, 4.0):
        circ = W.hea(1, 1, np.array([th, 0.0]))
        g_ps = oracle.grad_param_shift(circ, ham, [0])[0]
        g_fd = oracle.grad_fd(circ, ham, [0])[0]
        assert abs(g_ps + math.sin(th)) <= 1e-14
        assert abs(g_fd + math.sin(th)) <= 1e-9


def test_grad_shift_vs_fd(rng):
    n, layers = 4, 2
    circ = W.hea(n, layers, rng.uniform(0, 2 * math.pi, 2 * n * layers))
    ham = W.random_pauli_local(n, 12, 3, rng)
    g_ps = oracle.grad_param_shift(circ, ham)
    g_fd = oracle.grad_fd(circ, ham)
    assert np.max(np.abs(g_ps - g_fd)) <= 1e-8


def test_grad_vs_dense_derivative(rng):
    # Differentiate <psi|H|psi> with the dense operator and the analytic
    # derivative of one rotation, dR/dtheta = -i/2 P R.
    n, layers = 3, 2
    circ = W.hea(n, layers, rng.uniform(0, 2 * math.pi, 2 * n * layers))
    ham = W.random_pauli_dense(n, 10, rng)
    hd = brute.hamiltonian_operator(ham, n)
    g_ps = oracle.grad_param_shift(circ, ham)
    for p in range(len(circ.theta)):
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1
        dpsi = np.zeros_like(psi)
        for g in circ.gates:
            op = brute.gate_operator(g.matrix, g.targets, g.controls, n)
            psi, dpsi = op @ psi, op @ dpsi
            if g.param == p:
                dop = brute.gate_operator(-0.5j * brute.PAULI[g.axis] @ g.matrix, g.targets, (), n)
                dpsi = dpsi + dop @ np.linalg.solve(op, psi)
        want = 2 * np.real(np.vdot(psi, hd @ dpsi))
        assert abs(g_ps[p] - want) <= 1e-12


# ------------------------------------------------------------- generators
def test_workload_shapes_and_determinism():
    c1 = W.config1_random()
    assert c1.n == 30 and c1.counts() == {"haar": 1200, "cnot": 580}
    c2 = W.config2()
    assert c2.n == 32 and c2.counts() == {"haar": 1280, "cz": 620}
    c4, h4 = W.config4()
    assert len(c4.theta) == 480 and c4.counts()["cz"] == 230 and len(h4) == 200
    assert np.array_equal(W.config4()[0].theta, c4.theta)
    a = W.config0()[0].gates[17].matrix
    b = W.config0()[0].gates[17].matrix
    assert np.array_equal(a, b)
    assert np.allclose(a.conj().T @ a, np.eye(2), atol=1e-15)


def test_oracle_threads_change_no_result():
    """oracle.set_threads shares out only the outer loop of a gate (index
    groups written by one thread each): the state is bit-identical to the
    serial run."""
    n = 14
    c = W.config1_random(n, layers=4)
    for g in W.qft(n).gates[:40]:
        c.gates.append(g)
    psi1 = oracle.run(c)
    assert oracle.set_threads(4) == 4
    try:
        psi4 = oracle.run(c)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(psi1, psi4)
