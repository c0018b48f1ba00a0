"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: complex128 amplitudes within 1e-12 of the oracle (max abs); complex64
states within 1e-5 normwise relative error; reductions accumulated in double;
samples identical except at a CDF boundary closer than 1e-10 * total, where
both answers are correct.  At the 30-qubit sizes of the benchmark, where the
oracle cannot run the whole circuit, the checks are sampled amplitudes
against a closed form (QFT of a basis state) and the U^dag U = 1 property.
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


def make(n, **kw):
    kw.setdefault("use_torch_stream", False)
    s = Q.Simulator(n_max=kw.pop("n_max", max(n, 1)), **kw)
    s.allocate(n)
    return s


def check_c128(got, want, tol=1e-12):
    err = float(np.max(np.abs(got - want)))
    assert err <= tol, "max |diff| = %g" % err


def check_c64(got, want, tol=1e-5):
    rel = float(np.linalg.norm(got.astype(np.complex128) - want) / np.linalg.norm(want))
    assert rel <= tol, "normwise relative error %g" % rel


def check_samples(got, want, psi, u):
    p = np.abs(psi.astype(np.complex128)) ** 2
    cdf = np.cumsum(p)
    total = cdf[-1]
    bad = np.nonzero(got != want)[0]
    for s in bad:
        i = int(min(got[s], want[s]))
        r = u[s] * total
        assert abs(r - cdf[i]) <= 1e-10 * total, "shot %d: %d vs %d" % (s, got[s], want[s])
    assert len(bad) <= max(2, len(u) // 1000)


def random_circuit(rng, n, count, kmax=3):
    c = W.Circuit(n)
    for _ in range(count):
        kind = rng.integers(0, 7) if n >= 2 else rng.choice([0, 5, 6])
        if kind == 0:
            k = int(rng.integers(1, min(kmax, n) + 1))
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
        elif kind == 4 and n >= 3:
            qs = rng.permutation(n)[:3].tolist()
            c.add(W.haar_2x2(rng), qs[:1], qs[1:])
        elif kind == 5:
            c.add(W.haar_2x2(rng), (int(rng.integers(0, min(n, 3))),))   # low targets
        else:
            q = int(rng.integers(0, n))
            c.add(W.rz(float(rng.uniform(0, 6))), (q,))
    return c


MODES = [("pergate", 1, 0), ("fused", 2, 0), ("fused", 3, 0), ("fused", 4, 0), ("fused", 5, 0),
         ("tiled", 1, 0), ("tiled", 2, 0), ("tiled", 3, 0), ("tiled", 4, 0), ("tiled", 5, 0),
         ("tiled", 3, 6), ("tiled", 5, 10)]


@pytest.mark.parametrize("mode,k_max,tile_bits", MODES)
@pytest.mark.parametrize("n", [3, 9, 14, 18])
def test_random_circuits_c128(mode, k_max, tile_bits, n):
    rng = np.random.default_rng(1000 * n + 10 * k_max + tile_bits)
    circ = random_circuit(rng, n, 80 if n < 18 else 40)
    log("case", mode, k_max, tile_bits, n)
    s = make(n, mode=mode, k_max=k_max, tile_bits=tile_bits)
    s.run(circ)
    got = s.get_state()
    want = oracle.run(circ)
    check_c128(got, want)
    s.close()


@pytest.mark.parametrize("n,k_max,dtype", [(18, 3, "c128"), (20, 4, "c128"), (18, 5, "c64")])
def test_relabeling_plans_on_the_lds_kernel(n, k_max, dtype):
    """Fusion wider than 2 qubits sends passes to the LDS-tile kernel (MFMA
    for the 3- to 5-qubit ops); with relabeling those passes store their
    tiles to the new positions (the host model covers only the register
    kernel, so this path is checked here).  The relabeling plan must be the
    one taken (fewer passes than with fixed positions)."""
    circ = W.config1_random(n, layers=30)
    log("case relabel lds", n, k_max, dtype)
    fixed = make(n, mode="tiled", k_max=k_max, dtype=dtype, relabel=False)
    fixed.run(circ)
    _, p_fixed = fixed.plan()
    fixed.close()
    s = make(n, mode="tiled", k_max=k_max, dtype=dtype)
    s.run(circ)
    _, p_moved = s.plan()
    assert p_moved < p_fixed
    got = s.get_state()
    s.close()
    if dtype == "c128":
        check_c128(got, oracle.run(circ))
    else:
        check_c64(got, oracle.run(circ))


@pytest.mark.parametrize("mode,k_max", [("pergate", 1), ("fused", 3), ("fused", 5), ("tiled", 3),
                                        ("tiled", 5)])
def test_random_circuits_c64(mode, k_max):
    n = 16
    rng = np.random.default_rng(77 + k_max)
    circ = random_circuit(rng, n, 80)
    log("case c64", mode, k_max)
    s = make(n, mode=mode, k_max=k_max, dtype="c64")
    s.run(circ)
    got = s.get_state()
    check_c64(got, oracle.run(circ))
    s.close()


def diag_circuit(rng, n, count):
    """A Hadamard layer, then mostly diagonal gates: phases with 0-3 random
    controls and Rz, with an occasional dense 1-qubit gate.  Long runs of
    diagonal ops with differing controls reach the register-tile lowering,
    which merges them into diagonal ops of up to 8 table qubits."""
    c = W.Circuit(n)
    for q in range(n):
        c.add(W.H, (q,))
    for _ in range(count):
        kind = rng.integers(0, 10)
        if kind == 0:
            c.add(W.haar_2x2(rng), (int(rng.integers(0, n)),))
        elif kind <= 2:
            c.add(W.rz(float(rng.uniform(0, 6))), (int(rng.integers(0, n)),))
        else:
            nc = int(rng.integers(0, 4))
            qs = rng.permutation(n)[:nc + 1].tolist()
            c.add(W.phase(float(rng.uniform(0, 6))), qs[:1], qs[1:])
    return c


@pytest.mark.parametrize("mode,k_max,tile_bits", MODES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_one_and_two_qubit_states(mode, k_max, tile_bits, dtype):
    # states smaller than a tile, a register group and a wavefront: every
    # mode clamps its tile to the state and still matches the oracle
    for n in (1, 2):
        rng = np.random.default_rng(700 + 10 * n + k_max + tile_bits)
        circ = random_circuit(rng, n, 30)
        log("case", mode, k_max, tile_bits, dtype, n)
        s = make(n, mode=mode, k_max=k_max, tile_bits=tile_bits, dtype=dtype)
        s.run(W.Circuit(n))
        zero = np.zeros(1 << n, dtype=np.complex128)
        zero[0] = 1.0
        assert np.array_equal(s.get_state().astype(np.complex128), zero)
        s.run(circ)
        want = oracle.run(circ)
        got = s.get_state()
        if dtype == "c128":
            check_c128(got, want)
        else:
            check_c64(got, want)
        tol = 1e-13 if dtype == "c128" else 1e-6
        for q in range(n):
            assert abs(s.get_probability([q], [1]) - oracle.prob_bits(want, [q], [1])) <= tol
        u = rng.random(200)
        u[:2] = [0.0, np.nextafter(1.0, 0)]
        if dtype == "c128":
            check_samples(s.sample(u), oracle.sample(want, u), want, u)
        else:
            g = got.astype(np.complex128)
            check_samples(s.sample(u), oracle.sample(g, u), g, u)
        s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [13, 16])
def test_diagonal_runs_tiled(dtype, n):
    rng = np.random.default_rng(4242 + n)
    circ = diag_circuit(rng, n, 300)
    log("case diagonal runs", dtype, n)
    s = make(n, mode="tiled", k_max=2, dtype=dtype)
    s.run(circ)
    got = s.get_state()
    want = oracle.run(circ)
    if dtype == "c128":
        check_c128(got, want)
    else:
        check_c64(got, want)
    s.close()


@pytest.mark.parametrize("mode,k_max", [("pergate", 1), ("fused", 3), ("tiled", 2), ("tiled", 4)])
def test_apply_diag_matches_oracle(mode, k_max):
    n = 14
    rng = np.random.default_rng(515 + k_max)
    s = make(n, mode=mode, k_max=k_max)
    psi = oracle.zero_state(n)
    for q in range(n):
        s.apply(W.H, [q])
        oracle.apply(psi, W.H, [q])
    for _ in range(60):
        k = int(rng.integers(1, 4))
        nc = int(rng.integers(0, 3))
        qs = rng.permutation(n)[:k + nc].tolist()
        d = np.exp(1j * rng.uniform(0, 6, size=1 << k))
        s.apply_diag(d, qs[:k], qs[k:])
        oracle.apply(psi, np.diag(d), qs[:k], qs[k:])
        if rng.uniform() < 0.2:
            q = int(rng.integers(0, n))
            u = W.haar_2x2(rng)
            s.apply(u, [q])
            oracle.apply(psi, u, [q])
    log("case apply_diag", mode, k_max)
    check_c128(s.get_state(), psi)
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_long_single_pass_scheduling(dtype):
    # 12 qubits fit one tile: 1200 gates become one pass of several hundred
    # ops, longer than the lowering's scheduling window
    n = 12
    rng = np.random.default_rng(8080)
    circ = random_circuit(rng, n, 1200, kmax=2)   # register-kernel ops only
    log("case long pass", dtype)
    s = make(n, mode="tiled", k_max=2, dtype=dtype)
    s.run(circ)
    got = s.get_state()
    want = oracle.run(circ)
    if dtype == "c128":
        check_c128(got, want, tol=1e-11)
    else:
        check_c64(got, want)
    s.close()


def test_config0_state_probs_samples():
    circ, u = W.config0()
    log("case config0")
    s = make(16, mode="pergate")
    s.run(circ)
    got = s.get_state()
    want = oracle.run(circ)
    check_c128(got, want)
    pg = s.get_probabilities()
    assert np.max(np.abs(pg - oracle.probs(want))) <= 1e-13
    smp = s.sample(u)
    check_samples(smp, oracle.sample(want, u), want, u)
    s.close()


@pytest.mark.parametrize("mode", ["tiled", "fused"])
def test_config0_other_modes(mode):
    circ, u = W.config0()
    s = make(16, mode=mode, k_max=4)
    s.run(circ)
    got = s.get_state()
    want = oracle.run(circ)
    check_c128(got, want)
    check_samples(s.sample(u), oracle.sample(want, u), want, u)
    s.close()


def test_sampling_large_and_edges():
    rng = np.random.default_rng(5)
    n = 20
    circ = random_circuit(rng, n, 30)
    s = make(n)
    s.run(circ)
    want = oracle.run(circ)
    u = rng.random(3000)
    u[:3] = [0.0, 0.5, np.nextafter(1.0, 0)]
    check_samples(s.sample(u), oracle.sample(want, u), want, u)
    s.close()
    # sparse state: u close to 1 lands on the last nonzero amplitude
    s = make(12)
    st = np.zeros(1 << 12, dtype=np.complex128)
    st[[3, 700, 2049]] = [0.6, 0.0 + 0.64j, 0.48]
    st /= np.linalg.norm(st)
    s.set_state(st)
    uu = np.array([0.0, 0.3, 0.5, 0.99, np.nextafter(1.0, 0)])
    check_samples(s.sample(uu), oracle.sample(st, uu), st, uu)
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_expectation(dtype):
    rng = np.random.default_rng(11)
    for n, ham in [(10, W.random_pauli_dense(10, 64, rng)), (16, W.random_pauli_local(16, 200, 4, rng)),
                   (1, W.random_pauli_dense(1, 4, rng))]:
        circ = random_circuit(rng, n, 40)
        s = make(n, dtype=dtype)
        s.run(circ)
        got = s.expectation(ham)
        want, wim = oracle.expectation(oracle.run(circ), ham)
        tol = 1e-12 * max(1.0, np.sum(np.abs(ham.coeff))) if dtype == "c128" else \
            1e-5 * np.sum(np.abs(ham.coeff))
        assert abs(got - want) <= tol, (n, got, want)
        # the sum is Hermitian: its imaginary part vanishes up to rounding
        # (qubit id j is bit j here, so the masks go in unchanged)
        re, im = s.get_expectation_complex(ham.xmask, ham.zmask, ham.coeff)
        assert abs(re - got) <= 1e-13 * max(1.0, abs(got))
        assert abs(im) <= tol, (n, im)
        s.close()


def local_x_hamiltonian(n, terms, rng, xq):
    """Terms whose X and Y letters sit on the qubits xq only; Z letters
    anywhere; a Z-only term and two terms sharing an X mask included."""
    strings = []
    for t in range(terms):
        p = ["I"] * n
        for q in rng.choice(n, size=3, replace=False):
            p[int(q)] = "Z"
        if t % 5 != 0:
            for q in rng.choice(xq, size=int(rng.integers(1, 4)), replace=False):
                p[int(q)] = "XY"[int(rng.integers(0, 2))]
        strings.append("".join(p))
    strings.append(strings[1].replace("Z", "I"))
    return W.PauliSum.from_strings(strings, rng.standard_normal(len(strings)))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_expectation_local_x_terms(dtype):
    """Pauli sums of at most 16 terms whose X letters lie on at most 8 qubits
    take one read of the state (tiles holding every such qubit); against the
    oracle, at sizes with one and with many tiles, X letters low and high,
    and against the chunked path (the same sum with a 17th term)."""
    rng = np.random.default_rng(13)
    for n, xq in [(13, [0, 5, 12]), (20, [0, 2, 4, 6, 11, 13, 15, 17]), (22, [3, 9, 20, 21])]:
        circ = random_circuit(rng, n, 60)
        ham = local_x_hamiltonian(n, 15, rng, xq)
        assert len(ham) == 16
        s = make(n, dtype=dtype)
        s.run(circ)
        got = s.expectation(ham)
        re, im = s.get_expectation_complex(ham.xmask, ham.zmask, ham.coeff)
        want, _ = oracle.expectation(oracle.run(circ), ham)
        scale = max(1.0, float(np.sum(np.abs(ham.coeff))))
        tol = 1e-12 * scale if dtype == "c128" else 1e-5 * scale
        assert abs(got - want) <= tol, (n, got, want)
        assert abs(im) <= tol, (n, im)
        # a 17th term (zero coefficient) sends the sum to the chunked path
        big = W.PauliSum(np.append(ham.xmask, np.uint64(1 << (n - 1))),
                         np.append(ham.zmask, np.uint64(0)), np.append(ham.coeff, 0.0))
        other = s.expectation(big)
        assert abs(other - got) <= tol, (n, other, got)
        s.close()


def test_probability_masks():
    rng = np.random.default_rng(12)
    n = 14
    circ = random_circuit(rng, n, 50)
    s = make(n)
    s.run(circ)
    psi = oracle.run(circ)
    for qs, bs in [([], []), ([0], [1]), ([13], [0]), ([2, 9], [1, 0]), ([0, 1, 2, 3, 4], [1, 0, 1, 1, 0])]:
        got = s.get_probability(qs, bs)
        assert abs(got - oracle.prob_bits(psi, qs, bs)) <= 1e-13
    s.close()


def test_measure_collapse_matches_oracle():
    rng = np.random.default_rng(13)
    n = 12
    circ = random_circuit(rng, n, 50)
    s = make(n)
    s.run(circ)
    psi = oracle.run(circ)
    qs = [3, 0, 11, 7]
    u = rng.random(len(qs)).tolist()
    got_bits = s.measure(qs, u)
    want_bits = [oracle.measure(psi, q, x)[0] for q, x in zip(qs, u)]
    assert got_bits == want_bits
    check_c128(s.get_state(), psi)
    # measuring again repeats the outcome
    assert s.measure(qs, [0.999, 0.0, 0.5, 0.25]) == want_bits
    s.close()


@pytest.mark.parametrize("branch", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_teleportation(branch):
    # App. A.1 on the GPU path: Bob's qubit ends in the created state.
    u_create = W.haar_2x2(np.random.default_rng(99))
    s = make(3, mode="pergate")
    b1, b2, psi = 0, 1, 2
    s.apply(W.H, [b1])
    s.apply(W.X, [b2], [b1])
    s.apply(u_create, [psi])
    s.apply(W.X, [b1], [psi])
    s.apply(W.H, [psi])
    upsi = 0.0 if branch[0] == 0 else np.nextafter(1.0, 0)
    ub1 = 0.0 if branch[1] == 0 else np.nextafter(1.0, 0)
    m = s.measure([psi, b1], [upsi, ub1])
    assert m == list(branch)
    if m[1]:
        s.apply(W.X, [b2], [b1])
    if m[0]:
        s.apply(W.Z, [b2], [psi])
    st = s.get_state()
    base = m[1] * 1 + m[0] * 4
    bob = np.array([st[base], st[base + 2]])
    check_c128(bob, u_create @ np.array([1, 0]), 1e-14)
    s.close()


def test_state_beyond_device_memory_fails_cleanly():
    # 2^35 complex128 amplitudes (512 GiB) exceed one GPU's memory: the
    # first flush, which allocates the state, reports ENOMEM, and the device
    # stays usable for the next simulator
    log("case", "35 qubits c128, flush -> ENOMEM")
    s = make(35, dtype="c128")
    s.apply(W.H, [0], [])
    with pytest.raises(Q.QsvError) as ei:
        s.flush()
    assert ei.value.code == 2, str(ei.value)
    s.close()
    rng = np.random.default_rng(35)
    circ = random_circuit(rng, 10, 40)
    t = make(10)
    t.run(circ)
    check_c128(t.get_state(), oracle.run(circ))
    t.close()


def test_state_beyond_device_memory_message_names_free_memory():
    # the figure comes from hipMemGetInfo before any allocation is tried
    s = make(35, dtype="c128")
    s.apply(W.H, [0], [])
    with pytest.raises(Q.QsvError) as ei:
        s.flush()
    assert ei.value.code == 2 and "free of" in str(ei.value), str(ei.value)
    s.close()


def test_mem_limit_bounds_the_state():
    # 2^16 complex128 amplitudes take 1 MiB: a limit of exactly that fits, one
    # byte less does not
    rng = np.random.default_rng(36)
    circ = random_circuit(rng, 16, 40)
    ok = Q.Simulator(n_max=16, use_torch_stream=False, mem_limit=1 << 20)
    ok.allocate(16)
    ok.run(circ)
    check_c128(ok.get_state(), oracle.run(circ))
    ok.close()
    bad = Q.Simulator(n_max=16, use_torch_stream=False, mem_limit=(1 << 20) - 1)
    bad.allocate(16)
    bad.run(circ)
    with pytest.raises(Q.QsvError) as ei:
        bad.flush()
    assert ei.value.code == 2 and "mem_limit" in str(ei.value)
    bad.close()


@pytest.mark.parametrize("mode,k_max,fail_at", [("pergate", 1, 3), ("tiled", 2, 1)])
def test_failure_part_way_through_a_flush(monkeypatch, mode, k_max, fail_at):
    """A launch that fails after earlier kernels of the flush ran: the queue
    is dropped (its gates would run twice) and the state is refused until it
    is reset; then the handle works again.  The failure is injected on the
    host (the launch is skipped, no kernel fails)."""
    n = 16
    rng = np.random.default_rng(37)
    circ = random_circuit(rng, n, 60)
    monkeypatch.setenv("QSV_INJECT_LAUNCH_FAILURE", str(fail_at))
    s = Q.Simulator(n_max=n, mode=mode, k_max=k_max, tile_bits=12, use_torch_stream=False)
    monkeypatch.delenv("QSV_INJECT_LAUNCH_FAILURE")
    s.allocate(n)
    s.run(circ)
    with pytest.raises(Q.QsvError) as ei:
        s.flush()
    assert ei.value.code == 3 and "injected" in str(ei.value) and "invalid" in str(ei.value)
    assert s.plan()[0] == []                       # the queue is gone
    with pytest.raises(Q.QsvError) as ei:
        s.norm2()
    assert ei.value.code == 3 and "invalid" in str(ei.value)
    s.reset()
    s.run(circ)
    check_c128(s.get_state(), oracle.run(circ))
    s.close()


def test_allocate_deallocate_sequence():
    rng = np.random.default_rng(14)
    s = Q.Simulator(n_max=12, use_torch_stream=False)
    ids = s.allocate(6)
    ref = oracle.zero_state(6)
    circ = random_circuit(rng, 6, 30)
    s.run(circ)
    oracle.run(circ, ref)
    # put qubit 2 into |1> with an X after uncomputing nothing: a classical qubit
    s.apply(W.X, [ids[2]])
    oracle.apply(ref, W.X, [2])
    with pytest.raises(Q.NotClassicalError):
        s.deallocate(ids[4])          # entangled: must raise, state unchanged
    check_c128(s.get_state(), ref)
    # prepare a classical qubit: allocate, flip, deallocate
    new = s.allocate(2)
    ref = oracle.allocate(ref, 2)
    s.apply(W.X, [new[0]])
    oracle.apply(ref, W.X, [6])
    s.deallocate(new[0])
    v, ref = oracle.dealloc(ref, 6, 1e-12)
    assert v == 1
    check_c128(s.get_state(), ref)
    s.deallocate(new[1])
    v, ref = oracle.dealloc(ref, 6, 1e-12)
    assert v == 0
    check_c128(s.get_state(), ref)
    s.close()


@pytest.mark.parametrize("n", [5, 20])
def test_ghz_w_grover_closed_forms(n):
    s = make(n, mode="tiled")
    s.run(W.ghz(n))
    st = s.get_state()
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    check_c128(st, want, 1e-14)
    s.close()
    s = make(n, mode="fused", k_max=3)
    s.run(W.w_state(n))
    st = s.get_state()
    want = np.zeros(1 << n, dtype=np.complex128)
    for q in range(n):
        want[1 << q] = 1 / math.sqrt(n)
    check_c128(st, want, 1e-13)
    s.close()
    g = min(n, 9)
    marked = sum(1 << q for q in range(0, g, 2))
    s = make(g + 1, mode="tiled", k_max=2)
    j = int(math.floor(math.pi * math.sqrt(2 ** g) / 4))
    s.run(W.grover(g, marked, j))
    p = s.get_probability(list(range(g)), [(marked >> q) & 1 for q in range(g)])
    assert abs(p - math.sin((2 * j + 1) * math.asin(2 ** (-g / 2))) ** 2) <= 1e-12
    s.close()


def test_borrowed_torch_state():
    import torch
    n = 12
    buf = torch.empty(2 << n, dtype=torch.float64, device="cuda")
    s = Q.Simulator(n_max=n, state=buf)
    s.allocate(n)
    circ = random_circuit(np.random.default_rng(15), n, 40)
    s.run(circ)
    s.flush()
    s.synchronize()
    torch.cuda.synchronize()
    got = buf.cpu().numpy().view(np.complex128)
    check_c128(got, oracle.run(circ))
    s.close()


def test_config2_twin_c64_vs_oracle():
    n = 20
    circ = W.config2(n=n)
    want = oracle.run(circ)
    for mode, k in [("fused", 5), ("tiled", 5), ("tiled", 3)]:
        log("case config2 twin", mode, k)
        s = make(n, mode=mode, k_max=k, dtype="c64")
        s.run(circ)
        check_c64(s.get_state(), want)
        s.close()


# ------------------------------------------------------------- full size, 30 q
def test_qft_30q_sampled_closed_form():
    n = 30
    x, circ = W.config1_qft(n)
    log("case qft30 x=%d" % x)
    s = make(n, mode="tiled", k_max=4)
    s.run(W.basis_prep(n, x))
    s.run(circ)
    rng = np.random.default_rng(21)
    idx = rng.integers(0, 1 << n, size=4096, dtype=np.uint64)
    idx[:4] = [0, 1, (1 << n) - 1, 1 << (n - 1)]
    got = s.get_amplitudes(idx)
    y = idx.astype(object)
    ph = np.array([float((x * int(v)) % (1 << n)) for v in y]) / (1 << n)
    want = np.exp(2j * math.pi * ph) / (2 ** (n / 2))
    check_c128(got, want, 1e-12)
    assert abs(s.norm2() - 1.0) <= 1e-12
    s.close()


@pytest.mark.parametrize("mode,k_max", [("tiled", 3), ("pergate", 1)])
def test_brick_30q_then_inverse(mode, k_max):
    n = 30
    circ = W.config1_random(n)
    if mode == "pergate":
        circ.gates = circ.gates[:200]
    log("case brick30 inverse", mode, len(circ.gates))
    s = make(n, mode=mode, k_max=k_max)
    s.run(circ)
    assert abs(s.norm2() - 1.0) <= 1e-11
    for g in reversed(circ.gates):
        s.apply(g.matrix.conj().T, g.targets, g.controls)
    amp = s.get_amplitudes([0, 1, 12345])
    assert abs(amp[0] - 1.0) <= 1e-10 and np.max(np.abs(amp[1:])) <= 1e-10
    s.close()


# ------------------------------------------------------------- full size, 32 q
def test_qft_32q_c64_sampled_closed_form():
    """2^32 amplitudes (complex64, 32 GiB): every launch strides past 2^32
    threads' worth of work.  QFT of a basis state against its closed form."""
    n = 32
    x = int(np.random.default_rng(32).integers(0, 1 << n))
    log("case qft32 c64 x=%d" % x)
    s = make(n, mode="tiled", k_max=2, dtype="c64")
    s.run(W.basis_prep(n, x))
    s.run(W.qft(n))
    rng = np.random.default_rng(23)
    idx = rng.integers(0, 1 << n, size=4096, dtype=np.uint64)
    idx[:4] = [0, 1, (1 << n) - 1, 1 << (n - 1)]
    got = s.get_amplitudes(idx)
    ph = np.array([float((x * int(v)) % (1 << n)) for v in idx.astype(object)]) / (1 << n)
    want = np.exp(2j * math.pi * ph) / (2 ** (n / 2))
    check_c64(got, want)
    assert abs(s.norm2() - 1.0) <= 1e-5
    s.close()


def test_qft_33q_c128_sampled_closed_form():
    """The largest size of the workloads at full precision: 2^33 complex128
    amplitudes (128 GiB).  QFT of a basis state against its closed form on
    sampled amplitudes, then the norm."""
    n = 33
    x = int(np.random.default_rng(33).integers(0, 1 << n))
    log("case qft33 c128 x=%d" % x)
    s = make(n, mode="tiled", k_max=2, dtype="c128")
    s.run(W.basis_prep(n, x))
    s.run(W.qft(n))
    rng = np.random.default_rng(24)
    idx = rng.integers(0, 1 << n, size=4096, dtype=np.uint64)
    idx[:4] = [0, 1, (1 << n) - 1, 1 << (n - 1)]
    got = s.get_amplitudes(idx)
    ph = np.array([float((x * int(v)) % (1 << n)) for v in idx.astype(object)]) / (1 << n)
    want = np.exp(2j * math.pi * ph) / (2 ** (n / 2))
    check_c128(got, want)
    assert abs(s.norm2() - 1.0) <= 1e-12
    s.close()


def test_config2_32q_c64_then_inverse_and_measure():
    """The 32-qubit brick circuit and its inverse return |0...0> (within FP32
    rounding of 3800 gates); then a GHZ state is measured and collapsed."""
    n = 32
    circ = W.config2(n)
    log("case config2 32q inverse", len(circ.gates))
    s = make(n, mode="tiled", k_max=2, dtype="c64")
    s.run(circ)
    assert abs(s.norm2() - 1.0) <= 1e-4
    for g in reversed(circ.gates):
        s.apply(g.matrix.conj().T, g.targets, g.controls)
    amp = s.get_amplitudes([0, 1, (1 << n) - 1, 123456789])
    assert abs(amp[0] - 1.0) <= 1e-4 and np.max(np.abs(amp[1:])) <= 1e-4
    log("case ghz32 measure")
    s.reset()
    s.run(W.ghz(n))
    assert abs(s.get_probability([n - 1], [1]) - 0.5) <= 1e-6
    out = s.measure([n - 1], [0.75])
    want = 1 if 0.75 * 1.0 >= 0.5 else 0
    assert list(out) == [want]
    amp = s.get_amplitudes([0, (1 << n) - 1])
    assert abs(abs(amp[want]) - 1.0) <= 1e-6 and abs(amp[1 - want]) == 0.0
    s.close()


# ------------------------------------- the paper's benchmark circuit (Sec. 4.3.2)
def _fwht(a):
    """Unnormalised Walsh-Hadamard transform: out_y = sum_x (-1)^popcount(x & y) a_x."""
    h = 1
    while h < a.size:
        v = a.reshape(-1, 2, h)
        a = np.stack((v[:, 0, :] + v[:, 1, :], v[:, 0, :] - v[:, 1, :]), axis=1).reshape(-1)
        h *= 2
    return a


@pytest.mark.parametrize("mode,k_max", [("tiled", 2), ("pergate", 1)])
def test_simcomparison_22q_walsh_closed_form(mode, k_max):
    """H on every qubit, a chain of controlled Rz, H on every qubit:
    psi_y = 2^-n sum_x e^{i phi(x)} (-1)^{x.y}, with phi(x) collecting
    +-theta_i / 2 from every control bit x_i = 1 (the sign is the target bit)."""
    n = 22
    circ = W.simcomparison(n, np.random.default_rng(7))
    log("case simcomparison", n, mode)
    s = make(n, mode=mode, k_max=k_max)
    s.run(circ)
    got = s.get_state()
    s.close()
    xs = np.arange(1 << n, dtype=np.int64)
    phi = np.zeros(1 << n)
    for g in circ.gates:
        if g.name == "crz":
            c, t = g.controls[0], g.targets[0]
            half = np.angle(g.matrix[1, 1])           # Rz(theta)[1,1] = e^{i theta/2}
            on = ((xs >> c) & 1) == 1
            phi += np.where(on, np.where(((xs >> t) & 1) == 1, half, -half), 0.0)
    want = _fwht(np.exp(1j * phi)) / float(1 << n)
    check_c128(got, want, 1e-12)


# ------------------------------------------------- the headline path at size
_C1 = {}


def _config1(n):
    if n not in _C1:
        circ = W.config1_random(n)
        _C1[n] = (circ, oracle.run(circ))
    return _C1[n]


@pytest.mark.parametrize("n", [22, 23])
def test_headline_brick_register_tiles_vs_oracle(n):
    """The 40-layer Haar + CNOT brick circuit of the 30-qubit benchmark, at
    22 and 23 qubits, on the benchmark's path: mode tiled, k_max 2, 12-bit
    tiles of 16 amplitudes per thread, complex128.  2^(n-12) = 1024 / 2048
    tiles exceed the resident workgroups, so each persistent workgroup runs
    several tiles.  Every amplitude against the oracle at 1e-12 (A12)."""
    circ, want = _config1(n)
    log("case headline brick", n)
    s = make(n, mode="tiled", k_max=2, tile_bits=12, reg_bits=4, timing=True)
    s.run(circ)
    # the lowering the flush will run (host side, nothing executes): every
    # pass is a register-tile program, most ops split into real matrices
    _, info = s.check_tile_programs(None)
    assert info["reg_passes"] == info["passes"]
    assert info["real_ops"] >= 0.9 * (len(circ.gates) - n * 40) and info["diag_ops"] > 0
    got = s.get_state()
    _, launches, _ = s.kernel_times()["tile"]
    assert launches == info["passes"]
    check_c128(got, want)
    assert abs(s.norm2() - 1.0) <= 1e-12
    s.close()


def test_headline_brick_30q_tiled_equals_pergate_every_amplitude():
    """At the benchmark size (30 qubits, 16 GiB per state): the tiled k = 2
    state against the plain per-gate FP64 state, every one of the 2^30
    amplitudes, compared on the device in chunks (max |diff| <= 1e-12)."""
    import torch
    n = 30
    circ = W.config1_random(n)
    log("case headline brick 30q tiled vs pergate")
    bufs = []
    for mode, k in [("tiled", 2), ("pergate", 1)]:
        buf = torch.empty(2 << n, dtype=torch.float64, device="cuda")
        s = Q.Simulator(n_max=n, mode=mode, k_max=k, state=buf, use_torch_stream=False)
        s.allocate(n)
        s.run(circ)
        s.flush()
        s.synchronize()
        s.close()
        bufs.append(buf)
        log("  %s done" % mode)
    torch.cuda.synchronize()
    worst = 0.0
    chunk = 1 << 28
    for i in range(0, 2 << n, chunk):
        d = (bufs[0][i:i + chunk] - bufs[1][i:i + chunk]).view(-1, 2)
        worst = max(worst, float(torch.sqrt((d * d).sum(dim=1)).max()))
    norm = float((bufs[0] * bufs[0]).sum())
    del bufs
    torch.cuda.empty_cache()
    log("  max |tiled - pergate| = %.3g, norm2 = %.15f" % (worst, norm))
    assert worst <= 1e-12
    assert abs(norm - 1.0) <= 1e-11
