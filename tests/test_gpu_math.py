"""Emulated math gates (Sec. 4.3.3) on the GPU against the CPU oracle.

A math gate only moves amplitudes, so given the same input state the GPU
result must equal the oracle's bit for bit (complex128 and complex64).  The
inputs are set from the host; tables are random permutations, AddConstant and
modular multiplication (Shor's step, Sec. 5), on contiguous and scattered
registers, with and without controls, inside a queue of ordinary gates, on a
borrowed torch buffer, and at 30 qubits (sampled amplitudes against the
inverse table, then the inverse gate restoring the state bit for bit).
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


def random_state(rng, n, dtype=np.complex128):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(dtype)


CASES = [
    # n, register, controls, table kind
    (16, list(range(3, 13)), [], "perm"),               # contiguous, 10 bits
    (16, [14, 2, 9, 0, 5, 11], [7], "perm"),             # scattered, one control
    (16, [1, 4, 6, 8, 10], [0, 15], "add"),              # two controls
    (14, list(range(14)), [], "perm"),                   # the whole state
    (12, [5], [2], "x"),                                 # one bit: controlled X
    (15, [0, 1, 2, 3, 4, 5, 6, 7], [12], "mulmod"),      # Shor's modular multiplication
]


def _table(kind, w, rng):
    if kind == "perm":
        return rng.permutation(1 << w).astype(np.uint32)
    if kind == "add":
        return W.add_constant_table(w, 13)
    if kind == "x":
        return np.array([1, 0], dtype=np.uint32)
    return W.mul_mod_table(w, 7, 221)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_math_gate_bit_exact_vs_oracle(dtype, case):
    n, reg, ctrl, kind = CASES[case]
    log("math gate", dtype, CASES[case])
    rng = np.random.default_rng(100 + case)
    npd = np.complex128 if dtype == "c128" else np.complex64
    psi = random_state(rng, n, npd)
    tab = _table(kind, len(reg), rng)
    s = make(n, dtype=dtype)
    s.set_state(psi)
    s.apply_math(reg, tab, ctrl)
    got = s.get_state()
    s.close()
    want = oracle.apply_math(psi.astype(np.complex128), tab, reg, ctrl)
    assert np.array_equal(got.astype(np.complex128), want)


def test_math_gate_inside_a_gate_queue():
    """Gates before the math gate are flushed first, gates after it queue on
    the permuted state."""
    rng = np.random.default_rng(7)
    n = 13
    pre = W.random_brick(n, 3, rng, "cnot")
    post = W.random_brick(n, 2, rng, "cz")
    reg, ctrl, tab = [2, 3, 4, 5, 6, 7], [11], W.add_constant_table(6, 45)
    s = make(n)
    s.run(pre)
    s.apply_math(reg, tab, ctrl)
    s.run(post)
    got = s.get_state()
    s.close()
    want = oracle.run(pre)
    oracle.apply_math(want, tab, reg, ctrl)
    oracle.run(post, want)
    assert np.max(np.abs(got - want)) <= 1e-12


def test_math_add_constant_equals_gate_level_adder_on_gpu():
    """The emulated AddConstant and the gate-level Draper adder (QFT, phases,
    inverse QFT) run on the GPU agree to rounding."""
    rng = np.random.default_rng(8)
    n, reg, c = 14, [3, 4, 5, 6, 7, 8, 9, 10], 77
    psi = random_state(rng, n)
    a = make(n)
    a.set_state(psi)
    a.apply_math(reg, W.add_constant_table(len(reg), c))
    got_emu = a.get_state()
    a.close()
    b = make(n)
    b.set_state(psi)
    b.run(W.draper_add(n, c, reg))
    got_gates = b.get_state()
    b.close()
    assert np.max(np.abs(got_emu - got_gates)) <= 1e-12


def test_math_gate_on_borrowed_torch_state():
    import torch
    n = 12
    rng = np.random.default_rng(9)
    psi = random_state(rng, n)
    buf = torch.from_numpy(psi.view(np.float64).copy()).cuda()
    s = Q.Simulator(n_max=n, state=buf)
    s.allocate(n)
    s.set_state(psi)
    tab = rng.permutation(1 << 7).astype(np.uint32)
    reg = [0, 2, 4, 6, 8, 10, 11]
    s.apply_math(reg, tab, [1])
    s.synchronize()
    torch.cuda.synchronize()
    got = buf.cpu().numpy().view(np.complex128)
    s.close()
    assert np.array_equal(got, oracle.apply_math(psi.copy(), tab, reg, [1]))


def test_math_gate_30q_sampled_then_inverse():
    """30 qubits, complex128: Shor's modular multiplication on a 20-bit
    register, controlled by qubit 0; sampled amplitudes against the source
    index the inverse table gives, then the inverse multiplication restores
    the sampled amplitudes bit for bit."""
    rng = np.random.default_rng(10)
    n, w, N, a = 30, 20, 1048573, 5
    reg = list(range(6, 26))
    tab, inv = W.mul_mod_table(w, a, N), W.mul_mod_table(w, pow(a, -1, N), N)
    s = make(n)
    for q in range(n):                       # a product state with distinct amplitudes
        s.apply(W.haar_2x2(rng), [q])
    s.flush()
    idx = rng.integers(0, 1 << n, 4096, dtype=np.uint64)
    idx[0] = 0
    idx[1] = (1 << n) - 1
    inv_tab = np.argsort(tab).astype(np.uint64)   # inverse permutation
    src = []
    for j in idx.tolist():
        if j & 1:
            y = (j >> 6) & ((1 << w) - 1)
            x = int(inv_tab[y])
            j = (j & ~(((1 << w) - 1) << 6)) | (x << 6)
        src.append(j)
    before_src = s.get_amplitudes(np.array(src, dtype=np.uint64))
    before = s.get_amplitudes(idx)
    log("30q math gate: apply")
    s.apply_math(reg, tab, [0])
    after = s.get_amplitudes(idx)
    assert np.array_equal(after, before_src)
    log("30q math gate: inverse")
    s.apply_math(reg, inv, [0])
    back = s.get_amplitudes(idx)
    assert np.array_equal(back, before)
    assert abs(s.norm2() - 1.0) <= 1e-12
    s.close()
