"""CPU oracle for the state-vector simulator -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never loads it, and it shares
no code with the GPU path: it takes circuits and Pauli sums as produced by the
``workloads`` generators and computes, one gate at a time in complex128, what
the simulator must produce.

The arithmetic lives in ``qsv_oracle.c`` (plain C, built with gcc); this file
only marshals numpy arrays and strings calls together:

* ``run``           apply a circuit's gates in order (Sec. 4.3.2: gate-level
                    simulation of the whole state).
* ``expectation``   sum_t c_t <psi|P_t|psi> (Pauli sums, built term by term).
* ``measure``/``sample``/``dealloc``/``prob_bits``/``probs``: the reductions.
* ``grad_param_shift`` / ``grad_fd``: gradients of <H> by re-running the
  forward circuit; the shift rule is exact for exp(-i theta P / 2) gates.
* ``apply_math``    an emulated math gate (Sec. 4.3.3): a tabulated classical
                    bijection applied to a register of a superposition.
* ``dm_*``          density matrices (the noise simulator Sec. 4.3.2 names as
                    future work): gates as G rho G^dagger, channels as
                    sum_j K_j rho K_j^dagger, Tr(rho P) per Pauli string.
* ``kraus_sample``  one step of a stochastic noise trajectory (the stochastic
                    noise models named beside it): branch j of a channel with
                    probability ||K_j psi||^2, the state renormalised.

Parity status of every function is stated in the module docstring of the
test that pins it (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        c_d, c_i, c_u64 = ctypes.c_double, ctypes.c_int, ctypes.c_uint64
        lib.oracle_apply.argtypes = [P(c_d), c_i, P(c_d), c_i, P(c_i), c_i, P(c_i)]
        lib.oracle_apply.restype = c_i
        lib.oracle_set_threads.argtypes = [c_i]
        lib.oracle_set_threads.restype = c_i
        lib.oracle_probs.argtypes = [P(c_d), c_i, P(c_d)]
        lib.oracle_probs.restype = None
        lib.oracle_prob_bits.argtypes = [P(c_d), c_i, c_i, P(c_i), P(c_i)]
        lib.oracle_prob_bits.restype = c_d
        lib.oracle_expectation.argtypes = [P(c_d), c_i, c_i, P(c_u64), P(c_u64), P(c_d),
                                           P(c_d), P(c_d)]
        lib.oracle_expectation.restype = c_d
        lib.oracle_measure.argtypes = [P(c_d), c_i, c_i, c_d, P(c_d)]
        lib.oracle_measure.restype = c_i
        lib.oracle_sample.argtypes = [P(c_d), c_i, c_i, P(c_d), P(c_u64)]
        lib.oracle_sample.restype = c_i
        lib.oracle_dealloc.argtypes = [P(c_d), c_i, c_i, c_d, P(c_d)]
        lib.oracle_dealloc.restype = c_i
        lib.oracle_apply_math.argtypes = [P(c_d), c_i, c_i, P(c_i), P(ctypes.c_uint32), c_i,
                                          P(c_i)]
        lib.oracle_apply_math.restype = c_i
        lib.oracle_dm_apply.argtypes = [P(c_d), c_i, P(c_d), c_i, P(c_i), c_i, P(c_i)]
        lib.oracle_dm_apply.restype = c_i
        lib.oracle_dm_kraus.argtypes = [P(c_d), c_i, c_i, P(c_d), c_i, P(c_i)]
        lib.oracle_dm_kraus.restype = c_i
        lib.oracle_dm_expectation.argtypes = [P(c_d), c_i, c_i, P(c_u64), P(c_u64), P(c_d),
                                              P(c_d), P(c_d)]
        lib.oracle_dm_expectation.restype = c_d
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _nq(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    assert psi.size == 1 << n and psi.dtype == np.complex128 and psi.flags.c_contiguous
    return n


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def basis_state(n: int, x: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def set_threads(t: int) -> int:
    """Threads for the outer loop of ``apply`` (1, the default, is serial);
    returns the number in effect.  Results do not depend on it."""
    return int(_load().oracle_set_threads(int(t)))


def apply(psi: np.ndarray, matrix, targets: Sequence[int], controls: Sequence[int] = ()):
    """Apply one gate in place (qubit q = bit q)."""
    n = _nq(psi)
    u = np.ascontiguousarray(matrix, dtype=np.complex128)
    k = len(targets)
    assert u.shape == (1 << k, 1 << k)
    t = np.ascontiguousarray(targets, dtype=np.intc)
    c = np.ascontiguousarray(controls if len(controls) else [0], dtype=np.intc)
    qs = list(targets) + list(controls)
    assert len(set(qs)) == len(qs) and all(0 <= q < n for q in qs)
    rc = _load().oracle_apply(_dp(psi.view(np.float64)), n, _dp(u.view(np.float64)), k,
                              _ip(t), len(controls), _ip(c))
    if rc != 0:
        raise ValueError("oracle_apply rejected its arguments")
    return psi


def run(circuit, psi: Optional[np.ndarray] = None, gates: Optional[Iterable] = None):
    """Apply every gate of ``circuit`` (in issue order) to ``psi`` (default
    |0...0>).  Returns the state."""
    if psi is None:
        psi = zero_state(circuit.n)
    for g in (circuit.gates if gates is None else gates):
        apply(psi, g.matrix, g.targets, g.controls)
    return psi


def probs(psi: np.ndarray) -> np.ndarray:
    n = _nq(psi)
    out = np.empty(1 << n, dtype=np.float64)
    _load().oracle_probs(_dp(psi.view(np.float64)), n, _dp(out))
    return out


def prob_bits(psi: np.ndarray, qubits: Sequence[int], bits: Sequence[int]) -> float:
    n = _nq(psi)
    q = np.ascontiguousarray(qubits if len(qubits) else [0], dtype=np.intc)
    b = np.ascontiguousarray(bits if len(bits) else [0], dtype=np.intc)
    return _load().oracle_prob_bits(_dp(psi.view(np.float64)), n, len(qubits), _ip(q), _ip(b))


def norm2(psi: np.ndarray) -> float:
    return prob_bits(psi, [], [])


def expectation(psi: np.ndarray, ham, return_terms: bool = False):
    """Returns (sum_t c_t Re<P_t>, sum_t c_t Im<P_t>) [, per-term complex]."""
    n = _nq(psi)
    x = np.ascontiguousarray(ham.xmask, dtype=np.uint64)
    z = np.ascontiguousarray(ham.zmask, dtype=np.uint64)
    c = np.ascontiguousarray(ham.coeff, dtype=np.float64)
    nt = len(c)
    terms = np.zeros(max(nt, 1), dtype=np.complex128)
    im = ctypes.c_double(0.0)
    re = _load().oracle_expectation(_dp(psi.view(np.float64)), n, nt, _up(x), _up(z), _dp(c),
                                    _dp(terms.view(np.float64)), ctypes.byref(im))
    if return_terms:
        return re, im.value, terms[:nt]
    return re, im.value


def measure(psi: np.ndarray, qubit: int, u: float):
    """Collapse ``qubit`` in place; returns (outcome, p0, p1)."""
    n = _nq(psi)
    pp = np.zeros(2, dtype=np.float64)
    out = _load().oracle_measure(_dp(psi.view(np.float64)), n, int(qubit), float(u), _dp(pp))
    return out, float(pp[0]), float(pp[1])


def sample(psi: np.ndarray, u: np.ndarray) -> np.ndarray:
    n = _nq(psi)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(max(len(u), 1), dtype=np.uint64)
    rc = _load().oracle_sample(_dp(psi.view(np.float64)), n, len(u), _dp(u), _up(out))
    if rc != 0:
        raise MemoryError("oracle_sample")
    return out[:len(u)]


def dealloc(psi: np.ndarray, qubit: int, tau: float):
    """Returns (value, compacted state) or raises ValueError when the qubit is
    in superposition (Sec. 4.1.1)."""
    n = _nq(psi)
    out = np.zeros(1 << (n - 1), dtype=np.complex128)
    v = _load().oracle_dealloc(_dp(psi.view(np.float64)), n, int(qubit), float(tau),
                               _dp(out.view(np.float64)))
    if v < 0:
        raise ValueError("qubit %d is not in a classical state" % qubit)
    return v, out


def apply_math(psi: np.ndarray, table, qubits: Sequence[int], controls: Sequence[int] = ()):
    """Emulated math gate in place (Sec. 4.3.3): the register `qubits`
    (first = least significant) takes the value table[x] wherever the controls
    are 1.  `table` must be a permutation of range(2**len(qubits))."""
    n = _nq(psi)
    w = len(qubits)
    tab = np.ascontiguousarray(table, dtype=np.uint32)
    assert tab.shape == (1 << w,)
    q = np.ascontiguousarray(qubits, dtype=np.intc)
    c = np.ascontiguousarray(controls if len(controls) else [0], dtype=np.intc)
    qs = list(qubits) + list(controls)
    assert len(set(qs)) == len(qs) and all(0 <= x < n for x in qs)
    rc = _load().oracle_apply_math(_dp(psi.view(np.float64)), n, w, _ip(q),
                                   tab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                   len(controls), _ip(c))
    if rc != 0:
        raise ValueError("oracle_apply_math: bad arguments or the table is not a permutation")
    return psi


# ------------------------------------------------------------ density matrices
def _dn(rho: np.ndarray) -> int:
    n = int(rho.shape[0]).bit_length() - 1
    assert rho.shape == (1 << n, 1 << n) and rho.dtype == np.complex128 and rho.flags.c_contiguous
    return n


def dm_zero(n: int) -> np.ndarray:
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[0, 0] = 1.0
    return rho


def dm_apply(rho: np.ndarray, matrix, targets: Sequence[int], controls: Sequence[int] = ()):
    """rho <- G rho G^dagger in place, G the (controlled) gate."""
    n = _dn(rho)
    u = np.ascontiguousarray(matrix, dtype=np.complex128)
    t = np.ascontiguousarray(targets, dtype=np.intc)
    c = np.ascontiguousarray(controls if len(controls) else [0], dtype=np.intc)
    if _load().oracle_dm_apply(_dp(rho.view(np.float64)), n, _dp(u.view(np.float64)),
                               len(targets), _ip(t), len(controls), _ip(c)) != 0:
        raise ValueError("oracle_dm_apply rejected its arguments")
    return rho


def dm_kraus(rho: np.ndarray, kraus, targets: Sequence[int]):
    """rho <- sum_j K_j rho K_j^dagger in place (a quantum channel)."""
    n = _dn(rho)
    ks = np.ascontiguousarray(np.stack([np.asarray(k, dtype=np.complex128) for k in kraus]))
    t = np.ascontiguousarray(targets, dtype=np.intc)
    if _load().oracle_dm_kraus(_dp(rho.view(np.float64)), n, len(ks), _dp(ks.view(np.float64)),
                               len(targets), _ip(t)) != 0:
        raise ValueError("oracle_dm_kraus rejected its arguments")
    return rho


def dm_expectation(rho: np.ndarray, ham, return_terms: bool = False):
    """(sum_t c_t Re Tr(rho P_t), sum_t c_t Im Tr(rho P_t)) [, per-term]."""
    n = _dn(rho)
    x = np.ascontiguousarray(ham.xmask, dtype=np.uint64)
    z = np.ascontiguousarray(ham.zmask, dtype=np.uint64)
    c = np.ascontiguousarray(ham.coeff, dtype=np.float64)
    nt = len(c)
    terms = np.zeros(max(nt, 1), dtype=np.complex128)
    im = ctypes.c_double(0.0)
    re = _load().oracle_dm_expectation(_dp(rho.view(np.float64)), n, nt, _up(x), _up(z), _dp(c),
                                       _dp(terms.view(np.float64)), ctypes.byref(im))
    if return_terms:
        return re, im.value, terms[:nt]
    return re, im.value


def dm_run(events, n: int) -> np.ndarray:
    """Apply a noisy circuit (workloads.NoisyCircuit events: ("gate", U,
    targets, controls) or ("kraus", [K_j], targets)) to |0..0><0..0|."""
    rho = dm_zero(n)
    for ev in events:
        if ev[0] == "gate":
            dm_apply(rho, ev[1], ev[2], ev[3])
        else:
            dm_kraus(rho, ev[1], ev[2])
    return rho


def kraus_sample(psi: np.ndarray, kraus, targets: Sequence[int], u: float):
    """Replace the channel {K_j} on ``targets`` by one branch, in place.
    Branch j has probability p_j = ||K_j psi||^2; the branch taken is the
    smallest j whose running sum of p exceeds u * sum_j p_j, and psi becomes
    K_j psi / sqrt(p_j).  Returns (j, p)."""
    branches = []
    for K in kraus:
        phi = psi.copy()
        apply(phi, np.asarray(K, dtype=np.complex128), targets)
        branches.append(phi)
    p = np.array([norm2(b) for b in branches])
    total = float(p.sum())
    if not total > 0.0:
        raise ValueError("the channel leaves no probability")
    r = u * total
    run = 0.0
    pick = -1
    for j, pj in enumerate(p):
        run += pj
        if run > r:
            pick = j
            break
    if pick < 0:
        pick = int(np.nonzero(p > 0)[0][-1])
    psi[:] = branches[pick] / math.sqrt(p[pick])
    return pick, p


def allocate(psi: np.ndarray, count: int = 1) -> np.ndarray:
    """New qubits in |0> take the next highest bit positions."""
    out = np.zeros(psi.size << count, dtype=np.complex128)
    out[:psi.size] = psi
    return out


def energy(circuit, ham) -> float:
    psi = run(circuit)
    return expectation(psi, ham)[0]


def grad_param_shift(circuit, ham, params: Optional[Sequence[int]] = None) -> np.ndarray:
    """d<H>/d theta_p = [<H>(theta_p + pi/2) - <H>(theta_p - pi/2)] / 2, exact for
    gates exp(-i theta P / 2) (each parameter used by one gate)."""
    theta = np.asarray(circuit.theta, dtype=np.float64)
    params = range(len(theta)) if params is None else params
    out = []
    for p in params:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += math.pi / 2
        tm[p] -= math.pi / 2
        out.append(0.5 * (energy(circuit.with_theta(tp), ham) -
                          energy(circuit.with_theta(tm), ham)))
    return np.array(out)


def grad_fd(circuit, ham, params: Optional[Sequence[int]] = None, h: float = 1e-5) -> np.ndarray:
    """Central finite differences of <H> with step h."""
    theta = np.asarray(circuit.theta, dtype=np.float64)
    params = range(len(theta)) if params is None else params
    out = []
    for p in params:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        out.append((energy(circuit.with_theta(tp), ham) -
                    energy(circuit.with_theta(tm), ham)) / (2 * h))
    return np.array(out)
