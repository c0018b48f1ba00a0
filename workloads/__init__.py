"""Seeded synthetic inputs for the state-vector simulator.

This module only *generates* inputs: gate matrices, circuits (ordered gate
lists), Pauli-sum Hamiltonians and uniform random numbers.  It holds none of
the simulator's arithmetic (no gate application, no reduction), so both the
CPU oracle's tests and the GPU path can draw from it without sharing any of
the computation being checked.

Conventions (the paper leaves them open; the readings are fixed here once):

* A k-qubit gate matrix is 2^k x 2^k complex128, row-major; bit j of the row
  or column index belongs to ``targets[j]``.  Controls condition on |1>
  (the ``Control`` meta-instruction, Sec. 4.1.3).
* Qubit j of an n-qubit register is bit j of the amplitude index
  (little-endian), the register starting in |0...0> (Sec. 4, minimal example).
* Rotations: R_P(theta) = exp(-i theta P / 2); the phase gate
  R(phi) = diag(1, e^{i phi}).  ``Rx(0.5) | qubit`` appears in Sec. 4 without a
  definition; this is the usual one.
* Haar-random 2x2 unitaries follow Mezzadri's QR recipe (Notices AMS 2007).

Every generator takes its randomness from a ``numpy.random.Generator`` over
PCG64, seeded as ``SeedSequence(161208091 + config_index).spawn(4)``; the four
children feed, in order: gates/angles, the Hamiltonian, the basis state, and
the sampling/measurement uniforms.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 161208091

# --------------------------------------------------------------------------
# gate matrices
# --------------------------------------------------------------------------
_SQ2 = 1.0 / math.sqrt(2.0)
H = np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
T = np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=np.complex128)
# SWAP on (targets[0], targets[1]); row/col index r = b0 + 2*b1.
SWAP = np.array([[1, 0, 0, 0],
                 [0, 0, 1, 0],
                 [0, 1, 0, 0],
                 [0, 0, 0, 1]], dtype=np.complex128)
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}


def rx(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(theta: float) -> np.ndarray:
    return np.array([[np.exp(-0.5j * theta), 0], [0, np.exp(0.5j * theta)]],
                    dtype=np.complex128)


def phase(phi: float) -> np.ndarray:
    return np.array([[1, 0], [0, np.exp(1j * phi)]], dtype=np.complex128)


ROTATION = {"X": rx, "Y": ry, "Z": rz}


def haar_2x2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random U(2) matrix: QR of a complex Ginibre matrix, with the phases
    of R's diagonal moved into Q.  A is drawn before B."""
    a = rng.standard_normal((2, 2))
    b = rng.standard_normal((2, 2))
    zmat = (a + 1j * b) / math.sqrt(2.0)
    q, r = np.linalg.qr(zmat)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def haar_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    a = rng.standard_normal((dim, dim))
    b = rng.standard_normal((dim, dim))
    zmat = (a + 1j * b) / math.sqrt(2.0)
    q, r = np.linalg.qr(zmat)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


# --------------------------------------------------------------------------
# circuits
# --------------------------------------------------------------------------
@dataclass
class Gate:
    """One (controlled) k-qubit gate: ``matrix`` acts on ``targets`` when every
    qubit in ``controls`` is |1>.  Rotation gates exp(-i theta P/2) also carry
    the index of their angle in the circuit's parameter vector and the axis P,
    which the adjoint gradient needs."""
    matrix: np.ndarray
    targets: Tuple[int, ...]
    controls: Tuple[int, ...] = ()
    name: str = ""
    param: int = -1
    axis: str = ""

    @property
    def k(self) -> int:
        return len(self.targets)


@dataclass
class Circuit:
    n: int
    gates: List[Gate] = field(default_factory=list)
    theta: Optional[np.ndarray] = None   # rotation angles, indexed by Gate.param
    label: str = ""

    def add(self, matrix, targets, controls=(), name="", param=-1, axis=""):
        self.gates.append(Gate(np.asarray(matrix, dtype=np.complex128),
                               tuple(int(t) for t in targets),
                               tuple(int(c) for c in controls), name, param, axis))
        return self

    def counts(self):
        out = {}
        for g in self.gates:
            out[g.name] = out.get(g.name, 0) + 1
        return out

    def with_theta(self, theta: np.ndarray) -> "Circuit":
        """The same circuit with its rotation gates rebuilt at new angles."""
        c = Circuit(self.n, [], np.asarray(theta, dtype=np.float64).copy(), self.label)
        for g in self.gates:
            if g.param >= 0:
                c.add(ROTATION[g.axis](float(theta[g.param])), g.targets, g.controls,
                      g.name, g.param, g.axis)
            else:
                c.gates.append(g)
        return c


def streams(config_index: int):
    """The four seeded generators of a configuration (gates, Hamiltonian,
    basis state, uniforms)."""
    ss = np.random.SeedSequence(SEED_BASE + config_index)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]


def brick_pairs(n: int, layer: int):
    """Neighbour pairs (q, q+1) for q = layer%2, layer%2+2, ... (q+1 < n)."""
    return [(q, q + 1) for q in range(layer % 2, n - 1, 2)]


def random_brick(n: int, layers: int, rng: np.random.Generator,
                 two_qubit: str = "cnot") -> Circuit:
    """Layers of a Haar-random 2x2 gate on every qubit, then a two-qubit gate on
    alternating neighbour pairs: CNOT (control q, target q+1) or CZ."""
    c = Circuit(n, label=f"brick-{two_qubit}-{n}q-{layers}l")
    for layer in range(layers):
        for q in range(n):
            c.add(haar_2x2(rng), (q,), name="haar")
        for (a, b) in brick_pairs(n, layer):
            if two_qubit == "cnot":
                c.add(X, (b,), (a,), name="cnot")
            elif two_qubit == "cz":
                c.add(Z, (b,), (a,), name="cz")
            else:
                raise ValueError(two_qubit)
    return c


def qft(n: int, qubits: Optional[Sequence[int]] = None, inverse: bool = False) -> Circuit:
    """QFT|x> = 2^{-n/2} sum_y e^{+2 pi i x y / 2^n}|y> on ``qubits`` (bit j of x
    is qubits[j]): for j from high to low, H on q_j then controlled phases
    R(pi/2^{j-k}) from every lower q_k, then the bit-reversal swaps.  With
    ``inverse`` the gate list is reversed and every gate is replaced by its
    adjoint (the Dagger meta-instruction, Sec. 4.1.3)."""
    q = list(range(n)) if qubits is None else list(qubits)
    m = len(q)
    c = Circuit(max(q) + 1 if q else 0, label=f"qft-{m}")
    for j in range(m - 1, -1, -1):
        c.add(H, (q[j],), name="h")
        for k in range(j - 1, -1, -1):
            c.add(phase(math.pi / 2 ** (j - k)), (q[j],), (q[k],), name="cphase")
    for i in range(m // 2):
        c.add(SWAP, (q[i], q[m - 1 - i]), name="swap")
    if inverse:
        c.gates = [Gate(g.matrix.conj().T.copy(), g.targets, g.controls, g.name + "_dag")
                   for g in reversed(c.gates)]
    return c


def basis_prep(n: int, x: int) -> Circuit:
    """X on every set bit of x, preparing |x> from |0...0>."""
    c = Circuit(n, label=f"basis-{x}")
    for q in range(n):
        if (x >> q) & 1:
            c.add(X, (q,), name="x")
    return c


def draper_add(n: int, const: int, qubits: Optional[Sequence[int]] = None) -> Circuit:
    """Constant adder in Fourier space (Sec. 3): QFT, a phase R(2 pi c 2^j / 2^m)
    on register qubit j, inverse QFT; maps |x> to |x + c mod 2^m> on the
    register ``qubits`` (default 0..n-1; bit j of x is qubits[j])."""
    q = list(range(n)) if qubits is None else list(qubits)
    m = len(q)
    c = qft(n, q)
    c.n = max(n, c.n)
    c.label = f"draper-{m}-{const}"
    for j in range(m):
        ang = 2 * math.pi * ((const * (1 << j)) % (1 << m)) / (1 << m)
        c.add(phase(ang), (q[j],), name="phase")
    c.gates += qft(n, q, inverse=True).gates
    return c


# --------------------------------------------------------------------------
# noise channels (Kraus operators) and noisy circuits
# --------------------------------------------------------------------------
def depolarizing(p: float):
    """rho -> (1 - p) rho + p I/2 on one qubit."""
    a, b = math.sqrt(1 - 3 * p / 4), math.sqrt(p / 4)
    return [a * I2, b * X, b * Y, b * Z]


def amplitude_damping(gamma: float):
    """|1> decays to |0> with probability gamma."""
    return [np.array([[1, 0], [0, math.sqrt(1 - gamma)]], dtype=np.complex128),
            np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128)]


def dephasing(p: float):
    """Off-diagonal elements scaled by 1 - p."""
    return [math.sqrt(1 - p / 2) * I2, math.sqrt(p / 2) * Z]


def noisy_brick(n: int, layers: int, p: float, rng: np.random.Generator, gamma: float = 0.0):
    """Events of a noisy brick circuit: per layer a Haar 1-qubit gate on every
    qubit followed by depolarizing noise p on it, then CNOTs on alternating
    neighbour pairs, each followed by depolarizing noise on both qubits and,
    if gamma > 0, amplitude damping on the target.  Events are ("gate", U,
    targets, controls) and ("kraus", [K_j], targets)."""
    ev = []
    dep = depolarizing(p)
    for layer in range(layers):
        for q in range(n):
            ev.append(("gate", haar_2x2(rng), (q,), ()))
            ev.append(("kraus", dep, (q,)))
        for (a, b) in brick_pairs(n, layer):
            ev.append(("gate", X, (b,), (a,)))
            ev.append(("kraus", dep, (a,)))
            ev.append(("kraus", dep, (b,)))
            if gamma > 0:
                ev.append(("kraus", amplitude_damping(gamma), (b,)))
    return ev


def add_constant_table(w: int, const: int) -> np.ndarray:
    """The classical function of the AddConstant math gate (Sec. 3,
    Sec. 4.3.3), tabulated: x -> x + c mod 2^w."""
    x = np.arange(1 << w, dtype=np.uint64)
    return ((x + np.uint64(const % (1 << w))) % np.uint64(1 << w)).astype(np.uint32)


def mul_mod_table(w: int, a: int, modulus: int) -> np.ndarray:
    """x -> a x mod N for x < N and x itself for N <= x < 2^w, the modular
    multiplication of Shor's algorithm (Sec. 5) as a bijection of the w-bit
    register (gcd(a, N) = 1, N <= 2^w)."""
    assert math.gcd(a, modulus) == 1 and 0 < modulus <= (1 << w)
    x = np.arange(1 << w, dtype=np.uint64)
    out = x.copy()
    low = x < modulus
    out[low] = (np.uint64(a % modulus) * x[low]) % np.uint64(modulus)
    return out.astype(np.uint32)


def ghz(n: int) -> Circuit:
    """The Entangle operation of Sec. 4.3.1: H on qubit 0, then CNOT from qubit 0
    onto every other qubit."""
    c = Circuit(n, label=f"ghz-{n}")
    c.add(H, (0,), name="h")
    for q in range(1, n):
        c.add(X, (q,), (0,), name="cnot")
    return c


def w_state(n: int) -> Circuit:
    """X(q0); for i = 0..n-2: controlled-RY(theta_i) q_i -> q_{i+1} with
    cos(theta_i/2) = (n-i)^{-1/2}, then CNOT q_{i+1} -> q_i."""
    c = Circuit(n, label=f"w-{n}")
    c.add(X, (0,), name="x")
    for i in range(n - 1):
        th = 2 * math.acos(1 / math.sqrt(n - i))
        c.add(ry(th), (i + 1,), (i,), name="cry")
        c.add(X, (i,), (i + 1,), name="cnot")
    return c


def grover(n: int, marked: int, iterations: Optional[int] = None) -> Circuit:
    """Grover search (App. A.2) over n qubits x plus one oracle qubit prepared in
    |->.  Oracle: X on the zero bits of ``marked``, an n-controlled X onto the
    oracle qubit, undo the X gates.  Diffusion: H and X on every x qubit, a
    Z on x[-1] controlled by x[0..n-2], undo.  Iterations default to
    floor(pi sqrt(N) / 4)."""
    if iterations is None:
        iterations = int(math.floor(math.pi * math.sqrt(2 ** n) / 4))
    c = Circuit(n + 1, label=f"grover-{n}")
    anc = n
    c.add(X, (anc,), name="x")
    c.add(H, (anc,), name="h")
    for q in range(n):
        c.add(H, (q,), name="h")
    zeros = [q for q in range(n) if not (marked >> q) & 1]
    for _ in range(iterations):
        for q in zeros:
            c.add(X, (q,), name="x")
        c.add(X, (anc,), tuple(range(n)), name="mcx")
        for q in zeros:
            c.add(X, (q,), name="x")
        for q in range(n):
            c.add(H, (q,), name="h")
        for q in range(n):
            c.add(X, (q,), name="x")
        c.add(Z, (n - 1,), tuple(range(n - 1)), name="mcz")
        for q in range(n):
            c.add(X, (q,), name="x")
        for q in range(n):
            c.add(H, (q,), name="h")
    return c


def simcomparison(n: int, rng: np.random.Generator) -> Circuit:
    """The timed circuit of the paper's simulator comparison (Sec. 4.3.2):
    H on every qubit, a chain of controlled Rz(theta_i) with control q_i and
    target q_{i+1}, theta_i ~ U(0, 2 pi), H on every qubit."""
    c = Circuit(n, label=f"simcmp-{n}")
    for q in range(n):
        c.add(H, (q,), name="h")
    for i in range(n - 1):
        c.add(rz(float(rng.uniform(0, 2 * math.pi))), (i + 1,), (i,), name="crz")
    for q in range(n):
        c.add(H, (q,), name="h")
    return c


def hea(n: int, layers: int, theta: np.ndarray) -> Circuit:
    """Hardware-efficient ansatz: per layer, RY then RZ on every qubit, then a CZ
    ladder (i, i+1) for i = 0..n-2.  Angle index = 2*(layer*n + q) + {0: RY, 1: RZ}."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (2 * n * layers,)
    c = Circuit(n, theta=theta.copy(), label=f"hea-{n}q-{layers}l")
    for layer in range(layers):
        for q in range(n):
            p = 2 * (layer * n + q)
            c.add(ry(float(theta[p])), (q,), name="ry", param=p, axis="Y")
            c.add(rz(float(theta[p + 1])), (q,), name="rz", param=p + 1, axis="Z")
        for i in range(n - 1):
            c.add(Z, (i + 1,), (i,), name="cz")
    return c


# --------------------------------------------------------------------------
# Pauli sums
# --------------------------------------------------------------------------
@dataclass
class PauliSum:
    """sum_t coeff[t] * P_t.  P_t is given by two bit masks over qubits:
    X -> (x=1, z=0), Z -> (x=0, z=1), Y -> (x=1, z=1)."""
    xmask: np.ndarray   # uint64[T]
    zmask: np.ndarray   # uint64[T]
    coeff: np.ndarray   # float64[T]

    def __len__(self):
        return len(self.coeff)

    def strings(self, n: int) -> List[str]:
        out = []
        for x, z in zip(self.xmask.tolist(), self.zmask.tolist()):
            s = []
            for q in range(n):
                bx, bz = (x >> q) & 1, (z >> q) & 1
                s.append("IXZY"[bx + 2 * bz])
            out.append("".join(s))
        return out

    @staticmethod
    def from_strings(strings: Sequence[str], coeff: Sequence[float]) -> "PauliSum":
        """Build from strings whose character q is the letter on qubit q."""
        xs, zs = [], []
        for s in strings:
            x = z = 0
            for q, ch in enumerate(s):
                if ch in "XY":
                    x |= 1 << q
                if ch in "ZY":
                    z |= 1 << q
            xs.append(x)
            zs.append(z)
        return PauliSum(np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
                        np.asarray(coeff, dtype=np.float64))


def random_pauli_dense(n: int, terms: int, rng: np.random.Generator) -> PauliSum:
    """Each qubit's letter uniform over {I,X,Y,Z} (an all-I term is allowed);
    coefficients N(0,1).  Letters are drawn before coefficients."""
    letters = rng.integers(0, 4, size=(terms, n))
    coeff = rng.standard_normal(terms)
    strings = ["".join("IXYZ"[v] for v in row) for row in letters]
    return PauliSum.from_strings(strings, coeff)


def random_pauli_local(n: int, terms: int, max_weight: int,
                       rng: np.random.Generator) -> PauliSum:
    """Weight w ~ U{1..max_weight}, w distinct qubits uniform without
    replacement, letters uniform over {X,Y,Z}; coefficients N(0,1) drawn after
    all the strings."""
    strings = []
    for _ in range(terms):
        w = int(rng.integers(1, max_weight + 1))
        qs = rng.choice(n, size=w, replace=False)
        let = rng.integers(0, 3, size=w)
        s = ["I"] * n
        for q, l in zip(qs.tolist(), let.tolist()):
            s[q] = "XYZ"[l]
        strings.append("".join(s))
    coeff = rng.standard_normal(terms)
    return PauliSum.from_strings(strings, coeff)


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------
def config0(n: int = 16, layers: int = 20, shots: int = 1000):
    """16-qubit Haar+CNOT brick circuit, 20 layers; 1000 sampling uniforms."""
    g, _, _, u = streams(0)
    circ = random_brick(n, layers, g, "cnot")
    return circ, u.random(shots)


def config1_random(n: int = 30, layers: int = 40):
    """30-qubit Haar+CNOT brick circuit, 40 layers (1200 Haar + 580 CNOT)."""
    g, _, _, _ = streams(1)
    return random_brick(n, layers, g, "cnot")


def config1_qft(n: int = 30):
    """A random basis state |x>, x ~ U{0..2^n-1}, and the n-qubit QFT circuit.
    The state is prepared by the caller (X gates or a set-state); the QFT has
    n H + n(n-1)/2 controlled phases + floor(n/2) swaps."""
    _, _, b, _ = streams(1)
    x = int(b.integers(0, 1 << n))
    return x, qft(n)


def config2(n: int = 32, layers: int = 40):
    """32-qubit Haar + CZ brick circuit, 40 layers (1280 Haar + 620 CZ).
    Smaller ``n`` gives the twin used against the CPU oracle."""
    g, _, _, _ = streams(2)
    return random_brick(n, layers, g, "cz")


def config3(count: int = 4096, n_lo: int = 8, n_hi: int = 20, layers: int = 6,
            terms: int = 64):
    """``count`` HEA circuits with n ~ U{n_lo..n_hi}, ``layers`` layers of
    angles ~ U(0, 2 pi), each with a ``terms``-term dense random Pauli sum.
    Qubit counts are drawn first, then every circuit's angles in order."""
    g, hrng, _, _ = streams(3)
    ns = g.integers(n_lo, n_hi + 1, size=count)
    circuits, hams = [], []
    for n in ns.tolist():
        th = g.uniform(0, 2 * math.pi, size=2 * n * layers)
        circuits.append(hea(n, layers, th))
    for n in ns.tolist():
        hams.append(random_pauli_dense(n, terms, hrng))
    return circuits, hams


def config4(n: int = 24, layers: int = 10, terms: int = 200, max_weight: int = 4):
    """24-qubit HEA, 10 layers (480 angles ~ U(0, 2 pi)) and a 200-term Pauli sum
    of weight <= 4 with N(0,1) coefficients."""
    g, hrng, _, _ = streams(4)
    th = g.uniform(0, 2 * math.pi, size=2 * n * layers)
    return hea(n, layers, th), random_pauli_local(n, terms, max_weight, hrng)
