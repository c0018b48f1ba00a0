"""Brute-force references for pinning the oracle: every operator is built as a
dense 2^n x 2^n matrix from Kronecker products and index permutations, with
numpy only.  Shares nothing with ``oracle/`` (which loops over amplitudes) or
with the GPU library.  Keep n <= 10."""
import numpy as np

PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def local_operator(matrix, k, c):
    """Operator on (targets..., controls...) in local bit order (bit j of the
    local index = j-th listed qubit): U on the targets when every control is 1,
    identity otherwise.  np.kron(A, B) puts A on the high (control) bits."""
    dim_c = 1 << c
    p1 = np.zeros((dim_c, dim_c))
    p1[-1, -1] = 1.0
    return np.kron(p1, matrix) + np.kron(np.eye(dim_c) - p1, np.eye(1 << k))


def embed(op_local, qubits, n):
    """Dense n-qubit operator from an operator on ``qubits`` (local bit j =
    qubits[j]); the other qubits see the identity."""
    m = len(qubits)
    rest = [q for q in range(n) if q not in qubits]
    order = list(qubits) + rest          # local bit position -> global qubit
    full_local = np.kron(np.eye(1 << (n - m)), op_local)
    idx = np.arange(1 << n)
    loc = np.zeros(1 << n, dtype=np.int64)
    for lb, q in enumerate(order):
        loc |= ((idx >> q) & 1) << lb
    # full[i, j] = full_local[loc[i], loc[j]]
    return full_local[np.ix_(loc, loc)]


def gate_operator(matrix, targets, controls, n):
    return embed(local_operator(np.asarray(matrix), len(targets), len(controls)),
                 list(targets) + list(controls), n)


def circuit_operator(circuit):
    n = circuit.n
    full = np.eye(1 << n, dtype=np.complex128)
    for g in circuit.gates:
        full = gate_operator(g.matrix, g.targets, g.controls, n) @ full
    return full


def pauli_operator(string):
    """Dense operator of a Pauli string whose character q acts on qubit q."""
    op = np.ones((1, 1), dtype=np.complex128)
    for ch in string:            # qubit 0 first -> ends up on the lowest bit
        op = np.kron(PAULI[ch], op)
    return op


def hamiltonian_operator(ham, n):
    full = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for s, c in zip(ham.strings(n), ham.coeff.tolist()):
        full += c * pauli_operator(s)
    return full
