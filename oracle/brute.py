"""Brute-force pin for the oracle: full 2^n x 2^n matrices (n <= ~10).

Gate matrices here are *not* the closed forms used in ``sv_oracle.c``:
parametric gates are built as ``expm(-i t K)`` from their generators, which
are themselves Kronecker products of the Pauli matrices of eq. pauli_matrix;
fixed gates are sums of Kronecker products of projectors.  A full operator on
n qubits is assembled with ``np.kron`` with qubit 0 as the least significant
index bit (eq. sv).  TEST INFRASTRUCTURE ONLY.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
LETTER = {"I": I2, "X": PX, "Y": PY, "Z": PZ}


def two(a, b):
    """Operator a on the gate's first qubit (local bit 0) and b on its second
    (local bit 1): as a 4x4 matrix with local index l = b0 + 2 b1 this is
    kron(b, a)."""
    return np.kron(b, a)


def generator(kind: str) -> np.ndarray:
    if kind == "RX":
        return PX / 2
    if kind == "RY":
        return PY / 2
    if kind == "RZ":
        return PZ / 2
    if kind == "CPHASE":
        return -two(P1, P1)
    if kind == "GIVENS":
        return (two(PX, PY) - two(PY, PX)) / 4
    raise KeyError(kind)


def gate(kind: str, angle: float = 0.0) -> np.ndarray:
    if kind in ("RX", "RY", "RZ", "CPHASE", "GIVENS"):
        return expm(-1j * angle * generator(kind))
    if kind == "H":
        return (PX + PZ) / np.sqrt(2)
    if kind == "X":
        return PX
    if kind == "Y":
        return PY
    if kind == "Z":
        return PZ
    if kind == "S":
        return P0 + 1j * P1
    if kind == "T":
        return P0 + np.exp(1j * np.pi / 4) * P1
    if kind == "CNOT":           # first qubit controls
        return two(P0, I2) + two(P1, PX)
    if kind == "CZ":
        return two(P0, I2) + two(P1, PZ)
    if kind == "SWAP":
        return (two(I2, I2) + two(PX, PX) + two(PY, PY) + two(PZ, PZ)) / 2
    raise KeyError(kind)


def embed(n: int, local: np.ndarray, qubits) -> np.ndarray:
    """Full 2^n operator of a 1- or 2-qubit matrix on ``qubits`` (q[0] = local
    bit 0), as sum over matrix units |r><c| = kron of single-qubit units."""
    d = len(qubits)
    full = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for r in range(1 << d):
        for c in range(1 << d):
            if local[r, c] == 0:
                continue
            ops = [I2] * n
            for j, q in enumerate(qubits):
                u = np.zeros((2, 2), dtype=np.complex128)
                u[(r >> j) & 1, (c >> j) & 1] = 1.0
                ops[q] = u
            term = np.array([[1.0 + 0j]])
            for q in reversed(range(n)):     # qubit n-1 is the most significant factor
                term = np.kron(term, ops[q])
            full += local[r, c] * term
    return full


def circuit_unitary(n: int, gates, theta) -> np.ndarray:
    """Product of the embedded gate matrices.  A parametric gate's angle is
    scale * theta[param] + offset (gate tuple entries 4 and 3, defaults 1 and
    0); U1/U2 gates carry their matrix as entry 3."""
    U = np.eye(1 << n, dtype=np.complex128)
    for gt in gates:
        kind, qubits, p = gt[0], gt[1], gt[2]
        if kind in ("U1", "U2"):
            local = np.asarray(gt[3], dtype=np.complex128).reshape(2 * len(qubits), -1)
        else:
            if p is not None and p >= 0:
                ang = (gt[4] if len(gt) > 4 else 1.0) * theta[p] + (gt[3] if len(gt) > 3 else 0.0)
            else:
                ang = gt[3] if len(gt) > 3 else 0.0
            local = gate(kind, ang)
        U = embed(n, local, qubits) @ U
    return U


def pauli_matrix(n: int, x: int, z: int) -> np.ndarray:
    out = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        letter = "Y" if (xb and zb) else "X" if xb else "Z" if zb else "I"
        out = np.kron(out, LETTER[letter])
    return out


def hamiltonian_matrix(n: int, ham) -> np.ndarray:
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for x, z, a in zip(ham.x, ham.z, ham.coef):
        H += a * pauli_matrix(n, int(x), int(z))
    return H
