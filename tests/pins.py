"""Independent constructions used to pin the oracle (test-side only).

Nothing here is the oracle's own method: the expanded time-step unitary is
built with Kronecker products and a qubit-permutation matrix, the way
Sec. II-C writes it (I_above (x) Gate (x) I_below), rather than by the
oracle's index bit manipulation.
"""
from __future__ import annotations

import numpy as np


def controlled_local(m: np.ndarray, nc: int) -> np.ndarray:
    """Matrix on (targets as low bits, controls as high bits): m where all
    controls are 1, identity elsewhere."""
    d = m.shape[0]
    D = d << nc
    out = np.eye(D, dtype=complex)
    hi = ((1 << nc) - 1) * d
    out[hi:hi + d, hi:hi + d] = m
    return out


def perm_matrix(n: int, order) -> np.ndarray:
    """P with (P v)[new(i)] = v[i], where bit j of new(i) is bit order[j] of i
    and order lists all n qubits."""
    N = 1 << n
    P = np.zeros((N, N))
    for i in range(N):
        j = 0
        for pos, q in enumerate(order):
            j |= ((i >> q) & 1) << pos
        P[j, i] = 1.0
    return P


def kron_expand(m: np.ndarray, targets, controls, n: int) -> np.ndarray:
    """Full 2^n matrix of a (controlled) gate by brute force: permute the
    acted-on qubits to the low positions, take I (x) local, permute back."""
    targets, controls = list(targets), list(controls)
    local = controlled_local(np.asarray(m, dtype=complex), len(controls))
    acted = targets + controls
    rest = [q for q in range(n) if q not in acted]
    order = acted + rest
    P = perm_matrix(n, order)
    big = np.kron(np.eye(1 << len(rest)), local)
    return P.T @ big @ P


PAULI = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def pauli_dense(n: int, xmask: int, zmask: int) -> np.ndarray:
    """Dense Pauli string: Y where both bits are set, X or Z where one is;
    qubit q is the q-th factor from the right of the Kronecker product."""
    out = np.eye(1, dtype=complex)
    for q in range(n - 1, -1, -1):
        xb, zb = (xmask >> q) & 1, (zmask >> q) & 1
        p = "Y" if xb and zb else "X" if xb else "Z" if zb else "I"
        out = np.kron(out, PAULI[p])
    return out


def hamiltonian_dense(n: int, terms) -> np.ndarray:
    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for xm, zm, c in terms:
        H += c * pauli_dense(n, xm, zm)
    return H
