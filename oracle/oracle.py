"""Plain CPU oracle for the DiaQ hot path (arXiv:2405.01250).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It
shares no code with the HIP library (no gate table, no helper, no header)
and never calls it; the two meet only on the seeded inputs the tests hand
to both.

What each function follows
--------------------------
* ``gate_matrix`` -- the gate table (standard OpenQASM-2-style matrices; the
  paper itself defines none, so both sides implement the same written
  table independently).
* ``apply_gate`` / ``apply_circuit`` -- state-vector evolution (Sec. II-A):
  each gate is the time-step unitary I_above (x) Gate (x) I_below
  (Sec. II-C), applied by amplitude-index bit manipulation in C.
* ``gate_element`` / ``dense_matrix`` / ``dia_from_dense`` -- the expanded
  time-step matrix and its DiaQ form (Sec. IV): diagonal d holds
  A[t + max(0,-d), t + max(0,d)], which is exactly numpy's ``diagonal``.
* ``dia_spmv`` -- the DiaQ sparse matrix-vector product (the operation of
  Alg. 2), written from the format's definition (Sec. IV) as a row loop.
* ``pauli_apply`` / ``expect`` / ``energy`` -- <psi|H|phi> for a Pauli sum.
* ``param_shift_grad`` / ``fd_grad`` -- gradients of <H> by the two-term
  parameter-shift rule and by central differences.
* ``unitary_chain`` / ``density_chain`` / ``count_diagonals`` /
  ``count_nonzeros`` / ``trace_product`` -- matrix-level simulation
  (Sec. II-A): the circuit unitary as the running dense product of the
  time-step matrices, rho <- G rho G^dagger, and the diagonal count and
  non-zero count whose per-step curves Sec. III-A plots.

Precision: fp64 / complex128 everywhere.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "diaq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _c():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        lib.orc_apply_gate.argtypes = [P, ci, P, ci, P, ci, P]
        lib.orc_apply_gate.restype = None
        lib.orc_dia_spmv.argtypes = [i64, ci, P, P, P, P, P]
        lib.orc_dia_spmv.restype = None
        lib.orc_pauli_sum_apply.argtypes = [ci, ci, P, P, P, P, P]
        lib.orc_pauli_sum_apply.restype = None
        lib.orc_inner.argtypes = [i64, P, P, P]
        lib.orc_inner.restype = None
        lib.orc_set_threads.argtypes = [ci]
        lib.orc_set_threads.restype = None
        lib.orc_get_threads.argtypes = []
        lib.orc_get_threads.restype = ci
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the C oracle's parallel loops (results do not depend on it)."""
    _c().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_c().orc_get_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Gate table
# --------------------------------------------------------------------------

_NTARGETS = {"I": 1, "H": 1, "X": 1, "Y": 1, "Z": 1, "S": 1, "SDG": 1, "T": 1, "TDG": 1,
             "SX": 1, "RX": 1, "RY": 1, "RZ": 1, "P": 1, "U3": 1,
             "SWAP": 2, "RXX": 2, "RYY": 2, "RZZ": 2}


def gate_matrix(kind: str, params=(), matrix=None) -> np.ndarray:
    """Local matrix of a gate; multi-qubit rows are indexed with the first
    target as the least-significant bit."""
    p = list(params) + [0.0] * (3 - len(params))
    t = p[0]
    c, s = math.cos(t / 2), math.sin(t / 2)
    r2 = 1 / math.sqrt(2)
    if kind == "I":
        return np.eye(2, dtype=complex)
    if kind == "H":
        return np.array([[r2, r2], [r2, -r2]], dtype=complex)
    if kind == "X":
        return np.array([[0, 1], [1, 0]], dtype=complex)
    if kind == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=complex)
    if kind == "Z":
        return np.array([[1, 0], [0, -1]], dtype=complex)
    if kind == "S":
        return np.array([[1, 0], [0, 1j]], dtype=complex)
    if kind == "SDG":
        return np.array([[1, 0], [0, -1j]], dtype=complex)
    if kind == "T":
        return np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=complex)
    if kind == "TDG":
        return np.array([[1, 0], [0, np.exp(-1j * math.pi / 4)]], dtype=complex)
    if kind == "SX":
        return 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=complex)
    if kind == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=complex)
    if kind == "RY":
        return np.array([[c, -s], [s, c]], dtype=complex)
    if kind == "RZ":
        return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=complex)
    if kind == "P":
        return np.array([[1, 0], [0, np.exp(1j * t)]], dtype=complex)
    if kind == "U3":
        th, ph, la = p[0], p[1], p[2]
        cc, ss = math.cos(th / 2), math.sin(th / 2)
        return np.array([[cc, -np.exp(1j * la) * ss],
                         [np.exp(1j * ph) * ss, np.exp(1j * (ph + la)) * cc]], dtype=complex)
    if kind == "SWAP":
        m = np.zeros((4, 4), dtype=complex)
        m[0, 0] = m[3, 3] = 1
        m[1, 2] = m[2, 1] = 1
        return m
    if kind == "RXX":
        # cos(t/2) I - i sin(t/2) X(x)X ; X(x)X maps local r to r xor 3
        m = c * np.eye(4, dtype=complex)
        for r in range(4):
            m[r, r ^ 3] += -1j * s
        return m
    if kind == "RYY":
        # entry by entry: <r|Y(x)Y|q> = <r0|Y|q0> <r1|Y|q1>
        y = np.array([[0, -1j], [1j, 0]], dtype=complex)
        yy = np.zeros((4, 4), dtype=complex)
        for r in range(4):
            for q in range(4):
                yy[r, q] = y[r & 1, q & 1] * y[r >> 1, q >> 1]
        return c * np.eye(4, dtype=complex) - 1j * s * yy
    if kind == "RZZ":
        ph = [np.exp(-0.5j * t), np.exp(0.5j * t), np.exp(0.5j * t), np.exp(-0.5j * t)]
        return np.diag(np.array(ph, dtype=complex))
    if kind == "MATRIX":
        return np.array(matrix, dtype=complex)
    raise ValueError("unknown gate kind %r" % kind)


def generator_matrix(kind: str) -> np.ndarray:
    """G with U(a) = exp(-i a G / 2) for the rotation kinds."""
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
    Z = np.array([[1, 0], [0, -1]], dtype=complex)
    if kind == "RX":
        return X
    if kind == "RY":
        return Y
    if kind == "RZ":
        return Z
    if kind == "P":
        return np.diag([0, -2]).astype(complex)
    if kind in ("RXX", "RYY", "RZZ"):
        a = {"RXX": X, "RYY": Y, "RZZ": Z}[kind]
        # first target is the least-significant local bit: kron(second, first)
        return np.kron(a, a)
    raise ValueError("gate kind %r has no generator" % kind)


def _gate_fields(g):
    kind = g.kind
    targets = tuple(g.targets)
    controls = tuple(getattr(g, "controls", ()) or ())
    params = tuple(getattr(g, "params", ()) or ())
    matrix = getattr(g, "matrix", None)
    return kind, targets, controls, params, matrix


# --------------------------------------------------------------------------
# State evolution
# --------------------------------------------------------------------------

def apply_matrix(psi: np.ndarray, n: int, m: np.ndarray, targets, controls=()) -> None:
    """In place: psi <- (local matrix m on targets, controlled) psi."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 1 << n
    k = len(targets)
    m = np.ascontiguousarray(m, dtype=np.complex128)
    assert m.shape == (1 << k, 1 << k)
    t = np.array(targets, dtype=np.intc)
    cs = np.array(controls if controls else [0], dtype=np.intc)
    _c().orc_apply_gate(_ptr(psi), n, _ptr(m), k, _ptr(t), len(controls), _ptr(cs))


def apply_gate(psi: np.ndarray, n: int, g) -> None:
    kind, targets, controls, params, matrix = _gate_fields(g)
    apply_matrix(psi, n, gate_matrix(kind, params, matrix), targets, controls)


def apply_circuit(psi: np.ndarray, n: int, gates, copy: bool = True) -> np.ndarray:
    """Return U_G ... U_1 psi (state-vector simulation, Sec. II-A)."""
    out = np.array(psi, dtype=np.complex128, copy=True) if copy else psi
    for g in gates:
        apply_gate(out, n, g)
    return out


def basis_state(n: int, index: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[index] = 1.0
    return psi


# --------------------------------------------------------------------------
# Expanded matrices and the DiaQ format
# --------------------------------------------------------------------------

def dense_matrix(n: int, gates) -> np.ndarray:
    """The 2^n x 2^n matrix of a gate sequence: column j is U e_j."""
    N = 1 << n
    A = np.zeros((N, N), dtype=np.complex128)
    for j in range(N):
        A[:, j] = apply_circuit(basis_state(n, j), n, gates, copy=False)
    return A


def gate_element(n: int, g, i: int, j: int) -> complex:
    """A[i, j] of one expanded gate, from the gate applied to e_j.  Only the
    at most 8 amplitudes reachable from j are formed, so any n works."""
    kind, targets, controls, params, matrix = _gate_fields(g)
    m = gate_matrix(kind, params, matrix)
    if any(not (j >> c) & 1 for c in controls):
        return complex(1.0 if i == j else 0.0)
    tmask = 0
    for t in targets:
        tmask |= 1 << t
    if (i ^ j) & ~tmask:
        return 0j
    loc_i = sum(((i >> t) & 1) << r for r, t in enumerate(targets))
    loc_j = sum(((j >> t) & 1) << r for r, t in enumerate(targets))
    return complex(m[loc_i, loc_j])


def dia_from_dense(A: np.ndarray, keep_zero: bool = False):
    """DiaQ form of a dense matrix (Sec. IV): the sorted diagonal indices
    with a non-zero element, and for each the compact diagonal."""
    N = A.shape[0]
    offs, vals = [], []
    for d in range(-(N - 1), N):
        v = np.diagonal(A, d)
        if keep_zero or np.any(v != 0):
            offs.append(d)
            vals.append(np.array(v))
    return offs, vals


def pack_dia(offs, vals):
    """Pack compact diagonals: (offsets int64, starts int64, values)."""
    starts = np.zeros(len(offs) + 1, dtype=np.int64)
    for k, v in enumerate(vals):
        starts[k + 1] = starts[k] + len(v)
    packed = np.concatenate(vals) if vals else np.zeros(0, np.complex128)
    return np.array(offs, dtype=np.int64), starts, np.ascontiguousarray(packed, dtype=np.complex128)


def dia_spmv(N: int, offsets, starts, values, x) -> np.ndarray:
    """y = A x for a packed DiaQ matrix: y[i] = sum_k A[i, i+d_k] x[i+d_k]
    over the diagonals k with 0 <= i + d_k < N (Sec. IV's layout gives
    A[i, i+d] as element i - max(0,-d) of diagonal d)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    starts = np.ascontiguousarray(starts, dtype=np.int64)
    values = np.ascontiguousarray(values, dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.zeros(N, dtype=np.complex128)
    _c().orc_dia_spmv(N, len(offsets), _ptr(offsets), _ptr(starts), _ptr(values), _ptr(x), _ptr(y))
    return y


# --------------------------------------------------------------------------
# Observables and gradients
# --------------------------------------------------------------------------

def _terms_arrays(terms):
    xs = np.array([t[0] for t in terms], dtype=np.uint64)
    zs = np.array([t[1] for t in terms], dtype=np.uint64)
    cs = np.array([t[2] for t in terms], dtype=np.float64)
    return xs, zs, cs


def pauli_apply(n: int, terms, phi: np.ndarray) -> np.ndarray:
    """H phi for H = sum coef * i^{|x&z|} X^x Z^z; terms = [(x, z, coef)]."""
    xs, zs, cs = _terms_arrays(terms)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    out = np.empty_like(phi)
    _c().orc_pauli_sum_apply(n, len(terms), _ptr(xs), _ptr(zs), _ptr(cs), _ptr(phi), _ptr(out))
    return out


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    out = np.zeros(2)
    _c().orc_inner(a.size, _ptr(a), _ptr(b), _ptr(out))
    return complex(out[0], out[1])


def expect(n: int, terms, psi: np.ndarray, phi: np.ndarray | None = None) -> complex:
    """<psi|H|phi> (phi defaults to psi)."""
    if phi is None:
        phi = psi
    return inner(psi, pauli_apply(n, terms, phi))


def energy(psi0: np.ndarray, n: int, gates, terms) -> float:
    psi = apply_circuit(psi0, n, gates)
    return expect(n, terms, psi).real


def _with_angle(g, delta: float):
    """Copy of gate g with params[0] shifted by delta."""
    import copy as _copy
    h = _copy.copy(g)
    p = list(g.params)
    p[0] = p[0] + delta
    h.params = tuple(p)
    return h


def param_shift_grad(psi0: np.ndarray, n: int, gates, terms, nparams: int) -> np.ndarray:
    """dE/dtheta by the two-term shift rule, one occurrence at a time:
    dE/da = (E(a + pi/2) - E(a - pi/2)) / 2 for U = exp(-i a G/2) whose G/2
    has two eigenvalues one apart (Paulis, and P's diag(0,-2)), times the
    occurrence's chain factor, summed over occurrences of a parameter."""
    grad = np.zeros(nparams)
    gates = list(gates)
    for idx, g in enumerate(gates):
        if getattr(g, "param_index", -1) < 0:
            continue
        if getattr(g, "controls", ()) and g.kind != "P":
            # a controlled Pauli rotation has frequencies 1/2 and 1
            raise ValueError("two-term shift rule does not hold for a controlled rotation")
        plus = gates[:idx] + [_with_angle(g, math.pi / 2)] + gates[idx + 1:]
        minus = gates[:idx] + [_with_angle(g, -math.pi / 2)] + gates[idx + 1:]
        d = 0.5 * (energy(psi0, n, plus, terms) - energy(psi0, n, minus, terms))
        grad[g.param_index] += g.param_scale * d
    return grad


def fd_grad(psi0: np.ndarray, n: int, gates, terms, nparams: int, h: float = 1e-3,
            theta=None, rebuild=None) -> np.ndarray:
    """Central differences (E(theta + h e_j) - E(theta - h e_j)) / 2h.

    With ``theta`` and ``rebuild(theta) -> gates`` the parameter vector is
    perturbed and the circuit rebuilt (shared angles move together);
    otherwise each occurrence is shifted by h * param_scale."""
    grad = np.zeros(nparams)
    if rebuild is not None:
        theta = np.asarray(theta, dtype=np.float64)
        for j in range(nparams):
            tp = theta.copy()
            tp[j] += h
            tm = theta.copy()
            tm[j] -= h
            grad[j] = (energy(psi0, n, rebuild(tp), terms) - energy(psi0, n, rebuild(tm), terms)) / (2 * h)
        return grad
    gates = list(gates)
    for j in range(nparams):
        plus, minus = [], []
        for g in gates:
            if getattr(g, "param_index", -1) == j:
                plus.append(_with_angle(g, h * g.param_scale))
                minus.append(_with_angle(g, -h * g.param_scale))
            else:
                plus.append(g)
                minus.append(g)
        grad[j] = (energy(psi0, n, plus, terms) - energy(psi0, n, minus, terms)) / (2 * h)
    return grad


# --------------------------------------------------------------------------
# Matrix-level simulation (Sec. II-A; the Sec. III-A sparsity curves)
# --------------------------------------------------------------------------

def count_nonzeros(A: np.ndarray, tol: float = 0.0) -> int:
    """Elements with |a| > tol (a != 0 when tol = 0)."""
    return int(np.count_nonzero(np.abs(A) > tol)) if tol > 0 else int(np.count_nonzero(A))


def count_diagonals(A: np.ndarray, tol: float = 0.0) -> int:
    """Diagonals (dIndex = col - row) holding an element counted by
    count_nonzeros."""
    N = A.shape[0]
    keep = (np.abs(A) > tol) if tol > 0 else (A != 0)
    r, c = np.nonzero(keep)
    return int(np.unique(c - r).size) if r.size else 0


def unitary_chain(n: int, gates, tol: float = 0.0, start: np.ndarray | None = None):
    """U_t = G_t U_{t-1} from U_0 = start (identity by default), G_t the
    dense expanded time-step matrix of gate t.  Returns (U, records) with
    records[t] = (diagonals, non-zeros) of U_t."""
    U = np.eye(1 << n, dtype=np.complex128) if start is None else np.array(start, dtype=np.complex128)
    rec = []
    for g in gates:
        U = dense_matrix(n, [g]) @ U
        rec.append((count_diagonals(U, tol), count_nonzeros(U, tol)))
    return U, rec


def density_chain(rho: np.ndarray, n: int, gates, tol: float = 0.0):
    """rho_t = G_t rho_{t-1} G_t^dagger, dense; returns (rho, records)."""
    R = np.array(rho, dtype=np.complex128)
    rec = []
    for g in gates:
        G = dense_matrix(n, [g])
        R = G @ R @ G.conj().T
        rec.append((count_diagonals(R, tol), count_nonzeros(R, tol)))
    return R, rec


def trace_product(A: np.ndarray, B: np.ndarray) -> complex:
    """Tr(A B)."""
    return complex(np.trace(A @ B))
