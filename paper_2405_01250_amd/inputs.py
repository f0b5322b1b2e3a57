"""Seeded synthetic inputs: gate lists, states and observables.

This module holds data only -- which gates, on which qubits, with which
angles, in which order, and seeded random numbers.  It contains none of the
method's arithmetic (no gate matrices, no expansion, no products), so the
oracle and the HIP library can both be fed from it.

The workloads stand in for the paper's SupermarQ and QASMBench circuits
(Sec. II-B), which are not reproduced here:

* ``ghz``            -- the GHZ ladder (H, then a CNOT chain).
* ``qft``            -- the textbook quantum Fourier transform.
* ``random_layered`` -- U3 on every qubit plus alternating CX brickwork.
* ``hea``            -- hardware-efficient ansatz (RY, RZ, CZ ring) with a
                        ZZ + X observable, for gradients.
* ``qaoa_batch``     -- MaxCut QAOA on random 3-regular graphs.
* ``tfim``           -- Trotterised 1D transverse-field Ising model, the
                        shape of the paper's HAM benchmark.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Gate:
    """One gate: kind name, target and control qubits, angles.

    ``targets[0]`` is the least-significant local bit of a multi-qubit gate.
    ``param_index >= 0`` marks a differentiable rotation whose angle is
    ``param_scale * theta[param_index]``."""
    kind: str
    targets: tuple
    controls: tuple = ()
    params: tuple = ()
    param_index: int = -1
    param_scale: float = 1.0
    matrix: object = None


def h(q):
    return Gate("H", (q,))


def x(q):
    return Gate("X", (q,))


def cx(c, t):
    return Gate("X", (t,), (c,))


def cz(a, b):
    return Gate("Z", (b,), (a,))


def cp(lam, a, b):
    return Gate("P", (b,), (a,), (lam,))


def swap(a, b):
    return Gate("SWAP", (a, b))


def u3(theta, phi, lam, q):
    return Gate("U3", (q,), (), (theta, phi, lam))


# --------------------------------------------------------------------------
# States
# --------------------------------------------------------------------------

def random_state(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Real parts then imaginary parts i.i.d. N(0,1) from
    ``default_rng(seed)``, normalised to unit 2-norm."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    psi = np.empty(N, dtype=np.complex128)
    psi.real = rng.standard_normal(N)
    psi.imag = rng.standard_normal(N)
    psi /= np.linalg.norm(psi)
    return psi.astype(dtype)


def zero_state(n: int, dtype=np.complex128) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=dtype)
    psi[0] = 1.0
    return psi


# --------------------------------------------------------------------------
# Circuits
# --------------------------------------------------------------------------

def ghz(n: int):
    """H on qubit 0, then CX(0 -> k) for k = 1..n-1."""
    return [h(0)] + [cx(0, k) for k in range(1, n)]


def qft(n: int):
    """For q = n-1 .. 0: H(q), then CP(pi / 2^m) on (q - m, q) for
    m = 1..q; finally SWAP(q, n-1-q) for q < n/2."""
    gates = []
    for q in range(n - 1, -1, -1):
        gates.append(h(q))
        for m in range(1, q + 1):
            gates.append(cp(math.pi / (1 << m), q - m, q))
    for q in range(n // 2):
        gates.append(swap(q, n - 1 - q))
    return gates


def random_layered(n: int, layers: int, seed: int):
    """Layer l: U3(theta, phi, lambda) on q = 0..n-1, angles drawn per qubit
    in that order from U[0, 2pi); then CX(2i -> 2i+1) for even l and
    CX(2i+1 -> 2i+2) for odd l."""
    rng = np.random.default_rng(seed)
    gates = []
    for layer in range(layers):
        ang = rng.uniform(0.0, TWO_PI, size=(n, 3))
        for q in range(n):
            gates.append(u3(float(ang[q, 0]), float(ang[q, 1]), float(ang[q, 2]), q))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            gates.append(cx(a, a + 1))
    return gates


def hea(n: int, layers: int, seed: int, ring: bool = True):
    """Hardware-efficient ansatz.  Each layer: RY on every qubit, RZ on every
    qubit, then (if ``ring``) CZ(q, q+1 mod n) for every q.  Parameters are
    layer-major [RY q0..q(n-1), RZ q0..q(n-1)], drawn U[0, 2pi).

    The observable H = sum_i a_i Z_i Z_{i+1} (i < n-1) + sum_i b_i X_i with
    a then b drawn N(0,1) from the same generator.

    Returns (gates, theta, terms) with terms = [(xmask, zmask, coef)]."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, TWO_PI, size=2 * n * layers)
    a = rng.standard_normal(n - 1)
    b = rng.standard_normal(n)
    gates = hea_gates(n, layers, theta, ring)
    terms = [(0, (1 << i) | (1 << (i + 1)), float(a[i])) for i in range(n - 1)]
    terms += [(1 << i, 0, float(b[i])) for i in range(n)]
    return gates, theta, terms


def hea_gates(n: int, layers: int, theta, ring: bool = True):
    gates = []
    for layer in range(layers):
        base = 2 * n * layer
        for q in range(n):
            gates.append(Gate("RY", (q,), (), (float(theta[base + q]),), base + q, 1.0))
        for q in range(n):
            gates.append(Gate("RZ", (q,), (), (float(theta[base + n + q]),), base + n + q, 1.0))
        if ring:
            for q in range(n):
                gates.append(cz(q, (q + 1) % n))
    return gates


def random_regular3(n: int, rng) -> list:
    """Random simple 3-regular graph on n (even) vertices: configuration
    model pairing of 3n stubs, redrawn until there is no loop or repeated
    edge.  Returns sorted edge tuples (u < v)."""
    if n % 2:
        raise ValueError("a 3-regular graph needs an even vertex count")
    while True:
        stubs = np.repeat(np.arange(n), 3)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        edges = set()
        ok = True
        for u, v in pairs:
            u, v = int(u), int(v)
            if u == v:
                ok = False
                break
            e = (min(u, v), max(u, v))
            if e in edges:
                ok = False
                break
            edges.add(e)
        if ok:
            return sorted(edges)


def qaoa_gates(n: int, edges, gammas, betas):
    """H on all qubits; per layer l: RZZ(2 gamma_l) on every edge (gradient
    slot 2l, chain factor 2), then RX(2 beta_l) on every qubit (slot 2l+1,
    chain factor 2)."""
    gates = [h(q) for q in range(n)]
    for layer, (g, b) in enumerate(zip(gammas, betas)):
        for (u, v) in edges:
            gates.append(Gate("RZZ", (u, v), (), (2.0 * float(g),), 2 * layer, 2.0))
        for q in range(n):
            gates.append(Gate("RX", (q,), (), (2.0 * float(b),), 2 * layer + 1, 2.0))
    return gates


def maxcut_terms(edges):
    """C = sum_{(u,v)} (1 - Z_u Z_v) / 2 as Pauli terms (identity included)."""
    terms = [(0, 0, 0.5 * len(edges))]
    terms += [(0, (1 << u) | (1 << v), -0.5) for (u, v) in edges]
    return terms


@dataclass
class QaoaInstance:
    n: int
    edges: list
    p: int
    gammas: np.ndarray
    betas: np.ndarray
    gates: list = field(default_factory=list)
    terms: list = field(default_factory=list)


def qaoa_batch(count: int = 512, seed: int = 512, widths=(10, 12, 14, 16, 18, 20, 22),
               pmax: int = 4):
    """``count`` MaxCut QAOA instances: width uniform over ``widths``, a
    random 3-regular graph, depth p uniform in 1..pmax, angles gamma and
    beta uniform in [0, pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(widths))
        edges = random_regular3(n, rng)
        p = int(rng.integers(1, pmax + 1))
        gammas = rng.uniform(0.0, math.pi, size=p)
        betas = rng.uniform(0.0, math.pi, size=p)
        inst = QaoaInstance(n, edges, p, gammas, betas)
        inst.gates = qaoa_gates(n, edges, gammas, betas)
        inst.terms = maxcut_terms(edges)
        out.append(inst)
    return out


def tfim(n: int, steps: int, dt: float = 0.1, J: float = 1.0, hx: float = 1.0):
    """First-order Trotter steps of the open-chain transverse-field Ising
    model H = -J sum Z_i Z_{i+1} - hx sum X_i: each step RZZ(-2 J dt) on
    (i, i+1), then RX(-2 hx dt) on every qubit, so that one step is
    exp(i J dt sum ZZ) followed by exp(i hx dt sum X)."""
    gates = []
    for _ in range(steps):
        for i in range(n - 1):
            gates.append(Gate("RZZ", (i, i + 1), (), (-2.0 * J * dt,)))
        for q in range(n):
            gates.append(Gate("RX", (q,), (), (-2.0 * hx * dt,)))
    return gates


def tfim_terms(n: int, J: float = 1.0, hx: float = 1.0):
    """The same Hamiltonian as Pauli terms [(xmask, zmask, coef)]."""
    return ([(0, (1 << i) | (1 << (i + 1)), -J) for i in range(n - 1)]
            + [(1 << q, 0, -hx) for q in range(n)])


def magnetization_terms(n: int):
    """Average magnetization (1/n) sum Z_i, the observable of the
    Hamiltonian-simulation benchmark."""
    return [(0, 1 << q, 1.0 / n) for q in range(n)]


# The TFIM workload the benchmark times: 28 spins at the critical field
# (J = hx = 1), 20 Trotter steps of dt = 0.05 from |0..0> (1100 gates).
TFIM_N, TFIM_STEPS, TFIM_DT = 28, 20, 0.05
