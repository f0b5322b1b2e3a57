"""Pins of the CPU oracle against facts fixed outside it: the paper's worked
examples, closed forms, brute-force Kronecker products, textbook gate
identities and invariants.  CPU only."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
import scipy.linalg

from paper_2405_01250_amd import inputs as W
from tests import pins

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    lines = [l.strip() for l in open(os.path.join(GOLD, name)) if l.strip() and not l.startswith("#")]
    mi = lines.index("matrix")
    di = lines.index("diaq")
    mat = [row.split() for row in lines[mi + 1:di]]
    dia = {}
    for row in lines[di + 1:]:
        f = row.split()
        dia[int(f[0])] = f[1:]
    return mat, dia


def _symbolic(mat):
    """Map each letter to a distinct prime-ish complex value, 0 to 0."""
    letters = sorted({c for row in mat for c in row if c != "0"})
    val = {c: complex(k + 2, 0.5 * (k + 1)) for k, c in enumerate(letters)}
    A = np.array([[0 if c == "0" else val[c] for c in row] for row in mat], dtype=complex)
    inv = {v: c for c, v in val.items()}
    return A, inv


# --------------------------------------------------------------------------
# Sec. III-B / Sec. IV worked examples: the DiaQ layout
# --------------------------------------------------------------------------

@pytest.mark.parametrize("fixture", ["paper_dia_example.txt", "paper_gate_application_example.txt"])
def test_dia_worked_examples(orc, fixture):
    mat, dia = _read_golden(fixture)
    A, inv = _symbolic(mat)
    offs, vals = orc.dia_from_dense(A)
    got = {d: [inv[complex(v)] for v in vs] for d, vs in zip(offs, vals)}
    assert got == dia
    # The SpMV of Alg. 2 on that DiaQ matrix equals the dense product.
    o, s, v = orc.pack_dia(offs, vals)
    x = np.arange(1, 5) + 1j * np.arange(4, 0, -1)
    assert np.allclose(orc.dia_spmv(4, o, s, v, x), A @ x, rtol=0, atol=1e-13)


def test_scipy_offsets_of_example(orc):
    # Sec. III-B lists offsets [0, -3, 3] for the same matrix.
    mat, _ = _read_golden("paper_dia_example.txt")
    A, _ = _symbolic(mat)
    offs, _ = orc.dia_from_dense(A)
    assert sorted(offs) == sorted([0, -3, 3])


def test_hadamard_patterns_fig2(orc):
    """Fig. 2: H at each of four positions, built with numpy's Kronecker
    product exactly as the caption writes it, has diagonals 0, +-dim_b; the
    oracle's bit-manipulation expansion of H on qubit log2(dim_b) agrees."""
    rows = [l.split() for l in open(os.path.join(GOLD, "paper_hadamard_patterns.txt"))
            if l.strip() and not l.startswith("#")]
    Hm = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    for name, *offs in rows:
        expect = [int(o) for o in offs]
        dim_b = expect[-1]
        dim_a = 16 // (2 * dim_b)
        A = np.kron(np.kron(np.eye(dim_a), Hm), np.eye(dim_b))
        got, _ = orc.dia_from_dense(A)
        assert got == expect, name
        q = int(math.log2(dim_b))
        B = orc.dense_matrix(4, [W.h(q)])
        assert np.array_equal(A, B), name


def test_phase_gates_principal_diagonal_only(orc):
    # Sec. III-A: a Z (phase) gate's time-step unitary is the principal diagonal.
    for g in [W.Gate("Z", (2,)), W.Gate("S", (1,)), W.Gate("T", (3,)), W.Gate("RZ", (0,), (), (0.7,)),
              W.cz(1, 3), W.cp(0.3, 0, 2), W.Gate("RZZ", (1, 2), (), (1.1,))]:
        offs, _ = orc.dia_from_dense(orc.dense_matrix(4, [g]))
        assert offs == [0]


def test_transpose_is_relabelling(orc):
    # Sec. IV: transpose negates the diagonal indices; compact diagonals unchanged.
    rng = np.random.default_rng(1)
    A = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    A[np.abs(np.subtract.outer(np.arange(16), np.arange(16))) % 4 != 0] = 0
    oa, va = orc.dia_from_dense(A)
    ot, vt = orc.dia_from_dense(A.T)
    assert ot == sorted(-d for d in oa)
    for d, v in zip(oa, va):
        assert np.array_equal(vt[ot.index(-d)], v)


# --------------------------------------------------------------------------
# Gate table against textbook identities (matrix exponentials, Euler angles)
# --------------------------------------------------------------------------

def test_gate_table_identities(orc):
    G = orc.gate_matrix
    I2 = np.eye(2)
    X, Y, Z = pins.PAULI["X"], pins.PAULI["Y"], pins.PAULI["Z"]
    close = lambda a, b: np.allclose(a, b, rtol=0, atol=1e-14)
    assert close(G("H") @ G("H"), I2)
    assert close(G("S") @ G("S"), Z)
    assert close(G("T") @ G("T"), G("S"))
    assert close(G("SDG"), G("S").conj().T)
    assert close(G("TDG"), G("T").conj().T)
    assert close(G("SX") @ G("SX"), X)
    assert close(G("X"), X) and close(G("Y"), Y) and close(G("Z"), Z)
    assert close(G("H"), (X + Z) / math.sqrt(2))
    for t in [0.0, 0.3, 1.7, math.pi, 4.4, -2.2]:
        assert close(G("RX", (t,)), scipy.linalg.expm(-0.5j * t * X))
        assert close(G("RY", (t,)), scipy.linalg.expm(-0.5j * t * Y))
        assert close(G("RZ", (t,)), scipy.linalg.expm(-0.5j * t * Z))
        assert close(G("P", (t,)), np.diag([1, np.exp(1j * t)]))
        for kind, P in [("RXX", X), ("RYY", Y), ("RZZ", Z)]:
            assert close(G(kind, (t,)), scipy.linalg.expm(-0.5j * t * np.kron(P, P)))
        assert close(G("U3", (t, -math.pi / 2, math.pi / 2)), G("RX", (t,)))
        assert close(G("U3", (t, 0, 0)), G("RY", (t,)))
        assert close(G("U3", (0, 0, t)), G("P", (t,)))
        for ph, la in [(0.4, 1.3), (2.9, -0.8)]:
            euler = np.exp(0.5j * (ph + la)) * G("RZ", (ph,)) @ G("RY", (t,)) @ G("RZ", (la,))
            assert close(G("U3", (t, ph, la)), euler)
    # generators: U(a) = exp(-i a G / 2)
    for kind in ["RX", "RY", "RZ", "P", "RXX", "RYY", "RZZ"]:
        a = 0.77
        assert close(G(kind, (a,)), scipy.linalg.expm(-0.5j * a * orc.generator_matrix(kind)))
    # SWAP exchanges the two qubits: SWAP (u (x) v) = v (x) u
    u = np.array([0.3, 0.4j + 0.1])
    v = np.array([0.6, -0.2 + 0.5j])
    assert close(G("SWAP") @ np.kron(v, u), np.kron(u, v))


# --------------------------------------------------------------------------
# Bit-manipulation evolution against brute-force Kronecker expansion
# --------------------------------------------------------------------------

_KINDS1 = ["H", "X", "Y", "Z", "S", "T", "SX", "RX", "RY", "RZ", "P", "U3"]
_KINDS2 = ["SWAP", "RXX", "RYY", "RZZ"]


def _random_gate(rng, n):
    r = rng.random()
    qs = list(rng.permutation(n))
    params = tuple(float(v) for v in rng.uniform(0, 2 * math.pi, 3))
    if r < 0.45:
        kind = _KINDS1[rng.integers(len(_KINDS1))]
        targets = (qs[0],)
    elif r < 0.75:
        kind = _KINDS2[rng.integers(len(_KINDS2))]
        targets = (qs[0], qs[1])
    else:
        kind = "MATRIX"
        k = int(rng.integers(1, 4))
        k = min(k, n - 1)
        m = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        q, _ = np.linalg.qr(m)
        return W.Gate("MATRIX", tuple(int(t) for t in qs[:k]),
                      tuple(int(c) for c in qs[k:k + int(rng.integers(0, min(3, n - k) + 1))]),
                      matrix=q)
    nt = len(targets)
    nc = int(rng.integers(0, min(3, n - nt) + 1))
    return W.Gate(kind, tuple(int(t) for t in targets), tuple(int(c) for c in qs[nt:nt + nc]), params)


@pytest.mark.parametrize("seed", range(12))
def test_apply_gate_matches_kronecker(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 8))
    psi = W.random_state(n, seed)
    for _ in range(6):
        g = _random_gate(rng, n)
        m = orc.gate_matrix(g.kind, g.params, g.matrix)
        full = pins.kron_expand(m, g.targets, g.controls, n)
        want = full @ psi
        orc.apply_gate(psi, n, g)
        assert np.allclose(psi, want, rtol=0, atol=1e-13)


def test_dense_matrix_and_gate_element_match_kronecker(orc):
    rng = np.random.default_rng(7)
    n = 5
    for _ in range(10):
        g = _random_gate(rng, n)
        m = orc.gate_matrix(g.kind, g.params, g.matrix)
        full = pins.kron_expand(m, g.targets, g.controls, n)
        assert np.allclose(orc.dense_matrix(n, [g]), full, rtol=0, atol=1e-14)
        for _ in range(40):
            i, j = (int(v) for v in rng.integers(0, 1 << n, 2))
            assert abs(orc.gate_element(n, g, i, j) - full[i, j]) < 1e-14
        # diagonal entries of the DiaQ form
        offs, vals = orc.dia_from_dense(full)
        for d, v in zip(offs, vals):
            for t in range(len(v)):
                assert abs(orc.gate_element(n, g, t + max(0, -d), t + max(0, d)) - v[t]) < 1e-14


def test_kronecker_offsets_scale_with_dim_b(orc):
    # Alg. 3: I_a (x) M (x) I_b occupies the diagonals dim_b * dIndex(M).
    rng = np.random.default_rng(3)
    M = rng.standard_normal((4, 4)) + 0j
    M[0, 2] = M[2, 0] = M[1, 3] = M[3, 1] = 0
    om, _ = orc.dia_from_dense(M)
    for dim_b in [1, 2, 4, 8]:
        A = np.kron(np.kron(np.eye(64 // (4 * dim_b)), M), np.eye(dim_b))
        oa, _ = orc.dia_from_dense(A)
        assert oa == [dim_b * d for d in om]


# --------------------------------------------------------------------------
# Closed forms and invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 5, 8, 12, 16])
def test_ghz_closed_form(orc, n):
    psi = orc.apply_circuit(W.zero_state(n), n, W.ghz(n))
    want = np.zeros(1 << n, dtype=complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) <= 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 13])
def test_qft_closed_form(orc, n):
    # QFT_{jk} = e^{2 pi i jk / N} / sqrt(N), i.e. numpy's ortho inverse FFT.
    x = W.random_state(n, 50 + n)
    got = orc.apply_circuit(x, n, W.qft(n))
    assert np.max(np.abs(got - np.fft.ifft(x, norm="ortho"))) <= 1e-13
    # basis states: uniform magnitude, phases e^{2 pi i j k / N}
    N = 1 << n
    for j in [0, 1, N - 1, N // 3]:
        out = orc.apply_circuit(orc.basis_state(n, j), n, W.qft(n))
        k = np.arange(N)
        assert np.max(np.abs(out - np.exp(2j * math.pi * j * k / N) / math.sqrt(N))) <= 1e-13


def test_qft_gate_count():
    g = W.qft(24)
    assert sum(1 for x in g if x.kind == "H") == 24
    assert sum(1 for x in g if x.kind == "P") == 276
    assert sum(1 for x in g if x.kind == "SWAP") == 12
    assert len(W.qft(29)) == 449


def test_random_layered_gate_count():
    g = W.random_layered(28, 20, 28)
    assert len(g) == 830
    assert sum(1 for x in g if x.kind == "U3") == 560


def test_norm_preserved_after_every_gate(orc):
    n = 10
    psi = W.random_state(n, 5)
    for g in W.random_layered(n, 3, 9) + W.qft(n) + W.hea(n, 2, 4)[0]:
        orc.apply_gate(psi, n, g)
        assert abs(np.linalg.norm(psi) - 1) <= 1e-13


# --------------------------------------------------------------------------
# The DiaQ SpMV (the product Alg. 2 computes) on random and expanded matrices
# --------------------------------------------------------------------------

def test_dia_spmv_matches_dense_product(orc):
    rng = np.random.default_rng(11)
    N = 64
    for nd in [1, 3, 7, 20]:
        offs = sorted(rng.choice(np.arange(-(N - 1), N), nd, replace=False).tolist())
        A = np.zeros((N, N), dtype=complex)
        for d in offs:
            L = N - abs(d)
            idx = np.arange(L)
            A[idx + max(0, -d), idx + max(0, d)] = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        o, v = orc.dia_from_dense(A, keep_zero=True)
        o, s, v = orc.pack_dia([d for d in o if d in offs], [v[o.index(d)] for d in offs])
        x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        assert np.allclose(orc.dia_spmv(N, o, s, v, x), A @ x, rtol=0, atol=1e-12)


def test_dia_spmv_propagates_non_finite_x(orc):
    """Every stored element of a row multiplies its x entry, zero-valued
    ones included (IEEE: 0 * Inf = NaN); entries that are not stored do
    not take part.  Brute force on a 6 x 6 matrix with an explicit zero
    diagonal: rows whose stored elements reach the Inf column are NaN, the
    others equal the finite dense product."""
    N = 6
    offs = [-2, 0, 3]
    rng = np.random.default_rng(5)
    vals = [np.zeros(N - 2, complex), rng.standard_normal(N) + 1j * rng.standard_normal(N),
            rng.standard_normal(N - 3) + 1j * rng.standard_normal(N - 3)]
    o, s, v = orc.pack_dia(offs, vals)
    for bad in (np.inf, np.nan):
        for col in range(N):
            x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
            x[col] = bad
            y = orc.dia_spmv(N, o, s, v, x)
            for i in range(N):
                cols = [i + d for d in offs if 0 <= i + d < N]
                if col in cols:
                    assert not np.isfinite(y[i]), (bad, col, i)
                else:
                    want = 0j
                    for d, vv in zip(offs, vals):
                        if 0 <= i + d < N:
                            want += vv[i - max(0, -d)] * x[i + d]
                    assert y[i] == want, (bad, col, i)


def test_ghz12_by_dia_spmv(orc):
    """The GHZ-12 workload run by the oracle's DiaQ SpMV on each gate's
    DiaQ expansion reaches the closed form."""
    n = 12
    N = 1 << n
    psi = W.zero_state(n)
    for g in W.ghz(n):
        # DiaQ expansion from single elements of the time-step matrix; H and
        # CX on target q occupy the diagonals 0, +-2^q
        q = g.targets[0]
        offs = [-(1 << q), 0, 1 << q]
        vals = []
        for d in offs:
            L = N - abs(d)
            vals.append(np.array([orc.gate_element(n, g, t + max(0, -d), t + max(0, d)) for t in range(L)]))
        o, s, v = orc.pack_dia(offs, vals)
        psi = orc.dia_spmv(N, o, s, v, psi)
    want = np.zeros(N, dtype=complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) <= 1e-15


# --------------------------------------------------------------------------
# Products of DiaQ matrices (Alg. 1 semantics by dense products)
# --------------------------------------------------------------------------

def test_fused_ghz10_sparsity(orc):
    # Sec. III-A: the GHZ(10) unitary stays >= 99.8 % sparse.
    n = 10
    U = orc.dense_matrix(n, W.ghz(n))
    nnz = int(np.count_nonzero(U))
    assert nnz == 2048
    assert 1 - nnz / U.size >= 0.998
    offs, _ = orc.dia_from_dense(U)
    assert len(offs) == 1025


def test_hh_is_identity(orc):
    U = orc.dense_matrix(6, [W.h(3), W.h(3)])
    offs, vals = orc.dia_from_dense(U)
    assert offs == [0]
    assert np.allclose(vals[0], 1, rtol=0, atol=1e-15)


def test_fused_group_diagonal_counts(orc):
    """Sec. VI, gate fusion: H followed by its controlled-phase ladder keeps
    the three diagonals of H (the phases are diagonal); two adjacent U3 and
    a CX on the same pair of qubits span the offsets -3..3."""
    n = 5
    ladder = [W.h(4)] + [W.cp(math.pi / 2 ** m, 4 - m, 4) for m in range(1, 5)]
    offs, _ = orc.dia_from_dense(orc.dense_matrix(n, ladder))
    assert offs == [-16, 0, 16]
    for cx in (W.cx(0, 1), W.cx(1, 0)):
        offs, _ = orc.dia_from_dense(orc.dense_matrix(n, [W.u3(0.3, 0.4, 0.5, 0), W.u3(0.6, 0.7, 0.8, 1), cx]))
        assert offs == [-3, -2, -1, 0, 1, 2, 3]


# --------------------------------------------------------------------------
# Matrix-level simulation: unitary chains and density matrices (Sec. II-A)
# --------------------------------------------------------------------------

def ghz_unitary(n):
    """Closed form of the GHZ circuit's unitary: H on qubit 0 sends |j> to
    (|j with bit 0 cleared> +- |j with bit 0 set>)/sqrt 2, and the CX ladder
    then flips bits 1..n-1 of the second term."""
    N = 1 << n
    j = np.arange(N)
    s = 1 / math.sqrt(2)
    U = np.zeros((N, N), dtype=complex)
    U[j & ~1, j] = s
    U[(j | 1) ^ (N - 2), j] += np.where(j & 1, -s, s)
    return U


def test_unitary_chain_ghz10_stays_sparse(orc):
    """Sec. III-A: the GHZ(10) unitary simulation stays at least 99.8 %
    sparse at every time step; the final unitary is the closed form, 2048
    non-zeros on 1025 diagonals."""
    n = 10
    U, rec = orc.unitary_chain(n, W.ghz(n))
    assert np.max(np.abs(U - ghz_unitary(n))) < 1e-15
    for nd, nnz in rec:
        assert nnz == 2048 and 1 - nnz / 4 ** n >= 0.998
    assert rec[-1] == (1025, 2048)


def test_unitary_chain_order_and_counts(orc):
    """Each new time step multiplies on the left (checked against products
    of Kronecker-built matrices), and the counts follow closed forms: H on
    every qubit is dense (4^n non-zeros on 2^(n+1) - 1 diagonals), X on every
    qubit the anti-identity (2^n non-zeros on 2^n diagonals)."""
    rng = np.random.default_rng(31)
    n = 4
    gates = [W.u3(*rng.uniform(0, 6, 3), 1), W.cx(0, 2), W.Gate("RY", (3,), (0,), (0.7,)), W.swap(1, 3), W.h(2)]
    want = np.eye(1 << n, dtype=complex)
    for g in gates:
        want = pins.kron_expand(orc.gate_matrix(g.kind, g.params), g.targets, g.controls, n) @ want
    U, _ = orc.unitary_chain(n, gates)
    assert np.max(np.abs(U - want)) < 1e-14
    n = 5
    _, rec = orc.unitary_chain(n, [W.h(q) for q in range(n)])
    assert rec[-1] == (2 ** (n + 1) - 1, 4 ** n)
    _, rec = orc.unitary_chain(n, [W.Gate("X", (q,)) for q in range(n)])
    assert rec[-1] == (2 ** n, 2 ** n)


def test_density_chain_pure_and_mixed(orc):
    """rho = |psi><psi| evolves into |U psi><U psi| (U psi from the
    bit-manipulation state path); the maximally mixed state is invariant;
    trace, Hermiticity and purity are kept, and Tr(H rho) is <U psi|H|U psi>."""
    n = 5
    gates = W.random_layered(n, 2, 7) + W.tfim(n, 2, 0.2)
    psi = W.random_state(n, 3)
    R, rec = orc.density_chain(np.outer(psi, psi.conj()), n, gates)
    phi = orc.apply_circuit(psi, n, gates)
    assert np.max(np.abs(R - np.outer(phi, phi.conj()))) < 1e-14
    assert abs(np.trace(R) - 1) < 1e-14 and np.max(np.abs(R - R.conj().T)) < 1e-15
    assert rec[-1] == (2 ** (n + 1) - 1, 4 ** n)
    N = 1 << n
    M, _ = orc.density_chain(np.eye(N) / N, n, gates)
    assert np.max(np.abs(M - np.eye(N) / N)) < 1e-15
    terms = W.tfim_terms(n)
    H = pins.hamiltonian_dense(n, terms)
    assert abs(orc.trace_product(H, R) - orc.expect(n, terms, phi)) < 1e-13
    assert abs(orc.trace_product(R, R) - 1) < 1e-13


# --------------------------------------------------------------------------
# Observables
# --------------------------------------------------------------------------

def test_inner_product_is_compensated(orc):
    """<a|a> for a = (1, 2^-30, ..., 2^-30) with 2^20 small entries is
    1 + 2^-40 exactly; every small square is below half an ulp of 1, so a
    plain running sum would return 1.  Random vectors agree with an exactly
    rounded sum (math.fsum) of the same products to a few ulps."""
    a = np.full(1 + (1 << 20), 2.0 ** -30, dtype=np.complex128)
    a[0] = 1.0
    assert orc.inner(a, a) == complex(1 + 2.0 ** -40, 0.0)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(1 << 18) + 1j * rng.standard_normal(1 << 18)
    y = rng.standard_normal(1 << 18) + 1j * rng.standard_normal(1 << 18)
    re = math.fsum(x.real * y.real + x.imag * y.imag)
    im = math.fsum(x.real * y.imag - x.imag * y.real)
    got = orc.inner(x, y)
    eps = np.finfo(float).eps
    assert abs(got.real - re) <= 4 * eps * abs(re) and abs(got.imag - im) <= 4 * eps * abs(im)


def test_pauli_apply_matches_dense(orc):
    rng = np.random.default_rng(21)
    n = 6
    terms = [(int(rng.integers(0, 64)), int(rng.integers(0, 64)), float(rng.standard_normal())) for _ in range(9)]
    H = pins.hamiltonian_dense(n, terms)
    phi = W.random_state(n, 3)
    psi = W.random_state(n, 4)
    assert np.allclose(orc.pauli_apply(n, terms, phi), H @ phi, rtol=0, atol=1e-13)
    assert abs(orc.expect(n, terms, psi, phi) - np.vdot(psi, H @ phi)) < 1e-13
    assert np.allclose(H, H.conj().T)


def _bloch_energy(n, layers, theta, terms):
    """Closed form for the ring-free HEA: a product state.  Per qubit the
    Bloch vector starts at (0,0,1); RY(t) turns it about y, RZ(p) about z."""
    r = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    for layer in range(layers):
        base = 2 * n * layer
        for q in range(n):
            t = theta[base + q]
            x, y, z = r[q]
            x, z = x * math.cos(t) + z * math.sin(t), -x * math.sin(t) + z * math.cos(t)
            p = theta[base + n + q]
            x, y = x * math.cos(p) - y * math.sin(p), x * math.sin(p) + y * math.cos(p)
            r[q] = (x, y, z)
    e = 0.0
    for xm, zm, c in terms:
        if xm == 0:
            qs = [q for q in range(n) if (zm >> q) & 1]
            e += c * np.prod([r[q, 2] for q in qs])
        else:
            q = int(math.log2(xm))
            e += c * r[q, 0]
    return e


def test_hea_without_ring_closed_form(orc):
    n, layers = 20, 8
    gates, theta, terms = W.hea(n, layers, 20, ring=False)
    e = orc.energy(W.zero_state(n), n, gates, terms)
    assert abs(e - _bloch_energy(n, layers, theta, terms)) < 1e-11


# --------------------------------------------------------------------------
# Gradients
# --------------------------------------------------------------------------

def test_param_shift_against_corrected_fd(orc):
    """For a parameter used once, E(theta) = c0 + c1 cos + c2 sin, so
    (E(t+h) - E(t-h)) / (2 sin h) is the exact derivative."""
    n, layers = 6, 2
    gates, theta, terms = W.hea(n, layers, 33)
    psi0 = W.zero_state(n)
    ps = orc.param_shift_grad(psi0, n, gates, terms, len(theta))
    h = 1e-2
    fd = orc.fd_grad(psi0, n, gates, terms, len(theta), h=h) * (h / math.sin(h))
    assert np.max(np.abs(ps - fd)) < 1e-10
    # and the plain FD bias is the expected h^2/6 relative size at most
    fd3 = orc.fd_grad(psi0, n, gates, terms, len(theta), h=1e-3)
    assert np.linalg.norm(fd3 - ps) / np.linalg.norm(ps) < 1e-6


def _qaoa_p1_closed_form(n, edges, gamma, beta):
    """MaxCut QAOA p = 1 (Wang, Hadfield, Jiang, Rieffel 2018), written for
    the cost unitary exp(-i g C); here the cost layer is exp(-i gamma sum ZZ),
    which is that form with g = -2 gamma up to a global phase."""
    g = -2.0 * gamma
    adj = {v: set() for v in range(n)}
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    tot = 0.0
    for u, v in edges:
        d = len(adj[u]) - 1
        e = len(adj[v]) - 1
        f = len(adj[u] & adj[v])
        c = 0.5 + 0.25 * math.sin(4 * beta) * math.sin(g) * (math.cos(g) ** d + math.cos(g) ** e)
        c -= 0.25 * math.sin(2 * beta) ** 2 * math.cos(g) ** (d + e - 2 * f) * (1 - math.cos(2 * g) ** f)
        tot += c
    return tot


def test_qaoa_p1_closed_form(orc):
    rng = np.random.default_rng(8)
    for n in [8, 10, 12]:
        for _ in range(3):
            edges = W.random_regular3(n, rng)
            gamma, beta = rng.uniform(0, math.pi, 2)
            gates = W.qaoa_gates(n, edges, [gamma], [beta])
            e = orc.energy(W.zero_state(n), n, gates, W.maxcut_terms(edges))
            assert abs(e - _qaoa_p1_closed_form(n, edges, gamma, beta)) < 1e-11
            assert -1e-12 <= e <= len(edges) + 1e-12


def _closed_form_grad(n, edges, gamma, beta, h=1e-3):
    """(dE/dgamma, dE/dbeta) of the p = 1 closed form by the five-point
    stencil (truncation O(h^4), about 1e-12 here; rounding about 1e-12)."""
    def d(f, t):
        return (-f(t + 2 * h) + 8 * f(t + h) - 8 * f(t - h) + f(t - 2 * h)) / (12 * h)
    return (d(lambda g: _qaoa_p1_closed_form(n, edges, g, beta), gamma),
            d(lambda b: _qaoa_p1_closed_form(n, edges, gamma, b), beta))


def test_param_shift_chain_factor_and_shared_sum_p1_closed_form(orc):
    """QAOA p = 1: gamma drives every RZZ (angle 2 gamma) and beta every RX
    (angle 2 beta), so each gradient entry sums |E| or n occurrences, each
    with chain factor 2.  Both the parameter-shift gradient and the
    theta-level central difference (angles rebuilt from theta) must equal
    the derivative of the Wang-Hadfield-Jiang-Rieffel closed form, which is
    independent of the oracle.  Dropping the chain factor halves the result;
    keeping only one occurrence per slot loses all but one edge or qubit."""
    rng = np.random.default_rng(81)
    for n in (6, 8, 10):
        edges = W.random_regular3(n, rng)
        gamma, beta = rng.uniform(0, math.pi, 2)
        terms = W.maxcut_terms(edges)
        psi0 = W.zero_state(n)
        gates = W.qaoa_gates(n, edges, [gamma], [beta])
        want = np.array(_closed_form_grad(n, edges, gamma, beta))
        ps = orc.param_shift_grad(psi0, n, gates, terms, 2)
        assert np.max(np.abs(ps - want)) < 1e-8, (n, ps, want)

        def rebuild(t):
            return W.qaoa_gates(n, edges, [t[0]], [t[1]])
        fd = orc.fd_grad(psi0, n, gates, terms, 2, h=1e-5, theta=[gamma, beta], rebuild=rebuild)
        assert np.max(np.abs(fd - want)) < 1e-8, (n, fd, want)


def test_param_shift_shared_slots_deeper_qaoa(orc):
    """p = 2 and 3: four or six shared slots, each summed over its layer's
    gates.  The parameter-shift gradient against the theta-level central
    difference pinned above (h = 1e-5: the bias, h^2/6 times the third
    derivative, and the rounding, about 1e-16 |E| / h, both stay under
    1e-8 here)."""
    rng = np.random.default_rng(82)
    for n, p in ((6, 2), (8, 3)):
        edges = W.random_regular3(n, rng)
        gam = rng.uniform(0, math.pi, p)
        bet = rng.uniform(0, math.pi, p)
        terms = W.maxcut_terms(edges)
        psi0 = W.zero_state(n)
        gates = W.qaoa_gates(n, edges, gam, bet)
        theta = np.empty(2 * p)
        theta[0::2], theta[1::2] = gam, bet

        def rebuild(t):
            return W.qaoa_gates(n, edges, t[0::2], t[1::2])
        ps = orc.param_shift_grad(psi0, n, gates, terms, 2 * p)
        fd = orc.fd_grad(psi0, n, gates, terms, 2 * p, h=1e-5, theta=theta, rebuild=rebuild)
        assert np.max(np.abs(ps - fd)) < 1e-7 * max(1.0, np.max(np.abs(ps))), (n, p, ps, fd)
        assert np.max(np.abs(ps)) > 1e-2


def test_param_shift_chain_factor_single_occurrence(orc):
    """Rotations with chain factors s in [0.5, 2], one occurrence each:
    E(theta_j) = c0 + c1 cos(s theta_j) + c2 sin(s theta_j), so the
    theta-level central difference times s h / sin(s h) is the exact
    derivative, whatever s is."""
    n = 5
    rng = np.random.default_rng(83)
    kinds = ["RX", "RY", "RZ", "RXX", "RYY", "RZZ", "P"]
    nparam = 12
    theta = rng.uniform(0, 2 * math.pi, nparam)
    scale = rng.uniform(0.5, 2.0, nparam)
    layout = []
    for j in range(nparam):
        kind = kinds[j % len(kinds)]
        qs = tuple(int(q) for q in rng.choice(n, 2 if kind in ("RXX", "RYY", "RZZ") else 1, replace=False))
        layout.append((kind, qs))

    prep = [W.u3(*rng.uniform(0, 2 * math.pi, 3), q) for q in range(n)]
    post = [W.u3(*rng.uniform(0, 2 * math.pi, 3), q) for q in range(n)]

    def rebuild(t):
        gates = list(prep)
        for j, (kind, qs) in enumerate(layout):
            gates.append(W.Gate(kind, qs, (), (float(scale[j] * t[j]),), j, float(scale[j])))
            gates.append(W.cx(qs[0], (qs[0] + 1) % n))
        return gates + post
    terms = [(0, 0b00011, 0.7), (0b00100, 0, -1.1), (0b01000, 0b01000, 0.4), (0b10001, 0b00001, 0.9)]
    psi0 = W.zero_state(n)
    gates = rebuild(theta)
    ps = orc.param_shift_grad(psi0, n, gates, terms, nparam)
    h = 1e-2
    fd = orc.fd_grad(psi0, n, gates, terms, nparam, h=h, theta=theta, rebuild=rebuild)
    fd *= scale * h / np.sin(scale * h)
    assert np.max(np.abs(ps - fd)) < 1e-10, np.max(np.abs(ps - fd))
    assert np.min(np.abs(ps)) > 1e-6


# --------------------------------------------------------------------------
# TFIM Trotter workload (Hamiltonian simulation, 1D transverse-field Ising)
# --------------------------------------------------------------------------

def test_tfim_trotter_converges_to_exact_evolution(orc):
    """First-order Trotter product against exp(-i t H) from a dense
    matrix exponential: the error stays below t^2/(2s) ||[A, B]|| (A the
    ZZ part, B the field part) and halves when the step count doubles.  A
    sign slip in either angle makes the error O(1)."""
    n, t, J, hx = 6, 0.8, 1.0, 0.7
    terms = W.tfim_terms(n, J, hx)
    A = pins.hamiltonian_dense(n, [tm for tm in terms if tm[0] == 0])
    B = pins.hamiltonian_dense(n, [tm for tm in terms if tm[0] != 0])
    comm = np.linalg.norm(A @ B - B @ A, 2)
    x = W.random_state(n, 6)
    exact = scipy.linalg.expm(-1j * t * (A + B)) @ x
    errs = []
    for s in (8, 16, 32):
        got = orc.apply_circuit(x, n, W.tfim(n, s, t / s, J, hx))
        e = np.linalg.norm(got - exact)
        assert e <= t * t / (2 * s) * comm, (s, e)
        errs.append(e)
    assert 0.4 < errs[1] / errs[0] < 0.6 and 0.4 < errs[2] / errs[1] < 0.6, errs


def test_tfim_without_coupling_closed_form(orc):
    """J = 0: independent spins precessing about x, so from |0..0> each
    <Z_i> = cos(2 hx t)."""
    n, s, dt, hx = 7, 9, 0.07, 1.3
    psi = orc.apply_circuit(W.zero_state(n), n, W.tfim(n, s, dt, J=0.0, hx=hx))
    m = orc.expect(n, W.magnetization_terms(n), psi).real
    assert abs(m - math.cos(2 * hx * s * dt)) < 1e-13


def test_tfim_without_field_is_a_phase(orc):
    """hx = 0: the evolution is diagonal, amplitude j picks up
    exp(i J t sum_i z_i z_{i+1}) with z = 1 - 2 bit."""
    n, s, dt, J = 8, 5, 0.11, 0.9
    x = W.random_state(n, 8)
    got = orc.apply_circuit(x, n, W.tfim(n, s, dt, J=J, hx=0.0))
    j = np.arange(1 << n)
    z = 1 - 2 * ((j[:, None] >> np.arange(n)) & 1)
    want = x * np.exp(1j * J * s * dt * np.sum(z[:, :-1] * z[:, 1:], axis=1))
    assert np.max(np.abs(got - want)) < 1e-14
