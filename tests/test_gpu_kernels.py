"""GPU parity of the single-matrix entry points (from_gate, from_pauli_sum,
spmv, fuse, expect) against the CPU oracle, through the C ABI."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests import pins
from tests.gpu_util import assert_state_close, dense_from_dia, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL64 = 1e-12   # complex128 amplitudes
TOL32 = 1e-5    # complex64 amplitudes


def _random_gate(rng, n, allow_matrix=True):
    kinds1 = ["H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SX", "RX", "RY", "RZ", "P", "U3", "I"]
    kinds2 = ["SWAP", "RXX", "RYY", "RZZ"]
    qs = [int(q) for q in rng.permutation(n)]
    params = tuple(float(v) for v in rng.uniform(0, 2 * math.pi, 3))
    r = rng.random()
    if r < 0.5 or n < 3:
        kind, nt = kinds1[rng.integers(len(kinds1))], 1
    elif r < 0.8 or not allow_matrix:
        kind, nt = kinds2[rng.integers(len(kinds2))], 2
    else:
        k = int(rng.integers(1, min(3, n - 1) + 1))
        m = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        q, _ = np.linalg.qr(m)
        nc = int(rng.integers(0, min(3, n - k) + 1))
        return W.Gate("MATRIX", tuple(qs[:k]), tuple(qs[k:k + nc]), matrix=q)
    nc = int(rng.integers(0, min(3, n - nt) + 1))
    return W.Gate(kind, tuple(qs[:nt]), tuple(qs[nt:nt + nc]), params)


# --------------------------------------------------------------------------
# from_gate: the expanded time-step matrix in DiaQ form
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_from_gate_matches_oracle_dense(seed):
    rng = np.random.default_rng(seed)
    for _ in range(8):
        n = int(rng.integers(1, 8))
        g = _random_gate(rng, n)
        A = D.from_gate(g, n)
        got = A.diagonals()
        want = orc.dense_matrix(n, [g])
        # every stored diagonal matches the oracle's diagonal element by element
        for d, v in got.items():
            assert np.max(np.abs(v - np.diagonal(want, d))) <= 1e-15, (g, d)
        # and nothing non-zero is missing
        assert np.max(np.abs(dense_from_dia(n, got) - want)) <= 1e-15


def test_from_gate_fig2_offsets_on_gpu():
    for q in range(4):
        A = D.from_gate(W.h(q), 4)
        assert A.offsets().tolist() == [-(1 << q), 0, 1 << q]
        vals = A.diagonals()
        assert np.allclose(np.abs(vals[0]), 1 / math.sqrt(2), atol=0, rtol=1e-15)


def test_from_gate_large_n_sampled():
    # n = 24: sampled elements against the oracle's element definition
    rng = np.random.default_rng(5)
    n = 24
    for g in [W.u3(0.3, 1.1, 2.2, 23), W.cx(3, 17), W.swap(2, 21), W.Gate("RZZ", (0, 23), (), (0.9,)),
              W.Gate("RXX", (5, 20), (), (0.4,))]:
        A = D.from_gate(g, n)
        diags = A.diagonals()
        for d, v in diags.items():
            ts = rng.integers(0, len(v), 64)
            for t in ts:
                i, j = int(t) + max(0, -d), int(t) + max(0, d)
                assert abs(v[t] - orc.gate_element(n, g, i, j)) <= 1e-15


def test_from_gate_complex64():
    g = W.u3(0.7, 0.2, -1.3, 2)
    A = D.from_gate(g, 5, dtype=torch.complex64)
    want = orc.dense_matrix(5, [g])
    assert np.max(np.abs(dense_from_dia(5, A.diagonals()) - want)) <= 1e-7


# --------------------------------------------------------------------------
# spmv (Alg. 2) on arbitrary DiaQ matrices, including transposes
# --------------------------------------------------------------------------

def _random_dia(rng, n, nd):
    N = 1 << n
    offs = sorted(int(o) for o in rng.choice(np.arange(-(N - 1), N), nd, replace=False))
    diags = {}
    for d in offs:
        L = N - abs(d)
        v = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        v[rng.random(L) < 0.2] = 0  # explicit zeros: stored elements like any other
        diags[d] = v
    return diags


@pytest.mark.parametrize("n,nd", [(1, 1), (3, 4), (6, 9), (8, 27), (9, 30), (10, 3), (11, 60), (12, 7)])
def test_spmv_random_dia(n, nd):
    rng = np.random.default_rng(n * 100 + nd)
    N = 1 << n
    nd = min(nd, 2 * N - 1)
    diags = _random_dia(rng, n, nd)
    A = D.from_dense_diagonals(n, diags)
    Ad = dense_from_dia(n, diags)
    x = W.random_state(n, n)
    xd = to_dev(x)
    o, s, v = orc.pack_dia(sorted(diags), [diags[d] for d in sorted(diags)])
    ref = orc.dia_spmv(N, o, s, v, x)
    scale = max(1.0, float(np.max(np.abs(ref))))
    got = to_host(D.spmv(A, xd))
    assert np.max(np.abs(got - ref)) <= 1e-13 * scale * nd
    for flags, M in [(D.TRANSPOSE, Ad.T), (D.CONJUGATE, Ad.conj()), (D.ADJOINT, Ad.conj().T)]:
        got = to_host(D.spmv(A, xd, flags=flags))
        assert np.max(np.abs(got - M @ x)) <= 1e-13 * scale * nd, flags
    # transpose views relabel the diagonals without copying
    At = A.transpose(conjugate=True)
    got = to_host(D.spmv(At, xd))
    assert np.max(np.abs(got - Ad.conj().T @ x)) <= 1e-13 * scale * nd
    assert sorted(At.diagonals()) == sorted(-d for d in diags)


@pytest.mark.parametrize("n", [9, 12, 16, 20])
def test_spmv_gates_match_oracle(n):
    rng = np.random.default_rng(n)
    x = W.random_state(n, 100 + n)
    xd = to_dev(x)
    qs = sorted({0, 1, 5, n // 2, n - 2, n - 1})
    gates = [W.u3(*rng.uniform(0, 6.28, 3), q) for q in qs]
    gates += [W.cx(qs[i], qs[-1 - i]) for i in range(len(qs) // 2)]
    gates += [W.swap(0, n - 1), W.Gate("RXX", (1, n - 2), (), (0.7,)), W.Gate("RZZ", (2, n - 1), (), (1.3,)),
              _random_gate(rng, n)]
    for g in gates:
        A = D.from_gate(g, n)
        got = to_host(D.spmv(A, xd))
        ref = x.copy()
        orc.apply_gate(ref, n, g)
        assert_state_close(got, ref, TOL64, str(g))
        # adjoint undoes the gate
        back = to_host(D.spmv(A, to_dev(got), flags=D.ADJOINT))
        assert_state_close(back, x, TOL64, "adjoint " + str(g))


def _classes(y):
    """Per component: 0 finite, 1 NaN, 2 +Inf, 3 -Inf."""
    out = []
    for c in (y.real, y.imag):
        k = np.zeros(c.shape, np.int8)
        k[np.isnan(c)] = 1
        k[np.isposinf(c)] = 2
        k[np.isneginf(c)] = 3
        out.append(k)
    return np.stack(out)


@pytest.mark.parametrize("bad", [np.inf, np.nan, complex(0, -np.inf)])
def test_spmv_caller_matrix_propagates_non_finite_x(bad):
    """A caller-built matrix multiplies every stored element with its x entry,
    explicit zeros included (Alg. 2; 0 * Inf = NaN): the non-finite pattern of
    y and its finite values match the oracle's product, in both dtypes' fp64
    case, also through the transposed view."""
    rng = np.random.default_rng(31)
    n = 10
    N = 1 << n
    diags = {}
    for d in (-300, -3, 0, 5, 257):
        L = N - abs(d)
        diags[d] = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    diags[5][:] = 0          # an explicit all-zero diagonal
    diags[-3][::7] = 0       # scattered explicit zeros
    A = D.from_dense_diagonals(n, diags)
    x = W.random_state(n, 8)
    for col in (0, 37, 518, N - 1):
        x[col] = bad
    o, s_, v = orc.pack_dia(sorted(diags), [diags[d] for d in sorted(diags)])
    ref = orc.dia_spmv(N, o, s_, v, x)
    got = to_host(D.spmv(A, to_dev(x)))
    assert (_classes(got) == _classes(ref)).all()
    fin = np.isfinite(ref)
    assert (~fin).any() and fin.any()
    assert np.max(np.abs(got[fin] - ref[fin])) <= 1e-13
    # the transposed view: A^T's stored elements are A's, so the oracle's
    # product on the relabelled diagonals
    tdiags = {-d: vv for d, vv in diags.items()}
    o, s_, v = orc.pack_dia(sorted(tdiags), [tdiags[d] for d in sorted(tdiags)])
    ref_t = orc.dia_spmv(N, o, s_, v, x)
    got_t = to_host(D.spmv(A, to_dev(x), flags=D.TRANSPOSE))
    assert (_classes(got_t) == _classes(ref_t)).all()
    fin = np.isfinite(ref_t)
    assert np.max(np.abs(got_t[fin] - ref_t[fin])) <= 1e-13


def test_spmv_expanded_gate_skips_structural_zeros():
    """A gate's expansion stores structural zeros (a diagonal +-2^q of a
    one-qubit gate is zero on the rows outside the gate's coupling); the
    product skips them, so a non-finite x entry reaches exactly the rows whose
    time-step matrix has a non-zero in its column, and every other row equals
    the product over the non-zero entries."""
    n = 10
    N = 1 << n
    x = W.random_state(n, 9)
    col = 300
    x[col] = np.inf
    xf = x.copy()
    xf[col] = 0
    for g in [W.u3(0.3, 1.1, 2.2, 3), W.cx(2, 7), W.swap(1, 8), W.Gate("RXX", (0, 9), (), (0.4,))]:
        Ad = orc.dense_matrix(n, [g])
        got = to_host(D.spmv(D.from_gate(g, n), to_dev(x)))
        hit = Ad[:, col] != 0
        assert not np.isfinite(got[hit]).any(), g
        assert np.max(np.abs(got[~hit] - (Ad @ xf)[~hit])) <= 1e-13, g


def test_spmv_complex64():
    n = 14
    x = W.random_state(n, 3)
    g = W.u3(0.4, 1.0, 2.0, 11)
    A = D.from_gate(g, n, dtype=torch.complex64)
    got = to_host(D.spmv(A, to_dev(x, torch.complex64)))
    ref = x.copy()
    orc.apply_gate(ref, n, g)
    assert_state_close(got, ref, TOL32, "c64")


def test_spmv_rejects_aliasing_and_mismatch():
    n = 6
    A = D.from_gate(W.h(2), n)
    x = to_dev(W.random_state(n, 1))
    with pytest.raises(D.DiaqError) as ei:
        D.spmv(A, x, x)
    assert ei.value.status == 1
    with pytest.raises(ValueError):
        D.spmv(A, to_dev(W.random_state(n + 1, 1)))
    # a principal-diagonal-only matrix may run in place
    Z = D.from_gate(W.Gate("RZ", (3,), (), (0.4,)), n)
    ref = to_host(x).copy()
    orc.apply_gate(ref, n, W.Gate("RZ", (3,), (), (0.4,)))
    D.spmv(Z, x, x)
    assert_state_close(to_host(x), ref, TOL64)


# --------------------------------------------------------------------------
# fuse (Alg. 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_fuse_matches_dense_product(seed):
    rng = np.random.default_rng(40 + seed)
    n = int(rng.integers(2, 8))
    g1, g2 = _random_gate(rng, n), _random_gate(rng, n)
    A, B = D.from_gate(g1, n), D.from_gate(g2, n)
    C = D.fuse(A, B)
    want = orc.dense_matrix(n, [g1, g2])
    got = dense_from_dia(n, C.diagonals())
    assert np.max(np.abs(got - want)) <= 1e-14
    # no stored diagonal is entirely zero
    for d, v in C.diagonals().items():
        assert np.any(v != 0)


def test_fuse_hh_identity_and_ghz10():
    n = 6
    Hq = D.from_gate(W.h(3), n)
    C = D.fuse(Hq, Hq)
    assert C.offsets().tolist() == [0]
    assert np.allclose(C.diagonals()[0], 1, rtol=0, atol=1e-15)
    # GHZ(10) fused gate by gate: 1025 diagonals, nnz = 2048 (>= 99.8 % sparse)
    n = 10
    gates = W.ghz(n)
    U = D.from_gate(gates[0], n)
    for g in gates[1:]:
        U = D.fuse(U, D.from_gate(g, n))
    diags = U.diagonals()
    assert len(diags) == 1025
    nnz = sum(int(np.count_nonzero(v)) for v in diags.values())
    assert nnz == 2048
    assert np.max(np.abs(dense_from_dia(n, diags) - orc.dense_matrix(n, gates))) <= 1e-14


def test_fuse_group_diagonal_counts():
    """Alg. 1 on expanded gates: H and its controlled-phase ladder stay on
    three diagonals; U3, U3 and CX on one pair of qubits span -3..3 (any
    further pair sum cancels to exact zeros and is dropped)."""
    n = 5
    ladder = [W.h(4)] + [W.cp(math.pi / 2 ** m, 4 - m, 4) for m in range(1, 5)]
    for gates, want in ((ladder, [-16, 0, 16]),
                        ([W.u3(0.3, 0.4, 0.5, 0), W.u3(0.6, 0.7, 0.8, 1), W.cx(0, 1)], list(range(-3, 4)))):
        U = D.from_gate(gates[0], n)
        for g in gates[1:]:
            U = D.fuse(U, D.from_gate(g, n))
        live = [d for d, v in U.diagonals().items() if np.max(np.abs(v)) > 1e-14]
        assert sorted(live) == want
        assert np.max(np.abs(dense_from_dia(n, U.diagonals()) - orc.dense_matrix(n, gates))) <= 1e-14


def test_fuse_not_multiplyable():
    A = D.from_gate(W.h(0), 4)
    B = D.from_gate(W.h(0), 5)
    with pytest.raises(D.DiaqError) as ei:
        D.fuse(A, B)
    assert ei.value.status == 2


def test_fuse_large_applied_equals_sequential():
    n = 18
    g1, g2 = W.u3(0.3, 0.9, 1.7, 15), W.cx(3, 15)
    C = D.fuse(D.from_gate(g1, n), D.from_gate(g2, n))
    assert C.offsets().tolist() == [-(1 << 15), 0, 1 << 15]
    x = W.random_state(n, 18)
    got = to_host(D.spmv(C, to_dev(x)))
    ref = orc.apply_circuit(x, n, [g1, g2])
    assert_state_close(got, ref, TOL64)


# --------------------------------------------------------------------------
# Pauli sums and expectation values
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [3, 6, 10])
def test_pauli_sum_matches_dense(n):
    rng = np.random.default_rng(n)
    N = 1 << n
    terms = [(int(rng.integers(0, N)), int(rng.integers(0, N)), float(rng.standard_normal())) for _ in range(12)]
    terms.append((0, 0, 0.75))
    H = D.from_pauli_sum(n, terms)
    want = pins.hamiltonian_dense(n, terms)
    got = dense_from_dia(n, H.diagonals())
    assert np.max(np.abs(got - want)) <= 1e-14


@pytest.mark.parametrize("n", [4, 10, 16, 20])
def test_expect_matches_oracle(n):
    _, _, terms = W.hea(n, 1, n)
    H = D.from_pauli_sum(n, terms)
    psi = W.random_state(n, 7)
    phi = W.random_state(n, 8)
    e = D.expect(H, to_dev(psi))
    ref = orc.expect(n, terms, psi)
    assert abs(e - ref) <= 1e-12 * max(1.0, abs(ref))
    assert abs(e.imag) <= 1e-12
    e2 = D.expect(H, to_dev(psi), to_dev(phi))
    ref2 = orc.expect(n, terms, psi, phi)
    assert abs(e2 - ref2) <= 1e-12 * max(1.0, abs(ref2))


def test_expect_deterministic():
    n = 18
    _, _, terms = W.hea(n, 1, 3)
    H = D.from_pauli_sum(n, terms)
    psi = to_dev(W.random_state(n, 9))
    vals = {D.expect(H, psi) for _ in range(4)}
    assert len(vals) == 1


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_spmv_xcd_runs_change_only_the_order(dtype):
    """Gates coupling rows 1, 2 or 4 tiles apart run with XCD-ordered tiles
    by default: the result must equal the plain launch order bit for bit,
    and the oracle."""
    n = 16
    ctx = D.context()
    saved = D.get_tuning(ctx)
    x = W.random_state(n, 8)
    try:
        for q in (7, 8, 9, 10, 11, 12):
            for g in (W.u3(0.4, 1.1, 2.3, q), W.cx(0, q), W.cx(q, 0)):
                A = D.from_gate(g, n, dtype=dtype)
                outs = []
                for knob in (-1, 0):
                    D.set_tuning(ctx, spmv_xcd_runs=knob)
                    outs.append(to_host(D.spmv(A, to_dev(x, dtype))))
                assert np.array_equal(outs[0], outs[1]), "q=%d %s" % (q, g.kind)
                ref = orc.apply_circuit(x, n, [g])
                assert np.max(np.abs(outs[1] - ref)) <= (TOL64 if dtype == torch.complex128 else 1e-5)
    finally:
        D.set_tuning(ctx, **saved)
    with pytest.raises(D.DiaqError):
        D.set_tuning(ctx, spmv_xcd_runs=2)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_spmv_far_partner_order_changes_only_the_order(dtype):
    """Gates whose partner rows lie 16 MiB or more apart alternate partner
    tiles on each XCD by default: bitwise the plain launch order, and the
    oracle (n = 22, 4-KiB tiles: qubits 20 and 21)."""
    n = 22
    ctx = D.context()
    saved = D.get_tuning(ctx)
    x = W.random_state(n, 9)
    try:
        D.set_tuning(ctx, spmv_group_bits=-1)  # no pairing inside a workgroup
        for q in (19, 20, 21):
            for g in (W.u3(0.4, 1.1, 2.3, q), W.cx(3, q)):
                A = D.from_gate(g, n, dtype=dtype)
                outs = []
                for knob in (-1, 0):
                    D.set_tuning(ctx, spmv_xcd_runs=knob)
                    outs.append(to_host(D.spmv(A, to_dev(x, dtype))))
                assert np.array_equal(outs[0], outs[1]), "q=%d %s" % (q, g.kind)
                ref = orc.apply_circuit(x, n, [g])
                assert np.max(np.abs(outs[1] - ref)) <= (TOL64 if dtype == torch.complex128 else 1e-5)
    finally:
        D.set_tuning(ctx, **saved)
