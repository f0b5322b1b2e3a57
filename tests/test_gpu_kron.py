"""GPU parity of the Alg. 3 path (plan.kron: gates applied in place
without expanded diagonals), alone and with fusion, and of the adjoint
gradient on that path."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host
from tests.test_gpu_kernels import _random_gate

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(autouse=True)
def per_gate_launches():
    """These tests exercise the per-operation Alg. 3 kernels, also on small
    states, so the one-launch LDS path for small states is switched off
    (tests/test_gpu_small.py covers it)."""
    ctx = D.context()
    saved = D.get_tuning(ctx)
    D.set_tuning(ctx, kron_small_qubits=-1)
    yield
    D.set_tuning(ctx, **saved)


@pytest.mark.parametrize("fuse", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_kron_random_circuits(fuse, seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(1, 15))
    gates = [_random_gate(rng, n) for _ in range(int(rng.integers(1, 50)))]
    x = W.random_state(n, seed)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=D.make_plan(kron=True, fuse=fuse, max_fused_qubits=3))
    assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), TOL64, "kron fuse=%s seed %d" % (fuse, seed))


@pytest.mark.parametrize("kmax", [1, 2, 3])
def test_kron_workloads(kmax):
    for name, n, gates, x in [("qft", 16, W.qft(16), W.random_state(16, 2)),
                              ("random_layered", 16, W.random_layered(16, 4, 9), W.zero_state(16)),
                              ("tfim", 14, W.tfim(14, 6), W.random_state(14, 5)),
                              ("hea", 12, W.hea(12, 2, 6)[0], W.zero_state(12))]:
        for fuse in (False, True):
            psi = to_dev(x)
            D.apply_circuit(gates, psi, plan=D.make_plan(kron=True, fuse=fuse, max_fused_qubits=kmax))
            assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), TOL64, "%s k=%d fuse=%s" % (name, kmax, fuse))


def test_kron_complex64_and_large_n():
    n = 22
    gates = W.random_layered(n, 1, 22)
    x = W.zero_state(n)
    ref = orc.apply_circuit(x, n, gates)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=D.make_plan(kron=True))
    assert_state_close(to_host(psi), ref, TOL64, "kron n=22")
    psi32 = to_dev(x, torch.complex64)
    D.apply_circuit(gates, psi32, plan=D.make_plan(kron=True, fuse=True, max_fused_qubits=3))
    assert_state_close(to_host(psi32), ref, TOL32, "kron c64 n=22", l2tol=1e-4)


def test_kron_matches_plain_path_bitwise_structure():
    # same circuit, both paths, agree to rounding
    n = 18
    gates = W.qft(n)
    x = to_dev(W.random_state(n, 18))
    a, b = x.clone(), x.clone()
    D.apply_circuit(gates, a)
    D.apply_circuit(gates, b, plan=D.make_plan(kron=True, fuse=True))
    assert_state_close(to_host(a), to_host(b), TOL64, "plain vs kron")


@pytest.mark.parametrize("n,layers", [(6, 2), (12, 3)])
def test_kron_adjoint(n, layers):
    gates, theta, terms = W.hea(n, layers, 40 + n)
    H = D.from_pauli_sum(n, terms)
    psi0 = W.zero_state(n)
    e, g = D.adjoint_grad(gates, H, to_dev(psi0), len(theta), plan=D.make_plan(kron=True))
    assert abs(e - orc.energy(psi0, n, gates, terms)) <= 1e-12
    ps = orc.param_shift_grad(psi0, n, gates, terms, len(theta))
    assert np.linalg.norm(g - ps) <= 1e-10 * max(1.0, np.linalg.norm(ps))


def test_kron_adjoint_controlled_and_two_qubit_rotations():
    rng = np.random.default_rng(5)
    n = 7
    gates, pidx = [], 0
    for kind, nt, nc in [("RX", 1, 0), ("RYY", 2, 0), ("RZZ", 2, 0), ("RY", 1, 1), ("P", 1, 2), ("RXX", 2, 1)]:
        qs = [int(q) for q in rng.permutation(n)]
        gates.append(W.u3(*rng.uniform(0, 6, 3), qs[-1]))
        gates.append(W.Gate(kind, tuple(qs[:nt]), tuple(qs[nt:nt + nc]), (float(rng.uniform(0, 6)),), pidx, 1.3))
        pidx += 1
    terms = [(int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n)), float(rng.standard_normal()))
             for _ in range(6)]
    H = D.from_pauli_sum(n, terms)
    psi0 = W.random_state(n, 8)
    e, g = D.adjoint_grad(gates, H, to_dev(psi0), pidx, plan=D.make_plan(kron=True))
    e2, g2 = D.adjoint_grad(gates, H, to_dev(psi0), pidx)
    assert abs(e - orc.energy(psi0, n, gates, terms)) <= 1e-12
    fd = orc.fd_grad(psi0, n, gates, terms, pidx, h=1e-4)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))
    assert np.max(np.abs(g - g2)) <= 1e-12


# --------------------------------------------------------------------------
# Groups of four and five qubits (dense local matrices)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kmax", [4, 5])
@pytest.mark.parametrize("seed", range(5))
def test_kron_big_groups_random_circuits(kmax, seed):
    rng = np.random.default_rng(1900 + seed)
    n = int(rng.integers(3, 14))
    gates = [_random_gate(rng, n) for _ in range(int(rng.integers(20, 80)))]
    if n >= 6:  # a gate of six qubits with its controls stays as it is
        q = [int(v) for v in rng.permutation(n)[:6]]
        m = np.linalg.qr(rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)))[0]
        gates.insert(len(gates) // 2, W.Gate("MATRIX", tuple(q[:3]), tuple(q[3:]), matrix=m))
    x = W.random_state(n, seed)
    plan = D.make_plan(kron=True, fuse=True, max_fused_qubits=kmax)
    nops, _ = D.plan_count(gates, n, plan)
    n3, _ = D.plan_count(gates, n, D.make_plan(kron=True, fuse=True, max_fused_qubits=3))
    assert nops <= len(gates)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=plan)
    assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), TOL64, "kmax=%d seed %d" % (kmax, seed))


@pytest.mark.parametrize("kmax", [4, 5])
def test_kron_big_groups_workloads(kmax):
    plan = D.make_plan(kron=True, fuse=True, max_fused_qubits=kmax)
    cases = [("qft", 16, W.qft(16), W.random_state(16, 2)),
             ("random_layered", 20, W.random_layered(20, 4, 5), W.zero_state(20)),
             ("tfim", 14, W.tfim(14, 6, 0.1), W.random_state(14, 6)),
             ("hea", 12, W.hea(12, 3, 9)[0], W.zero_state(12)),
             ("ghz", 12, W.ghz(12), W.zero_state(12))]
    for name, n, gates, x in cases:
        psi = to_dev(x)
        D.apply_circuit(gates, psi, plan=plan)
        assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), TOL64, "%s kmax=%d" % (name, kmax))
    # fewer operations than three-qubit groups on the layered circuit
    g = W.random_layered(28, 20, 28)
    n3, _ = D.plan_count(g, 28, D.make_plan(kron=True, fuse=True, max_fused_qubits=3))
    nk, _ = D.plan_count(g, 28, plan)
    assert nk < n3


def test_kron_big_groups_complex64():
    n = 18
    gates = W.random_layered(n, 3, 8) + W.qft(n)[:40]
    x = W.random_state(n, 8)
    ref = orc.apply_circuit(x, n, gates)
    psi = to_dev(x, torch.complex64)
    D.apply_circuit(gates, psi, plan=D.make_plan(kron=True, fuse=True, max_fused_qubits=5))
    assert_state_close(to_host(psi), ref, TOL32, "kmax=5 c64", l2tol=1e-4)


def _group_gates(S, n):
    """One fused group on the qubits S (U3 on each, CX chain through S),
    then two diagonal gates reaching outside S (folded as row factors when
    the group is full)."""
    gates = [W.u3(0.3, 0.2, 0.1, S[0])]
    for j in range(len(S) - 1):
        gates += [W.cx(S[j], S[j + 1]), W.u3(0.4 + j, 0.25 * j, 0.1 + j, S[j + 1])]
    outside = [q for q in range(n) if q not in S]
    gates += [W.cp(0.7, S[0], outside[-1]), W.Gate("RZ", (outside[0],), (), (1.1,))]
    return gates


@pytest.mark.parametrize("S", [(0,), (1,), (2,), (0, 1), (0, 5), (1, 2, 9), (0, 1, 2, 3), (2, 7, 8, 12),
                               (0, 1, 2, 3, 4), (0, 3, 6, 9, 11), (2, 4, 5, 10, 13), (0, 1, 2, 3, 5)])
def test_kron_staged_low_qubit_groups(S):
    """Groups touching qubits 0..2 are staged through LDS (a wave loads its
    64 cosets' amplitudes coalesced): at the smallest state that has 64
    cosets, and above it."""
    for n in sorted({max(max(S) + 2, len(S) + 6), 15}):
        gates = _group_gates(list(S), n)
        x = W.random_state(n, n + len(S))
        for kmax in (4, 5):
            psi = to_dev(x)
            D.apply_circuit(gates, psi, plan=D.make_plan(kron=True, fuse=True, max_fused_qubits=kmax))
            assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), TOL64, "S=%s n=%d kmax=%d" % (S, n, kmax))
        psi32 = to_dev(x, torch.complex64)
        D.apply_circuit(gates, psi32, plan=D.make_plan(kron=True, fuse=True, max_fused_qubits=5))
        assert_state_close(to_host(psi32), orc.apply_circuit(x, n, gates), TOL32, "S=%s n=%d c64" % (S, n))


@pytest.mark.parametrize("kmax", [2, 3, 4, 5])
def test_factor_tables_on_wave_varying_and_uniform_qubits(kmax):
    """Operations whose folded diagonal factors sit on the lowest qubits
    (which differ across a wave's cosets), on high qubits only (the same for
    a whole wave), or on both, in one to three tables, with plain and
    controlled cores: every table path against the oracle, complex128 and
    complex64."""
    n = 18
    rng = np.random.default_rng(70 + kmax)
    gates = []
    for t in (17, 16, 15, 2, 0):
        gates.append(W.h(t))
        for k in range(n):
            if k != t and rng.random() < 0.7:
                gates.append(W.cp(float(rng.uniform(0, 6)), k, t))
        gates += [W.Gate("RZZ", (9, 11), (), (0.37,)), W.Gate("RZ", (1,), (), (1.1,)), W.cz(3, 10),
                  W.cp(0.2, 4, 8)]
    # controlled cores followed by ladders over 16 other qubits (three
    # tables): their rows with the controls off still take the factors
    gates += [W.cx(15, 17)] + [W.cp(0.1 + 0.3 * k, k, 17) for k in range(17) if k != 15]
    gates += [W.Gate("RZZ", (9, 10), (), (0.8,)), W.cx(5, 16), W.cp(1.3, 0, 16), W.cz(7, 11)]
    gates += [W.Gate("RY", (11,), (3, 6), (0.7,))] + [W.cp(0.2 + 0.1 * k, k, 11) for k in range(n)
                                                      if k not in (3, 6, 11)]
    x = W.random_state(n, 71)
    ref = orc.apply_circuit(x, n, gates)
    plan = D.make_plan(kron=True, fuse=True, max_fused_qubits=kmax)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=plan)
    assert_state_close(to_host(psi), ref, TOL64, "kmax=%d" % kmax)
    psi32 = to_dev(x, torch.complex64)
    D.apply_circuit(gates, psi32, plan=plan)
    assert_state_close(to_host(psi32), ref, TOL32, "kmax=%d c64" % kmax, l2tol=1e-4)
