"""Degenerate inputs on every path: empty circuits and empty gate ranges,
one- and two-qubit registers under every plan (group sizes larger than the
register), a matrix with no stored diagonal, an adjoint sweep with no gate
or no differentiable gate, and an empty circuit graph."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

PLANS = [None, dict(fuse=True, max_fused_qubits=2), dict(fuse=True, max_fused_qubits=3), dict(kron=True),
         dict(kron=True, fuse=True, max_fused_qubits=3), dict(kron=True, fuse=True, max_fused_qubits=4),
         dict(kron=True, fuse=True, max_fused_qubits=5)]


def _plan(kw):
    return None if kw is None else D.make_plan(**kw)


@pytest.mark.parametrize("kw", PLANS)
def test_empty_circuit_and_empty_range_leave_state(kw):
    n = 9
    x = W.random_state(n, 1)
    psi = to_dev(x)
    D.apply_circuit([], psi, plan=_plan(kw))
    assert np.array_equal(to_host(psi), x)
    gates = W.random_layered(n, 2, 3)
    D.apply_circuit(gates, psi, plan=_plan(kw), begin=5, end=5)
    assert np.array_equal(to_host(psi), x)


@pytest.mark.parametrize("kw", PLANS)
@pytest.mark.parametrize("n", [1, 2])
def test_tiny_registers_every_plan(kw, n):
    rng = np.random.default_rng(10 + n)
    gates = [W.u3(*rng.uniform(0, 6, 3), 0), W.h(n - 1), W.Gate("RZ", (0,), (), (0.4,))]
    if n == 2:
        gates += [W.cx(0, 1), W.swap(0, 1), W.Gate("RZZ", (0, 1), (), (0.9,)), W.cp(0.3, 1, 0)]
    x = W.random_state(n, n)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=_plan(kw))
    assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), TOL64, "n=%d %s" % (n, kw))


def test_matrix_without_diagonals():
    n = 5
    A = D.from_dense(np.zeros((1 << n, 1 << n)))
    assert A.offsets().tolist() == []
    x = to_dev(W.random_state(n, 2))
    y = D.spmv(A, x)
    assert not torch.any(y != 0)
    e = D.expect(A, x)
    assert e == 0


@pytest.mark.parametrize("kron", [False, True])
def test_adjoint_without_gates_or_parameters(kron):
    n = 6
    terms = [(0, 0b11, 0.7), (1 << 2, 0, -0.4)]
    H = D.from_pauli_sum(n, terms)
    x = W.random_state(n, 3)
    plan = D.make_plan(kron=True) if kron else None
    e, g = D.adjoint_grad([], H, to_dev(x), 0, plan=plan)
    assert abs(e - orc.expect(n, terms, x).real) <= 1e-12 and g.size == 0
    gates = W.random_layered(n, 2, 4)  # no differentiable gate
    e, g = D.adjoint_grad(gates, H, to_dev(x), 0, plan=plan)
    assert abs(e - orc.energy(x, n, gates, terms)) <= 1e-12 and g.size == 0


def test_empty_circuit_graph():
    n = 8
    x = W.random_state(n, 5)
    psi = to_dev(x)
    g = D.CircuitGraph([], psi)
    g.launch()
    torch.cuda.synchronize()
    assert np.array_equal(to_host(psi), x)
    g.close()


def test_device_copy():
    """diaq_copy: bitwise copy of 16-byte aligned buffers; misaligned,
    ragged or overlapping buffers are rejected and leave dst untouched."""
    x = to_dev(W.random_state(11, 6))
    y = torch.zeros_like(x)
    D.copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    empty = torch.zeros(0, dtype=torch.complex128, device="cuda:0")
    D.copy(empty, empty.clone())
    raw = torch.zeros(4096, dtype=torch.uint8, device="cuda:0")
    dst = torch.ones(4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(D.DiaqError):
        D.copy(raw[8:], dst[:-8])  # source 8 bytes off 16-byte alignment
    with pytest.raises(D.DiaqError):
        D.copy(raw[:24], dst[:24])  # not a multiple of 16 bytes
    with pytest.raises(D.DiaqError):
        D.copy(raw[:2048], raw[1024:3072])  # overlap
    torch.cuda.synchronize()
    assert bool(torch.all(dst == 1))


@pytest.mark.parametrize("kw", PLANS)
def test_all_zero_gate_matrix(kw):
    """A custom gate whose matrix is all zero has no stored diagonal: the
    state becomes zero on every plan, eagerly and replayed from a graph
    (which then holds a fill kernel, not a memset node)."""
    n = 9
    gates = [W.h(0), W.Gate("MATRIX", (3,), (), matrix=np.zeros((2, 2))), W.h(2)]
    x = W.random_state(n, 12)
    want = orc.apply_circuit(x, n, gates)
    assert not np.any(want)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=_plan(kw))
    assert not np.any(to_host(psi))
    psi = to_dev(x)
    g = D.CircuitGraph(gates, psi, plan=_plan(kw))
    for _ in range(2):
        psi.copy_(to_dev(x))
        g.launch()
        torch.cuda.synchronize()
        assert not np.any(to_host(psi))
    g.close()
