"""Every selectable shape of the DiaQ product kernel (Alg. 2 with row
ownership), forced through the tuning knobs: rows per lane 1, 2, 4; one or
three diagonals per chunk; non-temporal value / y streams on and off; tile
groups of G = 1, 2, 4, 8 over the coupling qubits (by threshold and by
per-qubit mask); XCD-aware tile orders on and off, XCD-contiguous and
interleaved-halves tile orders.  Each variant only
changes which lane computes a row and in which order tiles run, never the
arithmetic of a row (ascending diagonals, the same fused multiply-adds), so
every variant must equal the default one bit for bit, and the default must
match the oracle's state (complex128 1e-12, complex64 1e-5) after gates
with one, two and three coupling qubits at and above the tile."""
from __future__ import annotations

import itertools

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host

pytestmark = pytest.mark.gpu

N_QUBITS = 22


def _unitary(rng, k):
    m = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    q, _ = np.linalg.qr(m)
    return q


def _gates():
    rng = np.random.default_rng(2222)
    n = N_QUBITS
    return [
        W.u3(0.3, 1.2, -0.7, n - 1),                                 # far partner (pair order)
        W.u3(1.1, 0.4, 2.0, 9),                                      # tile distance 2 (XCD runs)
        W.u3(2.2, -0.3, 0.9, 13),
        W.swap(18, n - 1),                                           # one coupling, offset 2^21 - 2^18
        W.Gate("RXX", (19, n - 1), (), (0.8,)),                       # two coupling qubits
        W.Gate("MATRIX", (19, 20, n - 1), (), matrix=_unitary(rng, 3)),  # three coupling qubits
        W.cx(3, 20),
        W.cx(20, 2),
        W.Gate("RZZ", (0, n - 1), (), (1.3,)),                        # principal diagonal only
        W.Gate("MATRIX", (5, 19), (n - 1,), matrix=_unitary(rng, 2)),  # controlled, mixed low/high
        W.u3(0.5, 0.6, 0.7, 0),
        W.Gate("RYY", (8, 20), (), (2.1,)),
    ]


@pytest.fixture(scope="module")
def case():
    n = N_QUBITS
    gates = _gates()
    x0 = W.random_state(n, 2200)
    return n, gates, x0, orc.apply_circuit(x0, n, gates)


@pytest.fixture()
def restore_tuning():
    ctx = D.context()
    saved = D.get_tuning(ctx)
    yield ctx
    D.set_tuning(ctx, **saved)


_DEFAULT = dict(spmv_rows=0, spmv_group_bits=0, spmv_chunk=0, spmv_nontemporal=0, spmv_group_min_qubit=0,
                spmv_xcd_runs=0, spmv_group_qubits=0, spmv_order=0)

# tile grouping: none; G up to 8 over coupling qubits >= 18; G <= 2; G <= 4;
# per-qubit mask (qubits 19 and 21)
_GROUPINGS = {
    "nogroup": dict(spmv_group_bits=-1),
    "G8": dict(spmv_group_bits=0, spmv_group_min_qubit=18),
    "G2": dict(spmv_group_bits=1, spmv_group_min_qubit=18),
    "G4": dict(spmv_group_bits=2, spmv_group_min_qubit=18),
    "mask": dict(spmv_group_bits=0, spmv_group_qubits=(1 << 19) | (1 << 21)),
}


def _run(ctx, gates, x0, n, dtype, plan, **knobs):
    t = dict(_DEFAULT)
    t.update(knobs)
    D.set_tuning(ctx, **t)
    psi = to_dev(x0, dtype)
    D.apply_circuit(gates, psi, plan=plan)
    return to_host(psi)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
@pytest.mark.parametrize("rows", [1, 2, 4])
def test_spmv_variants_bitwise_and_oracle(case, restore_tuning, dtype, rows):
    n, gates, x0, ref = case
    ctx = restore_tuning
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    base = _run(ctx, gates, x0, n, dtype, None)
    assert_state_close(base, ref, tol, "default knobs", l2tol=tol if dtype == torch.complex128 else 1e-4)
    for chunk, nt, (gname, grouping), (xcd, order) in itertools.product((1, 3), (0, -1), _GROUPINGS.items(),
                                                                         ((0, 0), (-1, 0), (0, 1), (0, 2))):
        knobs = dict(spmv_rows=rows, spmv_chunk=chunk, spmv_nontemporal=nt, spmv_xcd_runs=xcd, spmv_order=order,
                     **grouping)
        got = _run(ctx, gates, x0, n, dtype, None, **knobs)
        assert np.array_equal(got, base), knobs


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_spmv_variants_fused_ops(case, restore_tuning, dtype):
    """Fused operations of up to three non-diagonal qubits (up to 27
    diagonals, several tiles apart) under every grouping and row count."""
    n, gates, x0, ref = case
    ctx = restore_tuning
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    plan = D.make_plan(fuse=True, max_fused_qubits=3)
    base = _run(ctx, gates, x0, n, dtype, plan)
    assert_state_close(base, ref, tol, "fuse3 default", l2tol=tol if dtype == torch.complex128 else 1e-4)
    for rows, chunk, (gname, grouping) in itertools.product((1, 2, 4), (1, 3), _GROUPINGS.items()):
        knobs = dict(spmv_rows=rows, spmv_chunk=chunk, **grouping)
        got = _run(ctx, gates, x0, n, dtype, plan, **knobs)
        assert np.array_equal(got, base), knobs
