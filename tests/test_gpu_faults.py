"""Fault injection forced from the host: invalid gates anywhere in a
circuit, an expansion larger than device memory, a parameter index past
the gradient vector, and a NaN in the input state.  Every error must come
back as a status (no partial work: the state is bitwise unchanged), the
context must stay usable afterwards, and a NaN must reach the norm rather
than be dropped by any kernel."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host

pytestmark = pytest.mark.gpu

PLANS = [None, dict(fuse=True, max_fused_qubits=2), dict(fuse=True, max_fused_qubits=3), dict(kron=True),
         dict(kron=True, fuse=True, max_fused_qubits=3), dict(kron=True, fuse=True, max_fused_qubits=5)]

BAD_GATES = [
    W.Gate("H", (12,)),                       # qubit out of range (n = 12)
    W.Gate("SWAP", (3, 3)),                   # duplicate target
    W.Gate("X", (4,), (4,)),                  # control equals target
    W.Gate("MATRIX", (1, 2)),                 # custom gate without a matrix
]


def _plan(kw):
    return None if kw is None else D.make_plan(**kw)


@pytest.mark.parametrize("kw", PLANS)
def test_bad_gate_anywhere_leaves_state_untouched(kw):
    """Every gate is checked before the first launch: a bad gate at the end
    of a long circuit returns INVALID_ARGUMENT with the state as it was."""
    n = 12
    good = W.random_layered(n, 3, 21) + W.qft(n)[:30]
    x = W.random_state(n, 22)
    psi = to_dev(x)
    for bad in BAD_GATES:
        for pos in (len(good), len(good) // 2):
            gates = good[:pos] + [bad] + good[pos:]
            with pytest.raises(D.DiaqError) as ei:
                D.apply_circuit(gates, psi, plan=_plan(kw))
            assert ei.value.status == 1, (bad, ei.value)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(psi), x), "state changed by a rejected call (%s, %s)" % (bad, kw)
    # the context still runs the valid circuit correctly afterwards
    D.apply_circuit(good, psi, plan=_plan(kw))
    assert_state_close(to_host(psi), orc.apply_circuit(x, n, good), 1e-12, "after rejected calls")


def test_oversize_expansion_is_out_of_memory_and_recoverable():
    """A U3 expanded at n = 34 needs 3 * 2^34 complex128 values (824 GB),
    more than the device holds: OUT_OF_MEMORY, and the next calls on the
    same context see no stale error."""
    with pytest.raises(D.DiaqError) as ei:
        D.from_gate(W.u3(0.3, 0.2, 0.1, 0), 34)
    assert ei.value.status == 3, ei.value
    with pytest.raises(D.DiaqError) as ei:
        D.from_gate(W.h(0), 35)
    assert ei.value.status == 1
    n = 10
    g = W.u3(0.7, -0.4, 1.1, 6)
    A = D.from_gate(g, n)
    x = W.random_state(n, 23)
    y = D.spmv(A, to_dev(x))
    assert_state_close(to_host(y), orc.apply_circuit(x, n, [g]), 1e-12, "after OOM")


@pytest.mark.parametrize("kron", [False, True])
def test_parameter_index_past_the_gradient_is_rejected(kron):
    n = 6
    gates = W.random_layered(n, 1, 24) + [W.Gate("RY", (2,), (), (0.5,), param_index=3)]
    H = D.from_pauli_sum(n, [(0, 0b11, 0.7)])
    plan = D.make_plan(kron=True) if kron else None
    with pytest.raises(D.DiaqError) as ei:
        D.adjoint_grad(gates, H, to_dev(W.random_state(n, 25)), 3, plan=plan)
    assert ei.value.status == 1
    e, g = D.adjoint_grad(gates, H, to_dev(W.random_state(n, 25)), 4, plan=plan)
    assert np.isfinite(e) and g.shape == (4,)


@pytest.mark.parametrize("kw", PLANS)
def test_nan_in_state_reaches_the_norm(kw):
    """One NaN amplitude in the input: after the circuit the norm is NaN
    (no kernel drops it), while the same circuit on the clean state keeps
    the norm at 1."""
    n = 11
    gates = W.random_layered(n, 2, 26)
    x = W.random_state(n, 27)
    bad = x.copy()
    bad[345] = complex(np.nan, 0.0)
    psi = to_dev(bad)
    D.apply_circuit(gates, psi, plan=_plan(kw))
    assert np.isnan(np.linalg.norm(to_host(psi)))
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=_plan(kw))
    assert abs(np.linalg.norm(to_host(psi)) - 1.0) <= 1e-12
