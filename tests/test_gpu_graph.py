"""Circuit graphs (diaq_circuit_graph_*): one application of a gate list
recorded as a HIP graph and replayed.  Each replay must equal the eager
diaq_apply_circuit of the same plan bit for bit (same kernels, same
arguments), and the oracle to the FP64 bar, also when other eager work on
the same context (which may grow and rewrite the context's workspaces) runs
between replays."""
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

PLANS = {
    "plain": None,
    "fuse2": dict(fuse=True, max_fused_qubits=2),
    "fuse3": dict(fuse=True, max_fused_qubits=3),
    "kron": dict(kron=True),
    "kron+fuse3": dict(kron=True, fuse=True, max_fused_qubits=3),
    "kron+fuse4": dict(kron=True, fuse=True, max_fused_qubits=4),
    "kron+fuse5": dict(kron=True, fuse=True, max_fused_qubits=5),
}


def _plan(name):
    kw = PLANS[name]
    return None if kw is None else D.make_plan(**kw)


def _cases():
    return [("ghz12", 12, W.ghz(12), W.zero_state(12)),
            ("qft13", 13, W.qft(13), W.random_state(13, 3)),
            ("layered+qft14", 14, W.random_layered(14, 3, 5) + W.qft(14)[:40], W.random_state(14, 4))]


@pytest.mark.parametrize("plan", list(PLANS))
def test_graph_replay_matches_eager_and_oracle(plan):
    for name, n, gates, x in _cases():
        want = orc.apply_circuit(x, n, gates)
        eager = to_dev(x)
        D.apply_circuit(gates, eager, plan=_plan(plan))
        psi = to_dev(x)
        g = D.CircuitGraph(gates, psi, plan=_plan(plan))
        assert g.nodes() >= 1
        # other eager work on the same context between replays: a larger
        # circuit that grows the context's own workspaces
        other = to_dev(W.random_state(n + 2, 7))
        for rep in range(3):
            psi.copy_(to_dev(x))
            g.launch()
            torch.cuda.synchronize()
            got = to_host(psi)
            assert np.array_equal(got, to_host(eager)), "%s %s replay %d differs from eager" % (name, plan, rep)
            assert_state_close(got, want, TOL64, "%s %s replay %d" % (name, plan, rep))
            D.apply_circuit(W.random_layered(n + 2, 2, rep) + W.qft(n + 2)[:20], other, plan=_plan(plan))
        g.close()


def test_graph_back_to_back_replays_compose():
    """Two replays without a reset apply the circuit twice."""
    n = 11
    gates = W.random_layered(n, 2, 3) + W.qft(n)[:25]
    x = W.random_state(n, 9)
    psi = to_dev(x)
    g = D.CircuitGraph(gates, psi, plan=D.make_plan(kron=True, fuse=True, max_fused_qubits=3))
    g.launch()
    g.launch()
    torch.cuda.synchronize()
    want = orc.apply_circuit(orc.apply_circuit(x, n, gates), n, gates)
    assert_state_close(to_host(psi), want, TOL64, "two replays")
    g.close()


def test_graph_complex64():
    n = 13
    gates = W.random_layered(n, 2, 8) + W.qft(n)[:30]
    x = W.random_state(n, 2)
    want = orc.apply_circuit(x, n, gates)
    for plan in ("plain", "kron+fuse3"):
        psi = to_dev(x, torch.complex64)
        eager = to_dev(x, torch.complex64)
        D.apply_circuit(gates, eager, plan=_plan(plan))
        g = D.CircuitGraph(gates, psi, plan=_plan(plan))
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(psi), to_host(eager))
        assert np.max(np.abs(to_host(psi) - want)) <= 1e-5
        g.close()


def test_graph_rejects_bad_arguments():
    n = 6
    psi = to_dev(W.zero_state(n))
    with pytest.raises(D.DiaqError):
        D.CircuitGraph([W.Gate("H", (n,), ())], psi)  # qubit out of range
    with pytest.raises(D.DiaqError):
        D.CircuitGraph(W.ghz(n), psi, scratch=psi)  # state and scratch alias
