"""GPU parity of the batched persistent launch (diaq_batch_create/run)
against the CPU oracle, eagerly and through graph replay."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.test_oracle_pins import _qaoa_p1_closed_form

pytestmark = pytest.mark.gpu


def _qaoa_circuits(count, seed, widths=(4, 6, 8, 10, 12, 14), pmax=3):
    insts = W.qaoa_batch(count, seed, widths=widths, pmax=pmax)
    circs = [(i.n, i.gates, i.terms, 2 * i.p) for i in insts]
    theta = np.concatenate([np.ravel(np.column_stack([i.gammas, i.betas])) for i in insts])
    return insts, circs, theta


def _check_against_oracle(insts, ev, grads, tol_e=1e-11, tol_g=1e-10, shift_max_n=10):
    for i, inst in enumerate(insts):
        psi0 = W.zero_state(inst.n)
        e = orc.energy(psi0, inst.n, inst.gates, inst.terms)
        assert abs(ev[i] - e) <= tol_e * max(1.0, abs(e)), (i, inst.n, inst.p)
        if inst.n > shift_max_n:
            continue
        ps = orc.param_shift_grad(psi0, inst.n, inst.gates, inst.terms, 2 * inst.p)
        assert np.max(np.abs(grads[i] - ps)) <= tol_g * max(1.0, np.max(np.abs(ps))), (i, inst.n)


def test_batch_qaoa_matches_oracle():
    insts, circs, _ = _qaoa_circuits(24, 11)
    b = D.Batch(circs)
    ev, grads = b.run()
    _check_against_oracle(insts, ev, grads)


def test_batch_theta_and_graph_replays():
    insts, circs, theta = _qaoa_circuits(16, 12)
    eager = D.Batch(circs)
    graph = D.Batch(circs, graph=True)
    rng = np.random.default_rng(3)
    for rep in range(3):
        th = theta if rep == 0 else rng.uniform(0, math.pi, theta.size)
        ev_e, g_e = eager.run(th)
        ev_g, g_g = graph.run(th)
        assert np.array_equal(ev_e, ev_g), rep
        for a, b in zip(g_e, g_g):
            assert np.array_equal(a, b), rep
        # each replay against the oracle on rebuilt circuits
        k = 0
        for i, inst in enumerate(insts[:6]):
            t = th[k:k + 2 * inst.p]
            gates = W.qaoa_gates(inst.n, inst.edges, t[0::2], t[1::2])
            e = orc.energy(W.zero_state(inst.n), inst.n, gates, inst.terms)
            assert abs(ev_g[i] - e) <= 1e-11 * max(1.0, abs(e))
            k += 2 * inst.p
        # eager GPU work between replays
        psi = torch.zeros(1 << 10, dtype=torch.complex128, device="cuda")
        psi[0] = 1
        D.apply_circuit(W.ghz(10), psi)


def test_batch_p1_closed_form():
    rng = np.random.default_rng(9)
    circs, want = [], []
    for n in [6, 8, 10, 12, 16]:
        edges = W.random_regular3(n, rng)
        g, bta = rng.uniform(0, math.pi, 2)
        circs.append((n, W.qaoa_gates(n, edges, [g], [bta]), W.maxcut_terms(edges), 2))
        want.append(_qaoa_p1_closed_form(n, edges, g, bta))
    ev, _ = D.Batch(circs).run()
    assert np.max(np.abs(ev - np.array(want))) <= 1e-11


def test_batch_general_gates():
    """Other one- and two-qubit kinds (controls included) and observables."""
    rng = np.random.default_rng(21)
    circs, refs = [], []
    for c in range(10):
        n = int(rng.integers(2, 15))
        gates, pidx = [], 0
        for _ in range(30):
            qs = [int(q) for q in rng.permutation(n)]
            r = rng.random()
            if r < 0.3:
                gates.append(W.u3(*rng.uniform(0, 6, 3), qs[0]))
            elif r < 0.45 and n >= 2:
                gates.append(W.cx(qs[0], qs[1]))
            elif r < 0.55 and n >= 2:
                gates.append(W.swap(qs[0], qs[1]))
            elif r < 0.65 and n >= 3:
                gates.append(W.Gate("X", (qs[0],), (qs[1], qs[2])))
            else:
                kind = ["RX", "RY", "RZ", "P", "RXX", "RYY", "RZZ"][int(rng.integers(7))]
                nt = 2 if kind in ("RXX", "RYY", "RZZ") else 1
                if nt > n:
                    continue
                gates.append(W.Gate(kind, tuple(qs[:nt]), (), (float(rng.uniform(0, 6)),), pidx, 1.5))
                pidx += 1
        terms = [(0, int(rng.integers(0, 1 << n)), float(rng.standard_normal())) for _ in range(5)]
        circs.append((n, gates, terms, pidx))
        refs.append((n, gates, terms, pidx))
    ev, grads = D.Batch(circs).run()
    for i, (n, gates, terms, np_) in enumerate(refs):
        psi0 = W.zero_state(n)
        assert abs(ev[i] - orc.energy(psi0, n, gates, terms)) <= 1e-11
        if np_:
            ps = orc.param_shift_grad(psi0, n, gates, terms, np_)
            assert np.max(np.abs(grads[i] - ps)) <= 1e-10 * max(1.0, np.max(np.abs(ps)))


def test_batch_wide_circuits_on_side_streams():
    """Circuits of 15+ qubits run gate by gate with the grid-wide Alg. 3
    kernels on side streams, next to the persistent kernel."""
    insts, circs, theta = _qaoa_circuits(10, 77, widths=(8, 12, 16, 18), pmax=2)
    rng = np.random.default_rng(78)
    for graph in (False, True):
        b = D.Batch(circs, graph=graph)
        for rep in range(2):
            th = theta if rep == 0 else rng.uniform(0, math.pi, theta.size)
            ev, grads = b.run(th)
            k = 0
            for i, inst in enumerate(insts):
                t = th[k:k + 2 * inst.p]
                k += 2 * inst.p
                gates = W.qaoa_gates(inst.n, inst.edges, t[0::2], t[1::2])
                psi0 = W.zero_state(inst.n)
                e = orc.energy(psi0, inst.n, gates, inst.terms)
                assert abs(ev[i] - e) <= 1e-11 * max(1.0, abs(e)), (graph, rep, inst.n)
                if inst.n == 16 and rep == 0:
                    ps = orc.param_shift_grad(psi0, inst.n, gates, inst.terms, 2 * inst.p)
                    assert np.max(np.abs(grads[i] - ps)) <= 1e-10 * max(1.0, np.max(np.abs(ps))), (graph, inst.n)


def test_batch_rejects_wide_gates():
    with pytest.raises(D.DiaqError):
        D.Batch([(6, [W.Gate("MATRIX", (0, 1, 2), matrix=np.eye(8))], [(0, 1, 1.0)], 0)])
    with pytest.raises(ValueError):
        D.Batch([(4, [W.h(0)], [(1, 0, 1.0)], 0)])
