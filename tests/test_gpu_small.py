"""The one-launch path of plan.kron on small states: the whole circuit in
one workgroup's LDS, gate by gate (Alg. 3 cosets), gates packed into the
kernel arguments with one launch per run that fits.  Checked against the
oracle for every gate shape (one to three targets, up to three controls,
diagonal and dense, custom matrices), at every register size the path
takes, in complex128 and complex64, on circuits long enough to need several
launches, replayed from a recorded circuit graph, and against the
per-operation Alg. 3 kernels."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host
from tests.test_gpu_kernels import _random_gate

pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    c = D.context()
    saved = D.get_tuning(c)
    yield c
    D.set_tuning(c, **saved)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 12, 13])
def test_small_random_circuits(ctx, n):
    rng = np.random.default_rng(4000 + n)
    gates = [_random_gate(rng, n) for _ in range(120)]
    x = W.random_state(n, n)
    ref = orc.apply_circuit(x, n, gates)
    for plan in (D.make_plan(kron=True), D.make_plan(kron=True, fuse=True, max_fused_qubits=5)):
        psi = to_dev(x)
        D.apply_circuit(gates, psi, plan=plan)
        assert_state_close(to_host(psi), ref, 1e-12, "n=%d" % n)
    psi32 = to_dev(x, torch.complex64)
    D.apply_circuit(gates, psi32, plan=D.make_plan(kron=True))
    assert_state_close(to_host(psi32), ref, 1e-5, "n=%d c64" % n, l2tol=1e-4)


def test_small_matches_per_operation_kernels(ctx):
    """Every circuit of the benchmark shapes: the LDS path against the
    per-operation kernels (small path off) and the oracle."""
    for name, n, gates, x in [("ghz", 12, W.ghz(12), W.zero_state(12)),
                              ("qft", 13, W.qft(13), W.random_state(13, 3)),
                              ("layered", 13, W.random_layered(13, 6, 4), W.zero_state(13)),
                              ("tfim", 12, W.tfim(12, 6), W.random_state(12, 5)),
                              ("hea", 11, W.hea(11, 3, 7)[0], W.zero_state(11))]:
        ref = orc.apply_circuit(x, n, gates)
        plan = D.make_plan(kron=True)
        D.set_tuning(ctx, kron_small_qubits=0)
        a = to_dev(x)
        D.apply_circuit(gates, a, plan=plan)
        D.set_tuning(ctx, kron_small_qubits=-1)
        b = to_dev(x)
        D.apply_circuit(gates, b, plan=plan)
        D.set_tuning(ctx, kron_small_qubits=0)
        assert_state_close(to_host(a), ref, 1e-12, name)
        assert_state_close(to_host(b), ref, 1e-12, name + " per op")


def test_small_ghz_closed_form_and_launches(ctx):
    n = 12
    psi = to_dev(W.zero_state(n))
    D.profile_start(ctx)
    D.apply_circuit(W.ghz(n), psi, plan=D.make_plan(kron=True))
    p = D.profile_stop(ctx)
    got = to_host(psi)
    want = np.zeros(1 << n, complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(got - want)) <= 1e-15
    assert p["spmv_launches"] == 1  # the 12 gates fit one launch
    # a long circuit takes several launches and still matches
    gates = W.random_layered(10, 12, 9)
    x = W.random_state(10, 9)
    psi = to_dev(x)
    D.profile_start(ctx)
    D.apply_circuit(gates, psi, plan=D.make_plan(kron=True))
    p = D.profile_stop(ctx)
    assert p["spmv_launches"] > 1
    assert_state_close(to_host(psi), orc.apply_circuit(x, 10, gates), 1e-12, "layered-10 multi-launch")


def test_small_graph_replays(ctx):
    n = 11
    gates = W.random_layered(n, 4, 2) + W.qft(n)
    x = W.random_state(n, 2)
    ref = orc.apply_circuit(x, n, gates)
    psi = to_dev(x)
    g = D.CircuitGraph(gates, psi, n=n, plan=D.make_plan(kron=True))
    for rep in range(3):
        psi.copy_(to_dev(x))
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert_state_close(to_host(psi), ref, 1e-12, "replay %d" % rep)
        # eager work between replays
        D.apply_circuit(W.ghz(n), to_dev(W.zero_state(n)), plan=D.make_plan(kron=True))
    g.close()


def test_small_limit_and_knob(ctx):
    """n = 14 (complex128 needs 256 KiB of LDS) takes the per-operation
    kernels; the knob caps the register the path takes."""
    for n in (14, 9):
        gates = W.random_layered(n, 2, 1)
        x = W.random_state(n, 1)
        ref = orc.apply_circuit(x, n, gates)
        for knob in (0, 8, -1):
            D.set_tuning(ctx, kron_small_qubits=knob)
            D.profile_start(ctx)
            psi = to_dev(x)
            D.apply_circuit(gates, psi, plan=D.make_plan(kron=True))
            p = D.profile_stop(ctx)
            assert_state_close(to_host(psi), ref, 1e-12, "n=%d knob %d" % (n, knob))
            one_launch = n <= 13 and knob != -1 and (knob == 0 or n <= knob)
            assert (p["spmv_launches"] < len(gates)) == one_launch, (n, knob, p["spmv_launches"])
    with pytest.raises(D.DiaqError):
        D.set_tuning(ctx, kron_small_qubits=15)
