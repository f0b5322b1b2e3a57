"""Every selectable shape of the Alg. 3 kernels, forced through the tuning
knobs: dense 4- and 5-qubit groups one lane per coset, with their rows
split over the waves of a block (8 or 4 rows per wave), or as fp64
matrix-core products (matrix re-read from LDS or held in registers), or
as pipelined matrix-core products (fp32 for complex64); the LDS staging
threshold for groups of up to four qubits (never, default, up to qubit 5);
non-temporal state streams of the per-coset kernels on and off.  Each
variant runs workloads whose groups sit on the lowest qubits, in the
middle and at the top, with folded diagonal factors on wave-varying and
wave-uniform qubits, against the oracle's state (complex128 1e-12,
complex64 1e-5)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host
from tests.test_gpu_kron import _group_gates

pytestmark = pytest.mark.gpu

_KNOBS = {
    "default": {},
    "percoset": {"kron_split": 1},
    "split8": {"kron_split": 2},
    "split4": {"kron_split": 3},
    "nostage": {"kron_stage_qubit": -1},
    "stage6": {"kron_stage_qubit": 6},
    "nt": {"kron_nontemporal": 1},
    "plain_io": {"kron_nontemporal": -1, "kron_split": 2},
    "mfma": {"kron_split": 4},
    "mfma_hold": {"kron_split": 5},
    "split8_gauss": {"kron_split": 6},
    "mfma_pipe": {"kron_split": 7},
    "order_xcd": {"kron_order": 1, "kron_stage_qubit": -1},
    "order_halves": {"kron_order": 2, "kron_stage_qubit": -1},
    "order_scatter": {"kron_order": 3},
}


def _factor_circuit(n, rng):
    gates = []
    for t in (n - 1, n - 3, 5, 2, 0):
        gates.append(W.h(t))
        for k in range(n):
            if k != t and rng.random() < 0.5:
                gates.append(W.cp(float(rng.uniform(0, 6)), k, t))
        gates += [W.Gate("RZZ", (9, 11), (), (0.37,)), W.Gate("RZ", (1,), (), (1.1,)), W.cz(3, 10)]
    gates += [W.cx(n - 3, n - 1)] + [W.cp(0.1 + 0.3 * k, k, n - 1) for k in range(n - 1) if k != n - 3]
    return gates


@pytest.fixture(scope="module")
def cases():
    rng = np.random.default_rng(4242)
    out = []
    n = 17
    out.append(("layered", n, W.random_layered(n, 5, 17), W.zero_state(n)))
    out.append(("factors", n, _factor_circuit(n, rng), W.random_state(n, 18)))
    gates = []
    for S in [(0, 1, 2, 3, 4), (1, 2, 3, 4, 5), (0, 3, 6, 9, 11), (2, 4, 5, 10, 13), (12, 13, 14, 15, 16),
              (0, 1, 2, 3), (2, 7, 8, 12), (5, 6, 7, 8), (13, 14, 15, 16), (0, 5), (4,), (1, 2, 9)]:
        gates += _group_gates(list(S), n)
    out.append(("groups", n, gates, W.random_state(n, 19)))
    return [(name, n, g, x, orc.apply_circuit(x, n, g)) for name, n, g, x in out]


@pytest.fixture()
def ctx():
    c = D.context()
    saved = D.get_tuning(c)
    yield c
    D.set_tuning(c, **saved)


@pytest.mark.parametrize("knobs", list(_KNOBS), ids=list(_KNOBS))
def test_kron_variants_match_oracle(cases, ctx, knobs):
    t = D.get_tuning(ctx)
    t.update(kron_split=0, kron_stage_qubit=0, kron_nontemporal=0, kron_order=0)
    t.update(_KNOBS[knobs])
    D.set_tuning(ctx, **t)
    for name, n, gates, x, ref in cases:
        for kmax in (3, 4, 5):
            plan = D.make_plan(kron=True, fuse=True, max_fused_qubits=kmax)
            psi = to_dev(x)
            D.apply_circuit(gates, psi, plan=plan)
            assert_state_close(to_host(psi), ref, 1e-12, "%s kmax=%d %s" % (name, kmax, knobs))
        psi = to_dev(x)
        D.apply_circuit(gates, psi, plan=D.make_plan(kron=True))
        assert_state_close(to_host(psi), ref, 1e-12, "%s kron %s" % (name, knobs))
        psi32 = to_dev(x, torch.complex64)
        D.apply_circuit(gates, psi32, plan=D.make_plan(kron=True, fuse=True, max_fused_qubits=5))
        assert_state_close(to_host(psi32), ref, 1e-5, "%s kmax=5 c64 %s" % (name, knobs), l2tol=1e-4)


def test_kron_knobs_rejected_out_of_range(ctx):
    for bad in ({"kron_split": 8}, {"kron_stage_qubit": 7}, {"kron_nontemporal": 2}, {"kron_order": 4}):
        with pytest.raises(D.DiaqError):
            D.set_tuning(ctx, **bad)
