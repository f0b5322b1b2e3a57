"""Autotuner: kernel knobs (with the JSON cache) and per-circuit plans; the
tuned path must still match the oracle."""
from __future__ import annotations

import json

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_autotune_kernel_knobs_and_cache(tmp_path):
    cache = str(tmp_path / "tune.json")
    ctx = D.context()
    saved = D.get_tuning(ctx)
    try:
        t = D.autotune(16, cache_path=cache, ctx=ctx)
        assert t["spmv_rows"] in (1, 2, 4) and t["spmv_chunk"] in (1, 3)
        entries = json.load(open(cache))["entries"]
        assert len(entries) == 1 and "|n=16|c128" in entries[0]["key"]
        t2 = D.autotune(16, cache_path=cache, ctx=ctx)  # read back, no timing
        assert t2 == t
        D.autotune(12, cache_path=cache, ctx=ctx)
        assert len(json.load(open(cache))["entries"]) == 2
        # the tuned kernel still computes the product
        n = 16
        gates = W.random_layered(n, 2, 16)
        x = W.random_state(n, 16)
        psi = to_dev(x)
        D.apply_circuit(gates, psi)
        assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), 1e-12, "tuned")
    finally:
        D.set_tuning(ctx, **{k: v for k, v in saved.items()})


@pytest.mark.parametrize("allow_kron", [False, True])
def test_autotune_plan(allow_kron):
    n = 14
    gates = W.random_layered(n, 4, 3) + W.qft(n)
    plan = D.autotune_plan(gates, n, allow_kron=allow_kron, measure=3)
    assert plan.kron in (0, 1) and (allow_kron or plan.kron == 0)
    x = W.random_state(n, 3)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=plan)
    assert_state_close(to_host(psi), orc.apply_circuit(x, n, gates), 1e-12, "autotuned plan")
