"""The C ABI library loads and exports every entry point that include/diaq.h
declares; host-only entry points work without a GPU.  CPU only."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest
import torch

from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diaq.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(diaq_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(D.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return D.load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["diaq_from_gate", "diaq_spmv", "diaq_fuse", "diaq_apply_circuit", "diaq_expect",
                     "diaq_adjoint_grad"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", D.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT\s+(diaq_[a-z0-9_]+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(lib, n)
    # the binding knows every declared entry point
    assert set(_declared()) <= set(D.EXPORTED)


def test_no_torch_types_in_header():
    text = open(HEADER).read()
    assert "torch" not in text.lower().replace("torch's", "")
    assert "at::" not in text and "Tensor" not in text


def test_from_gate_query_offsets_fig2(lib):
    # Fig. 2: Hadamard on each qubit of 4 -> diagonals 0, +-2^q (host-only call)
    for q in range(4):
        offs, nv = D.from_gate_query(W.h(q), 4)
        assert offs.tolist() == [-(1 << q), 0, 1 << q]
        assert nv == 3 * 16 - 2 * (1 << q)


def test_from_gate_query_kinds(lib):
    n = 6
    cases = [
        (W.Gate("Z", (2,)), [0]),
        (W.Gate("RZ", (1,), (), (0.3,)), [0]),
        (W.cz(1, 4), [0]),
        (W.cp(0.4, 0, 5), [0]),
        (W.Gate("RZZ", (1, 3), (), (0.2,)), [0]),
        (W.Gate("X", (3,)), [-8, 8]),
        (W.Gate("Y", (0,)), [-1, 1]),
        (W.cx(0, 3), [-8, 0, 8]),
        (W.swap(1, 4), [-14, 0, 14]),
        (W.Gate("RXX", (0, 2), (), (0.5,)), [-5, -3, 0, 3, 5]),
        (W.u3(0.1, 0.2, 0.3, 5), [-32, 0, 32]),
    ]
    for g, want in cases:
        offs, _ = D.from_gate_query(g, n)
        assert offs.tolist() == want, g


def test_from_gate_query_rejects_bad_gates(lib):
    bad = [
        W.Gate("H", (6,)),                 # qubit out of range
        W.Gate("SWAP", (1, 1)),            # duplicate qubit
        W.Gate("X", (2,), (2,)),           # control == target
        W.Gate("H", (0, 1)),               # wrong target count
        W.Gate("X", (0,), (1, 2, 3, 4)),   # too many controls
    ]
    for g in bad:
        with pytest.raises(D.DiaqError) as ei:
            D.from_gate_query(g, 6)
        assert ei.value.status == 1
    with pytest.raises(D.DiaqError):
        D.from_gate_query(W.Gate("MATRIX", (0,)), 4)  # matrix missing


def test_create_without_gpu_fails_loudly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = lib.diaq_create(0, None, ctypes.byref(h))
    assert st != 0
    with pytest.raises(RuntimeError):
        D.context()


def test_struct_layouts_match_header(tmp_path):
    """Every struct the binding passes by pointer has the header's size and
    field offsets (a C program built from include/diaq.h prints them)."""
    structs = {"diaq_gate_t": D.diaq_gate_t, "diaq_plan_t": D.diaq_plan_t, "diaq_tuning_t": D.diaq_tuning_t,
               "diaq_profile_t": D.diaq_profile_t, "diaq_circuit_t": D.diaq_circuit_t,
               "diaq_chain_step_t": D.diaq_chain_step_t, "diaq_spmv_shape_t": D.diaq_spmv_shape_t}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "diaq.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            name, field, value = line.split()
            got[(name, field)] = int(value)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_plan_count_host_only(lib):
    """diaq_plan_count needs no GPU.  The plain and Alg. 3 byte models are
    recomputed here from the definitions (a one-qubit or CX gate on target
    t stores E = 3N - 2^(t+1) values; an Alg. 3 operation reads and writes
    the state once, a controlled one without factors only its control-on
    half); the fused operation counts are the planner's documented
    figures for the n = 28 layered circuit and QFT-24."""
    n, N, s = 28, 1 << 28, 16
    gates = W.random_layered(n, 20, 28)
    nops, b = D.plan_count(gates, n)
    assert nops == 830
    want = 0.0
    for g in gates:
        t = g.targets[0]
        E = 3 * N - 2 ** (t + 1)
        want += s * (2 * E + 2 * N)
    assert b == pytest.approx(want, rel=1e-12)
    nops, b = D.plan_count(gates, n, D.make_plan(kron=True))
    assert nops == 830
    want = sum(2 * s * N / (2 ** len(g.controls)) for g in gates)
    assert b == pytest.approx(want, rel=1e-12)
    counts = {(False, 2): 284, (False, 3): 154, (True, 4): 97, (True, 5): 78}
    for (kron, k), c in counts.items():
        assert D.plan_count(gates, n, D.make_plan(kron=kron, fuse=True, max_fused_qubits=k))[0] == c, (kron, k)
    assert D.plan_count(W.qft(24), 24, D.make_plan(kron=True, fuse=True, max_fused_qubits=3))[0] == 20
    # the five-qubit cost model: groups whose qubits are all >= 4 (n >= 9)
    # run on the matrix cores, one pass in complex64, so both precisions
    # keep the five-qubit grouping at n = 28; at n = 8 no group qualifies
    # and complex64 (1.8 passes per five-qubit group) keeps the four-qubit
    # grouping while complex128 (1.3) does not
    five = D.make_plan(kron=True, fuse=True, max_fused_qubits=5)
    assert D.plan_count(gates, n, five, dtype=torch.complex64)[0] == 78
    small = W.random_layered(8, 20, 28)
    assert D.plan_count(small, 8, five, dtype=torch.complex64)[0] == 22
    assert D.plan_count(small, 8, five, dtype=torch.complex128)[0] == 17
    for kw in (dict(fuse=True, max_fused_qubits=4), dict(kron=True, fuse=True, max_fused_qubits=6),
               dict(fuse=True, max_fused_qubits=-1)):
        with pytest.raises(D.DiaqError) as ei:
            D.plan_count(gates, n, D.make_plan(**kw))
        assert ei.value.status == 1, kw


_ONE = ["H", "X", "Y", "Z", "S", "T", "SX", "RX", "RY", "RZ", "P", "U3"]
_TWO = ["SWAP", "RXX", "RYY", "RZZ"]


def _random_gate_host(rng, n):
    """A random gate on distinct qubits: a named kind or a custom matrix of
    1..3 targets with a random zero pattern, with up to two controls."""
    qs = [int(q) for q in rng.permutation(n)]
    r = rng.random()
    if r < 0.4:
        kind = _ONE[int(rng.integers(len(_ONE)))]
        targets = qs[:1]
    elif r < 0.6 and n >= 2:
        kind = _TWO[int(rng.integers(len(_TWO)))]
        targets = qs[:2]
    else:
        kind = "MATRIX"
        k = int(rng.integers(1, min(3, n) + 1))
        targets = qs[:k]
    rest = qs[len(targets):]
    nc = int(rng.integers(0, min(2, len(rest)) + 1))
    controls = tuple(rest[:nc])
    params = tuple(float(a) for a in rng.uniform(0.1, 6.0, 3))
    matrix = None
    if kind == "MATRIX":
        d = 1 << len(targets)
        m = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        m[rng.random((d, d)) < 0.5] = 0
        matrix = m
    return W.Gate(kind, tuple(targets), controls, params, matrix=matrix)


def test_from_gate_query_matches_brute_force_expansion(lib):
    """The offset algebra of the expansion (host side, no GPU): for random
    named, controlled and custom-matrix gates at n = 2..6, the offsets
    diaq_from_gate_query reports are exactly the diagonals holding a
    non-zero of the oracle's dense expanded matrix (plus the principal one
    of a controlled gate, whose identity rows sit there), and the value
    count is the sum of their lengths N - |d|."""
    from oracle import oracle as orc
    rng = np.random.default_rng(2024)
    for trial in range(60):
        n = int(rng.integers(2, 7))
        g = _random_gate_host(rng, n)
        offs, nv = D.from_gate_query(g, n)
        A = orc.dense_matrix(n, [g])
        want, _ = orc.dia_from_dense(A)
        assert offs.tolist() == want, (trial, g)
        assert nv == sum((1 << n) - abs(d) for d in want), trial


def test_spmv_shape_host_only(lib):
    """diaq_spmv_shape needs no GPU.  The knob sets of the product-variant
    GPU tests reach every kernel shape (tile groups of 2, 4 and 8 across 1-3
    coupling qubits, 1, 2 and 4 rows per lane, chunks of 1 and 3, streams
    with and without non-temporal hints), workgroup counts cover the state
    exactly once, and principal-diagonal-only gates run in place."""
    from tests.test_gpu_spmv_variants import N_QUBITS, _DEFAULT, _GROUPINGS, _gates
    n = N_QUBITS
    shapes = set()
    for g in _gates():
        for rows in (1, 2, 4):
            for grouping in _GROUPINGS.values():
                for chunk in (1, 3):
                    for nt in (0, -1):
                        t = dict(_DEFAULT)
                        t.update(grouping)
                        t.update(spmv_rows=rows, spmv_chunk=chunk, spmv_nontemporal=nt)
                        s = D.spmv_shape(g, n, **t)
                        if s["in_place"]:
                            assert g.kind == "RZZ"
                            continue
                        rows_wg = s["rows_per_lane"] * s["group"] * 256
                        assert s["blocks"] * rows_wg == 1 << n, (g, t, s)
                        assert s["group"] == 1 << len(s["group_qubits"])
                        assert s["tile_log2"] == 8 + s["rows_per_lane"].bit_length() - 1
                        assert all(q >= s["tile_log2"] for q in s["group_qubits"])
                        shapes.add((s["rows_per_lane"], s["group"], s["chunk"], s["nontemporal"]))
    assert {g for _, g, _, _ in shapes} == {1, 2, 4, 8}, shapes
    assert {r for r, _, _, _ in shapes} == {1, 2, 4}, shapes
    assert {c for _, _, c, _ in shapes} == {1, 3}, shapes
    assert {t for _, _, _, t in shapes} == {0, 1}, shapes
    # the defaults at n = 28: one row per lane; a U3 on qubit 27 pairs its
    # tiles (coupling qubit >= 21); on qubit 9 the XCD runs take over
    s = D.spmv_shape(W.u3(0.1, 0.2, 0.3, 27), 28)
    assert (s["rows_per_lane"], s["group"], s["group_qubits"]) == (1, 2, [27])
    s = D.spmv_shape(W.u3(0.1, 0.2, 0.3, 9), 28)
    assert (s["group"], s["xcd_run_log2"]) == (1, 2)
    s = D.spmv_shape(W.Gate("RZ", (5,), (), (0.3,)), 28)
    assert s["in_place"] == 1
    # tile orders apply where neither XCD runs nor partner alternation do
    s = D.spmv_shape(W.u3(0.1, 0.2, 0.3, 14), 28, spmv_order=2, spmv_group_bits=-1)
    assert (s["xcd_run_log2"], s["pair_bit"], s["tile_order"]) == (0, 0, 2)
    s = D.spmv_shape(W.u3(0.1, 0.2, 0.3, 9), 28, spmv_order=2)
    assert (s["xcd_run_log2"], s["tile_order"]) == (2, 0)
    with pytest.raises(D.DiaqError):
        D.spmv_shape(W.u3(0.1, 0.2, 0.3, 28), 28)
    with pytest.raises(D.DiaqError):
        D.spmv_shape(W.u3(0.1, 0.2, 0.3, 3), 28, spmv_rows=3)


def test_spmv_shape_packed_complex64(lib):
    """Complex64 products with even offsets run on pairs of amplitudes: the
    units of a launch cover the state once, tiles and paired coupling qubits
    are reported in amplitudes; a coupling on qubit 0, complex128, or the
    knob at -1 keep one amplitude per access."""
    c64 = torch.complex64
    n = 28
    for q in (1, 5, 9, 14, 27):
        s = D.spmv_shape(W.u3(0.1, 0.2, 0.3, q), n, c64)
        assert s["packed"] == 1, q
        units = s["rows_per_lane"] * s["group"] * 256
        assert s["blocks"] * units * 2 == 1 << n, (q, s)
        assert s["tile_log2"] == 9 + s["rows_per_lane"].bit_length() - 1, (q, s)
        assert all(g >= s["tile_log2"] for g in s["group_qubits"]), (q, s)
    assert D.spmv_shape(W.u3(0.1, 0.2, 0.3, 27), n, c64)["group_qubits"] == [27]
    assert D.spmv_shape(W.u3(0.1, 0.2, 0.3, 0), n, c64)["packed"] == 0
    assert D.spmv_shape(W.cx(5, 0), n, c64)["packed"] == 0
    assert D.spmv_shape(W.cx(0, 5), n, c64)["packed"] == 1
    assert D.spmv_shape(W.u3(0.1, 0.2, 0.3, 5), n, c64, spmv_pack=-1)["packed"] == 0
    assert D.spmv_shape(W.u3(0.1, 0.2, 0.3, 5), n)["packed"] == 0
    s = D.spmv_shape(W.Gate("RZ", (5,), (), (0.3,)), n, c64)
    assert (s["in_place"], s["packed"], s["blocks"]) == (1, 1, (1 << (n - 1)) // 256)
    with pytest.raises(D.DiaqError):
        D.spmv_shape(W.u3(0.1, 0.2, 0.3, 5), n, c64, spmv_pack=1)


def test_small_circuit_kernel_reads_gates_from_the_argument_segment():
    """The one-launch small-state kernel reads its packed gates in place in
    the kernel-argument segment: no private (scratch) copy of its arguments,
    whose address would not be a constant-space address.  Checked on the
    compiler's resource report for gfx950 (host-only)."""
    src = os.path.join(ROOT, "paper_2405_01250_amd", "csrc", "small.hip")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = subprocess.run([hipcc, "-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
                          os.path.dirname(src), "--offload-arch=gfx950", "--cuda-device-only", "-c", src, "-o",
                          os.devnull, "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr[-2000:]
    scratch, cur = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and cur:
            scratch[cur] = int(m.group(1))
    kernels = {k: v for k, v in scratch.items() if "small_circuit_kernel" in k}
    assert len(kernels) == 2, scratch
    assert all(v == 0 for v in kernels.values()), kernels
