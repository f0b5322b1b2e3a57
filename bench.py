"""Benchmark of the DiaQ hot path on one MI355X.

Workload (one "step"): the random layered circuit on n = 28 qubits -- 20
layers of U3 on every qubit plus alternating CX brickwork, 830 gates, seed
28, complex128 -- applied to a resident state vector, every gate expanded
to its DiaQ diagonals and applied by the DiaQ SpMV; then the Ising energy
<psi| sum_i a_i Z_i Z_{i+1} |psi> of the result (one diagonal).

Prints one JSON line.  ``value`` is the whole step's effective HBM rate:
algorithmic bytes (expansion writes E elements, each product reads E
elements plus x and writes y) divided by wall time of the timed steps.
``roofline`` describes the dominant kernel, the DiaQ SpMV, from HIP events
recorded around each of its launches inside the timed region.
``cpu_baseline`` times the CPU oracle on a bounded sample of the same
circuit on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, vendor peak


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--layers", type=int, default=20)
    ap.add_argument("--seed", type=int, default=28)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU-oracle sample (0 disables it)")
    ap.add_argument("--extras", type=int, default=1, help="also time adjoint vs parameter shift (HEA n=20)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of autotuned product-kernel knobs (read if it holds this size, else written)")
    ap.add_argument("--mode", default="bench", choices=["bench", "copy", "sweep", "plan"],
                    help="copy: run a plain device copy of 2^n complex elements (counter calibration); "
                         "sweep: single-gate rates per target qubit (one JSON line per gate)")
    ap.add_argument("--sweep-plan", default="dia", choices=["dia", "kron", "groups"],
                    help="sweep: dia = expansion + DiaQ SpMV per gate; kron = Alg. 3 in-place product per "
                         "gate; groups = Alg. 3 fused dense groups of 3, 4 and 5 consecutive qubits")
    ap.add_argument("--sweep-dtypes", default="c128,c64", help="sweep: dtypes to run")
    ap.add_argument("--sweep-gates", default="", help="sweep: comma-separated gate shapes to run (default all)")
    ap.add_argument("--sweep-qubits", default="", help="sweep: first,last target qubit (default all)")
    ap.add_argument("--plan", default="kron+fuse4",
                    help="mode plan: the benchmark circuit under this plan only, e.g. kron, kron+fuse4, dia+fuse3")
    ap.add_argument("--knobs", default="", help="JSON object of tuning knobs set after autotuning "
                                                "(fields of diaq_tuning_t), e.g. '{\"kron_split\": 2}'")
    return ap.parse_args()


def copy_mode(a):
    """A plain copy of known size (torch's device copy, the counter
    calibration), then the library's own streaming copy kernel: each reads
    and writes 2^n elements."""
    import torch
    N = 1 << a.n
    tdt = torch.complex128 if a.dtype == "c128" else torch.complex64
    x = torch.ones(N, dtype=tdt, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    nb = x.numel() * x.element_size()
    # the library's streaming copy kernel, the copy reference of the tables
    from paper_2405_01250_amd import diaq as D
    D.copy(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        D.copy(x, y)
    torch.cuda.synchronize()
    dl = (time.perf_counter() - t0) / a.steps
    print(json.dumps({"mode": "copy", "bytes_read": nb, "bytes_written": nb, "copies": a.steps,
                      "GBps": round(2 * nb / dt / 1e9, 1), "diaq_copy_GBps": round(2 * nb / dl / 1e9, 1)}),
          flush=True)


def _traffic_from_profiles(kernel_src: str):
    """HBM traffic per SpMV launch measured with rocprofv3 counters, if the
    committed summary was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "spmv_hbm_traffic_n28.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    want = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    if kv.get("spmv_source_sha256_16") != want:
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(n, gates, budget_s, s_bytes, repeats=3):
    """The CPU oracle, as it stands, on the first gates of the same circuit:
    `repeats` bounded samples on every host core, then on one core.  GB/s
    follows the oracle's own byte model: it applies each gate in place,
    reading and writing the 2^n-element state once (2 N s bytes per gate).
    Also the oracle's parameter-shift gradient of the HEA n = 20 workload,
    timed on a few of its 640 shifted energies."""
    import numpy as np

    from oracle import oracle as orc
    from paper_2405_01250_amd import inputs as W

    orc.build()
    per_gate = 2.0 * (1 << n) * s_bytes

    def sample(budget):
        psi = W.zero_state(n)
        done = 0
        t0 = time.perf_counter()
        for g in gates:
            orc.apply_gate(psi, n, g)
            done += 1
            if time.perf_counter() - t0 >= budget:
                break
        return done, time.perf_counter() - t0

    def stats(runs):
        rates = np.array([d / t for d, t in runs])
        return {"value": round(float(rates.mean()) * per_gate / 1e9, 2),
                "std": round(float(rates.std()) * per_gate / 1e9, 2), "unit": "GB/s",
                "gates_per_s": round(float(rates.mean()), 3), "gates_per_s_std": round(float(rates.std()), 3),
                "runs": [{"gates": d, "s": round(t, 3)} for d, t in runs]}

    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    orc.set_threads(cores)
    cores = orc.get_threads()
    sample(1.0)  # warm-up: pages the state in
    all_cores = stats([sample(budget_s / repeats) for _ in range(repeats)])
    orc.set_threads(1)
    one = stats([sample(max(1.0, budget_s / (3 * repeats))) for _ in range(repeats)])
    orc.set_threads(cores)
    # the other workload shapes, whole circuits, two runs each (bounded:
    # GHZ-28 is 28 gates, QFT-24 312 gates on 2^24 amplitudes, and 8
    # circuits of the QAOA batch)
    others = {}
    for name, nn, gl, x0f in (("ghz28", 28, W.ghz(28), lambda: W.zero_state(28)),
                              ("qft24", 24, W.qft(24), lambda: W.random_state(24, 24))):
        runs = []
        for _ in range(2):
            psi = x0f()
            t0 = time.perf_counter()
            orc.apply_circuit(psi, nn, gl, copy=False)
            runs.append(time.perf_counter() - t0)
        r = np.array(runs)
        others[name] = {"gates": len(gl), "s": round(float(r.mean()), 4), "s_std": round(float(r.std()), 4),
                        "gates_per_s": round(len(gl) / float(r.mean()), 2),
                        "GBps": round(len(gl) * 2.0 * (1 << nn) * s_bytes / float(r.mean()) / 1e9, 2)}
        del psi
    insts = W.qaoa_batch(512, 512)[:8]
    t0 = time.perf_counter()
    for inst in insts:
        orc.energy(W.zero_state(inst.n), inst.n, inst.gates, inst.terms)
    dq = time.perf_counter() - t0
    others["qaoa_batch_sample"] = {"circuits": len(insts), "s": round(dq, 3), "circuits_per_s": round(len(insts) / dq, 2),
                                   "what": "energies (no gradients) of the first 8 circuits of the 512-circuit batch"}
    # gradient baseline: parameter shift needs 2 energies per occurrence
    hn, layers = 20, 8
    hg, theta, terms = W.hea(hn, layers, 20)
    x0 = W.zero_state(hn)
    t0 = time.perf_counter()
    k = 0
    while k < 4:
        orc.energy(x0, hn, hg, terms)
        k += 1
    e_s = (time.perf_counter() - t0) / k
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = dict(all_cores)
    out.update({"cores": cores, "kind": "oracle", "host_cpu": model,
                "host_cpus_visible": len(os.sched_getaffinity(0)),
                "sample": "%d runs of about %.0f s each: the first gates of the n=%d random layered circuit "
                          "from |0..0>, complex128, in-place bit-manipulation oracle (C, OpenMP); GB/s = "
                          "gates/s x 2 N s (the oracle's in-place read + write of the state); mean and std over "
                          "the runs" % (repeats, budget_s / repeats, n),
                "one_core": one,
                "workloads": others,
                "hea20_param_shift": {"energy_s": round(e_s, 3), "shifted_energies": 2 * len(theta),
                                      "grads_per_s": round(1.0 / (2 * len(theta) * e_s), 5),
                                      "sample": "%d energies of the HEA n=20 circuit (480 gates) timed on all "
                                                "cores; a full gradient takes 2 x %d of them" % (k, len(theta))}})
    return out


def _group_circuit(W, rng, qs):
    """Gates that the Alg. 3 planner fuses into one dense operation on the
    qubits qs: a CX chain along them (which opens one operation over all of
    them), a U3 on each, the chain again and a U3 on each again."""
    gates = []
    for _ in range(2):
        gates += [W.cx(qs[j], qs[j + 1]) for j in range(len(qs) - 1)]
        gates += [W.u3(*rng.uniform(0, 2 * math.pi, 3), q) for q in qs]
    return gates


def sweep_mode(a):
    """Single-operation sweep at 2^n amplitudes, rates from HIP events around
    every launch.  dia: each gate shape on each target qubit, expanded and
    applied by the DiaQ SpMV (algorithmic bytes s*E written by the expansion,
    s*(E + 2N) moved by the product).  kron: the same gates by Alg. 3 in
    place (2 s N per gate, 2 s N / 2 for a controlled one).  groups: a
    circuit on k = 3, 4, 5 consecutive qubits starting at each position,
    fused by the planner (one dense operation, or more where its cost model
    prefers narrower groups; `ops` says how many; 2 s N each).  Rates are
    per operation."""
    import numpy as np
    import torch

    from paper_2405_01250_amd import diaq as D
    from paper_2405_01250_amd import inputs as W

    n = a.n
    rng = np.random.default_rng(a.seed)
    ctx = D.context()
    dts = {"c128": torch.complex128, "c64": torch.complex64}
    for dt_name in a.sweep_dtypes.split(","):
        tdt = dts[dt_name]
        psi = torch.from_numpy(W.random_state(n, a.seed)).to("cuda:0").to(tdt)
        scratch = torch.empty_like(psi)
        D.autotune(n, dtype=tdt, cache_path=a.tune_cache, ctx=ctx)
        if a.knobs:
            D.set_tuning(ctx, **json.loads(a.knobs))
        tuning = D.get_tuning(ctx)
        print(json.dumps({"mode": "sweep", "dtype": dt_name, "n": n, "plan": a.sweep_plan, "tuning": tuning}),
              flush=True)
        cases = []
        if a.sweep_plan in ("dia", "kron"):
            shapes = [("U3", lambda q: W.u3(*rng.uniform(0, 2 * math.pi, 3), q)),
                      ("CX", lambda q: W.cx(0, q) if q else W.cx(1, 0)),
                      ("CXhi", lambda q: W.cx(n - 1 if q != n - 1 else n - 2, q)),
                      ("RZ", lambda q: W.Gate("RZ", (q,), (), (0.7,))),
                      ("CZ", lambda q: W.Gate("Z", (q,), (0 if q else 1,))),
                      ("SWAP", lambda q: W.swap(q, n - 1 - q) if q != n - 1 - q else W.swap(q, 0))]
            plan = D.make_plan(kron=True) if a.sweep_plan == "kron" else None
            for name, make in shapes:
                for q in range(n):
                    cases.append((name, q, [make(q)], plan))
        else:
            for k in (3, 4, 5):
                plan = D.make_plan(kron=True, fuse=True, max_fused_qubits=k)
                for q in range(n - k + 1):
                    gates = _group_circuit(W, rng, list(range(q, q + k)))
                    cases.append(("G%d" % k, q, gates, plan))
        if a.sweep_gates:
            keep = set(a.sweep_gates.split(","))
            cases = [c for c in cases if c[0] in keep]
        if a.sweep_qubits:
            lo, hi = (int(v) for v in a.sweep_qubits.split(","))
            cases = [c for c in cases if lo <= c[1] <= hi]
        for name, q, g, plan in cases:
            arr = D.gate_array(g)
            D.apply_circuit(g, psi, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
            torch.cuda.synchronize()
            D.profile_start(ctx)
            for _ in range(a.steps):
                D.apply_circuit(g, psi, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
            p = D.profile_stop(ctx)
            out = {"mode": "sweep", "plan": a.sweep_plan, "dtype": dt_name, "n": n, "gate": name, "q": q,
                   "ops": D.plan_count(g, n, plan, dtype=tdt)[0],
                   "spmv_us": round(p["spmv_ms"] / max(1, p["spmv_launches"]) * 1e3, 1),
                   "spmv_GBps": round(p["spmv_bytes"] / p["spmv_ms"] / 1e6, 1) if p["spmv_ms"] else None,
                   "expand_GBps": round(p["expand_bytes"] / p["expand_ms"] / 1e6, 1) if p["expand_ms"] else None}
            print(json.dumps(out), flush=True)
        del psi, scratch
        torch.cuda.empty_cache()


def _plan_of(name, D):
    """'dia', 'kron', 'dia+fuseK' or 'kron+fuseK' -> a diaq_plan_t."""
    base, _, fuse = name.partition("+fuse")
    if base not in ("dia", "kron"):
        raise SystemExit("unknown plan %r" % name)
    kw = {"kron": base == "kron"}
    if fuse:
        kw.update(fuse=True, max_fused_qubits=int(fuse))
    return D.make_plan(**kw)


def plan_mode(a):
    """The benchmark circuit under one plan (--plan) for --warmup untimed
    and --steps timed runs: logical gates/s, and the operations' algorithmic
    rate from HIP events around every launch (Alg. 3: 2 N s per operation,
    N s for a controlled one without factors)."""
    import torch

    from paper_2405_01250_amd import diaq as D
    from paper_2405_01250_amd import inputs as W

    n = a.n
    tdt = torch.complex128 if a.dtype == "c128" else torch.complex64
    gates = W.random_layered(n, a.layers, a.seed)
    arr = D.gate_array(gates)
    plan = _plan_of(a.plan, D)
    ctx = D.context()
    D.autotune(n, dtype=tdt, cache_path=a.tune_cache, ctx=ctx)
    if a.knobs:
        D.set_tuning(ctx, **json.loads(a.knobs))
    state = torch.zeros(1 << n, dtype=tdt, device="cuda:0")
    state[0] = 1
    scratch = torch.empty_like(state)
    nops, nbytes = D.plan_count(gates, n, plan, dtype=tdt)
    for _ in range(max(1, a.warmup)):
        D.apply_circuit(gates, state, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    D.profile_start(ctx)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        D.apply_circuit(gates, state, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    p = D.profile_stop(ctx)
    print(json.dumps({"mode": "plan", "plan": a.plan, "dtype": a.dtype, "n": n, "gates": len(gates), "ops": nops,
                      "steps": a.steps, "ms_per_step": round(dt / a.steps * 1e3, 3),
                      "gates_per_s": round(len(gates) * a.steps / dt, 2),
                      "op_launches": p["spmv_launches"], "op_avg_us": round(p["spmv_ms"] / max(1, p["spmv_launches"]) * 1e3, 2),
                      "op_GBps": round(p["spmv_bytes"] / p["spmv_ms"] / 1e6, 1) if p["spmv_ms"] else None,
                      "op_bytes_per_launch": p["spmv_bytes"] / max(1, p["spmv_launches"]),
                      "tuning": D.get_tuning(ctx)}), flush=True)


def main():
    a = _args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if a.mode == "copy":
        copy_mode(a)
        return
    if a.mode == "sweep":
        sweep_mode(a)
        return
    if a.mode == "plan":
        plan_mode(a)
        return
    import numpy as np
    import torch

    from paper_2405_01250_amd import diaq as D
    from paper_2405_01250_amd import inputs as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    n = a.n
    N = 1 << n
    s = 16 if a.dtype == "c128" else 8
    tdt = torch.complex128 if a.dtype == "c128" else torch.complex64
    gates = W.random_layered(n, a.layers, a.seed)
    arr = D.gate_array(gates)

    def e_of(g):
        offs, nv = D.from_gate_query(g, n)
        return nv

    E = [e_of(g) for g in gates]
    step_bytes = sum(s * e + s * (e + 2 * N) for e in E)  # expansion + product
    spmv_bytes = sum(s * (e + 2 * N) for e in E)

    # observable: Ising energy sum a_i Z_i Z_{i+1} (one diagonal)
    rng = np.random.default_rng(a.seed)
    coef = rng.standard_normal(n - 1)
    terms = [(0, (1 << i) | (1 << (i + 1)), float(coef[i])) for i in range(n - 1)]
    Hzz = D.from_pauli_sum(n, terms, dtype=tdt)

    state = torch.zeros(N, dtype=tdt, device=dev)
    state[0] = 1
    scratch = torch.empty_like(state)
    ctx = D.context()

    # product-kernel knobs chosen by the autotuner at this size (untimed)
    tuning = D.autotune(n, dtype=tdt, cache_path=a.tune_cache, ctx=ctx)
    if a.knobs:
        D.set_tuning(ctx, **json.loads(a.knobs))
        tuning = D.get_tuning(ctx)

    def step():
        D.apply_circuit(gates, state, n=n, scratch=scratch, marshalled=arr, ctx=ctx)
        return D.expect(Hzz, state)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    D.profile_start(ctx)
    t0 = time.perf_counter()
    energies, step_ms = [], []
    for _ in range(a.steps):
        ts = time.perf_counter()
        energies.append(step())  # reads the energy back: the step ends synchronised
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = D.profile_stop(ctx)
    dt = t1 - t0
    ms_per_step = dt / a.steps * 1e3
    norm = float(torch.linalg.vector_norm(state).item())

    spmv_avg_ms = prof["spmv_ms"] / max(1, prof["spmv_launches"])
    spmv_bytes_per_launch = prof["spmv_bytes"] / max(1, prof["spmv_launches"])
    achieved = spmv_bytes_per_launch / (spmv_avg_ms * 1e-3) / 1e9
    traffic = _traffic_from_profiles(os.path.join(ROOT, "paper_2405_01250_amd", "csrc", "spmv.hip"))

    out = {
        "metric": "DiaQ SpMV effective HBM GB/s + gates/s at n=28; adjoint grads/s vs plain",
        "value": round(step_bytes * a.steps / dt / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.dtype,
        "data": "synthetic",
        "config": {"workload": "random layered circuit n=%d, %d layers (U3 on every qubit + CX brickwork), "
                               "%d gates, seed %d, |0..0>, plain per-gate expansion + DiaQ SpMV, then "
                               "<Z_iZ_i+1> energy" % (n, a.layers, len(gates), a.seed),
                   "n": n, "gates": len(gates), "layers": a.layers},
        "gates_per_s": round(len(gates) * a.steps / dt, 2),
        "step_ms": {"mean": round(float(np.mean(step_ms)), 3), "std": round(float(np.std(step_ms)), 3),
                    "median": round(float(np.median(step_ms)), 3), "steps": len(step_ms)},
        "tuning": tuning,
        "spmv_GBps": round(achieved, 1),
        "expand_GBps": round(prof["expand_bytes"] / (prof["expand_ms"] * 1e-3) / 1e9, 1)
        if prof["expand_ms"] else None,
        "spmv_share_of_step": round(prof["spmv_ms"] / (dt * 1e3), 3),
        "check": {"final_norm": norm, "energy": energies[-1].real},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "spmv_kernel (DiaQ SpMV, Alg. 2)",
                     "bytes_per_launch": spmv_bytes_per_launch, "avg_launch_ms": round(spmv_avg_ms, 4),
                     "launches": prof["spmv_launches"]},
    }
    if abs(norm - 1) > 1e-9:
        out["check"]["error"] = "norm drifted"

    if a.extras:
        p = D.autotune_plan(gates, n, dtype=tdt, allow_kron=True, measure=3, ctx=ctx)
        out["autotuned_plan"] = {"fuse": p.fuse, "max_fused_qubits": p.max_fused_qubits, "kron": p.kron}
        xs = min(a.steps, 3)  # timed runs of each extra
        out["variants"] = [fused_extra(D, gates, state, scratch, ctx, n, xs, **kw)
                           for kw in ({"fuse": True, "max_fused_qubits": 2}, {"fuse": True, "max_fused_qubits": 3},
                                      {"kron": True}, {"kron": True, "fuse": True, "max_fused_qubits": 2},
                                      {"kron": True, "fuse": True, "max_fused_qubits": 3},
                                      {"kron": True, "fuse": True, "max_fused_qubits": 4},
                                      {"kron": True, "fuse": True, "max_fused_qubits": 5})]
        if a.dtype == "c128":
            out["c64"] = c64_extra(D, W, torch, gates, xs)
        out["tfim"] = tfim_extra(D, W, torch, ctx, state, scratch, tdt)
        out["ghz12"] = ghz_extra(D, W, torch)
        if a.dtype == "c128":
            out["qft"] = qft_extra(D, W, torch, ctx)
        out["matrix"] = matrix_extra(D, W)
        out["adjoint"] = adjoint_extra(D, W, torch, dev)
        out["batch"] = batch_extra(D, W, torch, dev)
    if a.cpu_seconds > 0:
        del state, scratch, Hzz
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(n, gates, a.cpu_seconds, s)
    print(json.dumps(out), flush=True)


def fused_extra(D, gates, state, scratch, ctx, n, steps, **kw):
    """The same circuit under another plan -- gate-level fusion (plan.fuse)
    and/or Alg. 3 in-place products (plan.kron): logical gates/s and the
    algorithmic rate of the operations actually run."""
    import torch
    plan = D.make_plan(**kw)
    kmax = kw.get("max_fused_qubits", 0)
    nops, nbytes = D.plan_count(gates, n, plan)
    arr = D.gate_array(gates)
    D.apply_circuit(gates, state, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    D.profile_start(ctx)
    t0 = time.perf_counter()
    for _ in range(steps):
        D.apply_circuit(gates, state, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = D.profile_stop(ctx)
    pg = prof["spmv_bytes"] / (prof["spmv_ms"] * 1e-3) / 1e9 if prof["spmv_ms"] else None
    if kw.get("kron"):
        kern = ("kron_split_kernel / kron_mfmap_kernel / kron_apply_kernel / kron_lds_kernel (Alg. 3, dense "
                "groups of up to %d qubits)" % kmax if kmax > 3
                else "kron_apply_kernel / kron_lds_kernel / kron_diag_kernel (Alg. 3)")
    else:
        kern = "spmv_kernel (DiaQ SpMV, Alg. 2)"
    return {"plan": ("kron" if kw.get("kron") else "dia") + ("+fuse%d" % kmax if kw.get("fuse") else ""),
            "ops": nops, "gates": len(gates), "ms_per_step": round(dt / steps * 1e3, 3),
            "gates_per_s": round(len(gates) * steps / dt, 2), "GBps": round(nbytes * steps / dt / 1e9, 1),
            "product_GBps": round(pg, 1) if pg else None,
            "product_frac": round(pg / HBM_PEAK_GBPS, 4) if pg else None, "product_kernel": kern,
            "expand_GBps": round(prof["expand_bytes"] / (prof["expand_ms"] * 1e-3) / 1e9, 1)
            if prof["expand_ms"] else None}


def c64_extra(D, W, torch, gates, steps):
    """The same circuit on the plain path in complex64 (8-byte amplitudes):
    gates/s and the kernels' rates, with the autotuned knobs for complex64
    (the complex128 knobs are restored afterwards); also its time under the
    Alg. 3 plans with groups of up to four and up to five qubits."""
    n = max(max(g.targets + tuple(g.controls)) for g in gates) + 1
    ctx = D.context()
    saved = D.get_tuning(ctx)
    D.autotune(n, dtype=torch.complex64, ctx=ctx)
    psi = torch.zeros(1 << n, dtype=torch.complex64, device="cuda:0")
    psi[0] = 1
    scratch = torch.empty_like(psi)
    arr = D.gate_array(gates)
    D.apply_circuit(gates, psi, n=n, scratch=scratch, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    D.profile_start(ctx)
    t0 = time.perf_counter()
    for _ in range(steps):
        D.apply_circuit(gates, psi, n=n, scratch=scratch, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    p = D.profile_stop(ctx)
    norm = float(torch.linalg.vector_norm(psi.to(torch.complex128)).item())
    # the Alg. 3 plan with groups of up to four qubits, in complex64
    plan = D.make_plan(kron=True, fuse=True, max_fused_qubits=4)
    D.apply_circuit(gates, psi, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        D.apply_circuit(gates, psi, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    dk = time.perf_counter() - t0
    # and with groups of up to five qubits (those whose qubits are all >= 4
    # on the fp32 matrix cores)
    plan5 = D.make_plan(kron=True, fuse=True, max_fused_qubits=5)
    D.apply_circuit(gates, psi, n=n, scratch=scratch, plan=plan5, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        D.apply_circuit(gates, psi, n=n, scratch=scratch, plan=plan5, marshalled=arr, ctx=ctx)
    torch.cuda.synchronize()
    d5 = time.perf_counter() - t0
    D.set_tuning(ctx, **saved)
    del psi, scratch
    torch.cuda.empty_cache()
    return {"workload": "random layered n=%d, %d gates, complex64, plain path" % (n, len(gates)),
            "gates_per_s": round(len(gates) * steps / dt, 2), "ms_per_step": round(dt / steps * 1e3, 1),
            "spmv_GBps": round(p["spmv_bytes"] / p["spmv_ms"] / 1e6, 1),
            "expand_GBps": round(p["expand_bytes"] / p["expand_ms"] / 1e6, 1), "final_norm": norm,
            "kron_fuse4_gates_per_s": round(len(gates) * steps / dk, 1), "kron_fuse4_ms": round(dk / steps * 1e3, 2),
            "kron_fuse5_gates_per_s": round(len(gates) * steps / d5, 1), "kron_fuse5_ms": round(d5 / steps * 1e3, 2)}


def tfim_extra(D, W, torch, ctx, state, scratch, tdt):
    """Hamiltonian-simulation workload: Trotterised 1D TFIM (28 spins,
    J = hx = 1, 20 steps of dt = 0.05, 1100 gates) from |0..0>, run under
    each plan; the average magnetization must agree across plans."""
    n, steps, dt_ = W.TFIM_N, W.TFIM_STEPS, W.TFIM_DT
    gates = W.tfim(n, steps, dt_)
    M = D.from_pauli_sum(n, W.magnetization_terms(n), dtype=tdt)
    arr = D.gate_array(gates)
    out = {"workload": "1D TFIM Trotter circuit, n=%d, %d steps of dt=%g, J=hx=1, |0..0>, %d gates "
                       "(RZZ chain + RX layer per step); observable: average magnetization" % (n, steps, dt_, len(gates)),
           "gates": len(gates), "plans": []}
    mags = []
    for kw in ({}, {"fuse": True, "max_fused_qubits": 3}, {"kron": True},
               {"kron": True, "fuse": True, "max_fused_qubits": 3},
               {"kron": True, "fuse": True, "max_fused_qubits": 5}):
        plan = D.make_plan(**kw) if kw else None
        nops, nbytes = D.plan_count(gates, n, plan, dtype=tdt)
        for _ in range(2):  # the first run sizes the workspaces; the second is timed
            state.zero_()
            state[0] = 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            D.apply_circuit(gates, state, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        mags.append(D.expect(M, state).real)
        out["plans"].append({"plan": ("kron" if kw.get("kron") else "dia")
                             + ("+fuse%d" % kw["max_fused_qubits"] if kw.get("fuse") else ""),
                             "ops": nops, "ms": round(dt * 1e3, 2), "gates_per_s": round(len(gates) / dt, 1),
                             "GBps": round(nbytes / dt / 1e9, 1)})
    out["magnetization"] = mags[0]
    out["max_magnetization_diff"] = max(abs(m - mags[0]) for m in mags)
    return out


def ghz_extra(D, W, torch, reps=200):
    """GHZ-12 (H then 11 CX from |0..0>, a 64 KiB state): microseconds per
    gate when the host plans and launches every call, against the same
    launches replayed from a recorded circuit graph."""
    n = 12
    gates = W.ghz(n)
    arr = D.gate_array(gates)
    psi = torch.zeros(1 << n, dtype=torch.complex128, device="cuda:0")
    scratch = torch.empty_like(psi)
    out = {"workload": "GHZ-12 from |0..0>, %d gates" % len(gates), "plans": []}
    for name, plan in (("dia", None), ("kron", D.make_plan(kron=True)),
                       ("kron+fuse3", D.make_plan(kron=True, fuse=True, max_fused_qubits=3))):
        def reset():
            psi.zero_()
            psi[0] = 1

        reset()
        D.apply_circuit(gates, psi, n=n, scratch=scratch, plan=plan, marshalled=arr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            D.apply_circuit(gates, psi, n=n, scratch=scratch, plan=plan, marshalled=arr)
        torch.cuda.synchronize()
        eager = (time.perf_counter() - t0) / reps
        g = D.CircuitGraph(gates, psi, scratch=scratch, n=n, plan=plan)
        g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.launch()
        torch.cuda.synchronize()
        graph = (time.perf_counter() - t0) / reps
        reset()
        g.launch()
        host = psi.cpu().numpy()
        err = max(abs(host[0] - 2 ** -0.5), abs(host[-1] - 2 ** -0.5), float(abs(host[1:-1]).max()))
        out["plans"].append({"plan": name, "graph_nodes": g.nodes(), "eager_us_per_gate": round(eager / len(gates) * 1e6, 2),
                             "graph_us_per_gate": round(graph / len(gates) * 1e6, 2),
                             "max_err_vs_closed_form": err})
        g.close()
    return out


def qft_extra(D, W, torch, ctx):
    """QFT-24 and QFT-29 (textbook order: H and controlled-phase ladder per
    qubit, then the reversing swaps) on a random state: logical gates/s and
    the algorithmic rate of each plan, one timed run after a sizing run."""
    rows = []
    for n, seed in ((24, 24), (29, 29)):
        gates = W.qft(n)
        arr = D.gate_array(gates)
        psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda:0")
        scratch = torch.empty_like(psi)
        g = torch.Generator(device="cuda:0")
        g.manual_seed(seed)
        for kw in ({}, {"fuse": True, "max_fused_qubits": 2}, {"kron": True},
                   {"kron": True, "fuse": True, "max_fused_qubits": 3},
                   {"kron": True, "fuse": True, "max_fused_qubits": 4},
                   {"kron": True, "fuse": True, "max_fused_qubits": 5}):
            plan = D.make_plan(**kw) if kw else None
            nops, nbytes = D.plan_count(gates, n, plan)
            for _ in range(2):
                psi.copy_(torch.randn(1 << n, dtype=torch.complex128, device="cuda:0", generator=g))
                psi /= torch.linalg.vector_norm(psi)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                D.apply_circuit(gates, psi, n=n, scratch=scratch, plan=plan, marshalled=arr, ctx=ctx)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            rows.append({"qft": n, "gates": len(gates),
                         "plan": ("kron" if kw.get("kron") else "dia")
                         + ("+fuse%d" % kw["max_fused_qubits"] if kw.get("fuse") else ""),
                         "ops": nops, "ms": round(dt * 1e3, 2), "gates_per_s": round(len(gates) / dt, 1),
                         "GBps": round(nbytes / dt / 1e9, 1),
                         "norm": round(float(torch.linalg.vector_norm(psi).item()), 12)})
        del psi, scratch
        torch.cuda.empty_cache()
    return rows


def matrix_extra(D, W):
    """Matrix-level simulation through chained Alg. 1 products: the circuit
    unitary of GHZ, TFIM and QFT circuits with the per-step diagonal count
    and sparsity, and density-matrix evolution of a pure TFIM state."""
    import numpy as np
    rows = []
    for name, n, gates in [("GHZ", 10, W.ghz(10)), ("GHZ", 14, W.ghz(14)), ("TFIM", 10, W.tfim(10, 2, 0.1)),
                           ("QFT", 10, W.qft(10)), ("QFT", 12, W.qft(12))]:
        N = 1 << n
        t0 = time.perf_counter()
        U, rec = D.unitary(gates, n)
        dt = time.perf_counter() - t0
        rows.append({"unitary": "%s-%d" % (name, n), "gates": len(gates), "ms": round(dt * 1e3, 2),
                     "ms_per_gate": round(dt * 1e3 / len(gates), 3), "final_ndiag": int(rec[-1]["ndiag"]),
                     "final_nnz": int(rec[-1]["nnz"]), "min_sparsity": round(float(1 - rec["nnz"].max() / N ** 2), 6),
                     "diaq_stored_values": int(rec[-1]["nvalues"]), "dense_values": N * N})
        del U
    n = 8
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1
    rho = D.from_dense(np.outer(psi, psi))
    gates = W.tfim(n, 3, 0.1)
    t0 = time.perf_counter()
    R, rec = D.density_evolve(gates, rho, drop_tol=1e-14)
    dt = time.perf_counter() - t0
    I = D.from_dense(np.eye(1 << n))
    M = D.from_pauli_sum(n, W.magnetization_terms(n))
    rows.append({"density": "TFIM-%d, 3 steps, |0..0><0..0|" % n, "gates": len(gates), "ms": round(dt * 1e3, 2),
                 "final_ndiag": int(rec[-1]["ndiag"]), "trace": D.trace_product(I, R).real,
                 "purity": D.trace_product(R, R).real, "magnetization": D.trace_product(M, R).real})
    return rows


def batch_extra(D, W, torch, dev, reps=3):
    """512 QAOA circuits (widths 10..22, p 1..4): one persistent launch
    (eager and graph-replayed) against the plain per-gate path (expansion +
    SpMV per gate, adjoint sweep per circuit)."""
    import numpy as np
    insts = W.qaoa_batch(512, 512)
    circs = [(i.n, i.gates, i.terms, 2 * i.p) for i in insts]
    theta = np.concatenate([np.ravel(np.column_stack([i.gammas, i.betas])) for i in insts])
    out = {"workload": "512 MaxCut QAOA circuits, widths {10..22}, 3-regular graphs, p in 1..4, seed 512",
           "circuits": len(insts), "params": int(theta.size)}
    for graph in (False, True):
        b = D.Batch(circs, graph=graph)
        ev, gr = b.run(theta)
        t0 = time.perf_counter()
        for _ in range(reps):
            ev, gr = b.run(theta)
        dt = (time.perf_counter() - t0) / reps
        key = "graph" if graph else "eager"
        out[key + "_ms"] = round(dt * 1e3, 2)
        out[key + "_circuits_per_s"] = round(len(insts) / dt, 1)
        del b
    # plain per-gate path: every circuit through diaq_adjoint_grad
    mats = [D.from_pauli_sum(i.n, i.terms) for i in insts]
    work = torch.empty(3 << 22, dtype=torch.complex128, device=dev)
    psi0s = {}
    for i in insts:
        if i.n not in psi0s:
            p = torch.zeros(1 << i.n, dtype=torch.complex128, device=dev)
            p[0] = 1
            psi0s[i.n] = p
    max_err = 0.0
    t0 = time.perf_counter()
    for k, i in enumerate(insts):
        e, g = D.adjoint_grad(i.gates, mats[k], psi0s[i.n], 2 * i.p, work=work[: 3 << i.n])
        max_err = max(max_err, abs(e - ev[k]), float(np.max(np.abs(g - gr[k]))))
    dt = time.perf_counter() - t0
    out["plain_per_gate_ms"] = round(dt * 1e3, 2)
    out["plain_circuits_per_s"] = round(len(insts) / dt, 1)
    out["speedup_graph_vs_plain"] = round(dt * 1e3 / out["graph_ms"], 1)
    out["max_abs_diff_vs_plain"] = max_err
    return out


def adjoint_extra(D, W, torch, dev):
    """Adjoint gradient of the HEA (n=20, 8 layers, 320 parameters) against
    the plain per-gate path: one adjoint sweep vs the 2 * 320 forward passes
    the parameter-shift rule needs (timed forward pass x 640).  The gate
    list is marshalled once, as for the circuit timings."""
    n, layers = 20, 8
    gates, theta, terms = W.hea(n, layers, 20)
    H = D.from_pauli_sum(n, terms)
    psi0 = torch.zeros(1 << n, dtype=torch.complex128, device=dev)
    psi0[0] = 1
    work = torch.empty(3 << n, dtype=torch.complex128, device=dev)
    marshalled = D.gate_array(gates)
    D.adjoint_grad(gates, H, psi0, len(theta), work=work, marshalled=marshalled)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        e, g = D.adjoint_grad(gates, H, psi0, len(theta), work=work, marshalled=marshalled)
    t_adj = (time.perf_counter() - t0) / reps
    psi = psi0.clone()
    scratch = torch.empty_like(psi)
    arr = D.gate_array(gates)
    D.apply_circuit(gates, psi, scratch=scratch, marshalled=arr)
    D.expect(H, psi)
    t0 = time.perf_counter()
    for _ in range(reps):
        psi.copy_(psi0)
        D.apply_circuit(gates, psi, scratch=scratch, marshalled=arr)
        D.expect(H, psi)
    t_fwd = (time.perf_counter() - t0) / reps
    kplan = D.make_plan(kron=True)
    D.adjoint_grad(gates, H, psi0, len(theta), work=work, plan=kplan, marshalled=marshalled)
    t0 = time.perf_counter()
    for _ in range(reps):
        ek, gk = D.adjoint_grad(gates, H, psi0, len(theta), work=work, plan=kplan, marshalled=marshalled)
    t_kadj = (time.perf_counter() - t0) / reps
    return {"workload": "HEA n=20, 8 layers (RY, RZ, CZ ring), 320 params, H = sum a ZZ + sum b X",
            "adjoint_grads_per_s": round(1 / t_adj, 3), "adjoint_ms": round(t_adj * 1e3, 2),
            "forward_ms": round(t_fwd * 1e3, 2),
            "param_shift_grads_per_s": round(1 / (2 * len(theta) * t_fwd), 4),
            "speedup_vs_param_shift": round(2 * len(theta) * t_fwd / t_adj, 1),
            "kron_adjoint_grads_per_s": round(1 / t_kadj, 3), "kron_adjoint_ms": round(t_kadj * 1e3, 2),
            "kron_max_abs_grad_diff": float(abs(gk - g).max()),
            "energy": e}


if __name__ == "__main__":
    main()
