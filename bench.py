"""Benchmark: QAOA max-cut layer throughput at n = 30 on one MI355X.

Workload: random 3-regular graph on 30 vertices (seed 3, pairing model) with
U[0,1) FP64 edge weights, p = 10 layers, gamma/beta uniform in [0, pi);
the state starts at |+>^30 and the run ends with <C> on the host.
One step = one full run (all HBM passes + the <C> reduction).

value  = layer amplitude-updates per second, p * 2^n / t_step, complex64
         state (the complex128 figure is reported beside it).
roofline: the pass kernel, algorithmic bytes (one read + one write of the
         state per pass, write-only for the first) / HIP-event kernel time.
serve  : the serving workload (Poisson arrivals of mixed n in [14, 28],
         p in [1, 12], 30% gradient requests, complex64, 200 GiB budget).
cpu_baseline: the FP64 oracle on the host cores, on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAOA layer amp-updates/s + HBM GB/s at n=30; served ⟨C⟩ req/s, p50/p99"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=2048)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c128", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-gates", action="store_true")
    ap.add_argument("--no-optimize", action="store_true")
    ap.add_argument("--no-sample", action="store_true")
    ap.add_argument("--profile-out", default=os.path.join(ROOT, "gpurun_out", "bench_passes.json"))
    return ap.parse_args()


def time_runs(q, torch, sim, g, b, steps, warmup):
    """Wall time per run over `steps` runs, plus every forward-pass launch's
    kernel time from HIP events recorded on the library's stream around each
    launch inside those same timed runs."""
    for _ in range(warmup):
        sim.expect(g, b)
    q.qaoa_set_profiling(sim.handle, True)
    torch.cuda.synchronize()
    ms_all, by_all = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        q.qaoa_run(sim.handle, g, b)
        e, nrm = q.qaoa_expect(sim.handle)          # synchronises: events are complete
        ms, by = q.qaoa_pass_times(sim.handle)
        ms_all.append(ms)
        by_all.append(by)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    q.qaoa_set_profiling(sim.handle, False)
    return t, e, nrm, np.array(ms_all), np.array(by_all)


def pass_kinds(pass_ms):
    """Mean kernel ms per kind of pass in the three-set schedule (high set
    first, low set, high set with two layers' segments, ..., high set last):
    the write-only first pass, the low-set passes, the merged high-set passes
    and the last pass (with <C>)."""
    ms = list(pass_ms)
    if len(ms) < 3:
        return {"all": ms}
    mid = ms[1:-1]
    return {"first": ms[0], "low_set": float(np.mean(mid[0::2])),
            "high_set_merged": float(np.mean(mid[1::2])) if len(mid) > 1 else None, "last": ms[-1]}


def pmc_traffic(path):
    """Scaled HBM bytes per forward-pass launch from a committed rocprofv3
    counter summary, or None when the kernel source changed since it was taken."""
    import hashlib
    try:
        txt = open(path).read()
    except OSError:
        return None, "no counter summary"
    fields = dict(re.findall(r"^- (\w+): (\S+)$", txt, re.M))
    src = os.path.join(ROOT, "paper_2312_03019_amd", "csrc", "qaoa_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha:
        return None, "kernel source changed since the counters were taken"
    return float(fields["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)


def serve_bench(q, W, nreq):
    trace = W.serving_trace(nreq, seed=5)
    budget = 200 << 30
    out = {}
    # saturated: everything arrives at t = 0
    srv = q.Server(budget, max_slots=256, prec="c64")
    t0 = srv.clock()
    tix = [srv.submit(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta, r.want_grad,
                      arrival=t0) for r in trace]
    res = [srv.wait(t) for t in tix]
    st = srv.stats()
    srv.close()
    bad = sum(1 for x in res if x["status"] != 0)
    X = st["req_per_s"]
    out["saturated"] = {"req_per_s": X, "p50_s": st["p50_s"], "p99_s": st["p99_s"], "failed": bad}
    # open loop: Poisson arrivals at 0.8 X, submitted on schedule
    lam = 0.8 * X
    rng = W.SplitMix64(55)
    gaps = [-math.log(1.0 - rng.u01()) / lam for _ in trace]
    srv = q.Server(budget, max_slots=256, prec="c64")
    t0 = srv.clock()
    t = t0
    tix = []
    for r, gap in zip(trace, gaps):
        t += gap
        while srv.clock() < t:
            time.sleep(min(0.0005, max(0.0, t - srv.clock())))
        tix.append(srv.submit(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta, r.want_grad,
                              arrival=t))
    res = [srv.wait(x) for x in tix]
    st = srv.stats()
    srv.close()
    kinds = {}
    for r, x in zip(trace, res):
        kinds.setdefault("grad" if r.want_grad else "expect", []).append(x["t_done"] - x["t_arrival"])
    out["poisson"] = {"rate_req_per_s": lam, "req_per_s": st["req_per_s"], "p50_s": st["p50_s"],
                      "p99_s": st["p99_s"], "failed": sum(1 for x in res if x["status"] != 0),
                      "p99_expect_s": float(np.percentile(kinds.get("expect", [0]), 99)),
                      "p99_grad_s": float(np.percentile(kinds.get("grad", [0]), 99))}
    out["requests"] = nreq
    out["workload"] = ("Poisson arrivals; family uniform {3-regular (even n), G(n,0.3), complete}; "
                       "n U{14..28}; weights U[0,1); p U{1..12}; 30% gradient; complex64; budget 200 GiB")
    return out


def grad_bench(q, torch, W):
    """Adjoint gradients on the n=24 G(24, 0.3) p=8 workload, 64 parameter sets."""
    prob, params = W.grad_gnp_n24()
    out = {"workload": "n=24 G(24,0.3) unweighted (seed 4), p=8, 64 parameter sets U[0,pi); "
                       "state 128/256 MiB (cache-resident, not an HBM roofline point)"}
    for prec in ("c64", "c128"):
        sim = q.Simulator(prob.n, prob.edges, None, prec)
        sim.grad(*params[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g, b in params:
            sim.grad(g, b)
        t = time.perf_counter() - t0
        q.qaoa_set_profiling(sim.handle, True)
        sim.grad(*params[0])
        ms, by = q.qaoa_pass_times(sim.handle)
        q.qaoa_set_profiling(sim.handle, False)
        passes, _ = sim.plan(len(params[0][0]))
        fm, fb, bm, bb = ms[:passes], by[:passes], ms[passes:], by[passes:]
        out[prec] = {"grads_per_s": len(params) / t, "ms_per_grad": 1e3 * t / len(params),
                     "forward_gbps": fb.sum() / (fm.sum() * 1e-3) / 1e9,
                     "backward_gbps": bb.sum() / (bm.sum() * 1e-3) / 1e9 if len(bm) else None,
                     "forward_ms": float(fm.sum()), "backward_ms": float(bm.sum())}
        sim.close()
    return out


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def gates_bench(q, torch, W, prob, g, b):
    """The fused passes against the gate-by-gate circuit (one sweep per gate),
    complex64: the p-scan of the n=30 workload (times normalised to the gate
    path at p=1, as the paper's p-level figures do) and complete graphs at
    the paper's table configuration (K_N, N = 21..30, p=5, unweighted)."""
    out = {}
    rng = W.SplitMix64(77)
    gg, bb = W.uniform_angles(20, rng)
    sim = q.Simulator(prob.n, prob.edges, prob.weights, "c64")
    t_gate = {p: _time(torch, lambda p=p: (sim.run_gates(gg[:p], bb[:p]), q.qaoa_expect(sim.handle)), 2)
              for p in (1, 2, 3)}
    t_fused = {p: _time(torch, lambda p=p: sim.expect(gg[:p], bb[:p]), 3) for p in range(1, 21)}
    v, _ = sim.max_cut()
    sim.close()
    base = t_gate[1]
    out["p_scan"] = {
        "workload": f"n={prob.n} weighted 3-regular (seed 3), gamma/beta U[0,pi) (seed 77), complex64",
        "gate_path_ms": {p: t * 1e3 for p, t in t_gate.items()},
        "fused_ms": {p: t * 1e3 for p, t in t_fused.items()},
        "fused_over_gate_p1": {p: t / base for p, t in t_fused.items()},
        "gate_over_gate_p1": {p: t / base for p, t in t_gate.items()},
        "max_cut": v,
    }
    # complete graphs K_N, N = 21..30, p = 5, unweighted: the configuration of the
    # paper's timing tables, here both circuits on the same device
    gk, bk = W.uniform_angles(5, W.SplitMix64(78))
    scan = {}
    for n in range(21, 31):
        kn = W.complete(n)
        sk = q.Simulator(n, kn, None, "c64")
        gate = lambda: (sk.run_gates(gk, bk), q.qaoa_expect(sk.handle))
        if n < 27:
            tg = _time(torch, gate, 2)
        else:                      # seconds per run: one timed run (kernels already loaded)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gate()
            torch.cuda.synchronize()
            tg = time.perf_counter() - t0
        eg = q.qaoa_expect(sk.handle)[0]
        tf = _time(torch, lambda: sk.expect(gk, bk), 5)
        ef = sk.expect(gk, bk)[0]
        passes, _ = sk.plan(5)
        sk.close()
        m = n * (n - 1) // 2
        scan[n] = {"gate_path_ms": tg * 1e3, "fused_ms": tf * 1e3, "speedup": tg / tf, "expect_gate": eg,
                   "expect_fused": ef, "rel_diff_over_edges": abs(eg - ef) / m,
                   "sweeps_gate_path": n + 5 * (m + n), "passes_fused": passes}
        print(f"[bench] K_{n} p=5: gate path {tg * 1e3:.1f} ms, fused {tf * 1e3:.2f} ms", file=sys.stderr, flush=True)
    out["complete_p5_scan"] = {"workload": "K_N unweighted, N = 21..30, p = 5, gamma/beta U[0,pi) (seed 78), "
                                           "complex64; gate path = H, then per level one sweep per RZZ and per RX",
                               "by_n": scan}
    return out


def optimize_bench(q, W):
    """Approximation ratio <C>*/max C of optimised angles vs p (Adam over the
    adjoint gradient, 8 starts batched through the server), n=20 3-regular."""
    from paper_2312_03019_amd import optimize as opt
    e = W.random_regular(20, 3, W.SplitMix64(79))
    out = {"workload": "n=20 random 3-regular unweighted (seed 79), Adam lr 0.04, 8 starts x 100 steps, complex64"}
    for p in (1, 2, 3, 4, 5):
        t0 = time.perf_counter()
        r = opt.optimize(q, 20, e, None, p=p, starts=8, steps=100, lr=0.04, seed=p)
        out[p] = {"expect": r.expect, "ratio": r.ratio, "seconds": time.perf_counter() - t0,
                  "gamma": r.gamma.tolist(), "beta": r.beta.tolist()}
    out["max_cut"] = r.max_cut
    return out


def sample_bench(q, torch, W, prob, g, b, count=1 << 20):
    """Bitstrings from |psi|^2 of the n=30 workload's final state: 2^20 samples
    (inverse CDF: one FP64 pass over the state for chunk sums, then one wave per
    sample), and the best cut among them against the maximum cut."""
    sim = q.Simulator(prob.n, prob.edges, prob.weights, "c64")
    rng = np.random.default_rng(80)
    u = rng.random(count)
    try:
        sim.run(g, b)
        sim.sample(u[:1024])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z = sim.sample(u)
        t = time.perf_counter() - t0
        mc, _ = sim.max_cut()
    finally:
        sim.close()
    z = z.astype(np.int64)
    cut = np.zeros(count)
    for (uu, vv), w in zip(prob.edges, prob.weights):
        cut += w * (((z >> int(uu)) ^ (z >> int(vv))) & 1)
    return {"samples": count, "seconds": t, "samples_per_s": count / t, "best_sampled_cut": float(cut.max()),
            "mean_sampled_cut": float(cut.mean()), "max_cut": mc,
            "note": "uniforms from numpy default_rng(80); time includes the CDF pass over the 8 GiB state"}


def copy_ceiling(q, torch, nbytes=4 << 30, reps=5):
    """Device-to-device streaming copy with the library's probe kernel (GB/s, read + write)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    q.qaoa_copy_probe(src, dst, nbytes, st)
    st.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        q.qaoa_copy_probe(src, dst, nbytes, st)
    b.record(st)
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(W, prob, g, b, layers=2):
    """The FP64 oracle on the same graph, for the first `layers` layers and <C>."""
    import oracle
    t0 = time.perf_counter()
    oracle.run_expect(prob.n, prob.edges, prob.weights, g[:layers], b[:layers])
    dt = time.perf_counter() - t0
    return {"value": layers * (2 ** prob.n) / dt, "unit": "layer amp-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle on the same n={prob.n} graph, the first {layers} of the {len(g)} layers "
                      f"(same angles) plus <C>: {dt:.1f} s; value = {layers} * 2^{prob.n} / t"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2312_03019_amd as q
    import workloads as W

    torch.cuda.set_device(0)
    prob, g, b = W.weighted_3reg_n30(n=a.n, p=a.p)
    stream = torch.cuda.current_stream()
    res = {}
    for prec in (["c64"] if a.no_c128 else ["c64", "c128"]):
        sim = q.Simulator(prob.n, prob.edges, prob.weights, prec, stream=stream)
        t, e, nrm, ms, by = time_runs(q, torch, sim, g, b, a.steps, a.warmup)
        passes, sizes = sim.plan(a.p)
        res[prec] = {"t": t, "expect": e, "norm": nrm, "pass_ms": ms.mean(axis=0).tolist(),
                     "pass_ms_all": ms.tolist(), "pass_bytes": by[0].tolist(), "passes": passes, "sets": sizes,
                     "launch_ms_mean": float(ms.mean()), "launch_bytes_mean": float(by.mean())}
        if prec == "c64":
            keep64 = sim
        else:
            res["fidelity_c64_c128"] = keep64.fidelity(sim)
        del sim
    del keep64
    torch.cuda.empty_cache()

    copy_gbs = copy_ceiling(q, torch)
    torch.cuda.empty_cache()
    r64 = res["c64"]
    # algorithmic bytes per launch / mean launch duration, over every forward-pass launch of the timed runs
    achieved = r64["launch_bytes_mean"] / (r64["launch_ms_mean"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": a.p * 2 ** a.n / r64["t"],
        "unit": "layer amp-updates/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r64["t"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"n={a.n} random 3-regular (seed 3) with U[0,1) FP64 weights, p={a.p}, "
                               f"gamma/beta U[0,pi), complex64 state, |+>^n start, <C> to host",
                   "passes_per_run": r64["passes"], "qubit_sets": r64["sets"]},
        "hbm_gbps": achieved,
        "expect_c64": r64["expect"],
    }
    if "c128" in res:
        r128 = res["c128"]
        line["c128"] = {"value": a.p * 2 ** a.n / r128["t"], "ms_per_step": r128["t"] * 1e3,
                        "hbm_gbps": r128["launch_bytes_mean"] / (r128["launch_ms_mean"] * 1e-3) / 1e9,
                        "expect": r128["expect"]}
        line["c64_over_c128_speedup"] = r128["t"] / r64["t"]
        line["delta_expect_c64_c128"] = r64["expect"] - r128["expect"]
        line["one_minus_fidelity_c64_c128"] = 1.0 - res["fidelity_c64_c128"]
    traffic, tsrc = (None, "counters apply to the n=30 p=10 workload only")
    if a.n == 30 and a.p == 10:
        traffic, tsrc = pmc_traffic(os.path.join(ROOT, "profiles", "k_fwd_weighted3reg_n30_p10_c64_counters.md"))
    line["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS,
                        "traffic": None if traffic is None else traffic / 1e9,
                        "traffic_unit": "GB per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-kernel scaled)",
                        "traffic_source": tsrc,
                        "kernel": "k_fwd (one launch per HBM pass, all shapes)",
                        "launches_timed": a.steps * r64["passes"],
                        "algorithmic_bytes_per_launch": r64["launch_bytes_mean"],
                        "mean_launch_ms": r64["launch_ms_mean"],
                        "copy_ceiling_gbps": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                        "pass_ms_by_kind": pass_kinds(r64["pass_ms"]) if len(r64["sets"]) == 3 else None,
                        "per_launch_bytes": "2*2^n*8 read+write (write-only 2^n*8 for the first pass)"}
    if not a.no_grad:
        line["grad"] = grad_bench(q, torch, W)
    if not a.no_gates:
        line["gates"] = gates_bench(q, torch, W, prob, g, b)
    if not a.no_optimize:
        line["optimize"] = optimize_bench(q, W)
    if not a.no_sample:
        line["sample"] = sample_bench(q, torch, W, prob, g, b)
    if not a.no_serve:
        line["serve"] = serve_bench(q, W, a.serve_requests)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(W, prob, g, b)
    os.makedirs(os.path.dirname(a.profile_out), exist_ok=True)
    with open(a.profile_out, "w") as f:
        json.dump({k: v for k, v in res.items()}, f)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
