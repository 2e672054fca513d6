"""Benchmark: QAOA max-cut layer throughput at n = 30 on one MI355X.

Workload: random 3-regular graph on 30 vertices (seed 3, pairing model) with
U[0,1) FP64 edge weights, p = 10 layers, gamma/beta uniform in [0, pi);
the state starts at |+>^30 and the run ends with <C> on the host.
One step = one full run (all HBM passes + the <C> reduction).

value   : layer amplitude-updates per second, p * 2^n / t_step, complex64
          state (the complex128 figure is reported beside it).
roofline: the dominant pass kernel (largest share of the run's kernel time):
          its algorithmic bytes per launch (one read + one write of the state,
          write-only for the first pass) / its mean HIP-event launch time;
          every pass kernel and every pass of the run are listed beside it.
Other legs: the n = 26 precision comparison, a fresh context's time including
the graph upload, adjoint gradients (n = 24 accuracy against the FP64 oracle
and central differences; n = 28 HBM rates), the gate-by-gate circuit and the
p-scan with the approximation ratio, optimised ratios, sampling, serving
(Poisson arrivals of mixed n in [14, 28], p in [1, 12], 30% gradient
requests, complex64, 200 GiB budget), and the FP64 oracle on the host cores
on a bounded sample (cpu_baseline).
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
# the library's default chunk size for pipelined pass pairs (both precisions)
CHUNK_BYTES = {"c64": 128 << 20, "c128": 128 << 20}


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
    ap.add_argument("--no-n26", action="store_true")
    ap.add_argument("--only-grad-hbm", action="store_true",
                    help="run only the n=28 gradient leg and print its JSON (for profiling the adjoint sweep)")
    ap.add_argument("--profile-out", default=os.path.join(ROOT, "gpurun_out", "bench_passes.json"))
    return ap.parse_args()


def time_plain(q, torch, sim, g, b, steps, warmup):
    """Wall time per step (run, then <C> to the host) over `steps` steps after
    `warmup` untimed ones, with no profiling events in the queues."""
    for _ in range(warmup):
        sim.expect(g, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        q.qaoa_run(sim.handle, g, b)
        e, nrm = q.qaoa_expect(sim.handle)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, e, nrm


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


def pass_table(q, sim, pass_ms, pass_bytes):
    """Every pass of the timed runs: qubit set, kernel, mean ms, GB/s and fraction of peak."""
    rows = []
    for i, (ms, by) in enumerate(zip(pass_ms, pass_bytes)):
        st, name = q.qaoa_pass_kernel(sim.handle, i)
        gbs = by / (ms * 1e-3) / 1e9
        rows.append({"i": i, "set": st, "kernel": name, "ms": ms, "bytes": by, "gbps": gbs,
                     "frac": gbs / HBM_PEAK_GBS})
    return rows


def kernel_table(rows):
    """Per pass kernel: launches per run, mean ms, algorithmic bytes per launch,
    GB/s, fraction of peak and share of the run's kernel time."""
    tot = sum(r["ms"] for r in rows)
    out = {}
    for r in rows:
        k = out.setdefault(r["kernel"], {"launches": 0, "ms_sum": 0.0, "bytes_sum": 0.0})
        k["launches"] += 1
        k["ms_sum"] += r["ms"]
        k["bytes_sum"] += r["bytes"]
    for name, k in out.items():
        ms, by = k.pop("ms_sum"), k.pop("bytes_sum")
        k["mean_ms"] = ms / k["launches"]
        k["bytes_per_launch"] = by / k["launches"]
        k["gbps"] = by / (ms * 1e-3) / 1e9
        k["frac"] = k["gbps"] / HBM_PEAK_GBS
        k["share"] = ms / tot
    return out


def pmc_traffic(path, kernel):
    """Scaled HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    try:
        txt = open(path).read()
    except OSError:
        return None, "no counter summary"
    src = os.path.join(ROOT, "paper_2312_03019_amd", "csrc", "qaoa_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    m = re.search(r"^- kernel_source_sha256: (\S+)$", txt, re.M)
    if not m or m.group(1) != sha:
        return None, "kernel source changed since the counters were taken"
    m = re.search(r"^- traffic " + re.escape(kernel) + r": (\S+)$", txt, re.M)
    if not m:
        return None, f"no counters for {kernel}"
    return float(m.group(1)), os.path.relpath(path, ROOT)


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
    kinds, small = {}, []
    for r, x in zip(trace, res):
        kinds.setdefault("grad" if r.want_grad else "expect", []).append(x["t_done"] - x["t_arrival"])
        if not r.want_grad and r.problem.n <= 14:      # whole request in one workgroup
            small.append(x["t_done"] - x["t_arrival"])
    out["poisson"] = {"rate_req_per_s": lam, "req_per_s": st["req_per_s"], "p50_s": st["p50_s"],
                      "p99_s": st["p99_s"], "failed": sum(1 for x in res if x["status"] != 0),
                      "p99_expect_s": float(np.percentile(kinds.get("expect", [0]), 99)),
                      "p99_grad_s": float(np.percentile(kinds.get("grad", [0]), 99)),
                      "one_workgroup_requests": len(small),
                      "p50_one_workgroup_s": float(np.percentile(small, 50)) if small else None,
                      "p99_one_workgroup_s": float(np.percentile(small, 99)) if small else None}
    out["requests"] = nreq
    out["workload"] = ("Poisson arrivals; family uniform {3-regular (even n), G(n,0.3), complete}; "
                       "n U{14..28}; weights U[0,1); p U{1..12}; 30% gradient; complex64; budget 200 GiB")
    return out


def _golden():
    import json as _json
    with open(os.path.join(ROOT, "tests", "golden", "oracle_fullsize.json")) as f:
        return _json.load(f)


def _err_stats(diffs, E):
    a = np.abs(np.concatenate([np.ravel(d) for d in diffs])) / E
    return {"max_over_E": float(a.max()), "median_over_E": float(np.median(a))}


def grad_bench(q, torch, W):
    """Adjoint gradients on the n=24 G(24, 0.3) p=8 workload, 64 parameter sets:
    throughput, and the error of every one of the 16 partials of every set
    against the stored FP64 oracle adjoint, against the stored FP64 oracle
    central differences (h = 1e-6; the first four sets) and against central
    differences of the complex128 device run (h = 1e-6; all 64 sets)."""
    prob, params = W.grad_gnp_n24()
    gold = _golden()
    ref = gold["grad_gnp_n24"]["sets"]
    ref_fd = gold.get("grad_gnp_n24_fd", {}).get("sets", [])
    E = float(prob.num_edges)
    out = {"workload": "n=24 G(24,0.3) unweighted (seed 4), p=8, 64 parameter sets U[0,pi); "
                       "state 128/256 MiB (cache-resident, not an HBM roofline point); errors are "
                       "|d - d_ref| / |E| over all 16 partials of every set"}
    grads = {}
    for prec in ("c64", "c128"):
        sim = q.Simulator(prob.n, prob.edges, None, prec)
        sim.grad(*params[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [sim.grad(g, b) for g, b in params]
        t = time.perf_counter() - t0
        grads[prec] = res
        q.qaoa_set_profiling(sim.handle, True)
        sim.grad(*params[0])
        ms, by = q.qaoa_pass_times(sim.handle)
        q.qaoa_set_profiling(sim.handle, False)
        passes, _ = sim.plan(len(params[0][0]))
        fm, fb, bm, bb = ms[:passes], by[:passes], ms[passes:], by[passes:]
        d_or = [np.concatenate([r[1] - np.array(x["dgamma"]), r[2] - np.array(x["dbeta"])])
                for r, x in zip(res, ref)]
        d_fd = [np.concatenate([res[x["set"]][1] - np.array(x["dgamma"]), res[x["set"]][2] - np.array(x["dbeta"])])
                for x in ref_fd]
        out[prec] = {"grads_per_s": len(params) / t, "ms_per_grad": 1e3 * t / len(params),
                     "forward_gbps": fb.sum() / (fm.sum() * 1e-3) / 1e9,
                     "backward_gbps": bb.sum() / (bm.sum() * 1e-3) / 1e9 if len(bm) else None,
                     "forward_ms": float(fm.sum()), "backward_ms": float(bm.sum()),
                     "err_vs_oracle_adjoint": _err_stats(d_or, E),
                     "err_expect_vs_oracle_over_E": float(max(abs(r[0] - x["expect"]) for r, x in zip(res, ref)) / E)}
        if d_fd:
            out[prec]["err_vs_oracle_fd"] = dict(_err_stats(d_fd, E), sets=len(d_fd))
        if prec == "c128":
            # central differences of the complex128 device run, every set
            h = 1e-6
            diffs = []
            for (g, b), r in zip(params, res):
                fd = np.zeros(2 * len(g))
                for l in range(len(g)):
                    for k, (arr, other) in enumerate(((g, b), (b, g))):
                        a1, a2 = arr.copy(), arr.copy()
                        a1[l] += h
                        a2[l] -= h
                        e1 = sim.expect(a1, other)[0] if k == 0 else sim.expect(other, a1)[0]
                        e2 = sim.expect(a2, other)[0] if k == 0 else sim.expect(other, a2)[0]
                        fd[k * len(g) + l] = (e1 - e2) / (2 * h)
                diffs.append((np.concatenate([r[1], r[2]]), fd))
            out["c128"]["err_vs_device_c128_fd"] = _err_stats([a - f for a, f in diffs], E)
            c64 = grads["c64"]
            out["c64"]["err_vs_device_c128_fd"] = _err_stats(
                [np.concatenate([x[1], x[2]]) - f for x, (_, f) in zip(c64, diffs)], E)
        sim.close()
        # the same 64 gradients submitted together to the serving loop, which runs
        # them side by side (shared step launches) instead of one after another
        for slots in (8, 64):
            srv = q.Server(64 << 30, max_slots=slots, prec=prec)
            srv.wait(srv.submit(prob.n, prob.edges, None, *params[0], want_grad=True))
            t0 = time.perf_counter()
            tix = [srv.submit(prob.n, prob.edges, None, g, b, want_grad=True) for g, b in params]
            got = [srv.wait(t) for t in tix]
            t = time.perf_counter() - t0
            srv.close()
            d_sv = [np.concatenate([np.asarray(x["dgamma"]) - np.array(r["dgamma"]),
                                    np.asarray(x["dbeta"]) - np.array(r["dbeta"])]) for x, r in zip(got, ref)]
            out[prec][f"served_{slots}_slots"] = {"grads_per_s": len(params) / t,
                                                 "err_vs_oracle_adjoint": _err_stats(d_sv, E)}
    return out


def grad_hbm_bench(q, torch, W, n=28, p=4, reps=3):
    """Adjoint gradient at an HBM-bound size: n=28 weighted 3-regular, p=4
    (2 GiB / 4 GiB per vector): per pass kernel of the forward and backward
    sweeps, mean ms and algorithmic GB/s (backward passes move both vectors)."""
    prob, g, b = W.weighted_3reg_n30(n=n, p=p)
    out = {"workload": f"n={n} random 3-regular (seed 3) with U[0,1) weights, p={p}, gamma/beta U[0,pi); "
                       f"bytes: forward 2*2^n*S per pass (+2^n*S for lam in the last), backward 4*2^n*S "
                       f"(2*2^n*S for the pass undoing the first)"}
    for prec in ("c64", "c128"):
        sim = q.Simulator(prob.n, prob.edges, prob.weights, prec)
        sim.grad(g, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sim.grad(g, b)
        t = (time.perf_counter() - t0) / reps
        # per-kernel figures from whole-pass launches (the timed gradients use the library default)
        q.qaoa_set_chunking(sim.handle, 0, 0)
        q.qaoa_set_profiling(sim.handle, True)
        sim.grad(g, b)
        ms, by = q.qaoa_pass_times(sim.handle)
        q.qaoa_set_profiling(sim.handle, False)
        rows = pass_table(q, sim, ms, by)
        passes, _ = sim.plan(p)
        fwd, bwd = rows[:passes], rows[passes:]
        out[prec] = {"ms_per_grad": t * 1e3, "forward_ms": float(sum(r["ms"] for r in fwd)),
                     "backward_ms": float(sum(r["ms"] for r in bwd)),
                     "backward_gbps": sum(r["bytes"] for r in bwd) / (sum(r["ms"] for r in bwd) * 1e-3) / 1e9,
                     "kernels": kernel_table(rows)}
        sim.close()
        torch.cuda.empty_cache()
    return out


def n26_bench(q, torch, W, steps=20):
    """The precision comparison workload: G(26, 0.5) unweighted, p=4, complex64
    against complex128: time per run, speedup, <C> of each against the stored
    FP64 oracle value, and 1 - fidelity between the two final states."""
    prob, g, b = W.gnp_n26()
    ref = _golden()["gnp_n26"]["expect"]
    out = {"workload": "n=26 G(26,0.5) unweighted (seed 2), p=4, gamma/beta U[0,pi); states 512 MiB / 1 GiB"}
    sims = {}
    for prec in ("c64", "c128"):
        sim = q.Simulator(prob.n, prob.edges, None, prec)
        t, e, nrm = time_plain(q, torch, sim, g, b, steps, 3)
        out[prec] = {"ms_per_run": t * 1e3, "expect": e, "abs_err_vs_oracle_over_E": abs(e - ref) / prob.num_edges,
                     "layer_amp_updates_per_s": len(g) * 2 ** prob.n / t}
        sims[prec] = sim
    out["c64_over_c128_speedup"] = out["c128"]["ms_per_run"] / out["c64"]["ms_per_run"]
    out["one_minus_fidelity"] = 1.0 - sims["c64"].fidelity(sims["c128"])
    for s_ in sims.values():
        s_.close()
    return out


def upload_inclusive(q, torch, W, prob, g, b):
    """A fresh context from qaoa_create to <C> on the host: graph validation and
    upload, the per-set tile cut tables, the state allocation, the run image
    upload and the run itself (the headline step excludes the first four)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = q.Simulator(prob.n, prob.edges, prob.weights, "c64")
    e, _ = sim.expect(g, b)
    t = time.perf_counter() - t0
    sim.close()
    torch.cuda.empty_cache()
    return {"ms": t * 1e3, "expect": e,
            "note": "complex64, fresh context: create + graph upload + tile cut tables + state allocation + run + <C>"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


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
    e_fused = {p: sim.expect(gg[:p], bb[:p])[0] for p in range(1, 21)}
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
        "expect": e_fused,
        "approx_ratio": {p: e / v for p, e in e_fused.items()},
        "ratio_note": "<C>/max C at the scan's seeded angles (not optimised)",
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


def copy_ceiling(q, torch, nbytes=4 << 30, reps=5, block_bytes=16384):
    """Device-to-device streaming copy with the library's probe kernel (GB/s, read + write)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    q.qaoa_copy_probe(src, dst, nbytes, st, block_bytes)
    st.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        q.qaoa_copy_probe(src, dst, nbytes, st, block_bytes)
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
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
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
    if a.only_grad_hbm:
        cg = copy_ceiling(q, torch, block_bytes=16384)      # also the counters' reference copy
        torch.cuda.empty_cache()
        print(json.dumps({"grad_hbm": grad_hbm_bench(q, torch, W), "copy_ceiling_gbps_16k_per_wg": cg}), flush=True)
        return
    prob, g, b = W.weighted_3reg_n30(n=a.n, p=a.p)
    stream = torch.cuda.current_stream()
    res = {}
    for prec in (["c64"] if a.no_c128 else ["c64", "c128"]):
        sim = q.Simulator(prob.n, prob.edges, prob.weights, prec, stream=stream)
        # the default path (pass pairs pipelined over chunks) gives the headline,
        # timed without profiling events; the same runs again with HIP events around every
        # pass (pass pair) give the per-pass table and the pair spans
        t, e, nrm = time_plain(q, torch, sim, g, b, a.steps, a.warmup)
        t_prof, e_prof, _, ms, by = time_runs(q, torch, sim, g, b, a.steps, 0)
        assert e_prof == e, "profiled and plain runs must agree bitwise"
        passes, sizes = sim.plan(a.p)
        F, fixed = q.qaoa_chunk_plan(a.n, prec, a.p, CHUNK_BYTES[prec]) if CHUNK_BYTES[prec] else (0, [])
        chunked = None
        if F:
            spans = [q.qaoa_pass_span(sim.handle, 2 * i + 1, 2 * i + 2) for i in range(len(fixed))]
            pair_bytes = [float(by[0][2 * i + 1] + by[0][2 * i + 2]) for i in range(len(fixed))]
            chunked = {"chunk_bytes": CHUNK_BYTES[prec], "chunks_per_pass": 1 << F, "ms_per_run": t * 1e3,
                       "pair_ms_mean": float(np.mean(spans)),
                       "pair_gbps": sum(pair_bytes) / (sum(spans) * 1e-3) / 1e9,
                       "first_pass_ms": float(ms.mean(axis=0)[0])}
            # whole-pass launches of the same workload: the per-kernel roofline
            q.qaoa_set_chunking(sim.handle, 0, 0)
            t1, e1, _ = time_plain(q, torch, sim, g, b, a.steps, a.warmup)
            _, _, _, ms, by = time_runs(q, torch, sim, g, b, a.steps, 0)
            q.qaoa_set_chunking(sim.handle, CHUNK_BYTES[prec], 0, 3)
            assert e1 == e, "chunked and whole-pass runs must agree bitwise"
            chunked["ms_per_run_whole_passes"] = t1 * 1e3
            chunked["speedup"] = t1 / t
        rows = pass_table(q, sim, ms.mean(axis=0), by[0])
        res[prec] = {"t": t, "t_prof": t_prof, "expect": e, "norm": nrm, "passes": passes, "sets": sizes, "rows": rows,
                     "kernels": kernel_table(rows), "pass_ms_all": ms.tolist(), "chunked": chunked,
                     "launch_ms_mean": float(ms.mean()), "launch_bytes_mean": float(by.mean())}
        print(f"[bench] n={a.n} p={a.p} {prec}: {t * 1e3:.2f} ms per run", file=sys.stderr, flush=True)
        if prec == "c64":
            keep64 = sim
        else:
            res["fidelity_c64_c128"] = keep64.fidelity(sim)
        del sim
    del keep64
    torch.cuda.empty_cache()

    copy16 = copy_ceiling(q, torch, block_bytes=16384)
    copy4 = copy_ceiling(q, torch, block_bytes=4096)
    torch.cuda.empty_cache()
    r64 = res["c64"]
    kern = r64["kernels"]
    dom = max(kern, key=lambda k: kern[k]["share"])     # the kernel with the largest share of kernel time
    dk = kern[dom]
    achieved = dk["gbps"]
    line = {
        "metric": METRIC,
        "value": a.p * 2 ** a.n / r64["t"],
        "unit": "layer amp-updates/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r64["t"] * 1e3,
        "ms_per_step_with_pass_events": r64["t_prof"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"n={a.n} random 3-regular (seed 3) with U[0,1) FP64 weights, p={a.p}, "
                               f"gamma/beta U[0,pi), complex64 state, |+>^n start, <C> to host",
                   "passes_per_run": r64["passes"], "qubit_sets": r64["sets"]},
        "hbm_gbps_all_passes": r64["launch_bytes_mean"] / (r64["launch_ms_mean"] * 1e-3) / 1e9,
        "expect_c64": r64["expect"],
    }
    if "c128" in res:
        r128 = res["c128"]
        line["c128"] = {"value": a.p * 2 ** a.n / r128["t"], "ms_per_step": r128["t"] * 1e3,
                        "ms_per_step_with_pass_events": r128["t_prof"] * 1e3,
                        "hbm_gbps_all_passes": r128["launch_bytes_mean"] / (r128["launch_ms_mean"] * 1e-3) / 1e9,
                        "expect": r128["expect"], "kernels": r128["kernels"],
                        "passes": [{k: r[k] for k in ("i", "set", "kernel", "ms", "gbps", "frac")} for r in r128["rows"]],
                        "chunked_pairs": r128.get("chunked")}
        line["c64_over_c128_speedup"] = r128["t"] / r64["t"]
        line["delta_expect_c64_c128"] = r64["expect"] - r128["expect"]
        line["one_minus_fidelity_c64_c128"] = 1.0 - res["fidelity_c64_c128"]
    traffic, tsrc = (None, "counters apply to the n=30 p=10 workload only")
    if a.n == 30 and a.p == 10:
        traffic, tsrc = pmc_traffic(os.path.join(ROOT, "profiles", "pass_kernels_weighted3reg_n30_p10_counters.md"),
                                    dom)
    line["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS,
                        "traffic": None if traffic is None else traffic / 1e9,
                        "traffic_unit": "GB per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-kernel scaled)",
                        "traffic_source": tsrc,
                        "kernel": dom,
                        "workgroups_per_launch": 2 ** (a.n - len(q.qaoa_tile_map(a.n, "c64", 0)[0])),
                        "launches": "whole-pass launches (every tile of the pass in one launch); the headline run "
                                    "pipelines each low-set/high-set pass pair over chunks on extra streams (chunked_pairs)",
                        "kernel_share_of_run": dk["share"],
                        "launches_timed": a.steps * dk["launches"],
                        "algorithmic_bytes_per_launch": dk["bytes_per_launch"],
                        "mean_launch_ms": dk["mean_ms"],
                        "per_launch_bytes": "2*2^n*8 read+write (write-only 2^n*8 for the first pass)",
                        "copy_ceiling_gbps_16k_per_wg": copy16, "copy_ceiling_gbps_4k_per_wg": copy4,
                        "frac_of_copy_4k": achieved / copy4,
                        "kernels": kern,
                        "passes": [{k: r[k] for k in ("i", "set", "kernel", "ms", "gbps", "frac")} for r in r64["rows"]],
                        "all_passes_gbps": line["hbm_gbps_all_passes"]}
    if r64.get("chunked"):
        line["chunked_pairs"] = dict(r64["chunked"], note=(
            "value is measured with the library default: each (low-set, high-set) pass pair runs chunk by chunk, "
            "the high-set pass of chunk k on one of two more streams beside the low-set pass of chunk k+1; pair_gbps = "
            "algorithmic bytes of both passes / the pair's span from HIP events; results bitwise equal to whole passes"))
    if a.n == 30 and a.p == 10:
        line["t_including_upload"] = upload_inclusive(q, torch, W, prob, g, b)
    if not a.no_n26:
        line["n26"] = n26_bench(q, torch, W)
        print("[bench] n26 done", file=sys.stderr, flush=True)
    if not a.no_grad:
        line["grad"] = grad_bench(q, torch, W)
        print("[bench] grad n24 done", file=sys.stderr, flush=True)
        line["grad_hbm"] = grad_hbm_bench(q, torch, W)
        print("[bench] grad n28 done", file=sys.stderr, flush=True)
    if not a.no_gates:
        line["gates"] = gates_bench(q, torch, W, prob, g, b)
    if not a.no_optimize:
        line["optimize"] = optimize_bench(q, W)
    if not a.no_sample:
        line["sample"] = sample_bench(q, torch, W, prob, g, b)
    if not a.no_serve:
        line["serve"] = serve_bench(q, W, a.serve_requests)
        print("[bench] serve done", file=sys.stderr, flush=True)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(W, prob, g, b)
    os.makedirs(os.path.dirname(a.profile_out), exist_ok=True)
    with open(a.profile_out, "w") as f:
        json.dump({k: v for k, v in res.items()}, f)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
