"""Write tests/golden/oracle_fullsize.json: FP64 oracle results at the full
workload sizes, which the oracle needs minutes to produce (too slow to rerun
inside the GPU tests).  Every value comes from oracle/ alone, on the seeded
inputs of workloads/:

  gnp_n26          G(26, 0.5) unweighted, p = 4: <C> and the norm
  weighted_3reg_n30  random 3-regular, U[0,1) weights, n = 30, p = 10: <C>, norm,
                   and its maximum cut (value, lowest maximising z)
  grad_gnp_n24     G(24, 0.3) unweighted, p = 8, 64 parameter sets: <C> and
                   the adjoint gradient (16 values) of every set

  grad_gnp_n24_fd  FP64 central differences (h = 1e-6) of <C> for the first
                   four of those parameter sets (32 oracle runs per set)
  weighted_3reg_n30_amp_p1  single amplitudes psi_z of the depth-1 state of the
                   n = 30 graph (its first gamma and beta) at six indices z (distinct
                   under the global flip), each summed over the 2^30 basis states
                   (oracle.amplitude_p1); _shifted: the same at the second layer's
                   angles (|sin beta| > |cos beta|), four indices
  gnp_n26_state_samples, weighted_3reg_n30_state_samples  16 amplitudes each of
                   the full-depth oracle states of those two workloads, at seeded
                   indices distinct under the global flip

Usage: python tests/golden/make_golden.py [--skip-n30] [--only-max-cut] [--only-fd] [--only-amp] [--only-state-samples]
(n = 30 needs ~24 GiB RAM)
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_fullsize.json")


def main():
    skip30 = "--skip-n30" in sys.argv
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    if "--only-fd" in sys.argv:
        prob, params = W.grad_gnp_n24()
        sets = []
        t0 = time.time()
        for i, (g, b) in enumerate(params[:4]):
            dg, db = oracle.grad_fd(prob.n, prob.edges, prob.weights, g, b, h=1e-6)
            sets.append({"set": i, "dgamma": dg.tolist(), "dbeta": db.tolist()})
            print(f"grad_gnp_n24 FD set {i} ({time.time() - t0:.1f} s)", flush=True)
        out["grad_gnp_n24_fd"] = {"h": 1e-6, "sets": sets}
        json.dump(out, open(OUT, "w"), indent=1)
        return
    if "--only-state-samples" in sys.argv:
        # amplitudes of the full oracle evolution at seeded indices (distinct under
        # the global flip): the n=26 p=4 and n=30 p=10 workloads at their full depth
        # (n = 30 holds the whole FP64 state: ~24 GiB)
        for key, make in (("gnp_n26_state_samples", W.gnp_n26), ("weighted_3reg_n30_state_samples", W.weighted_3reg_n30)):
            prob, g, b = make()
            n = prob.n
            t0 = time.time()
            psi = oracle.evolve(n, prob.edges, prob.weights, g, b)
            rng = W.SplitMix64(4242 + n)
            zs, seen = [], set()
            while len(zs) < 16:
                z = rng.next_u64() % (1 << n)
                if z in seen or ((1 << n) - 1 - z) in seen:
                    continue
                seen.add(z)
                zs.append(z)
            out[key] = {"p": len(g), "amplitudes": [{"z": z, "re": float(psi[z].real), "im": float(psi[z].imag)}
                                                    for z in zs]}
            del psi
            print(f"{key}: 16 amplitudes ({time.time() - t0:.1f} s)", flush=True)
            json.dump(out, open(OUT, "w"), indent=1)
        return
    if "--only-amp" in sys.argv:
        prob, g, b = W.weighted_3reg_n30()
        n = prob.n
        rng = W.SplitMix64(2024)
        # psi(z) = psi(~z) for every depth (the global flip commutes with C and the
        # mixer and fixes |+>^n), so the indices are taken from distinct flip orbits
        zs = [0, int("01" * (n // 2), 2)] + [rng.next_u64() % (1 << n) for _ in range(4)]
        amps = []
        t0 = time.time()
        for z in zs:
            a = oracle.amplitude_p1(n, prob.edges, prob.weights, g[0], b[0], z)
            amps.append({"z": z, "re": a.real, "im": a.imag})
            print(f"amplitude z={z}: {a!r} ({time.time() - t0:.1f} s)", flush=True)
        out["weighted_3reg_n30_amp_p1"] = {"gamma": g[0], "beta": b[0], "amplitudes": amps}
        # the second layer's angles: |sin beta| > |cos beta|, the shifted factored form
        amps2 = []
        for z in zs[:4]:
            a = oracle.amplitude_p1(n, prob.edges, prob.weights, g[1], b[1], z)
            amps2.append({"z": z, "re": a.real, "im": a.imag})
            print(f"amplitude (layer-2 angles) z={z}: {a!r} ({time.time() - t0:.1f} s)", flush=True)
        out["weighted_3reg_n30_amp_p1_shifted"] = {"gamma": g[1], "beta": b[1], "amplitudes": amps2}
        json.dump(out, open(OUT, "w"), indent=1)
        return
    if "--only-max-cut" in sys.argv:
        prob, _, _ = W.weighted_3reg_n30()
        ct = oracle.cut_table(prob.n, prob.edges, prob.weights)
        z = int(ct.argmax())
        out["weighted_3reg_n30_max_cut"] = {"value": float(ct[z]), "argmax": z}
        json.dump(out, open(OUT, "w"), indent=1)
        print(out["weighted_3reg_n30_max_cut"])
        return
    out["_about"] = ("FP64 oracle values written by tests/golden/make_golden.py (oracle/ only) "
                     "on the seeded inputs of workloads/")
    t0 = time.time()
    prob, g, b = W.gnp_n26()
    e, nrm = oracle.run_expect(prob.n, prob.edges, prob.weights, g, b)
    out["gnp_n26"] = {"n": prob.n, "num_edges": int(prob.num_edges), "p": len(g), "expect": e, "norm": nrm}
    print(f"gnp_n26: <C> = {e!r} ({time.time() - t0:.1f} s)", flush=True)

    prob, params = W.grad_gnp_n24()
    sets = []
    for i, (g, b) in enumerate(params):
        e, dg, db = oracle.grad(prob.n, prob.edges, prob.weights, g, b)
        sets.append({"expect": e, "dgamma": dg.tolist(), "dbeta": db.tolist()})
        print(f"grad_gnp_n24 set {i}: <C> = {e:.12f} ({time.time() - t0:.1f} s)", flush=True)
    out["grad_gnp_n24"] = {"n": prob.n, "num_edges": int(prob.num_edges), "p": len(params[0][0]), "sets": sets}
    json.dump(out, open(OUT, "w"), indent=1)

    if not skip30:
        prob, g, b = W.weighted_3reg_n30()
        e, nrm = oracle.run_expect(prob.n, prob.edges, prob.weights, g, b)
        out["weighted_3reg_n30"] = {"n": prob.n, "num_edges": int(prob.num_edges), "p": len(g), "expect": e,
                                    "norm": nrm}
        print(f"weighted_3reg_n30: <C> = {e!r} ({time.time() - t0:.1f} s)", flush=True)
        ct = oracle.cut_table(prob.n, prob.edges, prob.weights)
        z = int(ct.argmax())                      # lowest index of the maximum
        out["weighted_3reg_n30_max_cut"] = {"value": float(ct[z]), "argmax": z}
        del ct
        print(f"weighted_3reg_n30 max cut: {out['weighted_3reg_n30_max_cut']} ({time.time() - t0:.1f} s)", flush=True)
    json.dump(out, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
