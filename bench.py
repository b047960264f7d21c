#!/usr/bin/env python3
"""Throughput of the spin-lattice NEP step on one MI355X.

Workload: B20 FeGe-like crystal, 32x32x32 cells = 262,144 atoms (131,072
spins), periodic, seeded random model, 300 K Langevin lattice bath and
stochastic-LLG spin bath (damping 0.1), dt = 1 fs, FP64 end to end. One
step = the whole B A O S A B step (3 descriptor passes, read-out, spin
couplings, 4 colour sweeps, one backward pass, neighbour-list upkeep and the
lattice half-steps) for every atom. Inputs are resident on the device before
the timed region.

Prints one JSON line (see the keys below). --gpus N > 1 is refused: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2606_14073_amd import workload as W  # noqa: E402

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def pair_counts(s):
    """Neighbour statistics of the workload (for the algorithmic work model)."""
    from scipy.spatial import cKDTree
    p = np.mod(s.pos, s.box)
    tree = cKDTree(p, boxsize=s.box)
    fe = s.types == 0
    out = {}
    for rc, key in ((6.0, "R"), (4.5, "A")):
        pairs = tree.query_pairs(rc, output_type="ndarray")
        a, b = pairs[:, 0], pairs[:, 1]
        out[key] = 2 * len(pairs)                                   # ordered pairs
        out[key + "_fefe"] = 2 * int(np.sum(fe[a] & fe[b]))
        out[key + "_fe_centre"] = int(np.sum(fe[a])) + int(np.sum(fe[b]))   # pairs with an Fe centre
    return out


def work_model(pc, n, n_fe):
    """Algorithmic FLOPs of one launch of the angular-set backward kernel
    (FMA = 2 FLOP), counted once per (centre, neighbour) pair inside 4.5 A:
      per pair: radial basis with derivative (cos+sin, Chebyshev, 9 f and 9 df) 60;
      harmonics and their gradients 24 + 72 -> 150;
      per radial function n (7): g^A, dg^A (36), and for spin pairs g^sa, dg^sa (36);
      per (n, lm) contraction: u, v (4 FMA), sums sv, sl, w, su (6 FMA) = 20 FLOP;
      per pair gradient assembly 20."""
    per_pair = 60 + 150 + 7 * 36 + 7 * 24 * 20 + 20
    spin_pairs = pc["A_fefe"]
    return pc["A"] * per_pair + spin_pairs * 7 * 36


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--breakdown", action="store_true", help="print the kernel-group breakdown to stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} requested, but this build runs on one GPU only; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2606_14073_amd import nepspin

    s = W.config_fp64_bench()
    params = W.random_params()
    v0 = W.maxwell_boltzmann(s.types, 300.0)
    kw = dict(dt=1.0, T0=300.0, alpha_s=0.1, gamma_L=0.01, ensemble=1, K_corr=1, seed=W.SEED_PHILOX)
    model = nepspin.Model(params)
    K, Wm = args.steps, args.warmup

    def run(precision, prof_groups=()):
        sim = nepspin.Sim(model, s.types, s.pos, s.spin, s.box, s.pbc, vel=v0, colour=s.colour,
                          params=nepspin.integrator_params(**kw), precision=precision)
        if Wm:
            sim.integrate(Wm, observables=False)
        sim.profile(prof_groups)
        sim.profile_read()
        t0 = time.perf_counter()
        sim.integrate(K, observables=False)      # returns after the device finished
        t1 = time.perf_counter()
        prof = sim.profile_read()
        sim.profile(())
        return sim, t1 - t0, prof

    # FP64 (the headline workload); the dominant kernel is timed with HIP events
    dom = "bwd_angular"
    sim64, dt64, prof64 = run("fp64", (dom,))
    rate64 = s.n * K / dt64
    print(f"fp64: {K} steps in {dt64:.3f} s -> {rate64:.4e} atom-steps/s", file=sys.stderr, flush=True)

    pc = pair_counts(s)
    flops_launch = work_model(pc, s.n, int((s.types == 0).sum()))
    ms, nl = prof64[dom]
    avg_ms = ms / max(nl, 1)
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12
    roofline = {"kernel": "k_bwd_angular<double>", "bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": None, "avg_launch_ms": round(avg_ms, 4), "launches": nl,
                "flop_per_launch": flops_launch}

    extra = {}
    if args.breakdown:
        _, _, prof = run("fp64", tuple(nepspin.PROFILE_GROUPS))
        tot = sum(v[0] for v in prof.values())
        for g, (m_, n_) in prof.items():
            print(f"  {g:13s} {m_ / K:8.3f} ms/step  {100 * m_ / tot:5.1f}%  launches/step {n_ / K:.1f}",
                  file=sys.stderr)
        extra["breakdown_ms_per_step"] = {g: round(m_ / K, 4) for g, (m_, n_) in prof.items()}

    if not args.no_fp32:
        _, dt32, _ = run("fp32")
        extra["fp32_mixed"] = {"value": s.n * K / dt32, "ms_per_step": 1e3 * dt32 / K}
        print(f"fp32-mixed: {K} steps in {dt32:.3f} s -> {s.n * K / dt32:.4e} atom-steps/s",
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        O.build(force=False)
        sp = O.step_params(dt=1.0, T0=300.0, alpha=0.1, gammaL=0.01, ensemble=1, K_corr=1, seed=W.SEED_PHILOX)
        t0 = time.perf_counter()
        O.run(s.types, s.pos, v0, s.spin, s.box, s.pbc, params, s.colour, sp, args.cpu_steps)
        t1 = time.perf_counter()
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": s.n * args.cpu_steps / (t1 - t0), "unit": "atom-steps/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} step(s) of the same 262,144-atom workload from its initial state "
                         f"({t1 - t0:.1f} s, OpenMP over atoms)"}

    line = {
        "metric": "atom-steps/s per MI355X (FP64 spin-lattice NEP step)",
        "value": rate64,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": 1e3 * dt64 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded B20 FeGe-like lattice and random NEP weights)",
        "config": {"workload": "FeGe B20 32x32x32 cells, 262,144 atoms (131,072 spins), periodic, "
                               "300 K Langevin + stochastic LLG (alpha 0.1), dt 1 fs, K_corr 1",
                   "atoms": s.n, "precision": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
