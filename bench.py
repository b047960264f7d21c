#!/usr/bin/env python3
"""Throughput of the spin-lattice NEP step on one MI355X.

Headline workload: B20 FeGe-like crystal, 32x32x32 cells = 262,144 atoms
(131,072 spins), periodic, seeded random model, 300 K Langevin lattice bath
and stochastic-LLG spin bath (damping 0.1), dt = 1 fs, FP64 end to end. One
step = the whole B A O S A B step (three descriptor passes and read-outs,
two spin-coupling assemblies, four colour sweeps, one backward pass,
neighbour-list upkeep, half-steps and baths) for every atom. Inputs are
resident on the device before the timed region; the clock brackets
sl_integrate_steps, which returns after the device has finished.

Also reported: the FP32-mixed variant of the same workload, a bounded sample
of the replica-serving workload (p50/p99 step latency), the roofline of the
dominant kernel (HIP-event time over the timed region against an algorithmic
FLOP count) and the CPU oracle on the host cores.

Prints one JSON line. --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2606_14073_amd import workload as W  # noqa: E402

# MI355X published peaks
PEAK = {"fp64": 78.6, "fp32": 157.3, "hbm_gbs": 8000.0}
KERNEL_NAME = {"desc_radial": "k_desc_radial<{r}>", "desc_angular": "k_desc_angular<{r}>",
               "readout": "k_mlp<{r},104>", "bwd_radial": "k_bwd_radial<{r}>",
               "bwd_angular": "k_bwd_angular<{r},true>", "bwd_angular_1": "k_bwd_angular<{r},false>",
               "gather": "k_gather<{r}>", "couplings": "k_assemble_angular<{r}>", "pairs": "k_assemble_pairs<{r}>",
               "sweep": "k_sweep<{r}>", "nlist": "k_build_cells", "integrate": "k_kick"}


def kernel_name(group, real="double"):
    """the largest kernel of a profile group, named as in the kernel trace"""
    return KERNEL_NAME.get(group, group).replace("{r}", real)


def pair_counts(s):
    """Ordered neighbour pairs of the workload inside each cutoff."""
    from scipy.spatial import cKDTree
    p = np.mod(s.pos, s.box)
    tree = cKDTree(p, boxsize=s.box)
    fe = s.types == 0
    out = {}
    for rc, key in ((6.0, "R"), (4.5, "A")):
        pr = tree.query_pairs(rc, output_type="ndarray")
        a, b = pr[:, 0], pr[:, 1]
        out[key] = 2 * len(pr)
        out[key + "_fefe"] = 2 * int(np.sum(fe[a] & fe[b]))
        out[key + "_fege"] = 2 * int(np.sum(fe[a] ^ fe[b]))     # ordered pairs with one Fe, one Ge
        out[key + "_fe"] = out[key + "_fefe"] + out[key + "_fege"] // 2   # ordered pairs with an Fe centre
    out["N"] = s.n
    out["N_fe"] = int(fe.sum())
    return out


def flops_per_step(group, pc, k_corr=1):
    """Algorithmic FLOPs of one step's launches of a kernel group (FMA = 2),
    counted once per (centre, neighbour) pair inside the channel's cutoff and
    once per atom; the figures per pair are in the comments below. The
    descriptor and read-out groups run one full pass, one spin-step pass over
    the spin carriers and k_corr spin-step passes that reuse the structural
    angular terms."""
    N, Nfe = pc["N"], pc["N_fe"]
    fe_centre_fe = pc["R_fefe"]             # spin pairs, radial set
    fe_centre_ge = pc["R_fege"] // 2        # Fe centre, Ge neighbour
    if group == "desc_radial":
        # per pair: geometry/basis 80 + radial accumulation 18; Fe-Fe: spin scalars 25 +
        # four magnetic channels 72; Fe-Ge: single-ion 20; per atom contractions
        fe_part = pc["R_fe"] * 98 + fe_centre_fe * 97 + fe_centre_ge * 20 + Nfe * 2 * 5 * 162
        full = fe_part + (pc["R"] - pc["R_fe"]) * 98 + (N - Nfe) * 2 * 162
        return full + (1 + k_corr) * fe_part
    if group == "desc_angular":
        # per pair: geometry/basis 75, g^A 126, harmonics 50, A accumulation 336;
        # spin pairs: g^sa 133, B accumulation 336; per atom q^A, q^sa 672.
        # Reuse passes: spin pairs only (geometry, harmonics, g^sa, B) and q^sa
        full = pc["A"] * 587 + pc["A_fefe"] * 469 + N * 672
        spin = pc["A_fe"] * 587 + pc["A_fefe"] * 469 + Nfe * 672
        reuse = pc["A_fefe"] * (75 + 50 + 133 + 336) + Nfe * 336
        return full + spin + k_corr * reuse
    if group in ("bwd_angular", "bwd_angular_1"):
        # per pair: geometry/basis+derivative 110, g^A and dg^A 252, harmonics and
        # gradients 150, per lm contraction 44 x 24; spin pairs: g^sa, dg^sa 252 and
        # 28 x 24; per atom QA, QS 1008. Species 0 (spin carriers), then species 1.
        if group == "bwd_angular":
            return pc["A_fe"] * 1568 + pc["A_fefe"] * 924 + Nfe * 1008
        return (pc["A"] - pc["A_fe"]) * 1568 + (N - Nfe) * 1008
    if group == "bwd_radial":
        # per pair: geometry/basis+derivative 115, radial dg 18, record 20; Fe-Fe: 8 more
        # channel values 144 + force/field terms 90; Fe-Ge: 36 + 30; per atom contractions
        return pc["R"] * 153 + fe_centre_fe * 234 + fe_centre_ge * 66 + Nfe * 5 * 162 + N * 2 * 162
    if group == "couplings":
        # per spin-step pass: per spin carrier the exchange, DMI and anisotropic
        # contractions 486 and P = Fp^sa A 168; spin-angular part per Fe-Fe pair
        # inside rc_A: geometry/basis 75, g^sa 126, harmonics 50, contraction 336 + 48
        return (1 + k_corr) * (Nfe * (486 + 168) + pc["A_fefe"] * 635)
    if group == "pairs":
        # per spin-step pass: per spin carrier the two single-ion contractions 324;
        # per Fe-Fe pair geometry/basis 80, three coupling values and the single-ion
        # weight 72, its tensor 21, rhat 33; per Fe-Ge pair 80 + 18 + 21
        return (1 + k_corr) * (Nfe * 324 + fe_centre_fe * (173 + 33) + fe_centre_ge * 119)
    if group == "readout":
        # 2 x (104 x 64) FMA per atom + tanh, energy and gradient
        per = 2 * 2 * 104 * 64 + 64 * 30
        return N * per + (1 + k_corr) * Nfe * per
    return None


def sweep_bytes_per_launch(pc, n_colours, real_bytes=8):
    """Algorithmic HBM bytes of one colour-class launch of the spin sweep: per
    spin its couplings inside rc_R (J, D, K, rhat and the neighbour index) and
    the neighbours' spins, its self terms, own spin, noise, list entries, and
    the spin it writes back."""
    nfe = pc["N_fe"]
    nc = pc["R_fefe"] / nfe                      # couplings per spin
    per_spin = nc * (6 * real_bytes + 4 + 24) + 7 * real_bytes + 24 + 24 + 12 + 24
    return per_spin * nfe / n_colours


def sim_rate(model, nepspin, s, v, ip, precision, n_steps, warmup=2):
    """atom-steps/s of n_steps on a resident system (clock around the steps only)."""
    sim = nepspin.Sim(model, s.types, s.pos, s.spin, s.box, s.pbc, vel=v, colour=s.colour, params=ip,
                      precision=precision)
    if warmup:
        sim.integrate(warmup, observables=False)
    t0 = time.perf_counter()
    sim.integrate(n_steps, observables=False)
    t1 = time.perf_counter()
    sim.close()
    return s.n * n_steps / (t1 - t0)


def run_precision_form(model, nepspin, n_steps):
    """96^3 cells = 7,077,888 atoms at 300 K: FP64, FP32-mixed and the BF16
    variant side by side, with the errors of E, F, H against FP64."""
    s = W.config_precision()
    v = W.maxwell_boltzmann(s.types, 300.0)
    ip = nepspin.integrator_params(dt=1.0, T0=300.0, alpha_s=0.1, gamma_L=0.01, ensemble=1, seed=W.SEED_PHILOX)
    out = {"workload": "FeGe B20 96x96x96 cells, 7,077,888 atoms, periodic, 300 K, K_corr 1", "steps": n_steps}
    for prec, key in (("fp64", "fp64"), ("fp32", "fp32_mixed"), ("bf16h", "bf16_hidden")):
        out[key] = sim_rate(model, nepspin, s, v, ip, prec, n_steps)
    ref = model.eval(s.types, s.pos, s.spin, s.box, s.pbc, want=("E", "F", "H"))
    errs = {}
    for prec, key in (("fp32", "fp32_mixed"), ("bf16h", "bf16_hidden")):
        got = model.eval(s.types, s.pos, s.spin, s.box, s.pbc, precision=prec, want=("E", "F", "H"))
        errs[key] = {"dE_per_atom_eV": abs(got["E"] - ref["E"]) / s.n,
                     "F_rel_l2": float(np.linalg.norm(got["F"] - ref["F"]) / np.linalg.norm(ref["F"])),
                     "H_rel_l2": float(np.linalg.norm(got["H"] - ref["H"]) / np.linalg.norm(ref["H"]))}
    out["errors_vs_fp64"] = errs
    return out


def run_slab(model, nepspin, n_steps):
    """256x256x8 cells = 4,194,304 atoms, free z, 700 A helix, T 150 -> 280 K
    and B 0 -> 1 T over 20,000 steps, FP32-mixed."""
    s = W.config_slab()
    v = W.maxwell_boltzmann(s.types, 150.0)
    ip = nepspin.integrator_params(dt=1.0, T0=150.0, T1=280.0, B0=(0, 0, 0), B1=(0, 0, 1.0), n_ramp=20000,
                                   alpha_s=0.1, gamma_L=0.01, ensemble=1, seed=W.SEED_PHILOX)
    return {"workload": "FeGe B20 slab 256x256x8 cells, 4,194,304 atoms, periodic x,y, free z, helix 700 A, "
                        "T 150->280 K, B 0->1 T over 20,000 steps", "steps": n_steps,
            "fp32_mixed": sim_rate(model, nepspin, s, v, ip, "fp32", n_steps)}


def run_self_consistent(model, nepspin, s, v, kw, n_steps, k1_ms_per_step, tol=1e-12):
    """The spin step iterated to a tolerance on the same workload, plain and
    with Anderson mixing (depth 3): passes per step and the cost of a step
    against the fixed K_corr = 1 step."""
    out = {"workload": "same system and schedule, FP64, spin residual <= %g" % tol, "steps": n_steps}
    for key, depth in (("plain", 0), ("anderson_depth3", 3)):
        ip = nepspin.integrator_params(**dict(kw, sc_tol=tol, sc_max=50, sc_depth=depth))
        sim = nepspin.Sim(model, s.types, s.pos, s.spin, s.box, s.pbc, vel=v, colour=s.colour, params=ip,
                          precision="fp64")
        sim.integrate(2, observables=False)
        t0 = time.perf_counter()
        ob = sim.integrate(n_steps)
        t1 = time.perf_counter()
        sim.close()
        ms = 1e3 * (t1 - t0) / n_steps
        out[key] = {"value": s.n * n_steps / (t1 - t0), "unit": "atom-steps/s", "ms_per_step": round(ms, 3),
                    "passes_mean": float(ob[:, 9].mean()), "passes_min": int(ob[:, 9].min()),
                    "passes_max": int(ob[:, 9].max()), "final_change_max": float(ob[:, 10].max()),
                    "cost_vs_kcorr1": round(ms / k1_ms_per_step, 3)}
    return out


def run_structural(nepspin, n_steps, warmup=3):
    """The structural-only NEP (no magnetic channels) on a synthetic water
    liquid of 100^3 molecules = 3,000,000 atoms: 300 K Langevin, dt 0.5 fs,
    skin 0.5 A, FP64 and FP32-mixed. The paper's engine runs liquid water at
    4.38e6 atom-steps/s on one LX2 node (other hardware: context only)."""
    s = W.config_water_bench()
    m = nepspin.Model(W.random_params_structural())
    v = W.maxwell_boltzmann(s.types, 300.0, masses=W.MASS_WATER)
    ip = nepspin.integrator_params(dt=0.5, T0=300.0, gamma_L=0.02, ensemble=1, skin=0.5,
                                   mass=tuple(W.MASS_WATER), seed=W.SEED_PHILOX)
    out = {"workload": "synthetic water, 100^3 molecules = 3,000,000 atoms, random structural NEP, 300 K "
                       "Langevin, dt 0.5 fs, skin 0.5 A", "steps": n_steps, "unit": "atom-steps/s",
           "paper_lx2_node_context": 4.38e6}
    for prec, key in (("fp64", "fp64"), ("fp32", "fp32_mixed")):
        sim = nepspin.Sim(m, s.types, s.pos, None, s.box, s.pbc, vel=v, params=ip, precision=prec)
        sim.integrate(warmup, observables=False)
        t0 = time.perf_counter()
        sim.integrate(n_steps, observables=False)
        t1 = time.perf_counter()
        sim.close()
        out[key] = s.n * n_steps / (t1 - t0)
        out[key + "_ms_per_step"] = round(1e3 * (t1 - t0) / n_steps, 3)
    m.close()
    return out


def run_serving(model, nepspin, n_req, n_steps, rate, seed=7):
    """Poisson arrivals of the serving request mix (cubic FeGe cells, N
    log-uniform 2,048-262,144, T ~ U(50,300) K, B_z ~ U(0,1) T), FP32-mixed."""
    reqs = W.serving_requests(n_req, rate=rate, seed=seed, n_steps=n_steps)
    built = []
    for r in reqs:
        s = W.fege_lattice(r.cells, r.cells, r.cells, seed=r.seed, greedy=False)
        v = W.maxwell_boltzmann(s.types, r.T, seed=r.seed + 1)
        ip = nepspin.integrator_params(dt=1.0, T0=r.T, alpha_s=0.1, gamma_L=0.01, ensemble=1, B0=(0, 0, r.Bz),
                                       seed=r.seed)
        built.append((r, s, v, ip))
    sv = nepspin.Server(model, precision="fp32", steps_per_batch=10, max_slots=256)
    t0 = time.perf_counter()
    ids = []
    for r, s, v, ip in built:
        dt = r.t_arrival - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(sv.submit(s.types, s.pos, s.spin, s.box, s.pbc, vel=v, colour=s.colour, params=ip,
                             n_steps=r.n_steps))
    sv.drain()
    t1 = time.perf_counter()
    st = [sv.poll(k) for k in ids]
    stats = sv.stats()
    sv.close()
    lat50 = [x["step_latency_p50"] for x in st]
    lat99 = [x["step_latency_p99"] for x in st]
    wait = [x["t_admit"] - x["t_submit"] for x in st]
    atoms = sum(s.n for _, s, _, _ in built)
    return {"requests": n_req, "steps_each": n_steps, "arrival_rate_per_s": rate,
            "atoms_total": atoms, "wall_s": round(t1 - t0, 3),
            "atom_steps_per_s": stats["atom_steps"] / (t1 - t0),
            "p50_step_latency_ms": 1e3 * float(np.median(lat50)),
            "p99_step_latency_ms": 1e3 * float(np.percentile(lat99, 99)),
            "mean_queue_wait_s": float(np.mean(wait)),
            "failed": int(sum(x["state"] != nepspin.SL_DONE for x in st)),
            "failures": [{"request": k, "cells": built[k][0].cells, "T": round(built[k][0].T, 1),
                          "Bz": round(built[k][0].Bz, 3), "error": x["error"], "steps_done": x["steps_done"]}
                         for k, x in enumerate(st) if x["state"] != nepspin.SL_DONE]}


KERNEL_SOURCE = {"k_sweep": "kernels_int.hip"}     # every other measured kernel is in kernels_nep.hip


def kernel_source_hash(kernel="k_desc_angular<double>"):
    """Hash of the translation unit that holds `kernel` and the headers it
    includes, to tell whether stored counters are stale."""
    import hashlib
    base = kernel.split("<")[0]
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_14073_amd", "csrc")
    for f in (KERNEL_SOURCE.get(base, "kernels_nep.hip"), "common.h", "engine.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    if there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k or k.get("source_hash") != kernel_source_hash(kernel):
        return None
    return k.get("bytes_per_launch")


def copy_calibration():
    """A plain streaming kernel of known size (reads 1 GiB, writes 1 GiB), for
    scaling the traffic counters."""
    import torch
    n = 1 << 27     # 128 Mi doubles = 1 GiB
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-sc", action="store_true", help="skip the self-consistent midpoint leg")
    ap.add_argument("--no-water", action="store_true", help="skip the structural-only NEP leg")
    ap.add_argument("--water-steps", type=int, default=30)
    ap.add_argument("--water-only", action="store_true",
                    help="run only the structural-only NEP leg and print its result as one JSON line")
    ap.add_argument("--sc-steps", type=int, default=20)
    ap.add_argument("--no-large", action="store_true", help="skip the 7.1M-atom precision form and the 4.2M slab")
    ap.add_argument("--large-steps", type=int, default=20)
    ap.add_argument("--serving-requests", type=int, default=24)
    ap.add_argument("--serving-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--copy-calib", action="store_true", help="run only the copy kernel used to calibrate counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} requested, but this build runs on one GPU only; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration()
        return

    from paper_2606_14073_amd import nepspin
    if args.water_only:
        print(json.dumps(run_structural(nepspin, args.water_steps)), flush=True)
        return

    s = W.config_fp64_bench()
    params = W.random_params()
    v0 = W.maxwell_boltzmann(s.types, 300.0)
    kw = dict(dt=1.0, T0=300.0, alpha_s=0.1, gamma_L=0.01, ensemble=1, K_corr=1, seed=W.SEED_PHILOX)
    model = nepspin.Model(params)
    K, Wm = args.steps, args.warmup

    def run(precision, n_steps, prof_groups=()):
        sim = nepspin.Sim(model, s.types, s.pos, s.spin, s.box, s.pbc, vel=v0, colour=s.colour,
                          params=nepspin.integrator_params(**kw), precision=precision)
        if Wm:
            sim.integrate(Wm, observables=False)
        sim.profile(prof_groups)
        sim.profile_read()
        t0 = time.perf_counter()
        sim.integrate(n_steps, observables=False)      # returns after the device finished
        t1 = time.perf_counter()
        prof = sim.profile_read()
        sim.profile(())
        sim.close()
        return t1 - t0, prof

    # Untimed profiling pass: every kernel group bracketed by HIP events on the
    # library's stream, for the per-step breakdown and the dominant kernel.
    n_prof = max(10, min(K, 50))
    _, prof_all = run("fp64", n_prof, tuple(nepspin.PROFILE_GROUPS))
    tot = sum(v[0] for v in prof_all.values())
    print(f"fp64 profiling pass, {n_prof} steps:", file=sys.stderr)
    for g, (m_, n_) in prof_all.items():
        print(f"  {g:13s} {m_ / n_prof:8.3f} ms/step  {100 * m_ / tot:5.1f}%  launches/step {n_ / n_prof:.1f}",
              file=sys.stderr)
    dom = max(prof_all, key=lambda g: prof_all[g][0])

    # Timed FP64 headline; HIP events bracket only the dominant group's launches.
    dt64, prof = run("fp64", K, (dom,))
    rate64 = s.n * K / dt64
    print(f"fp64: {K} steps in {dt64:.3f} s -> {rate64:.4e} atom-steps/s (dominant: {dom})",
          file=sys.stderr, flush=True)

    pc = pair_counts(s)
    groups = {}
    for g, (ms, nl) in prof_all.items():
        fs = flops_per_step(g, pc, kw["K_corr"])
        if fs is None or nl == 0:
            continue
        per_step = nl / n_prof
        avg = ms / nl
        ach = fs * n_prof / (ms * 1e-3) / 1e12
        groups[g] = {"avg_launch_ms": round(avg, 4), "launches": nl, "flop_per_step": int(fs),
                     "achieved_tflops": round(ach, 3), "frac_fp64_peak": round(ach / PEAK["fp64"], 4),
                     "launches_per_step": per_step}
    kname = kernel_name(dom)
    fs_dom = flops_per_step(dom, pc, kw["K_corr"])
    ms_dom, nl_dom = prof.get(dom, (0.0, 0))
    fl = None if fs_dom is None or not nl_dom else fs_dom * K / nl_dom     # mean FLOPs per launch
    if dom == "sweep" and nl_dom:
        # one profiled sweep = 2 x n_colours - 1 launches of k_sweep (ascending, then
        # descending; the last colour's two visits share one launch)
        ncol = int(s.colour.max()) + 1
        nk = nl_dom * (2 * ncol - 1)
        avg = ms_dom / nk
        by = sweep_bytes_per_launch(pc, ncol)
        ach = by / (avg * 1e-3) / 1e9
        roofline = {"kernel": kname, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_gbs"],
                    "unit": "GB/s", "frac": round(ach / PEAK["hbm_gbs"], 4), "traffic": traffic_from_profile(kname),
                    "avg_launch_ms": round(avg, 5), "launches": nk, "bytes_per_launch": int(by)}
    elif fl is not None and nl_dom:
        avg = ms_dom / nl_dom
        ach = fl / (avg * 1e-3) / 1e12
        roofline = {"kernel": kname, "bound": "mfma" if dom == "readout" else "alu",
                    "achieved": round(ach, 3), "peak": PEAK["fp64"], "unit": "TFLOP/s",
                    "frac": round(ach / PEAK["fp64"], 4), "traffic": traffic_from_profile(kname),
                    "avg_launch_ms": round(avg, 4), "launches": nl_dom, "flop_per_launch": int(fl)}
    else:
        roofline = {"kernel": kname, "bound": None, "achieved": None, "peak": None, "unit": None,
                    "frac": None, "traffic": None, "note": "dominant group has no work model"}

    extra = {"breakdown_ms_per_step": {g: round(m_ / n_prof, 4) for g, (m_, n_) in prof_all.items()},
             "kernel_rooflines": groups}

    if not args.no_fp32:
        # same workload in FP32-mixed: an untimed profiling pass for its breakdown
        # and roofline, then the timed run
        _, p32 = run("fp32", n_prof, tuple(nepspin.PROFILE_GROUPS))
        dom32 = max(p32, key=lambda g: p32[g][0])
        dt32, _ = run("fp32", K)
        f32 = {"value": s.n * K / dt32, "ms_per_step": 1e3 * dt32 / K, "speedup_vs_fp64": dt64 / dt32,
               "breakdown_ms_per_step": {g: round(m_ / n_prof, 4) for g, (m_, n_) in p32.items()},
               "dominant": dom32}
        fs32 = flops_per_step(dom32, pc, kw["K_corr"])
        ms32, nl32 = p32[dom32]
        if dom32 == "sweep" and nl32:
            ncol = int(s.colour.max()) + 1
            nk = nl32 * (2 * ncol - 1)
            by = sweep_bytes_per_launch(pc, ncol, real_bytes=4)
            ach = by / (ms32 / nk * 1e-3) / 1e9
            f32["roofline"] = {"kernel": kernel_name("sweep", "float"), "bound": "hbm", "achieved": round(ach, 1),
                               "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(ach / PEAK["hbm_gbs"], 4),
                               "avg_launch_ms": round(ms32 / nk, 5), "launches": nk}
        elif fs32 is not None and nl32:
            ach = fs32 * n_prof / (ms32 * 1e-3) / 1e12
            f32["roofline"] = {"kernel": kernel_name(dom32, "float"),
                               "bound": "mfma" if dom32 == "readout" else "alu", "achieved": round(ach, 3),
                               "peak": PEAK["fp32"], "unit": "TFLOP/s", "frac": round(ach / PEAK["fp32"], 4),
                               "avg_launch_ms": round(ms32 / nl32, 4), "launches": nl32,
                               "note": "peak is the packed-FP32 vector rate; the kernels are built without "
                                       "packed FP32, whose plain vector rate is 78.6 TFLOP/s"}
        extra["fp32_mixed"] = f32
        print(f"fp32-mixed: {K} steps in {dt32:.3f} s -> {s.n * K / dt32:.4e} atom-steps/s (dominant: {dom32})",
              file=sys.stderr, flush=True)

    if not args.no_sc:
        extra["self_consistent"] = run_self_consistent(model, nepspin, s, v0, kw, args.sc_steps, 1e3 * dt64 / K)
        print(f"self-consistent: {extra['self_consistent']}", file=sys.stderr, flush=True)

    if not args.no_water:
        extra["structural_water"] = run_structural(nepspin, args.water_steps)
        print(f"structural-only NEP, water: {extra['structural_water']}", file=sys.stderr, flush=True)

    if not args.no_serving:
        extra["serving"] = run_serving(model, nepspin, args.serving_requests, args.serving_steps, 20.0)
        print(f"serving: {extra['serving']}", file=sys.stderr, flush=True)

    if not args.no_large:
        # a model of their own: its evaluation engine (up to 120 GB) is released afterwards
        big = nepspin.Model(params)
        extra["precision_form"] = run_precision_form(big, nepspin, args.large_steps)
        print(f"precision form: {extra['precision_form']}", file=sys.stderr, flush=True)
        extra["slab"] = run_slab(big, nepspin, args.large_steps)
        print(f"slab: {extra['slab']}", file=sys.stderr, flush=True)
        big.close()

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
               "sample": f"{args.cpu_steps} full step(s) of the same 262,144-atom workload from its initial state, "
                         f"{t1 - t0:.1f} s with OpenMP over atoms"}
        print(f"cpu oracle: {cpu}", file=sys.stderr, flush=True)

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
