#!/usr/bin/env python3
"""Throughput of the spin-lattice NEP step on one MI355X.

Headline workload: B20 FeGe-like crystal, 96x96x96 cells = 7,077,888 atoms
(3,538,944 spins), periodic, seeded random model plus the short-range
repulsion, 300 K Langevin lattice bath and stochastic-LLG spin bath (damping
0.1), dt = 1 fs, FP64 end to end, with the FP32-mixed path on the same
workload beside it (rate, and E/F/H errors against FP64). One step = the
whole B A O S A B step (three descriptor passes and read-outs, two
spin-coupling assemblies, four colour sweeps, one backward pass,
neighbour-list upkeep, half-steps and baths) for every atom. Inputs are
resident on the device before the timed region; the clock brackets
sl_integrate_steps, which returns after the device has finished.

Also reported: the 262,144-atom workload (FP64 and FP32-mixed), the
self-consistent midpoint, the 4,194,304-atom slab, the structural-only NEP on
synthetic water, a bounded sample of the replica-serving workload (p50/p99
step latency), the roofline of the dominant kernel (HIP-event time over the
timed region against an algorithmic FLOP or byte count) and the CPU oracle on
the host cores.

Prints one JSON line. --gpus N > 1 is refused: the library runs on one GPU.
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


# The library's sweep launcher gives colour classes of at least SWEEP_WIDER_MIN
# spins 4 lanes per spin (kernel k_sweep<real,4>), of at least SWEEP_WIDE_MIN
# 8, smaller ones 16.
SWEEP_WIDE_MIN, SWEEP_WIDER_MIN = 8192, 32768


def kernel_name(group, real="double", colour=None):
    """the largest kernel of a profile group, named as in the kernel trace
    (for the sweep, the lane layout of the largest colour class)"""
    if group == "sweep" and colour is not None:
        c = np.asarray(colour)
        big = np.bincount(c[c >= 0]).max()
        lanes = 4 if big >= SWEEP_WIDER_MIN else 8 if big >= SWEEP_WIDE_MIN else 16
        return f"k_sweep<{real},{lanes}>"
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


def step_model(pc, k_corr, ms_per_step):
    """Whole-step FLOPs per atom-step two ways: an estimate of the method's
    work (per-pair and per-atom figures with the run's neighbour counts: 3 forwards,
    3 read-outs, 2 assemblies at 0.6 of the magnetic forward, the backward at 3
    forwards, 4 sweep visits per spin), and the sum of this file's per-group
    work model plus the sweep; with the achieved rate against the FP64 peak"""
    N, Nfe = pc["N"], pc["N_fe"]
    r_at, a_at = pc["R"] / N, pc["A"] / N
    ff_r, ff_a = pc["R_fefe"] / Nfe, pc["A_fefe"] / Nfe
    mag = (Nfe / N) * (ff_r * (36 + 4 * 2 * 81 + 72) + ff_a * (126 + 336 + 10) + 672)
    fwd = r_at * (66 + 2 * 9 * 9) + mag + a_at * (56 + 2 * 63 + 60 + 2 * 7 * 24)
    mlp = 2 * 2 * 102 * 64
    sweep = (Nfe / N) * 2 * (1 + k_corr) * (ff_r * 30 + 320)
    estimate = (2 + k_corr) * (fwd + mlp) + (1 + k_corr) * 0.6 * mag + 3 * fwd + sweep
    groups = ("desc_radial", "desc_angular", "readout", "bwd_radial", "bwd_angular", "bwd_angular_1",
              "couplings", "pairs")
    counted = sum(flops_per_step(g, pc, k_corr) for g in groups) / N + sweep
    out = {}
    for key, f in (("method_estimate", estimate), ("work_model", counted)):
        t = f * N / (ms_per_step * 1e-3) / 1e12
        out[key] = {"flop_per_atom_step": round(f), "achieved_tflops": round(t, 3),
                    "frac_fp64_peak": round(t / PEAK["fp64"], 4)}
    return out


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


def closest_pair(pos, box):
    """closest atom pair of a slab periodic in x and y (free z), and its z extent"""
    from scipy.spatial import cKDTree
    L = np.asarray(box, dtype=float).reshape(-1)[:3]
    p = pos.copy()
    p[:, :2] %= L[:2]
    p[:, 2] -= p[:, 2].min()
    d, _ = cKDTree(p, boxsize=[L[0], L[1], p[:, 2].max() + 100.0]).query(p, k=2)
    return float(d[:, 1].min()), float(p[:, 2].max())


def run_slab_ramp(model, nepspin, n_steps, chunk=500):
    """The slab workload over n_steps of its 20,000-step T/B ramp in chunks of
    `chunk` steps, stopping at the first failure: per chunk the targets, the
    lattice temperature, the energy, the magnetisation and the recolourings,
    every 2,500 steps the closest pair (progress on stderr)."""
    s = W.config_slab()
    v = W.maxwell_boltzmann(s.types, 150.0)
    ip = nepspin.integrator_params(dt=1.0, T0=150.0, T1=280.0, B0=(0, 0, 0), B1=(0, 0, 1.0), n_ramp=20000,
                                   alpha_s=0.1, gamma_L=0.01, ensemble=1, seed=W.SEED_PHILOX)
    sim = nepspin.Sim(model, s.types, s.pos, s.spin, s.box, s.pbc, vel=v, colour=s.colour, params=ip,
                      precision="fp32")
    done, t_run, nrc, err, rows = 0, 0.0, 0, None, []
    while done < n_steps:
        k = min(chunk, n_steps - done)
        t0 = time.perf_counter()
        try:
            ob = sim.integrate(k)
        except RuntimeError as e:
            err = str(e)
            break
        t_run += time.perf_counter() - t0
        done += k
        nrc = sim.colour()[1]
        f = min(done, 20000) / 20000
        row = {"step": done, "T_target": round(150 + 130 * f, 1), "Bz_target": round(f, 4),
               "T_lattice": round(float(ob[-min(k, 100):, 4].mean()), 1),
               "E_pot_per_atom": round(float(ob[-1, 1]) / s.n, 5), "Mz_mean": round(float(ob[-1, 8]), 5),
               "recolourings": nrc}
        if done % 2500 == 0 or done == n_steps:
            row["closest_pair_A"], row["z_extent_A"] = (round(x, 3) for x in closest_pair(sim.state()[0], s.box))
        rows.append(row)
        print(f"slab: {row}, {s.n * done / t_run:.4e} atom-steps/s", file=sys.stderr, flush=True)
    sim.close()
    return {"workload": "FeGe B20 slab 256x256x8 cells, 4,194,304 atoms, periodic x,y, free z, helix 700 A, "
                        "T 150->280 K, B 0->1 T over 20,000 steps, FP32-mixed",
            "steps_run": done, "steps_asked": n_steps, "stopped_by": err,
            "atom_steps_per_s": s.n * done / t_run if t_run else None, "progress": rows}


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


def run_serving(model, nepspin, n_req, n_steps, rate, seed=7, budget_gb=0.0, max_slots=256):
    """Poisson arrivals of the serving request mix (cubic FeGe cells, N
    log-uniform 2,048-262,144, T ~ U(50,300) K, B_z ~ U(0,1) T), FP32-mixed.
    budget_gb caps the device memory the server may hold (0: free HBM less a
    reserve). Prints progress to stderr every 20 s while replicas run."""
    reqs = W.serving_requests(n_req, rate=rate, seed=seed, n_steps=n_steps)
    built = []
    for r in reqs:
        s = W.fege_lattice(r.cells, r.cells, r.cells, seed=r.seed, greedy=False)
        v = W.maxwell_boltzmann(s.types, r.T, seed=r.seed + 1)
        ip = nepspin.integrator_params(dt=1.0, T0=r.T, alpha_s=0.1, gamma_L=0.01, ensemble=1, B0=(0, 0, r.Bz),
                                       seed=r.seed)
        built.append((r, s, v, ip))
    sv = nepspin.Server(model, precision="fp32", steps_per_batch=10, max_slots=max_slots,
                        hbm_budget_bytes=int(budget_gb * (1 << 30)))
    t0 = time.perf_counter()
    ids = []
    last = t0
    for r, s, v, ip in built:
        dt = r.t_arrival - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(sv.submit(s.types, s.pos, s.spin, s.box, s.pbc, vel=v, colour=s.colour, params=ip,
                             n_steps=r.n_steps))
    while True:
        done = sum(sv.poll(k)["state"] >= nepspin.SL_DONE for k in ids)
        if done == len(ids):
            break
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            print(f"serving: {last - t0:.0f} s, {done}/{len(ids)} replicas done", file=sys.stderr, flush=True)
        time.sleep(0.01)
    sv.drain()
    t1 = time.perf_counter()
    st = [sv.poll(k) for k in ids]
    stats = sv.stats()
    host = sv.host_stats()
    sv.close()
    lat50 = [x["step_latency_p50"] for x in st]
    lat99 = [x["step_latency_p99"] for x in st]
    wait = [x["t_admit"] - x["t_submit"] for x in st]
    atoms = sum(s.n for _, s, _, _ in built)
    return {"requests": n_req, "steps_each": n_steps, "arrival_rate_per_s": rate,
            "hbm_budget_gb": budget_gb or "free HBM less the reserve", "max_slots": max_slots,
            "atoms_total": atoms, "wall_s": round(t1 - t0, 3),
            "atom_steps_per_s": stats["atom_steps"] / (t1 - t0),
            "p50_step_latency_ms": 1e3 * float(np.median(lat50)),
            "p99_step_latency_ms": 1e3 * float(np.percentile(lat99, 99)),
            "mean_queue_wait_s": float(np.mean(wait)), "max_queue_wait_s": float(np.max(wait)),
            "batched_steps": stats["batched_steps"], "batch_busy_s": round(stats["busy_s"], 3),
            "relayouts": host["relayouts"], "relayout_s": round(host["relayout_s"], 3),
            "host_gap_s": round(host["gap_s"], 3),
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


def traffic_from_profile(kernel, n_atoms):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    if there is none, it was taken on another workload size, or the kernel's
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    sets = d.get("workloads", [d])
    match = [w for w in sets if w.get("n_atoms") == n_atoms]
    if not match:
        return None
    k = match[0].get("kernels", {}).get(kernel)
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


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pair_counts_scaled(s, cells=16):
    """pair counts of a crystal too large for a k-d tree pass: those of a
    cells^3 crystal from the same generator, scaled by the atom count (the
    counts per atom of the periodic lattice do not depend on its size)"""
    small = pair_counts(W.fege_lattice(cells, cells, cells))
    f = s.n / small["N"]
    out = {k: int(round(v * f)) for k, v in small.items()}
    out["N"], out["N_fe"] = s.n, int((s.types == 0).sum())
    return out


def roofline_of(group, prof, pc, n_steps, k_corr, s, real="double"):
    """roofline of one kernel group from its HIP-event time over n_steps: the
    colour sweep against HBM (algorithmic bytes), the others against the FP64
    vector (or MFMA) peak with the work model of flops_per_step"""
    ms, nl = prof.get(group, (0.0, 0))
    rb = 8 if real == "double" else 4
    kname = kernel_name(group, real, s.colour)
    if not nl:
        return {"kernel": kname, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "note": "no timed launches"}
    if group == "sweep":
        # one timed sweep = 2 x n_colours - 1 launches of k_sweep (ascending, then
        # descending; the turning colour's two visits share one launch)
        ncol = int(s.colour.max()) + 1
        nk = nl * (2 * ncol - 1)
        avg = ms / nk
        by = sweep_bytes_per_launch(pc, ncol, real_bytes=rb)
        ach = by / (avg * 1e-3) / 1e9
        return {"kernel": kname, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_gbs"],
                "unit": "GB/s", "frac": round(ach / PEAK["hbm_gbs"], 4), "traffic": traffic_from_profile(kname, s.n),
                "avg_launch_ms": round(avg, 5), "launches": nk, "bytes_per_launch": int(by)}
    fs = flops_per_step(group, pc, k_corr)
    if fs is None:
        return {"kernel": kname, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "note": "group has no work model"}
    fl = fs * n_steps / nl            # mean FLOPs per launch
    avg = ms / nl
    ach = fl / (avg * 1e-3) / 1e12
    peak = PEAK["fp64"] if real == "double" else PEAK["fp32"]
    out = {"kernel": kname, "bound": "mfma" if group == "readout" else "alu", "achieved": round(ach, 3),
           "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": traffic_from_profile(kname, s.n),
           "avg_launch_ms": round(avg, 4), "launches": nl, "flop_per_launch": int(fl)}
    if real != "double":
        out["note"] = ("peak is the packed-FP32 vector rate; the kernels are built without packed FP32, whose "
                       "plain vector rate is 78.6 TFLOP/s")
    return out


def cpu_baseline(params, s1, s2, v2):
    """The oracle on the host cores: the 512-atom workload's 100 NVE steps in
    full on every thread OpenMP gets, 10 of them on one thread, and one step of
    the 262,144-atom workload (atom-steps/s of each)"""
    import subprocess
    from oracle import oracle as O
    O.build(force=False)
    zbl = W.SHORT_RANGE_FEGE
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sp1 = O.step_params(dt=1.0, B0=(0, 0, 1.0), K_corr=1, zbl=zbl)
    t0 = time.perf_counter()
    O.run(s1.types, s1.pos, np.zeros((s1.n, 3)), s1.spin, s1.box, s1.pbc, params, s1.colour, sp1, 100)
    dt1 = time.perf_counter() - t0
    full = s1.n * 100 / dt1
    # one thread: a child process, since OpenMP fixes its team size at start-up
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r); from oracle import oracle as O; "
            "from paper_2606_14073_amd import workload as W; s = W.config_small(); p = W.random_params(); "
            "sp = O.step_params(dt=1.0, B0=(0, 0, 1.0), K_corr=1, zbl=W.SHORT_RANGE_FEGE); t0 = time.perf_counter(); "
            "O.run(s.types, s.pos, np.zeros((s.n, 3)), s.spin, s.box, s.pbc, p, s.colour, sp, 10); "
            "print(s.n * 10 / (time.perf_counter() - t0))" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        one = float(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                   timeout=300, check=True).stdout.split()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError):
        one = None
    sp2 = O.step_params(dt=1.0, T0=300.0, alpha=0.1, gammaL=0.01, ensemble=1, K_corr=1, seed=W.SEED_PHILOX,
                        zbl=zbl)
    t0 = time.perf_counter()
    O.run(s2.types, s2.pos, v2, s2.spin, s2.box, s2.pbc, params, s2.colour, sp2, 1)
    t2 = time.perf_counter() - t0
    return {"value": full, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"the 512-atom workload (4x4x4 cells), its 100 NVE steps in full, {dt1:.1f} s on "
                      f"{cores} OpenMP threads; host CPU: {host_cpu_model()}",
            "one_thread": one, "one_thread_sample": "10 steps of the same 512-atom workload on 1 thread",
            "config_262144_one_step": s2.n / t2,
            "config_262144_sample": f"1 step of the 262,144-atom workload at 300 K, {t2:.1f} s on {cores} threads "
                                    "(a 10-step sample does not fit the benchmark's time)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-sc", action="store_true", help="skip the self-consistent midpoint leg")
    ap.add_argument("--no-water", action="store_true", help="skip the structural-only NEP leg")
    ap.add_argument("--no-262k", action="store_true", help="skip the 262,144-atom legs")
    ap.add_argument("--no-slab", action="store_true", help="skip the 4.2M-atom slab leg")
    ap.add_argument("--water-steps", type=int, default=30)
    ap.add_argument("--water-only", action="store_true",
                    help="run only the structural-only NEP leg and print its result as one JSON line")
    ap.add_argument("--crystal-only", action="store_true",
                    help="run only the 262,144-atom crystal legs (FP64 and FP32-mixed) and print them as one JSON line")
    ap.add_argument("--sc-steps", type=int, default=20)
    ap.add_argument("--side-steps", type=int, default=50, help="timed steps of the 262,144-atom and slab legs")
    ap.add_argument("--serving-requests", type=int, default=24)
    ap.add_argument("--serving-steps", type=int, default=100)
    ap.add_argument("--serving-budget-gb", type=float, default=0.0,
                    help="device-memory cap of the server (0: free HBM less a reserve)")
    ap.add_argument("--serving-slots", type=int, default=256)
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg and print its result as one JSON line")
    ap.add_argument("--slab-ramp", type=int, default=0, metavar="STEPS",
                    help="run only the slab workload over STEPS steps of its ramp (stops at the first failure) "
                         "and print the result as one JSON line")
    ap.add_argument("--copy-calib", action="store_true", help="run only the copy kernel used to calibrate counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} requested, but the library runs on one GPU only; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration()
        return

    from paper_2606_14073_amd import nepspin
    if args.water_only:
        print(json.dumps(run_structural(nepspin, args.water_steps)), flush=True)
        return

    params = W.random_params()
    model = nepspin.Model(params, short_range=W.SHORT_RANGE_FEGE)
    kw = dict(dt=1.0, T0=300.0, alpha_s=0.1, gamma_L=0.01, ensemble=1, K_corr=1, seed=W.SEED_PHILOX)
    K, Wm = args.steps, args.warmup

    def run(s, v, precision, n_steps, prof_groups=(), warm=Wm):
        sim = nepspin.Sim(model, s.types, s.pos, s.spin, s.box, s.pbc, vel=v, colour=s.colour,
                          params=nepspin.integrator_params(**kw), precision=precision)
        if warm:
            sim.integrate(warm, observables=False)
        sim.profile(prof_groups)
        sim.profile_read()
        t0 = time.perf_counter()
        sim.integrate(n_steps, observables=False)      # returns after the device finished
        t1 = time.perf_counter()
        prof = sim.profile_read()
        sim.profile(())
        sim.close()
        return t1 - t0, prof

    def breakdown(prof, n):
        tot = sum(v[0] for v in prof.values()) or 1.0
        return {g: {"ms_per_step": round(m_ / n, 4), "share": round(m_ / tot, 4), "launches_per_step": n_ / n}
                for g, (m_, n_) in prof.items()}

    s2 = W.config_fp64_bench()
    v2 = W.maxwell_boltzmann(s2.types, 300.0)

    def crystal_leg():
        pc2 = pair_counts(s2)
        n2 = args.side_steps
        leg = {"workload": "FeGe B20 32x32x32 cells, 262,144 atoms (131,072 spins), periodic, 300 K Langevin + "
                           "stochastic LLG (alpha 0.1), dt 1 fs, K_corr 1, short-range term", "steps": n2}
        _, p2 = run(s2, v2, "fp64", n2, tuple(nepspin.PROFILE_GROUPS))
        leg["breakdown_ms_per_step"] = {g: b["ms_per_step"] for g, b in breakdown(p2, n2).items()}
        for prec, key in (("fp64", "fp64"), ("fp32", "fp32_mixed")):
            dtx, _ = run(s2, v2, prec, n2)
            leg[key] = s2.n * n2 / dtx
            leg[key + "_ms_per_step"] = round(1e3 * dtx / n2, 3)
        dom2 = max(p2, key=lambda g: p2[g][0])
        leg["dominant"] = dom2
        leg["roofline"] = roofline_of(dom2, p2, pc2, n2, kw["K_corr"], s2)
        return leg

    if args.serving_only:
        print(json.dumps(run_serving(model, nepspin, args.serving_requests, args.serving_steps, 20.0,
                                     budget_gb=args.serving_budget_gb, max_slots=args.serving_slots)), flush=True)
        model.close()
        return
    if args.slab_ramp:
        print(json.dumps(run_slab_ramp(model, nepspin, args.slab_ramp)), flush=True)
        model.close()
        return

    if args.crystal_only:
        print(json.dumps(crystal_leg()), flush=True)
        model.close()
        return

    # Headline: the largest single-GPU workload, 96^3 cells = 7,077,888 atoms,
    # FP64, 300 K Langevin + stochastic LLG, K_corr 1. An untimed profiling
    # pass with HIP events around every kernel group gives the breakdown and
    # the dominant group; the timed run brackets only that group's launches.
    s3 = W.config_precision()
    v3 = W.maxwell_boltzmann(s3.types, 300.0)
    pc3 = pair_counts_scaled(s3)
    n_prof = max(5, min(K, 10))
    _, prof_all = run(s3, v3, "fp64", n_prof, tuple(nepspin.PROFILE_GROUPS), warm=2)
    dom = max(prof_all, key=lambda g: prof_all[g][0])
    print(f"fp64 profiling pass, 7,077,888 atoms, {n_prof} steps:", file=sys.stderr)
    for g, b in breakdown(prof_all, n_prof).items():
        print(f"  {g:13s} {b['ms_per_step']:8.3f} ms/step  {100 * b['share']:5.1f}%  launches/step "
              f"{b['launches_per_step']:.1f}", file=sys.stderr)
    dt64, prof = run(s3, v3, "fp64", K, (dom,))
    rate64 = s3.n * K / dt64
    print(f"fp64: {K} steps in {dt64:.3f} s -> {rate64:.4e} atom-steps/s (dominant: {dom})",
          file=sys.stderr, flush=True)
    roofline = roofline_of(dom, prof, pc3, K, kw["K_corr"], s3)
    groups = {}
    for g, (ms, nl) in prof_all.items():
        fs = flops_per_step(g, pc3, kw["K_corr"])
        if fs is None or nl == 0:
            continue
        ach = fs * n_prof / (ms * 1e-3) / 1e12
        groups[g] = {"avg_launch_ms": round(ms / nl, 4), "launches": nl, "flop_per_step": int(fs),
                     "achieved_tflops": round(ach, 3), "frac_fp64_peak": round(ach / PEAK["fp64"], 4)}
    extra = {"breakdown_ms_per_step": {g: b["ms_per_step"] for g, b in breakdown(prof_all, n_prof).items()},
             "kernel_rooflines": groups, "step_model": step_model(pc3, kw["K_corr"], 1e3 * dt64 / K)}

    if not args.no_fp32:
        _, p32 = run(s3, v3, "fp32", n_prof, tuple(nepspin.PROFILE_GROUPS), warm=2)
        dom32 = max(p32, key=lambda g: p32[g][0])
        dt32, pr32 = run(s3, v3, "fp32", K, (dom32,))
        f32 = {"value": s3.n * K / dt32, "unit": "atom-steps/s", "ms_per_step": 1e3 * dt32 / K,
               "speedup_vs_fp64": dt64 / dt32,
               "breakdown_ms_per_step": {g: b["ms_per_step"] for g, b in breakdown(p32, n_prof).items()},
               "dominant": dom32, "roofline": roofline_of(dom32, pr32, pc3, K, kw["K_corr"], s3, "float")}
        # errors of the FP32-mixed potential against FP64 on the same state
        ref = model.eval(s3.types, s3.pos, s3.spin, s3.box, s3.pbc, B=(0, 0, 0.5), want=("E", "Ei", "F", "H"))
        got = model.eval(s3.types, s3.pos, s3.spin, s3.box, s3.pbc, B=(0, 0, 0.5), precision="fp32",
                         want=("E", "Ei", "F", "H"))
        f32["errors_vs_fp64"] = {
            "dE_per_atom_eV": abs(got["E"] - ref["E"]) / s3.n,
            "max_dEi_eV": float(np.abs(got["Ei"] - ref["Ei"]).max()),
            "F_rel_l2": float(np.linalg.norm(got["F"] - ref["F"]) / np.linalg.norm(ref["F"])),
            "H_rel_l2": float(np.linalg.norm(got["H"] - ref["H"]) / np.linalg.norm(ref["H"])),
            "bounds": "|dE|/N <= 1e-6 eV, F and H rel-l2 <= 1e-5"}
        del ref, got
        model.close()
        model = nepspin.Model(params, short_range=W.SHORT_RANGE_FEGE)   # releases the 7M-atom eval arrays
        extra["fp32_mixed"] = f32
        print(f"fp32-mixed: {K} steps in {dt32:.3f} s -> {f32['value']:.4e} atom-steps/s (dominant: {dom32}); "
              f"errors {f32['errors_vs_fp64']}", file=sys.stderr, flush=True)

    if not args.no_262k:
        leg = crystal_leg()
        extra["fege_262k"] = leg
        print(f"262,144 atoms: {leg}", file=sys.stderr, flush=True)
        if not args.no_sc:
            extra["self_consistent"] = run_self_consistent(model, nepspin, s2, v2, kw, args.sc_steps,
                                                           leg["fp64_ms_per_step"])
            print(f"self-consistent: {extra['self_consistent']}", file=sys.stderr, flush=True)

    if not args.no_slab:
        extra["slab"] = run_slab(model, nepspin, args.side_steps)
        print(f"slab: {extra['slab']}", file=sys.stderr, flush=True)

    if not args.no_water:
        extra["structural_water"] = run_structural(nepspin, args.water_steps)
        print(f"structural-only NEP, water: {extra['structural_water']}", file=sys.stderr, flush=True)

    if not args.no_serving:
        extra["serving"] = run_serving(model, nepspin, args.serving_requests, args.serving_steps, 20.0,
                                       budget_gb=args.serving_budget_gb, max_slots=args.serving_slots)
        print(f"serving: {extra['serving']}", file=sys.stderr, flush=True)
    model.close()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(params, W.config_small(), s2, v2)
        print(f"cpu oracle: {cpu}", file=sys.stderr, flush=True)

    line = {
        "metric": "atom\u00b7steps/s per MI355X, FP64 vs FP32-mixed; p50/p99 replica step latency",
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
        "data": "synthetic (seeded B20 FeGe-like lattice, random NEP weights plus the short-range term)",
        "config": {"workload": "FeGe B20 96x96x96 cells, 7,077,888 atoms (3,538,944 spins), periodic, 300 K "
                               "Langevin + stochastic LLG (alpha 0.1), dt 1 fs, K_corr 1, FP64; FP32-mixed "
                               "beside it",
                   "atoms": s3.n, "precision": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
