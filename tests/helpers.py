"""Shared test helpers: error norms and local-cluster oracle evaluations."""
import numpy as np


def rel_inf(a, b):
    """||a - b||_inf / ||b||_inf"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max() if a.size else 0.0)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def min_image_delta(a, b, box, pbc):
    d = np.asarray(a) - np.asarray(b)
    for x in range(3):
        if pbc[x]:
            d[..., x] -= box[x] * np.rint(d[..., x] / box[x])
    return d


def pos_error(pos1, rp, pos0, box, pbc):
    """Position error of one step, relative to the step's own displacement:
    ||dr||_inf / ||r^{n+1} - r^n||_inf (minimum image), with r^{n+1} the
    reference. Stored coordinates round at ulp(|r|), about 3e-14 A on a 150 A
    box, i.e. ~1e-11 of a 1 fs displacement; that floor (4 ulp of the largest
    coordinate) is subtracted before the ratio is taken."""
    dpos = np.abs(min_image_delta(pos1, rp, box, pbc)).max()
    disp = np.abs(min_image_delta(rp, pos0, box, pbc)).max()
    floor = 4 * np.spacing(np.abs(rp).max())
    return max(dpos - floor, 0.0) / disp if disp > 0 else dpos


def cluster_around(types, pos, spin, box, pbc, k, radius):
    """Atoms within `radius` of atom k, unwrapped by minimum image into a free
    cluster centred on atom k (at the origin), so that its displacements to
    the others are the minimum-image ones bit for bit; returns (types, pos,
    spin, index of k in the cluster)."""
    d = min_image_delta(pos, pos[k], box, pbc)
    sel = np.nonzero((d * d).sum(axis=1) < radius * radius)[0]
    return types[sel], d[sel], spin[sel], int(np.nonzero(sel == k)[0][0])


def oracle_local(oracle, types, pos, spin, box, pbc, params, atoms, *, B=(0, 0, 0), mu_s=1.0, zbl=None):
    """Per-atom E_i, F_i, H_i of selected atoms of a large system, each from a
    free cluster of radius 2 rc + 1 A around it (everything that reaches it)."""
    Ei, F, H = [], [], []
    for k in atoms:
        ct, cp, cs, kk = cluster_around(types, pos, spin, box, pbc, k, 13.0)
        o = oracle.evaluate(ct, cp, cs, np.array([1e5] * 3), np.zeros(3, np.int32), params, B=B, mu_s=mu_s,
                            want=("E", "F", "H", "Ei"), zbl=zbl)
        Ei.append(o["Ei"][kk])
        F.append(o["F"][kk])
        H.append(o["H"][kk])
    return np.array(Ei), np.array(F), np.array(H)


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def approaching_pair(s, d_lo=6.62, d_hi=6.9, speed=0.015):
    """A colouring of system s (greedy at 6.6 A, so valid for lists up to
    rc_R + skin = 6.5 A) and velocities that drive one same-colour spin pair,
    first found at a distance in (d_lo, d_hi), head-on towards each other at
    `speed` A/fs each; every other atom starts at rest. Returns (colour, vel,
    (i, j))."""
    from paper_2606_14073_amd import workload as W
    col = W.colour_greedy(s.types, s.pos, s.box, s.pbc, 6.6)
    fe = np.nonzero(s.types == 0)[0]
    for i in fe:
        d = min_image_delta(s.pos[fe], s.pos[i], s.box, s.pbc)
        r = np.sqrt((d * d).sum(axis=1))
        cand = np.nonzero((col[fe] == col[i]) & (r > d_lo) & (r < d_hi))[0]
        if cand.size:
            j = fe[cand[0]]
            u = d[cand[0]] / r[cand[0]]
            vel = np.zeros((s.n, 3))
            vel[i] = speed * u
            vel[j] = -speed * u
            return col, vel, (int(i), int(j))
    raise AssertionError("no same-colour pair in range")
