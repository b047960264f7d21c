"""ctypes binding of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

RC_R = 6.0
RC_A = 4.5
N_DESC = 102
N_PARAMS = 15438
# The structural-only NEP (no magnetic channels): c^R[4][9][9], c^A[4][7][9],
# then per species W0[64][37], b0[64], w1[64], b1 -- the descriptor is q^R (9)
# and q^A (28), the first 37 entries of the spin-aware one.
N_DESC_STRUCT = 37
N_PARAMS_STRUCT = 324 + 252 + 2 * (64 * 37 + 64 + 64 + 1)


def expand_structural(p):
    """The structural-only model as the spin-aware one with every magnetic
    coefficient and every W0 column of a magnetic channel zero: with zero
    spins the two define the same energy."""
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS_STRUCT,)
    out = np.zeros(N_PARAMS)
    out[:576] = p[:576]
    o_in, o_out = 576, 576 + 4 * 324 + 252
    for t in range(2):
        w0 = p[o_in:o_in + 64 * 37].reshape(64, 37)
        big = np.zeros((64, N_DESC))
        big[:, :37] = w0
        out[o_out:o_out + 64 * N_DESC] = big.ravel()
        o_in += 64 * 37
        o_out += 64 * N_DESC
        out[o_out:o_out + 129] = p[o_in:o_in + 129]
        o_in += 129
        o_out += 129
    assert o_in == N_PARAMS_STRUCT and o_out == N_PARAMS
    return out


def _model(params, spin, n):
    """spin-aware parameters and spins for either model"""
    params = np.asarray(params, dtype=np.float64)
    if params.shape == (N_PARAMS_STRUCT,):
        return expand_structural(params), np.zeros((n, 3)), True
    return params, spin, False


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-ffp-contract=off keeps a*b+c unfused)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class StepParams(ct.Structure):
    _fields_ = [("dt", ct.c_double), ("T0", ct.c_double), ("T1", ct.c_double),
                ("B0", ct.c_double * 3), ("B1", ct.c_double * 3), ("alpha", ct.c_double),
                ("gammaL", ct.c_double), ("mu_s", ct.c_double), ("mid_tol", ct.c_double),
                ("rcR", ct.c_double), ("rcA", ct.c_double), ("n_ramp", ct.c_int64),
                ("seed", ct.c_uint64), ("ensemble", ct.c_int), ("K_corr", ct.c_int),
                ("mid_cap", ct.c_int), ("act", ct.c_int), ("sequential", ct.c_int), ("sc_max", ct.c_int),
                ("sc_tol", ct.c_double), ("sc_depth", ct.c_int), ("sc_reg", ct.c_double),
                ("structural", ct.c_int), ("mass", ct.c_double * 2), ("zbl", ct.c_double * 4),
                ("landau", ct.c_double * 2), ("lsf", ct.c_int), ("lsf_gamma", ct.c_double)]


class Obs(ct.Structure):
    _fields_ = [("step", ct.c_double), ("E_nep", ct.c_double), ("E_kin", ct.c_double),
                ("E_z", ct.c_double), ("T_lat", ct.c_double), ("T_spin", ct.c_double),
                ("M", ct.c_double * 3), ("passes", ct.c_double), ("change", ct.c_double),
                ("capped", ct.c_double), ("s_len", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ct.CDLL(LIB_PATH)
        P = ct.c_void_p
        L.or_eval.argtypes = [ct.c_int, P, P, P, P, P, P, ct.c_double, ct.c_double, ct.c_int,
                              ct.c_double, P, P, P, P, P, P, P, P, P, P]
        L.or_neighbors.argtypes = [ct.c_int, P, P, P, ct.c_double, ct.c_int, ct.c_int, P, P]
        L.or_philox.argtypes = [P, P, P]
        L.or_field_lin.argtypes = [ct.c_int, P, P, P, P, P, P, P, ct.c_double, ct.c_double, ct.c_int,
                                   ct.c_double, P, P]
        L.or_normals.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_uint64, ct.c_uint32, P]
        L.or_anderson_mix.argtypes = [ct.c_int, ct.c_int, P, P, P, P, ct.c_double, P, P]
        L.or_run.argtypes = [ct.c_int, P, P, P, P, P, P, P, P, ct.c_int, ct.POINTER(StepParams),
                             ct.POINTER(ct.c_int64), ct.c_int64, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def neighbors(pos, box, pbc, rc, use_cells=False, maxnb=256):
    """Neighbour sets r_ij < rc (minimum image), ascending j per atom."""
    pos = _f64(pos)
    n = pos.shape[0]
    cnt = np.zeros(n, np.int32)
    nbr = np.full((n, maxnb), -1, np.int32)
    rc_ = lib().or_neighbors(n, _p(pos), _p(_f64(box)), _p(_i32(pbc)), rc, int(use_cells), maxnb,
                             _p(cnt), _p(nbr))
    if rc_ != 0:
        raise RuntimeError("neighbour overflow")
    return [nbr[i, :cnt[i]].copy() for i in range(n)]


def _zbl(zbl):
    """short-range term (Z_0, Z_1, r_inner, r_outer) as a C array, or None"""
    if zbl is None:
        return None
    z = np.ascontiguousarray(zbl, dtype=np.float64)
    assert z.shape == (4,)
    return z


def evaluate(types, pos, spin, box, pbc, params, *, mu_s=1.0, B=(0.0, 0.0, 0.0), act=0,
             rcR=RC_R, rcA=RC_A, want=("E", "F", "H"), zbl=None, landau=None):
    """Energy, forces, fields (and optionally q, Fp, per-atom E) of one system;
    params of the spin-aware model, or of the structural-only one (spins are
    then ignored, and q / Fp keep the first 37 columns). zbl = (Z_0, Z_1,
    r_inner, r_outer) adds the short-range repulsion to E and E_i; landau =
    (a, b) the onsite moment-length term a|s|^2 + b|s|^4 of spin carriers."""
    types = _i32(types)
    pos = _f64(pos)
    n = types.shape[0]
    params, spin, structural = _model(params, spin, n)
    spin = _f64(spin)
    out = {}
    E = np.zeros(1)
    Ez = np.zeros(1)
    Ei = np.zeros(n) if "Ei" in want else None
    F = np.zeros((n, 3)) if "F" in want else None
    H = np.zeros((n, 3)) if "H" in want else None
    q = np.zeros((n, N_DESC)) if "q" in want else None
    Fp = np.zeros((n, N_DESC)) if "Fp" in want else None
    lib().or_eval(n, _p(types), _p(pos), _p(spin), _p(_f64(box)), _p(_i32(pbc)), _p(_f64(params)),
                  rcR, rcA, act, mu_s, _p(_f64(B)), _p(E), _p(Ez), _p(Ei), _p(F), _p(H), _p(q), _p(Fp),
                  _p(_zbl(zbl)), _p(None if landau is None else _f64(landau)))
    out["E"] = float(E[0])
    out["Ez"] = float(Ez[0])
    for k, v in (("Ei", Ei), ("F", F), ("H", H), ("q", q), ("Fp", Fp)):
        if v is not None:
            out[k] = v[:, :N_DESC_STRUCT] if structural and k in ("q", "Fp") else v
    return out


def field_lin(types, pos, spin_hat, spin, box, pbc, params, *, mu_s=1.0, B=(0.0, 0.0, 0.0),
              act=0, rcR=RC_R, rcA=RC_A):
    """Field of the frozen-Fp magnetic energy (Fp* taken at spin_hat) at spins `spin`."""
    types = _i32(types)
    n = types.shape[0]
    H = np.zeros((n, 3))
    lib().or_field_lin(n, _p(types), _p(_f64(pos)), _p(_f64(spin_hat)), _p(_f64(spin)), _p(_f64(box)),
                       _p(_i32(pbc)), _p(_f64(params)), rcR, rcA, act, mu_s, _p(_f64(B)), _p(H))
    return H


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().or_philox(_p(c), _p(k), _p(o))
    return o


def anderson_mix(dF, dG, f, g, reg):
    """One Anderson mixing step (see or_anderson_mix): dF, dG [m][n]; returns (x_next, gamma, used)."""
    dF = _f64(np.atleast_2d(dF))
    dG = _f64(np.atleast_2d(dG))
    m, n = dF.shape if dF.size else (0, len(f))
    x = np.zeros(n)
    gam = np.zeros(max(m, 1))
    used = lib().or_anderson_mix(n, m, _p(dF), _p(dG), _p(_f64(f)), _p(_f64(g)), ct.c_double(reg), _p(x), _p(gam))
    return x, gam[:m], used


def normals(seed, atom, step, stream):
    xi = np.zeros(3)
    lib().or_normals(seed, atom, step, stream, _p(xi))
    return xi


def step_params(*, dt=1.0, T0=0.0, T1=None, B0=(0, 0, 0), B1=None, alpha=0.0, gammaL=0.0,
                mu_s=1.0, mid_tol=1e-15, mid_cap=50, n_ramp=0, seed=0x5EED, ensemble=0,
                K_corr=1, act=0, sequential=0, rcR=RC_R, rcA=RC_A, sc_tol=0.0, sc_max=30, sc_depth=0,
                sc_reg=1e-10, structural=0, mass=(0.0, 0.0), zbl=None, landau=None, lsf=0,
                lsf_gamma=0.0) -> StepParams:
    sp = StepParams()
    if landau is not None:
        sp.landau[0], sp.landau[1] = landau
    sp.lsf = lsf
    sp.lsf_gamma = lsf_gamma
    if zbl is not None:
        for a in range(4):
            sp.zbl[a] = zbl[a]
    sp.dt = dt
    sp.T0 = T0
    sp.T1 = T0 if T1 is None else T1
    for a in range(3):
        sp.B0[a] = B0[a]
        sp.B1[a] = (B0 if B1 is None else B1)[a]
    sp.alpha = alpha
    sp.gammaL = gammaL
    sp.mu_s = mu_s
    sp.mid_tol = mid_tol
    sp.sc_tol = sc_tol
    sp.sc_max = sc_max
    sp.sc_depth = sc_depth
    sp.sc_reg = sc_reg
    sp.structural = structural
    sp.mass[0], sp.mass[1] = mass
    sp.mid_cap = mid_cap
    sp.rcR = rcR
    sp.rcA = rcA
    sp.n_ramp = n_ramp
    sp.seed = seed
    sp.ensemble = ensemble
    sp.K_corr = K_corr
    sp.act = act
    sp.sequential = sequential
    return sp


def run(types, pos, vel, spin, box, pbc, params, colour, sp: StepParams, n_steps, step0=0):
    """n_steps of the spin-lattice step; returns (pos, vel, spin, step, obs[n_steps]), obs columns
    step, E_nep, E_kin, E_z, T_lattice, T_spin, M[3], sweep passes, last change, rotations
    stopped at the cap, mean |s|."""
    types = _i32(types)
    n = types.shape[0]
    params, spin, structural = _model(params, spin, n)
    if structural:
        sp.structural = 1
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    spin = _f64(spin).copy()
    colour = _i32(colour if colour is not None else np.full(n, -1))
    ncol = int(colour.max()) + 1 if colour.size else 0
    st = ct.c_int64(step0)
    obs = (Obs * max(n_steps, 1))()
    lib().or_run(types.shape[0], _p(types), _p(pos), _p(vel), _p(spin), _p(_f64(box)), _p(_i32(pbc)),
                 _p(_f64(params)), _p(colour), ncol, ct.byref(sp), ct.byref(st), n_steps,
                 ct.cast(obs, ct.c_void_p))
    ob = np.array([[o.step, o.E_nep, o.E_kin, o.E_z, o.T_lat, o.T_spin, o.M[0], o.M[1], o.M[2], o.passes, o.change,
                    o.capped, o.s_len] for o in obs[:n_steps]]).reshape(n_steps, 13)
    return pos, vel, spin, st.value, ob
