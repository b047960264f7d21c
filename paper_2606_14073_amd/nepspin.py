"""Python binding of libnepspin.so (the C ABI in include/nepspin.h).

Argument marshalling only: every step of the computation runs in the HIP
library. Importing this module does not need a GPU; calling into the library
does, and fails loudly when the library or the device is missing.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnepspin.so")

SL_OK, SL_E_INVALID, SL_E_OOM, SL_E_BOX, SL_E_DEVICE, SL_E_NONFINITE, SL_E_NOTFOUND, SL_E_BUSY, \
    SL_E_OVERFLOW, SL_E_NOLIB = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
SL_FP64, SL_FP32_MIXED = 0, 1
SL_QUEUED, SL_RUNNING, SL_DONE, SL_FAILED = 0, 1, 2, 3

PRECISION = {"fp64": SL_FP64, "fp32": SL_FP32_MIXED}

EXPORTS = ["sl_last_error", "nep_model_create", "nep_model_destroy", "nep_spin_eval", "nep_spin_eval_noalloc",
           "nep_spin_descriptors",
           "sl_create", "sl_integrate_steps", "sl_get_state", "sl_set_state", "sl_destroy", "sl_server_create",
           "sl_replica_submit", "sl_replica_poll", "sl_replica_fetch", "sl_server_drain", "sl_server_stats",
           "sl_server_host_stats", "sl_server_destroy", "sl_profile_enable", "sl_profile_read", "sl_get_colour", "sl_replica_bytes"]

PROFILE_GROUPS = ["desc_radial", "desc_angular", "readout", "bwd_radial", "bwd_angular", "gather", "couplings",
                  "sweep", "nlist", "integrate", "pairs", "bwd_angular_1"]


def replica_bytes(n_atoms, precision="fp64"):
    """Device bytes a replica of n_atoms is charged against a server's HBM budget."""
    return int(load().sl_replica_bytes(int(n_atoms), PRECISION[precision]))


class NepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class HParams(ct.Structure):
    _fields_ = [("n_max_R", ct.c_int), ("n_max_A", ct.c_int), ("l_max", ct.c_int), ("basis_K", ct.c_int),
                ("n_hidden", ct.c_int), ("n_species", ct.c_int), ("rc_R", ct.c_double), ("rc_A", ct.c_double),
                ("structural", ct.c_int), ("sr_Z", ct.c_double * 2), ("sr_r_inner", ct.c_double),
                ("sr_r_outer", ct.c_double), ("moment_a", ct.c_double), ("moment_b", ct.c_double)]

N_PARAMS = 15438
N_PARAMS_STRUCT = 5570     # structural-only NEP: c^R, c^A, per species W0[64][37], b0, w1, b1


class SystemView(ct.Structure):
    _fields_ = [("n_atoms", ct.c_int64), ("types", ct.c_void_p), ("pos", ct.c_void_p), ("spin", ct.c_void_p),
                ("box", ct.c_double * 3), ("pbc", ct.c_int32 * 3), ("mu_s", ct.c_double), ("B", ct.c_double * 3)]


class Exec(ct.Structure):
    _fields_ = [("device_ptrs", ct.c_int), ("hip_stream", ct.c_void_p)]


class IntegratorParams(ct.Structure):
    _fields_ = [("dt", ct.c_double), ("T0", ct.c_double), ("T1", ct.c_double), ("B0", ct.c_double * 3),
                ("B1", ct.c_double * 3), ("alpha_s", ct.c_double), ("gamma_L", ct.c_double),
                ("n_ramp", ct.c_int64), ("ensemble", ct.c_int), ("K_corr", ct.c_int), ("mid_tol", ct.c_double),
                ("mid_cap", ct.c_int), ("seed", ct.c_uint64), ("skin", ct.c_double), ("sc_tol", ct.c_double),
                ("sc_max", ct.c_int), ("mass", ct.c_double * 2), ("sc_depth", ct.c_int), ("sc_reg", ct.c_double),
                ("longitudinal", ct.c_int), ("gamma_lsf", ct.c_double)]


class Observables(ct.Structure):
    _fields_ = [("step", ct.c_int64), ("E_pot", ct.c_double), ("E_kin", ct.c_double), ("E_zeeman", ct.c_double),
                ("T_lattice", ct.c_double), ("T_spin", ct.c_double), ("M", ct.c_double * 3),
                ("spin_passes", ct.c_int32), ("mid_capped", ct.c_int32), ("spin_change", ct.c_double),
                ("spin_length", ct.c_double)]


class ServerConfig(ct.Structure):
    _fields_ = [("hbm_budget_bytes", ct.c_size_t), ("max_slots", ct.c_int), ("precision", ct.c_int),
                ("steps_per_batch", ct.c_int), ("K_corr", ct.c_int)]


class ReplicaStatus(ct.Structure):
    _fields_ = [("state", ct.c_int), ("error", ct.c_int), ("steps_done", ct.c_int64), ("n_steps", ct.c_int64),
                ("t_submit", ct.c_double), ("t_admit", ct.c_double), ("t_done", ct.c_double),
                ("step_latency_p50", ct.c_double), ("step_latency_p99", ct.c_double),
                ("n_latency_samples", ct.c_int64)]


_lib = None


def load():
    """Load libnepspin.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_14073_amd/build.py "
                              "(the library has no CPU fallback)")
        # PyTorch ships its own libamdhip64.so.7; loading it first lets the
        # library bind to the same HIP runtime, so device pointers and streams
        # from torch are valid here (two runtimes in one process do not mix).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ct.CDLL(LIB_PATH)
        P, I64 = ct.c_void_p, ct.c_int64
        L.sl_last_error.restype = ct.c_char_p
        L.nep_model_create.argtypes = [ct.POINTER(HParams), P, ct.c_size_t, ct.POINTER(P)]
        L.nep_model_destroy.argtypes = [P]
        L.nep_spin_eval.argtypes = [P, ct.POINTER(SystemView), ct.c_int, P, P, P, P, ct.POINTER(Exec)]
        L.nep_spin_eval_noalloc.argtypes = [P, ct.POINTER(SystemView), ct.c_int, P, P, P, P, ct.POINTER(Exec)]
        L.nep_spin_descriptors.argtypes = [P, ct.POINTER(SystemView), ct.c_int, P, P, ct.POINTER(Exec)]
        L.sl_create.argtypes = [P, ct.POINTER(SystemView), P, P, ct.POINTER(IntegratorParams), ct.c_int,
                                ct.POINTER(P)]
        L.sl_integrate_steps.argtypes = [P, I64, P]
        L.sl_get_state.argtypes = [P, P, P, P, ct.POINTER(I64)]
        L.sl_set_state.argtypes = [P, P, P, P, I64]
        L.sl_destroy.argtypes = [P]
        L.sl_server_create.argtypes = [P, ct.POINTER(ServerConfig), ct.POINTER(P)]
        L.sl_replica_submit.argtypes = [P, ct.POINTER(SystemView), P, P, ct.POINTER(IntegratorParams), I64,
                                        ct.POINTER(ct.c_uint64)]
        L.sl_replica_poll.argtypes = [P, ct.c_uint64, ct.POINTER(ReplicaStatus)]
        L.sl_replica_fetch.argtypes = [P, ct.c_uint64, P, P, P, ct.POINTER(Observables)]
        L.sl_server_drain.argtypes = [P]
        L.sl_server_stats.argtypes = [P, ct.POINTER(I64), ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
        L.sl_server_destroy.argtypes = [P]
        L.sl_profile_enable.argtypes = [P, ct.c_uint]
        L.sl_profile_read.argtypes = [P, P, P]
        L.sl_get_colour.argtypes = [P, P, ct.POINTER(I64)]
        L.sl_replica_bytes.argtypes = [I64, ct.c_int]
        L.sl_replica_bytes.restype = ct.c_size_t
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise NepError(rc, load().sl_last_error().decode())


def _p(a):
    # data_as keeps the array alive for as long as the pointer object lives
    # (through the call), also when the array is a temporary conversion
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def system_view(types, pos, spin, box, pbc=(1, 1, 1), mu_s=1.0, B=(0.0, 0.0, 0.0)):
    """Build an sl_system_view; returns (view, keep-alive arrays)."""
    t, p = _i32(types), _f64(pos)
    s = _f64(spin) if spin is not None else None
    v = SystemView()
    v.n_atoms = t.shape[0]
    v.types = t.ctypes.data
    v.pos = p.ctypes.data
    v.spin = s.ctypes.data if s is not None else None
    for a in range(3):
        v.box[a] = float(box[a])
        v.pbc[a] = int(pbc[a])
        v.B[a] = float(B[a])
    v.mu_s = mu_s
    return v, (t, p, s)


def integrator_params(*, dt=1.0, T0=0.0, T1=None, B0=(0, 0, 0), B1=None, alpha_s=0.0, gamma_L=0.0, n_ramp=0,
                      ensemble=0, K_corr=1, mid_tol=1e-15, mid_cap=50, seed=0x5EED, skin=0.5, sc_tol=0.0,
                      sc_max=30, sc_depth=0, sc_reg=1e-10, mass=(0.0, 0.0), longitudinal=0, gamma_lsf=0.0):
    ip = IntegratorParams()
    ip.dt, ip.T0, ip.T1 = dt, T0, T0 if T1 is None else T1
    for a in range(3):
        ip.B0[a] = B0[a]
        ip.B1[a] = (B0 if B1 is None else B1)[a]
    ip.alpha_s, ip.gamma_L, ip.n_ramp, ip.ensemble = alpha_s, gamma_L, n_ramp, ensemble
    ip.K_corr, ip.mid_tol, ip.mid_cap, ip.seed, ip.skin = K_corr, mid_tol, mid_cap, seed, skin
    ip.sc_tol, ip.sc_max, ip.sc_depth, ip.sc_reg = sc_tol, sc_max, sc_depth, sc_reg
    ip.mass[0], ip.mass[1] = mass
    ip.longitudinal, ip.gamma_lsf = longitudinal, gamma_lsf
    return ip


class Model:
    """nep_model_create: the spin-aware NEP (15,438 parameters) or the
    structural-only one (5,570 parameters), told apart by the length.
    short_range = (Z_0, Z_1, r_inner, r_outer) adds the screened-Coulomb
    repulsion, landau = (a, b) the onsite moment-length term a|s|^2 + b|s|^4
    of spin carriers; None leaves either off."""

    def __init__(self, params, short_range=None, landau=None):
        L = load()
        p = _f64(params)
        self.structural = p.size == N_PARAMS_STRUCT
        hp = HParams(8, 6, 4, 8, 64, 2, 6.0, 4.5, int(self.structural))
        if short_range is not None:
            hp.sr_Z[0], hp.sr_Z[1], hp.sr_r_inner, hp.sr_r_outer = (float(x) for x in short_range)
        if landau is not None:
            hp.moment_a, hp.moment_b = (float(x) for x in landau)
        self.short_range, self.landau = short_range, landau
        h = ct.c_void_p()
        _check(L.nep_model_create(ct.byref(hp), _p(p), p.size, ct.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            load().nep_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self, types, pos, spin, box, pbc=(1, 1, 1), *, mu_s=1.0, B=(0, 0, 0), precision="fp64",
             want=("E", "F", "H"), noalloc=False):
        """nep_spin_eval (nep_spin_eval_noalloc if noalloc) with host buffers:
        dict with E (total), Ei, F, H."""
        v, keep = system_view(types, pos, spin, box, pbc, mu_s, B)
        n = v.n_atoms
        E = np.zeros(1)
        Ei = np.zeros(n) if "Ei" in want else None
        F = np.zeros((n, 3)) if "F" in want else None
        H = np.zeros((n, 3)) if "H" in want else None
        fn = load().nep_spin_eval_noalloc if noalloc else load().nep_spin_eval
        _check(fn(self.h, ct.byref(v), PRECISION[precision], _p(E), _p(Ei), _p(F), _p(H), None))
        out = {"E": float(E[0])}
        for k, a in (("Ei", Ei), ("F", F), ("H", H)):
            if a is not None:
                out[k] = a
        return out

    def eval_device(self, types, pos, spin, box, pbc, E, Ei, F, H, *, mu_s=1.0, B=(0, 0, 0), precision="fp64",
                    stream=0):
        """nep_spin_eval writing into device buffers (integer addresses, e.g. torch data_ptr())."""
        v, keep = system_view(types, pos, spin, box, pbc, mu_s, B)
        ex = Exec(1, ct.c_void_p(stream) if stream else None)
        P = ct.c_void_p
        _check(load().nep_spin_eval(self.h, ct.byref(v), PRECISION[precision], P(E) if E else None,
                                    P(Ei) if Ei else None, P(F) if F else None, P(H) if H else None, ct.byref(ex)))

    def descriptors(self, types, pos, spin, box, pbc=(1, 1, 1), *, precision="fp64"):
        v, keep = system_view(types, pos, spin, box, pbc)
        n = v.n_atoms
        nd = 37 if self.structural else 102
        q = np.zeros((n, nd))
        Fp = np.zeros((n, nd))
        _check(load().nep_spin_descriptors(self.h, ct.byref(v), PRECISION[precision], _p(q), _p(Fp), None))
        return q, Fp


def _obs_array(obs, n):
    """columns: step, E_pot, E_kin, E_zeeman, T_lattice, T_spin, M[3], spin sweep passes, last change,
    rotations stopped at the cap, mean |s|"""
    return np.array([[o.step, o.E_pot, o.E_kin, o.E_zeeman, o.T_lattice, o.T_spin, o.M[0], o.M[1], o.M[2],
                      o.spin_passes, o.spin_change, o.mid_capped, o.spin_length] for o in obs[:n]]).reshape(n, 13)


class Sim:
    """sl_create / sl_integrate_steps / sl_get_state / sl_set_state."""

    def __init__(self, model: Model, types, pos, spin, box, pbc=(1, 1, 1), vel=None, colour=None, *,
                 mu_s=1.0, B=(0, 0, 0), params: IntegratorParams | None = None, precision="fp64"):
        self.model = model
        v, keep = system_view(types, pos, spin, box, pbc, mu_s, B)
        self.n = v.n_atoms
        ip = params or integrator_params()
        vel_ = _f64(vel)
        col = _i32(colour)
        h = ct.c_void_p()
        _check(load().sl_create(model.h, ct.byref(v), _p(vel_), _p(col), ct.byref(ip), PRECISION[precision],
                                ct.byref(h)))
        self.h = h

    def integrate(self, n_steps, observables=True):
        obs = (Observables * max(n_steps, 1))() if observables else None
        _check(load().sl_integrate_steps(self.h, n_steps, ct.cast(obs, ct.c_void_p) if obs is not None else None))
        return _obs_array(obs, n_steps) if observables else None

    def state(self):
        n = self.n
        pos, vel, spin = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        st = ct.c_int64()
        _check(load().sl_get_state(self.h, _p(pos), _p(vel), _p(spin), ct.byref(st)))
        return pos, vel, spin, st.value

    def colour(self):
        """Current colouring (caller order, -1 on species 1) and the number of
        recolourings since creation."""
        col = np.zeros(self.n, dtype=np.int32)
        k = ct.c_int64()
        _check(load().sl_get_colour(self.h, col.ctypes.data_as(ct.c_void_p), ct.byref(k)))
        return col, k.value

    def profile(self, groups):
        """time the named kernel groups (PROFILE_GROUPS) with HIP events"""
        mask = 0
        for g in groups:
            mask |= 1 << PROFILE_GROUPS.index(g)
        _check(load().sl_profile_enable(self.h, mask))

    def profile_read(self):
        ms = np.zeros(len(PROFILE_GROUPS))
        n = np.zeros(len(PROFILE_GROUPS), np.int64)
        _check(load().sl_profile_read(self.h, _p(ms), _p(n)))
        return {g: (float(ms[k]), int(n[k])) for k, g in enumerate(PROFILE_GROUPS)}

    def set_state(self, pos, vel, spin, step):
        _check(load().sl_set_state(self.h, _p(_f64(pos)), _p(_f64(vel)), _p(_f64(spin)), int(step)))

    def close(self):
        if self.h:
            load().sl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """sl_server_create / sl_replica_submit / poll / fetch / drain."""

    def __init__(self, model: Model, *, hbm_budget_bytes=0, max_slots=64, precision="fp32", steps_per_batch=10,
                 K_corr=1):
        self.model = model
        cfg = ServerConfig(hbm_budget_bytes, max_slots, PRECISION[precision], steps_per_batch, K_corr)
        h = ct.c_void_p()
        _check(load().sl_server_create(model.h, ct.byref(cfg), ct.byref(h)))
        self.h = h
        self.sizes = {}

    def submit(self, types, pos, spin, box, pbc=(1, 1, 1), vel=None, colour=None, *, mu_s=1.0,
               params: IntegratorParams | None = None, n_steps=100):
        v, keep = system_view(types, pos, spin, box, pbc, mu_s)
        ip = params or integrator_params()
        rid = ct.c_uint64()
        _check(load().sl_replica_submit(self.h, ct.byref(v), _p(_f64(vel)), _p(_i32(colour)), ct.byref(ip),
                                        n_steps, ct.byref(rid)))
        self.sizes[rid.value] = v.n_atoms
        return rid.value

    def poll(self, rid):
        st = ReplicaStatus()
        _check(load().sl_replica_poll(self.h, rid, ct.byref(st)))
        return {k: getattr(st, k) for k, _ in ReplicaStatus._fields_}

    def fetch(self, rid):
        n = self.sizes[rid]
        pos, vel, spin = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        ob = Observables()
        _check(load().sl_replica_fetch(self.h, rid, _p(pos), _p(vel), _p(spin), ct.byref(ob)))
        return pos, vel, spin, _obs_array([ob], 1)[0]

    def drain(self):
        _check(load().sl_server_drain(self.h))

    def stats(self):
        a, b, c = ct.c_int64(), ct.c_double(), ct.c_double()
        _check(load().sl_server_stats(self.h, ct.byref(a), ct.byref(b), ct.byref(c)))
        return {"batched_steps": a.value, "atom_steps": b.value, "busy_s": c.value}

    def host_stats(self):
        """re-layouts, their seconds, and the seconds of all gaps between batches"""
        a, b, c = ct.c_int64(), ct.c_double(), ct.c_double()
        _check(load().sl_server_host_stats(self.h, ct.byref(a), ct.byref(b), ct.byref(c)))
        return {"relayouts": a.value, "relayout_s": b.value, "gap_s": c.value}

    def close(self):
        if self.h:
            load().sl_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
