"""Spins of variable length on the GPU (the onsite moment-length term
a|s|^2 + b|s|^4 and the longitudinal Langevin spin dynamics) against the FP64
oracle: every step, conservation of each spin's length without damping, the
relaxation to the minimum of the onsite term, and the equilibrium moments of
isolated spins. Also the midpoint cap: a field strong enough that the plain
fixed-point iteration stops at the cap while the library's Newton solve
converges, which each side reports."""
import math

import numpy as np
import pytest

from paper_2606_14073_amd import workload as W
from tests.helpers import min_image_delta, pos_error, rel_inf

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
LANDAU = (-1.0, 0.5)
KB = 8.617333262e-5
MUB = 5.7883818060e-5


def _model(nepspin, params=None, landau=LANDAU, short_range=W.SHORT_RANGE_FEGE):
    return nepspin.Model(W.random_params() if params is None else params, short_range=short_range,
                         landau=landau)


def _oracle_kw(kw):
    m = dict(kw)
    m["alpha"] = m.pop("alpha_s", 0.0)
    m["gammaL"] = m.pop("gamma_L", 0.0)
    m["lsf"] = m.pop("longitudinal", 0)
    m["lsf_gamma"] = m.pop("gamma_lsf", 0.0)
    m.pop("skin", None)
    return m


def _varied_lengths(s, lo=0.8, hi=1.2, seed=7):
    rng = np.random.default_rng(seed)
    lens = np.where(s.types == 0, rng.uniform(lo, hi, s.n), 0.0)
    return s.spin * lens[:, None], lens


@pytest.mark.parametrize("gamma", [0.0, 0.05])
def test_longitudinal_every_step_matches_oracle(oracle, gamma):
    """512 atoms, spins of lengths 0.8-1.2, 300 K lattice bath and (gamma > 0)
    the longitudinal spin bath: every step against one oracle step from the
    GPU's state, observables (mean |s| included) too"""
    from paper_2606_14073_amd import nepspin
    s = W.config_small()
    spin0, _ = _varied_lengths(s)
    p = W.random_params()
    m = _model(nepspin)
    kw = dict(dt=1.0, T0=300.0, gamma_L=0.01, ensemble=1, B0=(0, 0, 1.0), longitudinal=1, gamma_lsf=gamma)
    sim = nepspin.Sim(m, s.types, s.pos, spin0, s.box, s.pbc, vel=W.maxwell_boltzmann(s.types, 300.0),
                      colour=s.colour, params=nepspin.integrator_params(**kw))
    okw = oracle.step_params(zbl=W.SHORT_RANGE_FEGE, landau=LANDAU, **_oracle_kw(kw))
    prev = sim.state()
    worst = [0.0] * 5
    for k in range(12):
        ob = sim.integrate(1)[0]
        cur = sim.state()
        rp, rv, rs, _, rob = oracle.run(s.types, prev[0], prev[1], prev[2], s.box, s.pbc, p, s.colour, okw, 1,
                                        step0=prev[3])
        e = [pos_error(cur[0], rp, prev[0], s.box, s.pbc), rel_inf(cur[1], rv), np.abs(cur[2] - rs).max()]
        eo = max(abs(ob[c] - rob[0, c]) / abs(rob[0, c]) for c in (1, 2, 3, 5, 12))
        e += [eo, ob[11]]   # the oracle's plain iteration may stop at its cap; the library's Newton solve may not
        worst = [max(a, b) for a, b in zip(worst, e)]
        prev = cur
    m.close()
    print(f"longitudinal, gamma {gamma}: worst per-step pos {worst[0]:.2e} vel {worst[1]:.2e} spin {worst[2]:.2e} "
          f"observables {worst[3]:.2e}, capped rotations {worst[4]}", flush=True)
    assert max(worst[:4]) <= TOL64 and worst[4] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_eval_with_moment_length_term(oracle, precision):
    """one evaluation with spins of lengths 0.7-1.3 and the onsite
    moment-length term: E, E_i, F, H against the oracle (FP64 to 1e-12;
    FP32-mixed within its bounds); the term's own energy and field are
    checked against a|s|^2 + b|s|^4 and -(2a + 4b|s|^2) s"""
    from paper_2606_14073_amd import nepspin
    s = W.fege_lattice(4, 4, 4, seed=9)
    spin, lens = _varied_lengths(s, 0.7, 1.3, seed=9)
    p = W.random_params()
    B = (0.0, 0.2, 0.7)
    m = _model(nepspin)
    got = m.eval(s.types, s.pos, spin, s.box, s.pbc, B=B, precision=precision, want=("E", "Ei", "F", "H"))
    m.close()
    ref = oracle.evaluate(s.types, s.pos, spin, s.box, s.pbc, p, B=B, want=("E", "F", "H", "Ei"),
                          zbl=W.SHORT_RANGE_FEGE, landau=LANDAU)
    plain = oracle.evaluate(s.types, s.pos, spin, s.box, s.pbc, p, B=B, want=("E", "H", "Ei"),
                            zbl=W.SHORT_RANGE_FEGE)
    a, b = LANDAU
    fe = s.types == 0
    np.testing.assert_allclose((ref["Ei"] - plain["Ei"])[fe], a * lens[fe] ** 2 + b * lens[fe] ** 4, rtol=1e-12,
                               atol=1e-13)
    np.testing.assert_allclose((ref["H"] - plain["H"])[fe], -(2 * a + 4 * b * lens[fe, None] ** 2) * spin[fe],
                               rtol=1e-11, atol=1e-12)
    etot = ref["E"] + ref["Ez"]
    if precision == "fp64":
        assert rel_inf(got["Ei"], ref["Ei"]) <= TOL64
        assert abs(got["E"] - etot) <= TOL64 * abs(etot)
        assert rel_inf(got["F"], ref["F"]) <= TOL64
        assert rel_inf(got["H"], ref["H"]) <= TOL64
    else:
        assert abs(got["E"] - etot) / s.n <= 1e-6
        assert np.linalg.norm(got["F"] - ref["F"]) <= 1e-5 * np.linalg.norm(ref["F"])
        assert np.linalg.norm(got["H"] - ref["H"]) <= 1e-5 * np.linalg.norm(ref["H"])


def test_longitudinal_selfconsistent_matches_oracle(oracle):
    """the self-consistent midpoint (corrector passes until the spins change
    by at most 1e-13, plain and with Anderson mixing) with variable lengths:
    every step against one oracle step from the GPU's state"""
    from paper_2606_14073_amd import nepspin
    s = W.config_small()
    spin0, _ = _varied_lengths(s, seed=3)
    p = W.random_params()
    m = _model(nepspin)
    for depth in (0, 3):
        kw = dict(dt=1.0, T0=300.0, gamma_L=0.01, ensemble=1, B0=(0, 0, 1.0), longitudinal=1, gamma_lsf=0.05,
                  sc_tol=1e-13, sc_max=40, sc_depth=depth)
        sim = nepspin.Sim(m, s.types, s.pos, spin0, s.box, s.pbc, vel=W.maxwell_boltzmann(s.types, 300.0),
                          colour=s.colour, params=nepspin.integrator_params(**kw))
        okw = oracle.step_params(zbl=W.SHORT_RANGE_FEGE, landau=LANDAU, **_oracle_kw(kw))
        prev = sim.state()
        worst = [0.0] * 3
        passes = []
        for k in range(6):
            ob = sim.integrate(1)[0]
            cur = sim.state()
            rp, rv, rs, _, rob = oracle.run(s.types, prev[0], prev[1], prev[2], s.box, s.pbc, p, s.colour, okw,
                                            1, step0=prev[3])
            e = [pos_error(cur[0], rp, prev[0], s.box, s.pbc), rel_inf(cur[1], rv), np.abs(cur[2] - rs).max()]
            worst = [max(a, b) for a, b in zip(worst, e)]
            passes.append((int(ob[9]), int(rob[0, 9])))
            prev = cur
        sim.close()
        print(f"longitudinal, self-consistent, depth {depth}: worst per-step pos {worst[0]:.2e} "
              f"vel {worst[1]:.2e} spin {worst[2]:.2e}; passes (GPU, oracle) {passes}", flush=True)
        assert max(worst) <= TOL64
        assert all(abs(a - b) <= 1 for a, b in passes) and min(a for a, _ in passes) >= 2
    m.close()


def test_longitudinal_fp32_mixed_step_error(oracle):
    """FP32-mixed with variable lengths and the longitudinal bath: one step
    from the same state against the FP64 oracle"""
    from paper_2606_14073_amd import nepspin
    s = W.fege_lattice(7, 7, 7)
    spin0, _ = _varied_lengths(s, seed=5)
    p = W.random_params()
    m = _model(nepspin)
    kw = dict(dt=1.0, T0=300.0, gamma_L=0.01, ensemble=1, B0=(0, 0, 1.0), longitudinal=1, gamma_lsf=0.05)
    sim = nepspin.Sim(m, s.types, s.pos, spin0, s.box, s.pbc, vel=W.maxwell_boltzmann(s.types, 300.0),
                      colour=s.colour, params=nepspin.integrator_params(**kw), precision="fp32")
    a = sim.state()
    sim.integrate(1)
    b = sim.state()
    sim.close()
    m.close()
    rp, rv, rs, _, _ = oracle.run(s.types, a[0], a[1], a[2], s.box, s.pbc, p, s.colour,
                                  oracle.step_params(zbl=W.SHORT_RANGE_FEGE, landau=LANDAU, **_oracle_kw(kw)), 1,
                                  step0=a[3])
    ep, ev, es = pos_error(b[0], rp, a[0], s.box, s.pbc), rel_inf(b[1], rv), np.abs(b[2] - rs).max()
    print(f"longitudinal fp32 one step: pos {ep:.2e} vel {ev:.2e} spin {es:.2e}", flush=True)
    assert ep < 1e-5 and ev < 1e-5 and es < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_longitudinal_replica_batching_invariant(precision):
    """a replica with variable lengths served alone, served beside replicas
    with and without longitudinal dynamics, and run as a direct simulation:
    bitwise the same state"""
    from paper_2606_14073_amd import nepspin
    m = _model(nepspin)

    def req(cells, seed, lsf, T=250.0):
        s = W.fege_lattice(cells, cells, cells, seed=seed)
        spin, _ = _varied_lengths(s, seed=seed) if lsf else (s.spin, None)
        ip = nepspin.integrator_params(dt=1.0, T0=T, alpha_s=0.0 if lsf else 0.1, gamma_L=0.01, ensemble=1,
                                       B0=(0, 0, 0.5), longitudinal=lsf, gamma_lsf=0.05 if lsf else 0.0,
                                       seed=300 + seed)
        return s, spin, W.maxwell_boltzmann(s.types, T, seed=seed + 1), ip

    def submit(sv, r, n):
        s, spin, v, ip = r
        return sv.submit(s.types, s.pos, spin, s.box, s.pbc, vel=v, colour=s.colour, params=ip, n_steps=n)

    X, n = req(4, 21, 1), 9
    sv = nepspin.Server(m, precision=precision, steps_per_batch=4, max_slots=8)
    a = submit(sv, X, n)
    sv.drain()
    alone = sv.fetch(a)
    sv.close()
    sv = nepspin.Server(m, precision=precision, steps_per_batch=3, max_slots=8)
    ids = [submit(sv, req(5, 22, 0), 6)]
    b = submit(sv, X, n)
    ids.append(submit(sv, req(4, 23, 1, T=80.0), 11))
    sv.drain()
    mixed = sv.fetch(b)
    for k in ids:
        assert sv.poll(k)["state"] == nepspin.SL_DONE
    sv.close()
    s, spin, v, ip = X
    sim = nepspin.Sim(m, s.types, s.pos, spin, s.box, s.pbc, vel=v, colour=s.colour, params=ip, precision=precision)
    sim.integrate(n)
    direct = sim.state()
    sim.close()
    m.close()
    for x, y, z in zip(alone[:3], mixed[:3], direct[:3]):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    fe = s.types == 0
    assert np.ptp(np.linalg.norm(alone[2][fe], axis=1)) > 0.1   # the lengths stay spread


def test_longitudinal_lengths_kept_without_damping():
    """gamma = 0: only the rotations act; every spin keeps its own length"""
    from paper_2606_14073_amd import nepspin
    s = W.fege_lattice(6, 6, 6)
    spin0, lens = _varied_lengths(s, 0.7, 1.3)
    m = _model(nepspin)
    sim = nepspin.Sim(m, s.types, s.pos, spin0, s.box, s.pbc, vel=W.maxwell_boltzmann(s.types, 300.0),
                      colour=s.colour, params=nepspin.integrator_params(dt=1.0, T0=300.0, gamma_L=0.01, ensemble=1,
                                                                        longitudinal=1))
    ob = sim.integrate(200)
    spin = sim.state()[2]
    m.close()
    fe = s.types == 0
    assert np.abs(np.linalg.norm(spin[fe], axis=1) - lens[fe]).max() <= 1e-13
    assert ob[-1, 12] == pytest.approx(lens[fe].mean(), rel=1e-13)


def _isolated(n, seed, lengths=None):
    rng = np.random.default_rng(seed)
    g = np.arange(n)
    pos = np.stack([g % 10, (g // 10) % 10, g // 100], axis=1) * 8.0 + 5.0
    spin = rng.normal(size=(n, 3))
    spin /= np.linalg.norm(spin, axis=1, keepdims=True)
    if lengths is not None:
        spin *= np.asarray(lengths)[:, None]
    return pos, spin


def test_longitudinal_relaxation_to_minimum():
    """zero model, no field, T = 0: each length goes to sqrt(-a/2b), direction kept"""
    from paper_2606_14073_amd import nepspin
    a, b = -1.3, 0.4
    n = 20
    pos, spin = _isolated(n, 9, np.linspace(0.5, 2.0, n))
    m = nepspin.Model(np.zeros(15438), landau=(a, b))
    sim = nepspin.Sim(m, np.zeros(n, np.int32), pos, spin, np.zeros(3), (0, 0, 0), colour=np.zeros(n, np.int32),
                      params=nepspin.integrator_params(dt=1.0, longitudinal=1, gamma_lsf=0.2))
    sim.integrate(400)
    out = sim.state()[2]
    m.close()
    r = np.linalg.norm(out, axis=1)
    np.testing.assert_allclose(r, math.sqrt(-a / (2 * b)), rtol=1e-9)
    np.testing.assert_allclose(out / r[:, None], spin / np.linalg.norm(spin, axis=1)[:, None], atol=1e-12)


def test_longitudinal_equilibrium_moments():
    """isolated spins at 300 K in 400 T with the onsite term: <|s|>, <|s|^2>
    and <s.B^> against quadrature of exp(-(a|s|^2 + b|s|^4 - mu_B B.s)/kB T)
    over vectors s"""
    from scipy import integrate
    from paper_2606_14073_amd import nepspin
    a, b = LANDAU
    n, T, Bz = 1000, 300.0, 400.0
    kT, h = KB * T, MUB * Bz
    pos, spin = _isolated(n, 13)
    m = nepspin.Model(np.zeros(15438), landau=LANDAU)
    sim = nepspin.Sim(m, np.zeros(n, np.int32), pos, spin, np.zeros(3), (0, 0, 0), colour=np.zeros(n, np.int32),
                      params=nepspin.integrator_params(dt=1.0, T0=T, B0=(0, 0, Bz), longitudinal=1, gamma_lsf=0.03))
    sim.integrate(600, observables=False)
    r1, r2, mz = [], [], []
    for _ in range(24):
        sim.integrate(150, observables=False)
        sp = sim.state()[2]
        r = np.linalg.norm(sp, axis=1)
        r1.append(r.mean())
        r2.append((r * r).mean())
        mz.append(sp[:, 2].mean())
    m.close()

    def mom(f):
        w = lambda c, r: r * r * np.exp(-(a * r * r + b * r ** 4 + 0.5 - h * r * c) / kT)
        return (integrate.dblquad(lambda c, r: f(c, r) * w(c, r), 0.2, 2.0, -1, 1, epsabs=1e-12)[0]
                / integrate.dblquad(w, 0.2, 2.0, -1, 1, epsabs=1e-12)[0])
    want = (mom(lambda c, r: r), mom(lambda c, r: r * r), mom(lambda c, r: r * c))
    got = (np.mean(r1), np.mean(r2), np.mean(mz))
    err = [np.std(x) / math.sqrt(len(x)) for x in (r1, r2, mz)]
    print("GPU longitudinal equilibrium: got", got, "want", want, "stderr", err, flush=True)
    assert abs(got[0] - want[0]) < 4 * err[0] + 1.5e-3
    assert abs(got[1] - want[1]) < 4 * err[1] + 3e-3
    assert abs(got[2] - want[2]) < 4 * err[2] + 0.01


def test_midpoint_cap_reported(oracle):
    """A 30,000 T field with damping 0.5 and dt 2 fs: the oracle's plain
    fixed-point iteration of the midpoint equation stops at a cap of 8 with
    rotations unconverged (and reports them); with a cap of 400 it converges
    (to 1e-13; at 1e-15 rounding keeps a few iterations from settling).
    The library's Newton solve converges within the cap of 8, reports none,
    and matches the converged oracle step."""
    from paper_2606_14073_amd import nepspin
    s = W.config_small()
    p = W.random_params()
    m = nepspin.Model(p)
    kw = dict(dt=2.0, T0=100.0, alpha_s=0.5, gamma_L=0.01, ensemble=1, B0=(0, 0, 3.0e4), mid_tol=1e-13)
    sim = nepspin.Sim(m, s.types, s.pos, s.spin, s.box, s.pbc, vel=W.maxwell_boltzmann(s.types, 100.0),
                      colour=s.colour, params=nepspin.integrator_params(mid_cap=8, **kw))
    prev = sim.state()
    for k in range(3):
        ob = sim.integrate(1)[0]
        cur = sim.state()
        okw = _oracle_kw(kw)
        _, _, rs8, _, r8 = oracle.run(s.types, prev[0], prev[1], prev[2], s.box, s.pbc, p, s.colour,
                                      oracle.step_params(mid_cap=8, **okw), 1, step0=prev[3])
        rp, rv, rs, _, rob = oracle.run(s.types, prev[0], prev[1], prev[2], s.box, s.pbc, p, s.colour,
                                        oracle.step_params(mid_cap=400, **okw), 1, step0=prev[3])
        es = np.abs(cur[2] - rs).max()
        print(f"step {k}: capped GPU {ob[11]:.0f}, oracle cap 8 {r8[0, 11]:.0f}, cap 400 {rob[0, 11]:.0f}; "
              f"spin err vs converged {es:.2e}, oracle cap 8 vs converged {np.abs(rs8 - rs).max():.2e}", flush=True)
        assert ob[11] == 0 and rob[0, 11] == 0 and r8[0, 11] > 0
        assert es <= TOL64 and rel_inf(cur[1], rv) <= TOL64
        assert pos_error(cur[0], rp, prev[0], s.box, s.pbc) <= TOL64
        prev = cur
    m.close()
