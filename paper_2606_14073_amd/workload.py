"""Seeded synthetic inputs for the spin-lattice NEP workloads.

This module only draws inputs: B20 FeGe-like lattices, spin textures,
velocities, random model parameters and the Fe-sublattice colouring. It holds
none of the potential's or the integrator's arithmetic, so it can feed both
the HIP library and the CPU oracle without coupling them.

The paper's benchmark (helix-to-skyrmion transformation in FeGe, Sec. 6
"Benchmark application and setup") needs DFT-trained weights that are not
published; these generators stand in for it with seeded random weights and
synthetic crystals of the same structure and size.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Model sizes (descriptor layout and parameter vector order are fixed by the
# library header; they are repeated here only to size the random draw).
N_RADIAL = 9
N_ANGULAR = 7
N_BASIS = 9
N_HIDDEN = 64
N_DESC = 102
N_PAIR_TYPES = 4
N_PARAMS = (N_PAIR_TYPES * N_RADIAL * N_BASIS            # c^R
            + N_PAIR_TYPES * N_ANGULAR * N_BASIS         # c^A
            + 4 * N_PAIR_TYPES * N_RADIAL * N_BASIS      # c^ex, c^dm, c^an, c^si
            + N_PAIR_TYPES * N_ANGULAR * N_BASIS         # c^sa
            + 2 * (N_HIDDEN * N_DESC + 2 * N_HIDDEN + 1))  # per-species MLP
assert N_PARAMS == 15438

LATTICE_A = 4.70          # Angstrom, cubic B20 cell
U_FE = 0.1352             # Wyckoff 4a parameter of Fe (literature value)
U_GE = 0.8414             # Wyckoff 4a parameter of Ge
MASS = np.array([55.845, 72.630])   # u, IUPAC
KB = 8.617333262e-5       # eV/K
KAPPA = 9.648533212e-3    # (eV/Angstrom)/u -> Angstrom/fs^2

SEED_WEIGHTS = 0
SEED_STATE = 1
SEED_PHILOX = 0x5EED

# The optional short-range repulsion of the FeGe workloads: nuclear charges of
# Fe and Ge, and the interval over which the repulsion is switched off (A).
# With the seeded random weights alone, neighbours come closer than 1.5 A
# within 100-200 steps at 300 K (weight seeds 0-12 all do). Switched off over
# 1.0-2.0 A the term keeps pairs beyond 1.9 A, but the lattice still
# rearranges (rms displacement 1 A after 800 steps); switched off over
# 1.8-2.6 A, just above the nearest Fe-Ge distance of 2.39 A, it cages each
# atom among its neighbours: the 512-atom cell at 300 K keeps its closest pair
# beyond 2.3 A and its rms displacement below 0.45 A over 2,000 steps.
SHORT_RANGE_FEGE = (26.0, 32.0, 1.8, 2.6)


def b20_fractional(u: float) -> np.ndarray:
    """The four 4a sites of space group P2_1 3 for parameter u (mod 1)."""
    s = np.array([[u, u, u],
                  [0.5 + u, 0.5 - u, -u],
                  [-u, 0.5 + u, 0.5 - u],
                  [0.5 - u, -u, 0.5 + u]])
    return np.mod(s, 1.0)


@dataclasses.dataclass
class System:
    """One spin-lattice system, atoms in caller order."""
    types: np.ndarray      # [n] int32, 0 = Fe (carries a spin), 1 = Ge
    pos: np.ndarray        # [n,3] float64, Angstrom
    spin: np.ndarray       # [n,3] float64, unit vectors on Fe, zero on Ge
    box: np.ndarray        # [3] float64
    pbc: np.ndarray        # [3] int32
    cells: tuple           # (nx, ny, nz)
    colour: np.ndarray     # [n] int32, Fe colour class, -1 on Ge

    @property
    def n(self) -> int:
        return int(self.types.shape[0])


def fege_lattice(nx: int, ny: int, nz: int, *, seed: int = SEED_STATE,
                 noise: float = 0.02, pbc=(1, 1, 1), spins: str = "random",
                 helix_pitch: float = 700.0, greedy: bool = True) -> System:
    """B20 FeGe-like supercell.

    Atom index = ((cx*ny + cy)*nz + cz)*8 + site, sites 0-3 Fe and 4-7 Ge.
    Positions are lattice sites plus N(0, noise) per component. Fe spins are
    uniform on the sphere ("random") or a helix s = (0, cos 2pi x/p, sin 2pi x/p)
    along x ("helix"); Ge spins are zero. When the periodic colouring does not
    apply, the greedy one is drawn if `greedy`, else colour is None.
    """
    rng = np.random.default_rng(seed)
    frac = np.concatenate([b20_fractional(U_FE), b20_fractional(U_GE)])  # [8,3]
    cx, cy, cz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cell = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)  # [nc,3]
    lattice = (cell[:, None, :] + frac[None, :, :]) * LATTICE_A                    # [nc,8,3]
    pos = lattice.reshape(-1, 3).copy()
    n = pos.shape[0]
    pos += rng.normal(0.0, noise, size=pos.shape)
    types = np.tile(np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.int32), nx * ny * nz)
    box = np.array([nx, ny, nz], dtype=np.float64) * LATTICE_A
    pbc = np.asarray(pbc, dtype=np.int32)
    for a in range(3):
        if pbc[a]:
            pos[:, a] = np.mod(pos[:, a], box[a])
    spin = np.zeros((n, 3))
    fe = types == 0
    if spins == "random":
        v = rng.normal(size=(int(fe.sum()), 3))
        spin[fe] = v / np.linalg.norm(v, axis=1, keepdims=True)
    elif spins == "helix":
        x = lattice.reshape(-1, 3)[fe, 0]
        ph = 2.0 * np.pi * x / helix_pitch
        spin[fe] = np.stack([np.zeros_like(ph), np.cos(ph), np.sin(ph)], axis=1)
    elif spins == "ferro":
        spin[fe] = np.array([0.0, 0.0, 1.0])
    else:
        raise ValueError(spins)
    colour = colour_periodic(nx, ny, nz, pbc)
    if colour is None and greedy:
        colour = colour_greedy(types, pos, box, pbc, 7.0)
    return System(types, pos, spin, box, pbc, (nx, ny, nz), colour)


def colour_periodic(nx: int, ny: int, nz: int, pbc) -> np.ndarray | None:
    """colour = site + 4*(cx%2 + 2*(cy%2) + 4*(cz%2)) on Fe, -1 on Ge (32
    colours): two Fe of one colour sit on the same site two cells apart,
    2a = 9.4 A, so the colouring survives the drift of the random-weight model
    for hundreds of steps before a same-colour pair reaches the list shell.

    Valid only when every periodic cell count is even (the parity classes must
    wrap consistently); returns None otherwise.
    """
    for c, p in zip((nx, ny, nz), pbc):
        if p and c % 2:
            return None
    cx, cy, cz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    par = (cx % 2 + 2 * (cy % 2) + 4 * (cz % 2)).ravel()
    site = np.arange(8)
    col = site[None, :] + 4 * par[:, None]
    col[:, 4:] = -1
    return col.reshape(-1).astype(np.int32)


def colour_greedy(types, pos, box, pbc, radius: float, keep=None) -> np.ndarray:
    """Greedy colouring of the Fe graph (edges r < radius) in atom-index order.

    With `keep` (a colouring), a repair instead: spins keep their colour unless
    it is the colour of a neighbour, in which case, in atom-index order, they
    take the smallest colour none of their neighbours has.
    """
    from scipy.spatial import cKDTree
    fe = np.nonzero(types == 0)[0]
    p = pos[fe].copy()
    boxsize = None
    if np.all(pbc):
        boxsize = box.copy()
        p = np.mod(p, boxsize)
    elif np.any(pbc):
        # cKDTree wants one box for all axes: give free axes a huge period
        span = p.max(axis=0) - p.min(axis=0) + 4 * radius
        boxsize = np.where(np.asarray(pbc) > 0, box, np.maximum(span, 1.0) * 4)
        p = p - np.where(np.asarray(pbc) > 0, 0.0, p.min(axis=0))
        p = np.mod(p, boxsize)
    tree = cKDTree(p, boxsize=boxsize)
    pairs = tree.query_pairs(radius, output_type="ndarray")
    adj = [[] for _ in range(len(fe))]
    for a, b in pairs:
        adj[a].append(b)
        adj[b].append(a)
    col_fe = np.full(len(fe), -1, dtype=np.int64)
    if keep is not None:
        col_fe[:] = np.asarray(keep)[fe]
    for a in range(len(fe)):
        used = {col_fe[b] for b in adj[a] if col_fe[b] >= 0}
        if col_fe[a] >= 0 and col_fe[a] not in used:
            continue
        c = 0
        while c in used:
            c += 1
        col_fe[a] = c
    col = np.full(types.shape[0], -1, dtype=np.int32)
    col[fe] = col_fe
    return col


def maxwell_boltzmann(types: np.ndarray, T: float, seed: int = SEED_STATE + 1, masses=MASS) -> np.ndarray:
    """Velocities (Angstrom/fs) drawn at temperature T with zero total momentum."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses)[types][:, None]
    v = rng.normal(size=(types.shape[0], 3)) * np.sqrt(KAPPA * KB * T / m)
    p = (m * v).sum(axis=0) / m.sum()
    return v - p[None, :]


def random_params(seed: int = SEED_WEIGHTS, sigma: float = 0.1) -> np.ndarray:
    """All model parameters i.i.d. N(0, sigma) in the library's order."""
    return np.random.default_rng(seed).normal(0.0, sigma, N_PARAMS)


# Structural-only NEP on a water-like liquid -----------------------------------
# The paper compares throughput with DeePMD on liquid water using its NEP engine
# without the magnetic channels; the trained water model is not public, so a
# seeded random structural model on a synthetic water box stands in for it.

N_PARAMS_STRUCT = 324 + 252 + 2 * (64 * 37 + 64 + 64 + 1)
MASS_WATER = np.array([15.999, 1.008])   # O, H (u)
WATER_DENSITY = 0.1003                   # atoms per cubic Angstrom (liquid water, 300 K)


def random_params_structural(seed: int = SEED_WEIGHTS, sigma: float = 0.1) -> np.ndarray:
    """Structural-only model parameters i.i.d. N(0, sigma)."""
    return np.random.default_rng(seed).normal(0.0, sigma, N_PARAMS_STRUCT)


def water_box(n: int, *, seed: int = SEED_STATE, noise: float = 0.02) -> System:
    """n^3 water molecules, one per cell of a simple cubic grid whose spacing
    gives liquid-water density, each with a uniformly random orientation
    (O-H 0.9572 A, H-O-H 104.52 deg), plus N(0, noise) per component.
    Atom order molecule by molecule (O, H, H); species O = 0, H = 1; periodic;
    no spins and no colouring."""
    rng = np.random.default_rng(seed)
    a = (3.0 / WATER_DENSITY) ** (1.0 / 3.0)
    g = (np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
         + 0.5) * a
    nm = g.shape[0]
    half = np.deg2rad(104.52) / 2
    local = 0.9572 * np.array([[np.sin(half), np.cos(half), 0.0], [-np.sin(half), np.cos(half), 0.0]])
    # uniform random rotations from unit quaternions
    qv = rng.normal(size=(nm, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    Rm = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
                   np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
                   np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)
    h = np.einsum("mij,hj->mhi", Rm, local)                       # [nm, 2, 3]
    pos = np.concatenate([g[:, None, :], g[:, None, :] + h], axis=1).reshape(-1, 3)
    pos += rng.normal(0.0, noise, size=pos.shape)
    box = np.full(3, n * a)
    pos = np.mod(pos, box)
    types = np.tile(np.array([0, 1, 1], dtype=np.int32), nm)
    return System(types, pos, np.zeros_like(pos), box, np.ones(3, dtype=np.int32), (n, n, n), None)


def config_water_small() -> System:
    """5^3 molecules = 375 atoms."""
    return water_box(5)


def config_water_bench() -> System:
    """100^3 molecules = 3,000,000 atoms."""
    return water_box(100)


# Named workloads ------------------------------------------------------------

def config_small() -> System:
    """4x4x4 cells = 512 atoms, periodic, random spins."""
    return fege_lattice(4, 4, 4)


def config_fp64_bench() -> System:
    """32x32x32 cells = 262,144 atoms, periodic, random spins."""
    return fege_lattice(32, 32, 32)


def config_precision() -> System:
    """96x96x96 cells = 7,077,888 atoms, periodic, random spins."""
    return fege_lattice(96, 96, 96)


def config_slab() -> System:
    """256x256x8 cells = 4,194,304 atoms, periodic in x,y, free z, 70 nm helix."""
    return fege_lattice(256, 256, 8, pbc=(1, 1, 0), spins="helix", helix_pitch=700.0)


@dataclasses.dataclass
class Request:
    """One replica request of the serving workload."""
    t_arrival: float
    cells: int
    T: float
    Bz: float
    n_steps: int
    seed: int


def serving_requests(n: int = 512, rate: float = 20.0, seed: int = 7,
                     n_steps: int = 1000, nmin: int = 2048, nmax: int = 262144) -> list:
    """Poisson arrivals; N log-uniform on [nmin, nmax] rounded to a cubic cell
    count clipped to [6, 32]; T ~ U(50, 300) K; B_z ~ U(0, 1) T."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    logn = rng.uniform(math.log(nmin), math.log(nmax), n)
    cells = np.clip(np.rint(np.cbrt(np.exp(logn) / 8.0)), 6, 32).astype(int)
    T = rng.uniform(50.0, 300.0, n)
    B = rng.uniform(0.0, 1.0, n)
    return [Request(float(t[i]), int(cells[i]), float(T[i]), float(B[i]), n_steps, 1000 + i)
            for i in range(n)]
