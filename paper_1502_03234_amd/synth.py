"""Seeded synthetic inputs: Lennard-Jones liquid/vapor slabs and droplets.

This module only *creates* particle states (positions and velocities in a
periodic box). It holds none of the dynamic-cutoff method's arithmetic, so
both the CPU oracle and the HIP path read their inputs from here.

Workload shapes follow the liquid/vapor systems of the thesis (Section 6: a
Lennard-Jones liquid slab at T* = 0.7 between vapor regions, reduced units
sigma = epsilon = m = 1), re-scaled to the sizes used here:

* slab: a jittered FCC liquid slab |z - zc| < half_thickness at density 0.8
  with uniformly placed vapor outside it, Maxwell-Boltzmann velocities with
  zero net momentum, rescaled to exactly T* over 3N - 3 degrees of freedom;
* droplet: the N FCC sites nearest the box centre (a liquid sphere) in a
  cubic box filled with vapor.

Random numbers come from SplitMix64 (Steele, Lea & Flood 2014; the
constants below are that published generator's) mapped to 53-bit uniform
doubles; Gaussians come from the Box-Muller transform.  Each purpose draws
from its own stream so that adding draws to one purpose does not shift the
others.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1

# stream tags: one independent SplitMix64 sequence per purpose
_TAG_VACANCY, _TAG_JITTER, _TAG_VAPOR, _TAG_VELOCITY, _TAG_TRACE = 1, 2, 3, 4, 5


class SplitMix64:
    """Counter form of SplitMix64: output k (k = 1, 2, ...) is mix(state0 + k*gamma)."""

    def __init__(self, seed: int, tag: int = 0):
        self.state = (int(seed) * 0x100000001B3 + int(tag) * 0x9E3779B97F4A7C15) & _MASK
        self.count = 0

    def next_u64(self, n: int) -> np.ndarray:
        k = np.arange(self.count + 1, self.count + 1 + n, dtype=np.uint64)
        self.count += n
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * _GAMMA
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, n: int) -> np.ndarray:
        """n doubles uniform on [0, 1) with 53 random bits each."""
        return (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def normal(self, n: int) -> np.ndarray:
        """n standard normals (Box-Muller, both outputs of each pair used)."""
        m = (n + 1) // 2
        u1 = 1.0 - self.uniform(m)          # (0, 1]: log is finite
        u2 = self.uniform(m)
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.empty(2 * m)
        z[0::2] = r * np.cos(2.0 * math.pi * u2)
        z[1::2] = r * np.sin(2.0 * math.pi * u2)
        return z[:n]


@dataclass
class State:
    """A particle state in caller (id) order: x and v are float64 [3][n]."""
    x: np.ndarray
    v: np.ndarray
    box: tuple
    n_liquid: int
    n_vapor: int
    temperature: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[1]


def _into_box(x: np.ndarray, box) -> np.ndarray:
    out = np.empty_like(x)
    for k in range(3):
        c = np.mod(x[k], box[k])
        c[c >= box[k]] = 0.0
        out[k] = c
    return out


def _partial_fisher_yates(rng: SplitMix64, m: int, k: int) -> np.ndarray:
    """Indices of k items drawn without replacement from range(m)."""
    idx = np.arange(m, dtype=np.int64)
    u = rng.uniform(k)
    for i in range(k):
        r = i + int(u[i] * (m - i))
        idx[i], idx[r] = idx[r], idx[i]
    return idx[:k]


def _velocities(rng: SplitMix64, n: int, temperature: float) -> np.ndarray:
    v = rng.normal(3 * n).reshape(3, n) * math.sqrt(temperature)
    v -= v.mean(axis=1, keepdims=True)
    t_now = float(np.sum(v * v)) / (3 * n - 3)
    return v * math.sqrt(temperature / t_now)


def _place_vapor(rng: SplitMix64, fixed: np.ndarray, box, n_vapor: int, inside_excluded,
                 exclusion: float) -> np.ndarray:
    """Uniform vapor points outside an excluded region, rejecting any point closer than
    `exclusion` (minimum image) to an already placed particle. Candidates are taken in
    draw order, so the result only depends on the seed."""
    from scipy.spatial import cKDTree

    box = np.asarray(box, dtype=np.float64)
    tree = cKDTree(fixed.T, boxsize=box) if fixed.shape[1] else None
    cell = exclusion
    ncell = np.maximum(1, np.floor(box / cell).astype(np.int64))
    grid: dict = {}
    out = []
    while len(out) < n_vapor:
        m = max(1024, 2 * (n_vapor - len(out)))
        cand = rng.uniform(3 * m).reshape(m, 3) * box
        keep = ~inside_excluded(cand)
        cand = cand[keep]
        if tree is not None and len(cand):
            d, _ = tree.query(cand, k=1, distance_upper_bound=exclusion)
            cand = cand[~(d < exclusion)]
        for p in cand:
            p = np.where(p >= box, 0.0, p)
            c = tuple((np.floor(p / box * ncell).astype(np.int64)) % ncell)
            clash = False
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        key = ((c[0] + dx) % ncell[0], (c[1] + dy) % ncell[1], (c[2] + dz) % ncell[2])
                        for q in grid.get(key, ()):
                            dd = p - q
                            dd -= box * np.rint(dd / box)
                            if float(dd @ dd) < exclusion * exclusion:
                                clash = True
                                break
                        if clash:
                            break
                    if clash:
                        break
                if clash:
                    break
            if clash:
                continue
            grid.setdefault(c, []).append(p)
            out.append(p)
            if len(out) == n_vapor:
                break
    return np.asarray(out, dtype=np.float64).T.reshape(3, n_vapor)


LATTICE_A0 = (4.0 / 0.8) ** (1.0 / 3.0)


def slab(n_liquid: int, n_vapor: int, box, *, seed: int, temperature: float = 0.7,
         z_center: float | None = None, half_thickness: float = 12.5, jitter: float = 0.05,
         exclusion: float = 1.0) -> State:
    """Liquid slab |z - z_center| < half_thickness plus vapor elsewhere.

    Liquid sites: FCC (100) half-layers with in-plane spacing a = Lx / round(Lx / a0),
    a0 = (4/0.8)^(1/3), m = ceil(n_liquid / (2 n^2)) half-layers evenly spaced across the
    slab, alternating the two in-plane sublattices; the surplus sites are vacated by a
    seeded partial Fisher-Yates draw. Every coordinate gets uniform +-jitter.
    """
    box = tuple(float(b) for b in box)
    lx, ly, lz = box
    zc = lz / 2.0 if z_center is None else z_center
    nx = int(round(lx / LATTICE_A0))
    ny = int(round(ly / LATTICE_A0))
    ax, ay = lx / nx, ly / ny
    per_layer = 2 * nx * ny
    m = int(math.ceil(n_liquid / per_layer))
    dz = 2.0 * half_thickness / m
    ii, jj = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64), indexing="xy")
    ii, jj = ii.ravel(), jj.ravel()
    layers = []
    for l in range(m):
        z = zc - half_thickness + (l + 0.5) * dz
        if l % 2 == 0:
            a = np.stack([ii * ax, jj * ay])
            b = np.stack([(ii + 0.5) * ax, (jj + 0.5) * ay])
        else:
            a = np.stack([(ii + 0.5) * ax, jj * ay])
            b = np.stack([ii * ax, (jj + 0.5) * ay])
        xy = np.concatenate([a, b], axis=1)
        layers.append(np.vstack([xy, np.full((1, xy.shape[1]), z)]))
    sites = np.concatenate(layers, axis=1)
    n_sites = sites.shape[1]
    if n_sites < n_liquid:
        raise ValueError("lattice too small")
    vac = _partial_fisher_yates(SplitMix64(seed, _TAG_VACANCY), n_sites, n_sites - n_liquid)
    keep = np.ones(n_sites, dtype=bool)
    keep[vac] = False
    liq = sites[:, keep]
    liq = liq + (2.0 * SplitMix64(seed, _TAG_JITTER).uniform(3 * n_liquid).reshape(3, n_liquid) - 1.0) * jitter
    liq = _into_box(liq, box)

    def in_slab(p):
        return np.abs(p[:, 2] - zc) < half_thickness

    vap = _place_vapor(SplitMix64(seed, _TAG_VAPOR), liq, box, n_vapor, in_slab, exclusion)
    x = np.ascontiguousarray(np.concatenate([liq, vap], axis=1))
    v = np.ascontiguousarray(_velocities(SplitMix64(seed, _TAG_VELOCITY), x.shape[1], temperature))
    return State(x=x, v=v, box=box, n_liquid=n_liquid, n_vapor=n_vapor, temperature=temperature,
                 meta=dict(kind="slab", seed=seed, lattice=(nx, ny, m), n_sites=n_sites,
                           z_center=zc, half_thickness=half_thickness))


def droplet(n_drop: int, box_side: float, *, seed: int, rho_vapor: float = 0.01,
            temperature: float = 0.7, jitter: float = 0.05, exclusion: float = 1.0) -> State:
    """Liquid sphere made of the n_drop cubic-FCC sites (density 0.8) nearest the box centre
    (ties broken by site index), vapor at rho_vapor outside radius R + exclusion."""
    L = float(box_side)
    box = (L, L, L)
    n = int(round(L / LATTICE_A0))
    a = L / n
    g = np.arange(n, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    base = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    offs = [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)]
    sites = np.concatenate([(base + np.array(o)[:, None]) * a for o in offs], axis=1)
    c = L / 2.0
    r2 = np.sum((sites - c) ** 2, axis=0)
    order = np.lexsort((np.arange(sites.shape[1]), r2))[:n_drop]
    liq = sites[:, np.sort(order)]
    liq = liq + (2.0 * SplitMix64(seed, _TAG_JITTER).uniform(3 * n_drop).reshape(3, n_drop) - 1.0) * jitter
    liq = _into_box(liq, box)
    R = (3.0 * n_drop / (0.8 * 4.0 * math.pi)) ** (1.0 / 3.0)
    n_vapor = int(round(rho_vapor * (L ** 3 - n_drop / 0.8)))

    def in_drop(p):
        return np.sum((p - c) ** 2, axis=1) < (R + exclusion) ** 2

    vap = _place_vapor(SplitMix64(seed, _TAG_VAPOR), liq, box, n_vapor, in_drop, exclusion)
    x = np.ascontiguousarray(np.concatenate([liq, vap], axis=1))
    v = np.ascontiguousarray(_velocities(SplitMix64(seed, _TAG_VELOCITY), x.shape[1], temperature))
    return State(x=x, v=v, box=box, n_liquid=n_drop, n_vapor=n_vapor, temperature=temperature,
                 meta=dict(kind="droplet", seed=seed, radius=R, centre=c))


# -- degenerate test states ---------------------------------------------------------------------
def lattice(n_side: int, box_side: float, *, seed: int, jitter: float = 0.05,
            temperature: float = 0.7) -> State:
    """One particle near the centre of every box of a cubic n_side^3 grid of edge box_side /
    n_side (density (n_side / box_side)^3): every box holds exactly one particle, so the density
    image is constant and there is no interface."""
    L = float(box_side)
    h = L / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    n = x.shape[1]
    x = x + (2.0 * SplitMix64(seed, _TAG_JITTER).uniform(3 * n).reshape(3, n) - 1.0) * jitter
    v = _velocities(SplitMix64(seed, _TAG_VELOCITY), n, temperature)
    return State(x=np.ascontiguousarray(x), v=np.ascontiguousarray(v), box=(L, L, L), n_liquid=n,
                 n_vapor=0, temperature=temperature, meta=dict(kind="lattice", seed=seed))


def gas(n: int, box, *, seed: int, temperature: float = 0.7, exclusion: float = 1.0) -> State:
    """n particles uniform in the box with no two closer than `exclusion` (a dilute gas: no
    liquid anywhere)."""
    box = tuple(float(b) for b in box)
    x = _place_vapor(SplitMix64(seed, _TAG_VAPOR), np.zeros((3, 0)), box, n,
                     lambda p: np.zeros(len(p), bool), exclusion)
    v = _velocities(SplitMix64(seed, _TAG_VELOCITY), n, temperature)
    return State(x=np.ascontiguousarray(x), v=np.ascontiguousarray(v), box=box, n_liquid=0, n_vapor=n,
                 temperature=temperature, meta=dict(kind="gas", seed=seed))


def pair(r: float, box_side: float) -> State:
    """Two particles at rest a distance r apart along x, straddling the periodic x face."""
    L = float(box_side)
    x = np.array([[L - 0.5 * r, 0.5 * r], [0.5 * L, 0.5 * L], [0.5 * L, 0.5 * L]], dtype=np.float64)
    return State(x=x, v=np.zeros((3, 2)), box=(L, L, L), n_liquid=0, n_vapor=2, temperature=0.0,
                 meta=dict(kind="pair", r=r))


# -- named workloads --------------------------------------------------------------------------
# Slab workloads: 98 % of the particles in the liquid slab (|z - 30| < 12.5, density 0.8 on
# FCC sites with vacancies) and 2 % vapor, box Lx x Ly x 60.
SLABS = {
    "slab16k": dict(n=16_000, box=(28.0, 28.0, 60.0), seed=1001),
    "slab256k": dict(n=256_000, box=(112.0, 112.0, 60.0), seed=1002),
    "slab2m": dict(n=2_048_000, box=(320.0, 320.0, 60.0), seed=1003),
}


def named(name: str, temperature: float = 0.7) -> State:
    if name in SLABS:
        c = SLABS[name]
        n_liq = int(round(0.98 * c["n"]))
        return slab(n_liq, c["n"] - n_liq, c["box"], seed=c["seed"], temperature=temperature)
    if name == "thesis16k":
        # the thesis's test system (Section 6): 16,000 particles filling a 22 x 22 x 44 block
        # centred in a 22 x 22 x 88 box; lattice sites stand in for its random placement
        return slab(16_000, 0, (22.0, 22.0, 88.0), seed=1006, temperature=temperature,
                    half_thickness=22.0)
    if name == "thesis192k":
        # the same geometry scaled laterally to 192,000 particles (the size of the thesis's
        # speedup measurements, Section 6.2): a 76 x 76 x 44 block in a 76 x 76 x 88 box
        return slab(192_000, 0, (76.0, 76.0, 88.0), seed=1007, temperature=temperature,
                    half_thickness=22.0)
    if name == "droplet1m":
        return droplet(1_000_000, 166.0, seed=1005, temperature=temperature)
    raise KeyError(name)


def small_slab(n: int, box, seed: int, temperature: float = 0.7) -> State:
    """A slab with the same 98:2 split and geometry rule, at any size (test inputs)."""
    box = tuple(float(b) for b in box)
    n_liq = int(round(0.98 * n))
    ht = min(12.5, 0.25 * box[2])
    return slab(n_liq, n - n_liq, box, seed=seed, temperature=temperature, half_thickness=ht)


def serving_system(j: int, n_target: int, temperature: float) -> State:
    """Serving-trace system j: box L x L x 60 with L = max(14, round(28 sqrt(N/16000))),
    N_liq = round(0.8 L^2 25), N_vap = round(0.011662 L^2 35)."""
    L = max(14, int(round(28.0 * math.sqrt(n_target / 16000.0))))
    n_liq = int(round(0.8 * L * L * 25))
    n_vap = int(round(0.011662 * L * L * 35))
    return slab(n_liq, n_vap, (float(L), float(L), 60.0), seed=4000 + j, temperature=temperature)


def serving_droplet(j: int, n_target: int, temperature: float) -> State:
    """Serving-trace droplet j: n_target liquid particles (radius R for density 0.8) centred in a
    cubic box of side L = max(14, ceil(2 R + 16)) with vapor at 0.01 outside R + 1."""
    R = (3.0 * n_target / (0.8 * 4.0 * math.pi)) ** (1.0 / 3.0)
    L = max(14, int(math.ceil(2.0 * R + 16.0)))
    return droplet(n_target, float(L), seed=5000 + j, temperature=temperature)


def serving_trace(trace_seed: int, n_systems: int = 64, n_min: int = 4000, n_max: int = 200_000,
                  t_range=(0.65, 0.85)):
    """(N_target, T*) per system, N log-uniform on [n_min, n_max], T* uniform on t_range."""
    rng = SplitMix64(trace_seed, _TAG_TRACE)
    u = rng.uniform(2 * n_systems).reshape(2, n_systems)
    ns = np.exp(np.log(n_min) + u[0] * (np.log(n_max) - np.log(n_min)))
    ts = t_range[0] + u[1] * (t_range[1] - t_range[0])
    return [(int(round(a)), float(b)) for a, b in zip(ns, ts)]


def poisson_arrivals(trace_seed: int, n: int, rate: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    u = SplitMix64(trace_seed, _TAG_TRACE + 100).uniform(n)
    return np.cumsum(-np.log(1.0 - u) / rate)
