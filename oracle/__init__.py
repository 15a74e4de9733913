"""CPU FP64 oracle of the dynamic-cutoff-method hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may import
this package. The product path (``paper_1502_03234_amd``) never does; the two share no code.

``dcm_oracle.c`` (plain single-threaded C, FP64, no fast-math) is the oracle; this module
builds it with gcc on first use and marshals numpy arrays through ctypes. Every function
names the passage of the thesis it follows in the C source.

Parity status of each part (the pins live in ``tests/test_oracle_pins.py``): every function
below is pinned by closed forms, invariants, library routines or brute force.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dcm_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("epsilon", C.c_double), ("sigma", C.c_double),
                ("mass", C.c_double), ("rc_min", C.c_double), ("rc_max", C.c_double),
                ("alpha", C.c_double), ("bin", C.c_double), ("smooth_passes", C.c_int32),
                ("min_component", C.c_int32), ("detect_every", C.c_int32),
                ("pair_rule", C.c_int32), ("energy_shift", C.c_int32), ("dt", C.c_double),
                ("temperature", C.c_double), ("tdamp", C.c_double), ("thermostat", C.c_int32), ("cutoff_shape", C.c_int32),
                ("tail", C.c_int32), ("vapor_cutoff", C.c_int32), ("ms_nu", C.c_double),
                ("ms_iters", C.c_int32)]


class Thermo(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("virial", C.c_double * 6),
                ("pairs", C.c_int64), ("step", C.c_int64), ("xi", C.c_double), ("eta", C.c_double)]


class DetectOut(C.Structure):
    _fields_ = [("count", C.c_void_p), ("smooth", C.c_void_p), ("raw", C.c_void_p),
                ("label", C.c_void_p), ("dist", C.c_void_p), ("d", C.c_void_p),
                ("rc", C.c_void_p), ("km", C.c_double * 3), ("stats", C.c_int64 * 6),
                ("dist_v", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build(force=False)
        L = C.CDLL(path)
        P = C.POINTER(Params)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.orc_grid.argtypes = [P, vp, vp]
        L.orc_wrap.argtypes = [P, i64, vp]
        L.orc_bin.argtypes = [P, i64, vp, vp, vp]
        L.orc_smooth.argtypes = [vp, i32, vp, vp]
        L.orc_two_means.argtypes = [i64, vp, vp]
        L.orc_two_means.restype = i32
        L.orc_components.argtypes = [vp, vp, C.c_uint8, vp, vp]
        L.orc_components.restype = i64
        L.orc_segment.argtypes = [vp, vp, d, i32, vp, vp, vp]
        L.orc_distance.argtypes = [vp, vp, d, vp, vp]
        L.orc_distance.restype = i64
        L.orc_godunov.argtypes = [vp, vp]
        L.orc_godunov.restype = d
        L.orc_cutoff.argtypes = [P, d]
        L.orc_cutoff.restype = d
        L.orc_interp.argtypes = [vp, vp, vp, vp]
        L.orc_interp.restype = d
        L.orc_detect.argtypes = [P, i64, vp, C.POINTER(DetectOut)]
        L.orc_forces.argtypes = [P, i64, vp, vp, i64, vp, i32, vp, vp, vp, vp]
        L.orc_forces_images.argtypes = [P, i64, vp, d, i64, vp, vp, vp]
        L.orc_run.argtypes = [P, i64, vp, vp, vp, vp, i64, i32, i32, vp, vp]
        L.orc_tail_planar.argtypes = [P, d, d, d, d, vp, vp]
        L.orc_interp_grad.argtypes = [vp, vp, vp, vp, vp]
        L.orc_interp_grad.restype = d
        L.orc_tail.argtypes = [P, vp, vp, vp, i64, vp, vp, vp, vp]
        L.orc_ms_solve.argtypes = [vp, vp, vp, i32, vp]
        L.orc_mumford_shah.argtypes = [vp, vp, d, vp, vp, d, i32, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def params(box, *, epsilon=1.0, sigma=1.0, mass=1.0, rc_min=2.5, rc_max=6.0, alpha=-0.5,
           bin=1.0, smooth_passes=1, min_component=27, detect_every=2, pair_rule=0,
           energy_shift=0, dt=0.005, temperature=0.7, tdamp=0.5, thermostat=0,
           cutoff_shape=0, tail=0, vapor_cutoff=0, ms_nu=0.0, ms_iters=100) -> Params:
    p = Params()
    p.box[:] = [float(b) for b in box]
    p.epsilon, p.sigma, p.mass = epsilon, sigma, mass
    p.rc_min, p.rc_max, p.alpha, p.bin = rc_min, rc_max, alpha, bin
    p.smooth_passes, p.min_component = smooth_passes, min_component
    p.detect_every, p.pair_rule, p.energy_shift = detect_every, pair_rule, energy_shift
    p.dt = dt
    p.temperature, p.tdamp, p.thermostat = temperature, tdamp, thermostat
    p.cutoff_shape = cutoff_shape
    p.tail = tail
    p.vapor_cutoff = vapor_cutoff
    p.ms_nu, p.ms_iters = ms_nu, ms_iters
    return p


def grid(p: Params):
    dims = np.zeros(3, np.int32)
    h = np.zeros(3, np.float64)
    lib().orc_grid(C.byref(p), _p(dims), _p(h))
    return dims, h


def grid_shape(dims):
    """numpy shape of a grid array: [Nz][Ny][Nx]."""
    return (int(dims[2]), int(dims[1]), int(dims[0]))


def wrap(p: Params, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64).copy()
    lib().orc_wrap(C.byref(p), x.shape[1], _p(x))
    return x


def bin_particles(p: Params, x: np.ndarray):
    dims, _ = grid(p)
    x = np.ascontiguousarray(x, np.float64)
    count = np.zeros(int(np.prod(dims)), np.uint32)
    cell = np.zeros(x.shape[1], np.uint32)
    lib().orc_bin(C.byref(p), x.shape[1], _p(x), _p(count), _p(cell))
    return count, cell


def smooth(dims, passes: int, img: np.ndarray) -> np.ndarray:
    dims = np.asarray(dims, np.int32)
    img = np.ascontiguousarray(img, np.uint32).ravel()
    out = np.zeros_like(img)
    lib().orc_smooth(_p(dims), passes, _p(img), _p(out))
    return out


def two_means(g: np.ndarray):
    g = np.ascontiguousarray(g, np.uint32).ravel()
    km = np.zeros(3, np.float64)
    it = lib().orc_two_means(g.size, _p(g), _p(km))
    return km, it


def components(dims, s: np.ndarray, phase: int):
    dims = np.asarray(dims, np.int32)
    s = np.ascontiguousarray(s, np.uint8).ravel()
    comp = np.zeros(s.size, np.uint32)
    size = np.zeros(s.size, np.uint32)
    n = lib().orc_components(_p(dims), _p(s), phase, _p(comp), _p(size))
    return comp, size, n


def segment(dims, g: np.ndarray, t: float, min_component: int):
    dims = np.asarray(dims, np.int32)
    g = np.ascontiguousarray(g, np.uint32).ravel()
    raw = np.zeros(g.size, np.uint8)
    label = np.zeros(g.size, np.uint8)
    stats = np.zeros(4, np.int64)
    lib().orc_segment(_p(dims), _p(g), float(t), int(min_component), _p(raw), _p(label), _p(stats))
    return raw, label, stats


def distance(dims, h, cap: float, label: np.ndarray):
    dims = np.asarray(dims, np.int32)
    h = np.asarray(h, np.float64)
    label = np.ascontiguousarray(label, np.uint8).ravel()
    D = np.zeros(label.size, np.float64)
    rounds = lib().orc_distance(_p(dims), _p(h), float(cap), _p(label), _p(D))
    return D, rounds


def godunov(a, h=(1.0, 1.0, 1.0)) -> float:
    a = np.asarray(a, np.float64)
    h = np.asarray(h, np.float64)
    return lib().orc_godunov(_p(a), _p(h))


def cutoff(p: Params, d: float) -> float:
    return lib().orc_cutoff(C.byref(p), float(d))


def interp(dims, h, D: np.ndarray, xp) -> float:
    dims = np.asarray(dims, np.int32)
    h = np.asarray(h, np.float64)
    D = np.ascontiguousarray(D, np.float64).ravel()
    xp = np.asarray(xp, np.float64)
    return lib().orc_interp(_p(dims), _p(h), _p(D), _p(xp))


def ms_solve(dims, r: np.ndarray, w, iters: int, u0: np.ndarray) -> np.ndarray:
    """Relaxed two-phase segmentation (Eq. 13): minimise sum u r + sum_k w_k |D_k u| over
    u in [0, 1] by primal-dual iterations from u0; returns u."""
    dims = np.asarray(dims, np.int32)
    r = np.ascontiguousarray(r, np.float64).ravel()
    w = np.asarray(w, np.float64)
    u = np.ascontiguousarray(u0, np.float64).ravel().copy()
    lib().orc_ms_solve(_p(dims), _p(r), _p(w), int(iters), _p(u))
    return u


def mumford_shah(dims, h, Lmax: float, g: np.ndarray, km, nu: float, iters: int, raw: np.ndarray):
    """Eq. 13 on image g from the labels raw (threshold labels): (labels, relaxed u)."""
    dims = np.asarray(dims, np.int32)
    h = np.asarray(h, np.float64)
    g = np.ascontiguousarray(g, np.uint32).ravel()
    km = np.ascontiguousarray(km, np.float64)
    lab = np.ascontiguousarray(raw, np.uint8).ravel().copy()
    u = np.zeros(lab.size)
    lib().orc_mumford_shah(_p(dims), _p(h), float(Lmax), _p(g), _p(km), float(nu), int(iters),
                           _p(lab), _p(u))
    return lab, u


def interp_grad(dims, h, D: np.ndarray, xp):
    """Trilinear interpolation (Eq. 6) and the gradient of the interpolant: (value, grad[3])."""
    dims = np.asarray(dims, np.int32)
    h = np.asarray(h, np.float64)
    D = np.ascontiguousarray(D, np.float64).ravel()
    xp = np.asarray(xp, np.float64)
    g = np.zeros(3)
    v = lib().orc_interp_grad(_p(dims), _p(h), _p(D), _p(xp), _p(g))
    return v, g


def tail_planar(p: Params, rc: float, delta: float, rho_l: float, rho_v: float):
    """Eq. 21-22 for a planar interface at signed distance delta (> 0: in the liquid):
    (force along the normal into the liquid, du)."""
    fn = np.zeros(1)
    du = np.zeros(1)
    lib().orc_tail_planar(C.byref(p), float(rc), float(delta), float(rho_l), float(rho_v),
                          _p(fn), _p(du))
    return float(fn[0]), float(du[0])


def tail(p: Params, det: "Detection", x: np.ndarray, rc: np.ndarray):
    """Tail correction of every particle from a detection's distance fields (Eq. 21-22).
    Returns (f [3][n], du [n]); the pair-energy share of particle i is du[i] / 2."""
    if det.dist_v is None:
        raise ValueError("the detection was run without the tail correction's vapor distances")
    x = np.ascontiguousarray(x, np.float64)
    rc = np.ascontiguousarray(rc, np.float64)
    n = x.shape[1]
    f = np.zeros((3, n))
    du = np.zeros(n)
    km = np.ascontiguousarray(det.km, np.float64)
    lib().orc_tail(C.byref(p), _p(det.dist), _p(det.dist_v), _p(km), n, _p(x), _p(rc), _p(f), _p(du))
    return f, du


@dataclass
class Detection:
    count: np.ndarray
    smooth: np.ndarray
    raw: np.ndarray
    label: np.ndarray
    dist: np.ndarray
    d: np.ndarray
    rc: np.ndarray
    km: np.ndarray
    stats: np.ndarray
    dist_v: np.ndarray | None = None


def detect(p: Params, x: np.ndarray) -> Detection:
    """Interface detection of one (already wrapped) state: Eq. 9-12, 14-19, Alg. 3.1, Eq. 7."""
    dims, _ = grid(p)
    G = int(np.prod(dims))
    x = np.ascontiguousarray(x, np.float64)
    n = x.shape[1]
    det = Detection(np.zeros(G, np.uint32), np.zeros(G, np.uint32), np.zeros(G, np.uint8),
                    np.zeros(G, np.uint8), np.zeros(G), np.zeros(n), np.zeros(n),
                    np.zeros(3), np.zeros(6, np.int64),
                    np.zeros(G) if (p.tail or p.vapor_cutoff) else None)
    o = DetectOut(_p(det.count).value, _p(det.smooth).value, _p(det.raw).value,
                  _p(det.label).value, _p(det.dist).value, _p(det.d).value, _p(det.rc).value)
    o.dist_v = _p(det.dist_v).value if det.dist_v is not None else None
    lib().orc_detect(C.byref(p), n, _p(x), C.byref(o))
    det.km[:] = o.km[:]
    det.stats[:] = o.stats[:]
    return det


@dataclass
class Forces:
    f: np.ndarray      # [3][m]
    e: np.ndarray      # [m]
    w: np.ndarray      # [6][m]  (xx, yy, zz, xy, xz, yz)
    pairs: np.ndarray  # [m]


def forces(p: Params, x: np.ndarray, rc: np.ndarray, subset=None, method: int = 1) -> Forces:
    """Alg. 3.2 with per-particle cutoffs rc; method 0 = all pairs, 1 = link cells."""
    x = np.ascontiguousarray(x, np.float64)
    rc = np.ascontiguousarray(rc, np.float64)
    n = x.shape[1]
    sub = None if subset is None else np.ascontiguousarray(subset, np.int64)
    m = n if sub is None else sub.size
    out = Forces(np.zeros((3, m)), np.zeros(m), np.zeros((6, m)), np.zeros(m, np.int64))
    lib().orc_forces(C.byref(p), n, _p(x), _p(rc), m, None if sub is None else _p(sub), method,
                     _p(out.f), _p(out.e), _p(out.w), _p(out.pairs))
    return out


def forces_images(p: Params, x: np.ndarray, R: float, subset=None):
    """Exact reference forces (Eq. 20's F^exact): full LJ over all images within R.
    Returns (f [3][m], e [m])."""
    x = np.ascontiguousarray(x, np.float64)
    n = x.shape[1]
    sub = None if subset is None else np.ascontiguousarray(subset, np.int64)
    m = n if sub is None else sub.size
    f = np.zeros((3, m))
    e = np.zeros(m)
    lib().orc_forces_images(C.byref(p), n, _p(x), float(R), m, None if sub is None else _p(sub),
                            _p(f), _p(e))
    return f, e


def thermo_of(fr: Forces, v: np.ndarray, mass: float = 1.0) -> dict:
    return dict(ke=0.5 * mass * float(np.sum(v * v)), pe=float(np.sum(fr.e)),
                virial=fr.w.sum(axis=1), pairs=int(fr.pairs.sum()))


@dataclass
class RunState:
    x: np.ndarray
    v: np.ndarray
    rc: np.ndarray
    f: np.ndarray
    k: int
    xi: float = 0.0
    eta: float = 0.0


def prepare(p: Params, x: np.ndarray, v: np.ndarray, method: int = 1) -> RunState:
    """Force evaluation k = 0 of a new state: wrap, detect, forces."""
    x = wrap(p, x)
    det = detect(p, x)
    fr = forces(p, x, det.rc, method=method)
    f = fr.f.copy()
    if p.tail:
        f += tail(p, det, x, det.rc)[0]
    return RunState(x, np.ascontiguousarray(v, np.float64).copy(), det.rc.copy(), f, 0)


def run(p: Params, st: RunState, nsteps: int, method: int = 1):
    """Advance st in place by nsteps velocity-Verlet steps; returns the thermo records."""
    th = (Thermo * max(nsteps, 1))()
    nh = np.array([st.xi, st.eta], np.float64)
    lib().orc_run(C.byref(p), st.x.shape[1], _p(st.x), _p(st.v), _p(st.rc), _p(st.f), st.k,
                  nsteps, method, _p(nh), C.cast(th, C.c_void_p))
    st.k += nsteps
    st.xi, st.eta = float(nh[0]), float(nh[1])
    return [dict(ke=t.ke, pe=t.pe, virial=np.array(t.virial[:]), pairs=t.pairs, step=t.step,
                 xi=t.xi, eta=t.eta) for t in th[:nsteps]]
