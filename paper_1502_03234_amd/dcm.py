"""ctypes binding of libdcm.so (C ABI in include/dcm.h); argument marshalling only.

Every computation runs in the library's HIP kernels. PyTorch supplies device memory (the
workspace and the caller arrays) and the stream. Importing this module loads the library
and raises ImportError if it has not been built -- there is no other execution path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcm.so")

DCM_OK, DCM_PENDING = 0, 1
DCM_E_INVALID, DCM_E_WORKSPACE, DCM_E_HIP, DCM_E_BUDGET = -1, -2, -3, -4
DCM_E_NONFINITE, DCM_E_UNKNOWN_TICKET, DCM_E_NOT_CONVERGED = -5, -6, -7
DCM_FP64, DCM_FP32C = 0, 1
DCM_PAIR_I, DCM_PAIR_MAX = 0, 1
DCM_NVE, DCM_NOSE_HOOVER = 0, 1
DCM_CUTOFF_EXP, DCM_CUTOFF_LINEAR = 0, 1
DCM_NSTAGES = 11
STAGES = ["kick_drift_key", "sort", "smooth", "two_means", "segment", "distance", "cutoffs",
          "forces", "reduce", "tail", "list"]


class DcmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dcm status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("epsilon", C.c_double), ("sigma", C.c_double),
                ("mass", C.c_double), ("rc_min", C.c_double), ("rc_max", C.c_double),
                ("alpha", C.c_double), ("bin", C.c_double), ("smooth_passes", C.c_int32),
                ("min_component", C.c_int32), ("detect_every", C.c_int32),
                ("precision", C.c_int32), ("pair_rule", C.c_int32), ("energy_shift", C.c_int32),
                ("dt", C.c_double), ("temperature", C.c_double), ("tdamp", C.c_double),
                ("thermostat", C.c_int32), ("cutoff_shape", C.c_int32), ("tail", C.c_int32),
                ("vapor_cutoff", C.c_int32), ("ms_nu", C.c_double), ("ms_iters", C.c_int32),
                ("neighbor_list", C.c_int32), ("skin", C.c_double), ("list_capacity", C.c_int32)]


class Thermo(C.Structure):
    _fields_ = [("ke", C.c_double), ("pe", C.c_double), ("virial", C.c_double * 6),
                ("pairs", C.c_int64), ("step", C.c_int64), ("xi", C.c_double), ("eta", C.c_double)]


THERMO_DOUBLES = C.sizeof(Thermo) // 8     # 12 doubles per record


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("queued", C.c_int64), ("running", C.c_int64),
                ("batches", C.c_int64), ("bytes_in_use", C.c_size_t), ("groupings", C.c_int64),
                ("grouping_ms", C.c_double), ("grouped_steps", C.c_int64), ("eager_steps", C.c_int64)]


class DetectOut(C.Structure):
    _fields_ = [("count", C.c_void_p), ("smooth", C.c_void_p), ("raw", C.c_void_p),
                ("label", C.c_void_p), ("dist", C.c_void_p), ("rc", C.c_void_p),
                ("km", C.c_void_p), ("stats", C.c_void_p), ("dist_v", C.c_void_p)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")

_lib = C.CDLL(LIB_PATH)
_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_PP = C.POINTER(Params)
_SIGS = {
    "dcm_version": ([], C.c_char_p),
    "dcm_last_error": ([], C.c_char_p),
    "dcm_grid_dims": ([_PP, _vp], _i32),
    "dcm_workspace_bytes": ([_PP, _i64, C.POINTER(_sz)], _i32),
    "dcm_create": ([_PP, _i64, _vp, _sz, _vp, _vp, _vp, C.POINTER(_vp)], _i32),
    "dcm_create_from_state": ([_PP, _i64, _vp, _sz, _vp, _vp, _vp, _i64, _vp, C.POINTER(_vp)], _i32),
    "dcm_set_cutoffs": ([_vp, _vp, _vp], _i32),
    "dcm_detect_interface": ([_vp, _vp, C.POINTER(DetectOut)], _i32),
    "dcm_compute_forces": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "dcm_step": ([_vp, _i32, _vp, _vp], _i32),
    "dcm_exact_forces": ([_vp, C.c_double, _vp, _vp, _vp], _i32),
    "dcm_get_thermostat": ([_vp, _vp, _vp], _i32),
    "dcm_set_thermostat": ([_vp, _vp, _vp], _i32),
    "dcm_get_state": ([_vp, _vp, _vp, _vp, _vp, C.POINTER(_i64)], _i32),
    "dcm_check": ([_vp, _vp], _i32),
    "dcm_set_profiling": ([_vp, _i32], _i32),
    "dcm_stage_times": ([_vp, _vp, _vp], _i32),
    "dcm_destroy": ([_vp], _i32),
    "dcm_list_builds": ([_vp, C.POINTER(_i64)], _i32),
    "dcm_grid_workspace_bytes": ([_vp, C.POINTER(_sz)], _i32),
    "dcm_grid_smooth": ([_vp, _i32, _vp, _vp, _vp, _sz, _vp], _i32),
    "dcm_grid_smooth_noalloc": ([_vp, _i32, _vp, _vp, _vp], _i32),
    "dcm_grid_two_means": ([_vp, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "dcm_grid_segment": ([_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "dcm_grid_distance": ([_vp, _vp, C.c_double, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "dcm_server_create": ([_sz, _vp, _sz, _vp, C.POINTER(_vp)], _i32),
    "dcm_submit": ([_vp, _PP, _i64, _vp, _vp, _i32, C.POINTER(C.c_uint64)], _i32),
    "dcm_poll": ([_vp, C.c_uint64, _vp, _vp, C.POINTER(Thermo)], _i32),
    "dcm_server_query": ([_vp, C.POINTER(ServerStats)], _i32),
    "dcm_server_destroy": ([_vp], _i32),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def _check(status: int) -> int:
    if status < 0:
        raise DcmError(status, _lib.dcm_last_error().decode())
    return status


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device arrays must be contiguous CUDA/HIP tensors")
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream if hasattr(s, "cuda_stream") else int(s)


def params(box, *, epsilon=1.0, sigma=1.0, mass=1.0, rc_min=2.5, rc_max=6.0, alpha=-0.5, bin=1.0,
           smooth_passes=1, min_component=27, detect_every=2, precision=DCM_FP64,
           pair_rule=DCM_PAIR_I, energy_shift=0, dt=0.005, temperature=0.7, tdamp=0.5,
           thermostat=DCM_NVE, cutoff_shape=DCM_CUTOFF_EXP, tail=0, vapor_cutoff=0, ms_nu=0.0,
           ms_iters=100, neighbor_list=0, skin=0.3, list_capacity=0) -> Params:
    p = Params()
    p.box[:] = [float(b) for b in box]
    p.epsilon, p.sigma, p.mass = epsilon, sigma, mass
    p.rc_min, p.rc_max, p.alpha, p.bin = rc_min, rc_max, alpha, bin
    p.smooth_passes, p.min_component, p.detect_every = smooth_passes, min_component, detect_every
    p.precision, p.pair_rule, p.energy_shift, p.dt = precision, pair_rule, energy_shift, dt
    p.temperature, p.tdamp, p.thermostat = temperature, tdamp, thermostat
    p.cutoff_shape = cutoff_shape
    p.tail = tail
    p.vapor_cutoff = vapor_cutoff
    p.ms_nu, p.ms_iters = ms_nu, ms_iters
    p.neighbor_list, p.skin, p.list_capacity = neighbor_list, skin, list_capacity
    return p


# ---- one wrapper per C entry point, same names -------------------------------------------
def dcm_version() -> str:
    return _lib.dcm_version().decode()


def dcm_last_error() -> str:
    return _lib.dcm_last_error().decode()


def dcm_grid_dims(p: Params):
    dims = (C.c_int32 * 3)()
    _check(_lib.dcm_grid_dims(C.byref(p), dims))
    return tuple(dims)


def dcm_workspace_bytes(p: Params, n: int) -> int:
    b = C.c_size_t()
    _check(_lib.dcm_workspace_bytes(C.byref(p), int(n), C.byref(b)))
    return b.value


def dcm_create(p: Params, n: int, ws, x, v, stream=None) -> int:
    h = C.c_void_p()
    _check(_lib.dcm_create(C.byref(p), int(n), _ptr(ws), ws.numel() * ws.element_size(), _ptr(x),
                           _ptr(v), _stream(stream), C.byref(h)))
    return h.value


def dcm_create_from_state(p: Params, n: int, ws, x, v, rc, step: int, stream=None) -> int:
    h = C.c_void_p()
    _check(_lib.dcm_create_from_state(C.byref(p), int(n), _ptr(ws), ws.numel() * ws.element_size(),
                                      _ptr(x), _ptr(v), _ptr(rc), int(step), _stream(stream),
                                      C.byref(h)))
    return h.value


def dcm_set_cutoffs(h: int, rc, stream=None):
    _check(_lib.dcm_set_cutoffs(h, _stream(stream), _ptr(rc)))


def dcm_detect_interface(h: int, stream=None, **outs):
    o = DetectOut(*[_ptr(outs.get(f)) for f, _ in DetectOut._fields_])
    _check(_lib.dcm_detect_interface(h, _stream(stream), C.byref(o)))


def dcm_compute_forces(h: int, stream=None, f=None, e=None, w=None, pairs=None, thermo=None):
    _check(_lib.dcm_compute_forces(h, _stream(stream), _ptr(f), _ptr(e), _ptr(w), _ptr(pairs),
                                   _ptr(thermo)))


def dcm_exact_forces(h: int, R: float, stream=None, f=None, e=None):
    _check(_lib.dcm_exact_forces(h, float(R), _stream(stream), _ptr(f), _ptr(e)))


def dcm_step(h: int, nsteps: int, stream=None, thermo=None):
    _check(_lib.dcm_step(h, int(nsteps), _stream(stream), _ptr(thermo)))


def dcm_get_thermostat(h: int, stream=None):
    t = (C.c_double * 2)()
    _check(_lib.dcm_get_thermostat(h, _stream(stream), t))
    return float(t[0]), float(t[1])


def dcm_set_thermostat(h: int, xi: float, eta: float, stream=None):
    t = (C.c_double * 2)(float(xi), float(eta))
    _check(_lib.dcm_set_thermostat(h, _stream(stream), t))


def dcm_get_state(h: int, stream=None, x=None, v=None, rc=None) -> int:
    k = C.c_int64()
    _check(_lib.dcm_get_state(h, _stream(stream), _ptr(x), _ptr(v), _ptr(rc), C.byref(k)))
    return k.value


def dcm_check(h: int, stream=None):
    _check(_lib.dcm_check(h, _stream(stream)))


def dcm_set_profiling(h: int, on):
    """on: False/0 off, True/1 every stage, 2 the pair-force stage only."""
    _check(_lib.dcm_set_profiling(h, int(on)))


def dcm_stage_times(h: int):
    ms = (C.c_double * DCM_NSTAGES)()
    cnt = (C.c_int64 * DCM_NSTAGES)()
    _check(_lib.dcm_stage_times(h, ms, cnt))
    return {STAGES[q]: (ms[q], cnt[q]) for q in range(DCM_NSTAGES)}


def dcm_list_builds(h: int) -> int:
    b = C.c_int64(0)
    _check(_lib.dcm_list_builds(h, C.byref(b)))
    return b.value


def dcm_destroy(h: int):
    _check(_lib.dcm_destroy(h))


def dcm_grid_workspace_bytes(dims) -> int:
    d = (C.c_int32 * 3)(*dims)
    b = C.c_size_t()
    _check(_lib.dcm_grid_workspace_bytes(d, C.byref(b)))
    return b.value


def dcm_grid_smooth(dims, passes: int, img, out, ws, stream=None):
    d = (C.c_int32 * 3)(*dims)
    _check(_lib.dcm_grid_smooth(d, int(passes), _ptr(img), _ptr(out), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)))


def dcm_grid_smooth_noalloc(dims, passes: int, img, out, stream=None):
    d = (C.c_int32 * 3)(*dims)
    _check(_lib.dcm_grid_smooth_noalloc(d, int(passes), _ptr(img), _ptr(out), _stream(stream)))


def dcm_grid_two_means(dims, img, km, stats, ws, stream=None):
    d = (C.c_int32 * 3)(*dims)
    _check(_lib.dcm_grid_two_means(d, _ptr(img), _ptr(km), _ptr(stats), _ptr(ws),
                                   ws.numel() * ws.element_size(), _stream(stream)))


def dcm_grid_segment(dims, img, km, min_component: int, raw, label, stats, ws, stream=None):
    d = (C.c_int32 * 3)(*dims)
    _check(_lib.dcm_grid_segment(d, _ptr(img), _ptr(km), int(min_component), _ptr(raw), _ptr(label),
                                 _ptr(stats), _ptr(ws), ws.numel() * ws.element_size(),
                                 _stream(stream)))


def dcm_grid_distance(dims, h, cap: float, label, dist, sweeps, ws, stream=None):
    d = (C.c_int32 * 3)(*dims)
    hh = (C.c_double * 3)(*h)
    _check(_lib.dcm_grid_distance(d, hh, float(cap), _ptr(label), _ptr(dist), _ptr(sweeps), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)))


def dcm_server_create(budget: int, pool, stream=None) -> int:
    h = C.c_void_p()
    _check(_lib.dcm_server_create(int(budget), _ptr(pool), pool.numel() * pool.element_size(),
                                  _stream(stream), C.byref(h)))
    return h.value


def dcm_submit(sv: int, p: Params, x, v, nsteps: int) -> int:
    """x, v: host float64 [3][n] arrays (numpy); copied by the library."""
    import numpy as np
    x = np.ascontiguousarray(x, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    t = C.c_uint64()
    _check(_lib.dcm_submit(sv, C.byref(p), x.shape[1], x.ctypes.data, v.ctypes.data, int(nsteps),
                           C.byref(t)))
    return t.value


def dcm_poll(sv: int, ticket: int, n: int):
    """(status, x, v, thermo): status DCM_PENDING, or DCM_OK with host results."""
    import numpy as np
    x = np.empty((3, n))
    v = np.empty((3, n))
    th = Thermo()
    st = _lib.dcm_poll(sv, int(ticket), x.ctypes.data, v.ctypes.data, C.byref(th))
    if st == DCM_PENDING:
        return st, None, None, None
    _check(st)
    rec = dict(ke=th.ke, pe=th.pe, virial=list(th.virial), pairs=th.pairs, step=th.step, xi=th.xi,
               eta=th.eta)
    return st, x, v, rec


def dcm_server_query(sv: int) -> dict:
    s = ServerStats()
    _check(_lib.dcm_server_query(sv, C.byref(s)))
    return {f: getattr(s, f) for f, _ in ServerStats._fields_}


def dcm_server_destroy(sv: int):
    _check(_lib.dcm_server_destroy(sv))


# ---- convenience: a system whose workspace and state tensors torch allocates -------------
def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """Device workspace (torch allocations are 256-byte aligned)."""
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + int(nbytes)]


def thermo_records(t: torch.Tensor):
    """Decode a float64 tensor of k * THERMO_DOUBLES values into dicts."""
    a = t.detach().cpu().view(torch.float64).reshape(-1, THERMO_DOUBLES)
    ints = t.detach().cpu().view(torch.int64).reshape(-1, THERMO_DOUBLES)
    return [dict(ke=float(r[0]), pe=float(r[1]), virial=r[2:8].numpy().copy(),
                 pairs=int(i[8]), step=int(i[9]), xi=float(r[10]), eta=float(r[11]))
            for r, i in zip(a, ints)]


class System:
    """A DCM system on one GPU: caller tensors in, caller tensors out."""

    def __init__(self, p: Params, x, v, rc=None, step: int = 0, device="cuda", stream=None):
        x = torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()
        v = torch.as_tensor(v, dtype=torch.float64).to(device).contiguous()
        self.p, self.n, self.device = p, int(x.shape[1]), device
        self.stream = stream
        self.ws = workspace(dcm_workspace_bytes(p, self.n), device)
        if rc is None:
            self.h = dcm_create(p, self.n, self.ws, x, v, stream)
        else:
            rc = torch.as_tensor(rc, dtype=torch.float64).to(device).contiguous()
            self.h = dcm_create_from_state(p, self.n, self.ws, x, v, rc, step, stream)
        self.dims = dcm_grid_dims(p)
        self.G = self.dims[0] * self.dims[1] * self.dims[2]

    def close(self):
        if self.h:
            torch.cuda.synchronize()
            dcm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=self.device)

    def detect(self):
        o = dict(count=self._t(self.G, torch.int32), smooth=self._t(self.G, torch.int32),
                 raw=self._t(self.G, torch.uint8), label=self._t(self.G, torch.uint8),
                 dist=self._t(self.G, torch.float64), rc=self._t(self.n, torch.float64),
                 km=self._t(3, torch.float64), stats=self._t(6, torch.int64))
        if self.p.tail or self.p.vapor_cutoff:
            o["dist_v"] = self._t(self.G, torch.float64)
        dcm_detect_interface(self.h, self.stream, **o)
        return o

    def forces(self, per_atom=True, thermo=True):
        o = dict(f=self._t((3, self.n), torch.float64))
        if per_atom:
            o.update(e=self._t(self.n, torch.float64), w=self._t((6, self.n), torch.float64),
                     pairs=self._t(self.n, torch.int32))
        if thermo:
            o["thermo"] = self._t(THERMO_DOUBLES, torch.float64)
        dcm_compute_forces(self.h, self.stream, **o)
        return o

    def exact_forces(self, R: float, energy=False):
        """Eq. 20's reference: full LJ over every image within R (forces [3][n], energies [n])."""
        f = self._t((3, self.n), torch.float64)
        e = self._t(self.n, torch.float64) if energy else None
        dcm_exact_forces(self.h, R, self.stream, f=f, e=e)
        return (f, e) if energy else f

    def set_cutoffs(self, rc):
        dcm_set_cutoffs(self.h, torch.as_tensor(rc, dtype=torch.float64).to(self.device).contiguous(),
                        self.stream)

    def step(self, nsteps: int, thermo=True):
        th = self._t(max(nsteps, 1) * THERMO_DOUBLES, torch.float64) if thermo else None
        dcm_step(self.h, nsteps, self.stream, th)
        return th

    def state(self):
        x, v, rc = self._t((3, self.n), torch.float64), self._t((3, self.n), torch.float64), \
            self._t(self.n, torch.float64)
        k = dcm_get_state(self.h, self.stream, x, v, rc)
        return x, v, rc, k

    def check(self):
        dcm_check(self.h, self.stream)

    def thermostat(self):
        return dcm_get_thermostat(self.h, self.stream)

    def set_thermostat(self, xi: float, eta: float):
        dcm_set_thermostat(self.h, xi, eta, self.stream)
