"""ctypes binding of libhb (include/hb.h): same names, argument marshalling only.

Every step of the solver runs in the HIP kernels of libhb.so; this module only
converts Python/NumPy/torch arguments into the C ABI's plain pointers and
raises ``HBError`` on a negative status.  Arrays are C-ordered [nz][ny][nx]:
NumPy arrays are passed as host memory, CUDA/HIP torch tensors as device
memory.  There is no CPU fallback: ``load()`` fails when the library is
missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhb.so")

HB_OK = 0
HB_E_ARG, HB_E_CFL, HB_E_NOMEM, HB_E_HIP, HB_E_STATE, HB_E_BUSY, HB_E_NONFINITE = range(-1, -8, -1)
HB_F64, HB_F32C = 0, 1
HB_HOST, HB_DEVICE = 0, 1
HB_DTYPE_F64, HB_DTYPE_F32 = 0, 1
HB_ALLOW_UNSTABLE, HB_USE_GRAPH, HB_STAGEWISE, HB_PAIRWISE, HB_BC_PERIODIC = 1, 2, 4, 8, 16
HB_DEBUG_POISON = 32

_NAMES = {HB_E_ARG: "HB_E_ARG", HB_E_CFL: "HB_E_CFL", HB_E_NOMEM: "HB_E_NOMEM",
          HB_E_HIP: "HB_E_HIP", HB_E_STATE: "HB_E_STATE", HB_E_BUSY: "HB_E_BUSY",
          HB_E_NONFINITE: "HB_E_NONFINITE"}


class HBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class hb_config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("mu2", ctypes.c_double), ("lambda_", ctypes.c_double), ("inv_L2", ctypes.c_double),
                ("t0", ctypes.c_double), ("dt", ctypes.c_double), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("stream", ctypes.c_void_p)]


class hb_radial_config(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("flags", ctypes.c_uint32), ("dr", ctypes.c_double),
                ("mu2", ctypes.c_double), ("lambda_", ctypes.c_double), ("inv_L2", ctypes.c_double),
                ("t0", ctypes.c_double), ("dt", ctypes.c_double), ("steps", ctypes.c_int64)]


HB_RADIAL_MAX_NODES = 2700


class hb_diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("step", ctypes.c_int64), ("integral", ctypes.c_double),
                ("l2_phi", ctypes.c_double), ("l2_psi", ctypes.c_double),
                ("linf_phi", ctypes.c_double), ("linf_psi", ctypes.c_double),
                ("lap_max", ctypes.c_double), ("energy", ctypes.c_double),
                ("nonfinite", ctypes.c_int64), ("negative", ctypes.c_int64)]

    def asdict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib: Optional[ctypes.CDLL] = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SIGS = {
    "hb_create": [ctypes.POINTER(hb_config), ctypes.POINTER(_P)],
    "hb_set_initial": [_P, _P, _P, _I, _I],
    "hb_set_state": [_P, _P, _P, _I64, _I, _I],
    "hb_step": [_P, _I64],
    "hb_step_timed": [_P, _I64, ctypes.POINTER(ctypes.c_double)],
    "hb_read": [_P, _P, _P, _I, _I],
    "hb_time": [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)],
    "hb_sync": [_P],
    "hb_diagnostics": [_P, ctypes.POINTER(hb_diag)],
    "hb_bubbles": [_P, ctypes.c_double, ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
    "hb_set_tiling": [_P, _I, _I],
    "hb_default_tiling": [ctypes.POINTER(hb_config), ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "hb_autotune": [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "hb_destroy": [_P],
    "hb_footprint": [ctypes.POINTER(hb_config)],
    "hb_last_error": [],
    "hb_set_allocator": [_P, _P, _P],
    "hb_batch_create": [_I, ctypes.POINTER(hb_config), _P, ctypes.POINTER(_P)],
    "hb_batch_set_initial": [_P, _I, _P, _P, _I, _I],
    "hb_batch_step": [_P, _I64],
    "hb_batch_read": [_P, _I, _P, _P, _I, _I],
    "hb_batch_sync": [_P],
    "hb_batch_set_tiling": [_P, _I, _I],
    "hb_batch_autotune": [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "hb_batch_destroy": [_P],
    "hb_pool_create": [ctypes.c_size_t, _I, _P, ctypes.POINTER(_P)],
    "hb_pool_admit": [_P, ctypes.POINTER(hb_config), _P, _P, _I, _I, _I64, ctypes.POINTER(_I)],
    "hb_pool_advance": [_P, _I],
    "hb_pool_poll": [_P, ctypes.POINTER(_I), _I, ctypes.POINTER(_I)],
    "hb_pool_check": [_P, ctypes.POINTER(_I), _I, ctypes.POINTER(_I)],
    "hb_pool_stats": [_P, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_size_t)],
    "hb_pool_read": [_P, _I, _P, _P, _I, _I],
    "hb_pool_release": [_P, _I],
    "hb_pool_destroy": [_P],
    "hb_probe_bandwidth": [_I, ctypes.c_size_t, _I, ctypes.POINTER(ctypes.c_double)],
    "hb_radial_solve": [_I, ctypes.POINTER(hb_radial_config), _P, _P, _I, _P],
    "hb_radial_solve_noalloc": [_I, ctypes.POINTER(hb_radial_config), _P, _P, _P],
}


def exported_names():
    return list(_SIGS)


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhb.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhb.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_size_t if name == "hb_footprint" else (
            ctypes.c_char_p if name == "hb_last_error" else ctypes.c_int)
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise HBError(rc, load().hb_last_error().decode())
    return rc


def _arr(a):
    """(pointer, mem, dtype, keepalive) of a NumPy array or a torch tensor."""
    if a is None:
        return None, HB_HOST, HB_DTYPE_F64, None
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("arrays must be C-contiguous")
        if a.dtype == np.float64:
            dt = HB_DTYPE_F64
        elif a.dtype == np.float32:
            dt = HB_DTYPE_F32
        else:
            raise TypeError(f"unsupported dtype {a.dtype}")
        return a.ctypes.data, HB_HOST, dt, a
    import torch
    if isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        if a.dtype == torch.float64:
            dt = HB_DTYPE_F64
        elif a.dtype == torch.float32:
            dt = HB_DTYPE_F32
        else:
            raise TypeError(f"unsupported dtype {a.dtype}")
        return a.data_ptr(), (HB_DEVICE if a.is_cuda else HB_HOST), dt, a
    raise TypeError(f"unsupported array type {type(a)}")


# Points of every live grid, keyed by ("s", solver), ("b", batch, index) or
# ("p", pool, slot): the C ABI takes no array sizes, so the binding checks
# them before a kernel could read or write past a caller's array.
_GRIDS: dict = {}


def _points(cfg) -> int:
    return int(cfg.n[0]) * int(cfg.n[1]) * int(cfg.n[2])


def _pair(key, a, b, what):
    """Marshal one or two state arrays of the grid `key` (each may be None):
    (ptr_a, ptr_b, mem, dtype, keepalive).  Both must hold the grid's number of
    points and share memory kind and dtype."""
    if key not in _GRIDS:
        raise ValueError(f"{what}: unknown or destroyed handle")
    count = _GRIDS[key]
    ma, mb = _arr(a), _arr(b)
    for x in (a, b):
        if x is not None:
            n = x.size if isinstance(x, np.ndarray) else x.numel()
            if n != count:
                raise ValueError(f"{what}: array has {n} values, the grid has {count}")
    if a is not None and b is not None and ma[1:3] != mb[1:3]:
        raise ValueError(f"{what}: both arrays must share memory kind and dtype")
    mem, dt = (ma[1], ma[2]) if a is not None else (mb[1], mb[2])
    return ma[0], mb[0], mem, dt, (ma[3], mb[3])


def make_config(n: Sequence[int], lo: Sequence[float], hi: Sequence[float], mu2: float,
                lam: float, dt: float, t0: float = 0.0, inv_L2: float = 1.0,
                precision: int = HB_F64, flags: int = 0, stream: Optional[int] = None) -> hb_config:
    c = hb_config()
    c.n[:] = [int(v) for v in n]
    c.lo[:] = [float(v) for v in lo]
    c.hi[:] = [float(v) for v in hi]
    c.mu2, c.lambda_, c.inv_L2, c.t0, c.dt = float(mu2), float(lam), float(inv_L2), float(t0), float(dt)
    c.precision, c.flags, c.stream = int(precision), int(flags), stream
    return c


def config_from_workload(w, precision: int = HB_F64, flags: int = 0, stream=None) -> hb_config:
    return make_config(w.n, w.lo, w.hi, w.mu2, w.lam, w.dt, w.t0, w.inv_L2, precision, flags, stream)


# ---- single solve ---------------------------------------------------------------

def hb_create(cfg: hb_config) -> int:
    h = _P()
    _check(load().hb_create(ctypes.byref(cfg), ctypes.byref(h)))
    _GRIDS[("s", h.value)] = _points(cfg)
    return h.value


def hb_set_initial(h: int, phi0, phi1=None) -> None:
    if phi0 is None:
        raise ValueError("hb_set_initial: phi0 is required")
    p0, p1, m, d, _keep = _pair(("s", h), phi0, phi1, "hb_set_initial")
    _check(load().hb_set_initial(h, p0, p1, m, d))


def hb_set_state(h: int, phi, psi, n: int) -> None:
    if phi is None:
        raise ValueError("hb_set_state: phi is required")
    p0, p1, m, d, _keep = _pair(("s", h), phi, psi, "hb_set_state")
    _check(load().hb_set_state(h, p0, p1, int(n), m, d))


def hb_step(h: int, nsteps: int) -> None:
    _check(load().hb_step(h, int(nsteps)))


def hb_step_timed(h: int, nsteps: int):
    ms = (ctypes.c_double * 4)()
    _check(load().hb_step_timed(h, int(nsteps), ms))
    return list(ms)


def hb_read(h: int, phi=None, phi_t=None) -> None:
    """Fill the given output arrays (NumPy host or torch device)."""
    if phi is None and phi_t is None:
        return
    p0, p1, m, d, _keep = _pair(("s", h), phi, phi_t, "hb_read")
    _check(load().hb_read(h, p0, p1, m, d))


def hb_time(h: int):
    t = ctypes.c_double()
    n = _I64()
    _check(load().hb_time(h, ctypes.byref(t), ctypes.byref(n)))
    return t.value, n.value


def hb_sync(h: int) -> None:
    _check(load().hb_sync(h))


def hb_diagnostics(h: int, allow_nonfinite: bool = False) -> dict:
    d = hb_diag()
    rc = load().hb_diagnostics(h, ctypes.byref(d))
    if rc == HB_E_NONFINITE and allow_nonfinite:
        return d.asdict()
    _check(rc)
    return d.asdict()


def hb_bubbles(h: int, eps: float = 0.0):
    """(negative sets, positive sets): face-connected sets of {phi < -eps}
    and {phi > eps} in the current state (the paper's bubbles, section 1)."""
    neg, pos = _I64(), _I64()
    _check(load().hb_bubbles(h, float(eps), ctypes.byref(neg), ctypes.byref(pos)))
    return int(neg.value), int(pos.value)


def hb_set_tiling(h: int, by: int, zc: int) -> None:
    _check(load().hb_set_tiling(h, int(by), int(zc)))


def hb_autotune(h: int, trial_steps: int = 5):
    by, zc = _I(), _I()
    _check(load().hb_autotune(h, int(trial_steps), ctypes.byref(by), ctypes.byref(zc)))
    return by.value, zc.value


def hb_destroy(h: int) -> None:
    if h:
        _GRIDS.pop(("s", h), None)
        _check(load().hb_destroy(h))


def hb_default_tiling(cfg: hb_config):
    """(by, zc) that hb_create would choose for a single solve of cfg."""
    by, zc = _I(), _I()
    _check(load().hb_default_tiling(ctypes.byref(cfg), ctypes.byref(by), ctypes.byref(zc)))
    return by.value, zc.value


def hb_footprint(cfg: hb_config) -> int:
    return int(load().hb_footprint(ctypes.byref(cfg)))


def hb_last_error() -> str:
    return load().hb_last_error().decode()


# ---- device allocator -------------------------------------------------------------

HB_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
HB_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
# Every installed pair stays alive: the library hands each block back through
# the allocator that made it, also after another one is installed.
_HOOKS: list = []


def hb_set_allocator(alloc=None, release=None) -> None:
    """Install Python callables ``alloc(nbytes, stream) -> device address``
    (an int; 0 or an exception means failure) and ``release(ptr, nbytes)`` as
    the library's device allocator; both None restores hipMalloc/hipFree."""
    if (alloc is None) != (release is None):
        raise ValueError("hb_set_allocator: give both functions or neither")
    if alloc is None:
        _check(load().hb_set_allocator(None, None, None))
        return

    def _alloc(_ctx, nbytes, stream):
        try:
            return int(alloc(int(nbytes), stream or 0)) or None
        except Exception:
            return None

    def _release(_ctx, ptr, nbytes):
        try:
            release(int(ptr), int(nbytes))
        except Exception:
            pass

    pair = (HB_ALLOC_FN(_alloc), HB_FREE_FN(_release))
    _HOOKS.append(pair)
    _check(load().hb_set_allocator(ctypes.cast(pair[0], _P), ctypes.cast(pair[1], _P), None))


def use_torch_allocator() -> None:
    """Let torch's caching allocator own the library's device memory (blocks
    are tied to the stream the library allocates them for)."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)

    def release(ptr, _nbytes):
        torch.cuda.caching_allocator_delete(ptr)

    hb_set_allocator(alloc, release)


# ---- batched form -----------------------------------------------------------------

def hb_batch_create(cfgs: Sequence[hb_config], stream=None) -> int:
    arr = (hb_config * len(cfgs))(*cfgs)
    b = _P()
    _check(load().hb_batch_create(len(cfgs), arr, stream, ctypes.byref(b)))
    for i, c in enumerate(cfgs):
        _GRIDS[("b", b.value, i)] = _points(c)
    return b.value


def hb_batch_set_initial(b: int, i: int, phi0, phi1=None) -> None:
    if phi0 is None:
        raise ValueError("hb_batch_set_initial: phi0 is required")
    p0, p1, m, d, _keep = _pair(("b", b, int(i)), phi0, phi1, "hb_batch_set_initial")
    _check(load().hb_batch_set_initial(b, int(i), p0, p1, m, d))


def hb_batch_step(b: int, nsteps: int) -> None:
    _check(load().hb_batch_step(b, int(nsteps)))


def hb_batch_read(b: int, i: int, phi=None, phi_t=None) -> None:
    if phi is None and phi_t is None:
        return
    p0, p1, m, d, _keep = _pair(("b", b, int(i)), phi, phi_t, "hb_batch_read")
    _check(load().hb_batch_read(b, int(i), p0, p1, m, d))


def hb_batch_sync(b: int) -> None:
    _check(load().hb_batch_sync(b))


def hb_batch_set_tiling(b: int, by: int, zc: int) -> None:
    _check(load().hb_batch_set_tiling(b, int(by), int(zc)))


def hb_batch_autotune(b: int, trial_steps: int = 5):
    """Tune each precision group of the batch; returns ((by, zc) FP64,
    (by, zc) FP32c), (-1, -1) for a precision the batch does not hold."""
    by, zc = (_I * 2)(), (_I * 2)()
    _check(load().hb_batch_autotune(b, int(trial_steps), by, zc))
    return (by[0], zc[0]), (by[1], zc[1])


def _forget(kind, handle):
    for k in [k for k in _GRIDS if k[0] == kind and k[1] == handle]:
        del _GRIDS[k]


def hb_batch_destroy(b: int) -> None:
    if b:
        _forget("b", b)
        _check(load().hb_batch_destroy(b))


# ---- served form ----------------------------------------------------------------------

def hb_pool_create(hbm_budget: int, max_slots: int, stream=None) -> int:
    p = _P()
    _check(load().hb_pool_create(int(hbm_budget), int(max_slots), stream, ctypes.byref(p)))
    return p.value


def hb_pool_admit(p: int, cfg: hb_config, phi0, phi1, steps: int) -> Optional[int]:
    """Returns the slot, or None when the pool is busy (HB_E_BUSY)."""
    if phi0 is None:
        raise ValueError("hb_pool_admit: phi0 is required")
    key = ("p", p, None)
    _GRIDS[key] = _points(cfg)
    try:
        p0, p1, m, d, _keep = _pair(key, phi0, phi1, "hb_pool_admit")
    finally:
        del _GRIDS[key]
    slot = _I()
    rc = load().hb_pool_admit(p, ctypes.byref(cfg), p0, p1, m, d, int(steps), ctypes.byref(slot))
    if rc == HB_E_BUSY:
        return None
    _check(rc)
    _GRIDS[("p", p, slot.value)] = _points(cfg)
    return slot.value


def hb_pool_advance(p: int, k: int) -> None:
    _check(load().hb_pool_advance(p, int(k)))


def hb_pool_poll(p: int, cap: int = 1024):
    buf = (_I * cap)()
    n = _I()
    _check(load().hb_pool_poll(p, buf, cap, ctypes.byref(n)))
    return list(buf[: n.value])


def hb_pool_check(p: int, cap: int = 1024):
    """Slots whose state holds NaN/Inf; they stop stepping (see include/hb.h)."""
    buf = (_I * cap)()
    n = _I()
    _check(load().hb_pool_check(p, buf, cap, ctypes.byref(n)))
    return list(buf[: n.value])


def hb_pool_stats(p: int):
    a = _I()
    u = ctypes.c_size_t()
    _check(load().hb_pool_stats(p, ctypes.byref(a), ctypes.byref(u)))
    return a.value, u.value


def hb_pool_read(p: int, slot: int, phi=None, phi_t=None) -> None:
    if phi is None and phi_t is None:
        return
    p0, p1, m, d, _keep = _pair(("p", p, int(slot)), phi, phi_t, "hb_pool_read")
    _check(load().hb_pool_read(p, int(slot), p0, p1, m, d))


def hb_pool_release(p: int, slot: int) -> None:
    _check(load().hb_pool_release(p, int(slot)))
    _GRIDS.pop(("p", p, int(slot)), None)


def hb_pool_destroy(p: int) -> None:
    if p:
        _forget("p", p)
        _check(load().hb_pool_destroy(p))


# ---- convenience (marshalling only) -------------------------------------------------

def solve_host(w, nsteps: Optional[int] = None, precision: int = HB_F64, flags: int = 0,
               tiling=None):
    """Run a synth_inputs.Workload through the GPU path with host arrays in and out."""
    p0, p1 = w.initial()
    h = hb_create(config_from_workload(w, precision, flags))
    try:
        if tiling is not None:
            hb_set_tiling(h, *tiling)
        hb_set_initial(h, p0, p1)
        hb_step(h, w.steps if nsteps is None else nsteps)
        phi = np.empty_like(p0)
        psi = np.empty_like(p0)
        hb_read(h, phi, psi)
    finally:
        hb_destroy(h)
    return phi, psi


def hb_probe_bandwidth(kind: int, bytes_per_array: int, iters: int = 20) -> float:
    g = ctypes.c_double()
    _check(load().hb_probe_bandwidth(int(kind), int(bytes_per_array), int(iters), ctypes.byref(g)))
    return g.value


# ---- batched radial solves ------------------------------------------------------------

def make_radial_config(m: int, dr: float, mu2: float, lam: float, dt: float, steps: int,
                       t0: float = 0.0, inv_L2: float = 1.0, flags: int = 0) -> hb_radial_config:
    c = hb_radial_config()
    c.m, c.flags, c.dr, c.mu2, c.lambda_ = int(m), int(flags), float(dr), float(mu2), float(lam)
    c.inv_L2, c.t0, c.dt, c.steps = float(inv_L2), float(t0), float(dt), int(steps)
    return c


def hb_radial_solve(cfgs, phi, psi, stream=None) -> None:
    """Advance the solves in place; phi/psi: FP64 NumPy arrays (host) or torch
    tensors (device) holding the solves back to back."""
    arr = (hb_radial_config * len(cfgs))(*cfgs)
    if phi is None or psi is None:
        raise ValueError("hb_radial_solve: phi and psi are required")
    total = sum(int(c.m) for c in cfgs)
    for x in (phi, psi):
        n = x.size if isinstance(x, np.ndarray) else x.numel()
        if n != total:
            raise ValueError(f"hb_radial_solve: array has {n} values, the solves have {total} nodes")
    p0, m0, d0, _k0 = _arr(phi)
    p1, m1, d1, _k1 = _arr(psi)
    if d0 != HB_DTYPE_F64 or d1 != HB_DTYPE_F64 or m0 != m1:
        raise TypeError("phi and psi must be FP64 and in the same memory")
    _check(load().hb_radial_solve(len(cfgs), arr, p0, p1, m0, stream))


def hb_radial_solve_noalloc(cfgs, phi, psi, stream=None) -> None:
    """hb_radial_solve without device allocation: phi/psi must be FP64 torch
    device tensors holding the solves back to back; the library keeps the
    descriptors and c(t) tables in its fixed device scratch."""
    arr = (hb_radial_config * len(cfgs))(*cfgs)
    total = sum(int(c.m) for c in cfgs)
    for x in (phi, psi):
        if isinstance(x, np.ndarray) or x is None:
            raise TypeError("hb_radial_solve_noalloc: phi and psi must be device tensors")
        if x.numel() != total:
            raise ValueError(f"hb_radial_solve_noalloc: array has {x.numel()} values, the solves have "
                             f"{total} nodes")
    p0, m0, d0, _k0 = _arr(phi)
    p1, m1, d1, _k1 = _arr(psi)
    if d0 != HB_DTYPE_F64 or d1 != HB_DTYPE_F64 or m0 != HB_DEVICE or m1 != HB_DEVICE:
        raise TypeError("hb_radial_solve_noalloc: phi and psi must be FP64 device tensors")
    _check(load().hb_radial_solve_noalloc(len(cfgs), arr, p0, p1, stream))
