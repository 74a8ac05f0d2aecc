"""CPU oracle for the Higgs-boson RK4 solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg import
this package.  The GPU library and its Python binding never import it, and it
imports nothing from them.

* ``solve``      -- textbook classical RK4 + fourth-order 13-point Laplacian,
                    FP64, plain C (``hb_oracle.c``), OpenMP over z-planes with
                    no reductions (thread-count invariant).  Section 2.1.
* ``rhs``        -- one evaluation of f(t, v), eq. (rhs).
* ``laplacian``  -- the 13-point operator on a caller-filled padded array.
* ``radial``     -- the radial 1-D form of section 2.2 (NumPy).
* ``diagnostics``-- plain FP64 definitions of the observables.
* ``components`` -- bubble count: connected sets of each sign (section 1),
                    breadth-first flood fill in plain C.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_ZERO = 0
BC_PERIODIC = 1
ORDER_TEXTBOOK = 0
ORDER_PAPER_REUSE = 1
ORDER_AXES_REVERSED = 2

CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-std=c11", "-Wall"]


def build(verbose: bool = False) -> str:
    """Compile ``hb_oracle.c`` into ``liboracle.so`` with gcc."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib: Optional[ctypes.CDLL] = None


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i, d, ll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    lib.hbo_laplacian.argtypes = [i, i, i, d, d, d, dp, dp]
    lib.hbo_laplacian.restype = i
    lib.hbo_rhs.argtypes = [i, i, i, d, d, d, d, d, d, d, i, dp, dp, dp, dp]
    lib.hbo_rhs.restype = i
    lib.hbo_solve.argtypes = [i, i, i, d, d, d, d, d, d, d, d, ll, ll, i, i, dp, dp]
    lib.hbo_solve.restype = i
    lib.hbo_set_threads.argtypes = [i]
    lib.hbo_set_threads.restype = None
    lib.hbo_get_threads.argtypes = []
    lib.hbo_get_threads.restype = i
    lib.hbo_components.argtypes = [i, i, i, i, dp, d, ctypes.POINTER(ll), ctypes.POINTER(ll)]
    lib.hbo_components.restype = i
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> None:
    _load().hbo_set_threads(int(n))


def get_threads() -> int:
    return int(_load().hbo_get_threads())


def laplacian(upad: np.ndarray, h: Sequence[float]) -> np.ndarray:
    """13-point Laplacian of a padded array of shape (nz+4, ny+4, nx+4) whose
    2-cell halo the caller has filled.  Returns the (nz, ny, nx) interior."""
    upad = np.ascontiguousarray(upad, np.float64)
    nz, ny, nx = (s - 4 for s in upad.shape)
    out = np.empty((nz, ny, nx), np.float64)
    rc = _load().hbo_laplacian(nx, ny, nz, h[0], h[1], h[2], _ptr(upad), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"hbo_laplacian failed: {rc}")
    return out


def rhs(phi: np.ndarray, psi: np.ndarray, h: Sequence[float], mu2: float, lam: float,
        inv_L2: float, t: float, bc: int = BC_ZERO) -> Tuple[np.ndarray, np.ndarray]:
    """f(t, (phi, psi)) of eq. (rhs) on interior arrays."""
    phi = np.ascontiguousarray(phi, np.float64)
    psi = np.ascontiguousarray(psi, np.float64)
    nz, ny, nx = phi.shape
    f1 = np.empty_like(phi)
    f2 = np.empty_like(phi)
    rc = _load().hbo_rhs(nx, ny, nz, h[0], h[1], h[2], mu2, lam, inv_L2, t, bc,
                         _ptr(phi), _ptr(psi), _ptr(f1), _ptr(f2))
    if rc != 0:
        raise RuntimeError(f"hbo_rhs failed: {rc}")
    return f1, f2


def solve(phi0: np.ndarray, psi0: np.ndarray, h: Sequence[float], mu2: float, lam: float,
          dt: float, nsteps: int, t0: float = 0.0, inv_L2: float = 1.0, step0: int = 0,
          bc: int = BC_ZERO, order: int = ORDER_TEXTBOOK) -> Tuple[np.ndarray, np.ndarray]:
    """Advance (phi, psi) by ``nsteps`` classical RK4 steps; t_n = t0 + n dt for
    n = step0 .. step0 + nsteps - 1.  Returns new arrays."""
    phi = np.array(phi0, dtype=np.float64, order="C", copy=True)
    psi = np.array(psi0, dtype=np.float64, order="C", copy=True)
    nz, ny, nx = phi.shape
    if psi.shape != phi.shape:
        raise ValueError("phi and psi shapes differ")
    rc = _load().hbo_solve(nx, ny, nz, h[0], h[1], h[2], mu2, lam, inv_L2, t0, dt,
                           int(step0), int(nsteps), bc, order, _ptr(phi), _ptr(psi))
    if rc != 0:
        raise RuntimeError(f"hbo_solve failed: {rc}")
    return phi, psi


def components(phi: np.ndarray, eps: float = 0.0, bc: int = BC_ZERO) -> Tuple[int, int]:
    """Number of maximal face-connected node sets of {phi < -eps} and of
    {phi > eps} (the paper's bubbles, section 1; ``bc`` = BC_PERIODIC wraps
    neighbours).  Returns (negative sets, positive sets)."""
    phi = np.ascontiguousarray(phi, np.float64)
    if phi.ndim != 3:
        raise ValueError("phi must be a 3-D [nz][ny][nx] array")
    nz, ny, nx = phi.shape
    nneg, npos = ctypes.c_longlong(0), ctypes.c_longlong(0)
    rc = _load().hbo_components(nx, ny, nz, bc, _ptr(phi), float(eps), ctypes.byref(nneg),
                                ctypes.byref(npos))
    if rc != 0:
        raise RuntimeError(f"hbo_components failed: {rc}")
    return int(nneg.value), int(npos.value)


def solve_workload(w, nsteps: Optional[int] = None, order: int = ORDER_TEXTBOOK):
    """Run a ``synth_inputs.Workload`` through the oracle."""
    p0, p1 = w.initial()
    return solve(p0, p1, w.h, w.mu2, w.lam, w.dt, w.steps if nsteps is None else nsteps,
                 t0=w.t0, inv_L2=w.inv_L2, order=order)


def rel_maxnorm(phi, psi, phi_ref, psi_ref) -> float:
    """State-vector relative max norm
    max(|dphi|_inf, |dpsi|_inf) / max(|phi_ref|_inf, |psi_ref|_inf)."""
    num = max(float(np.max(np.abs(phi - phi_ref))), float(np.max(np.abs(psi - psi_ref))))
    den = max(float(np.max(np.abs(phi_ref))), float(np.max(np.abs(psi_ref))))
    return num / den if den > 0 else num
