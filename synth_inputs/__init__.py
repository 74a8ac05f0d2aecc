"""Seeded synthetic inputs for the Higgs-boson RK4 solver.

This module is the only code shared by the GPU path's tests/benchmarks and the
CPU oracle.  It holds grid coordinates, initial-data generators and the
workload descriptions; it contains none of the method's arithmetic (no
Laplacian, no right-hand side, no Runge-Kutta step).

Grid convention (cell-centred): an axis with ``n`` points on ``[lo, hi]`` has
spacing ``h = (hi - lo) / n`` and nodes ``x_i = lo + (i + 1/2) h`` for
``i = 0 .. n-1``.  Arrays are C-ordered ``[z][y][x]`` (x fastest), interior
points only.

Initial data follow the paper's section 3 (bump function, eq. (bump)) and the
synthetic workloads derived from it:

* ``gaussian_sum``   -- a seeded sum of isotropic Gaussian bumps
  ``A exp(-|x-c|^2 / (2 w^2))``; per bump the draws are, in this order,
  ``A ~ U(-1, 1)``, ``w ~ U(0.5, 2)``, ``c ~ U(-8, 8)^3`` from
  ``numpy.random.default_rng(seed)`` (PCG64).
* ``cinf_bump``      -- ``A exp(1 - 1/(1 - r^2/R^2))`` inside ``r < R``, else 0
  (maximum ``A`` at the centre).
* ``paper_bump``     -- the paper's section 3 bump
  ``exp(1/R^2 - 1/(R^2 - |x-C|^2))`` inside ``|x-C| < R``, else 0.
* ``example6_data``  -- the non-radial, sign-changing data of section 3,
  Example 6, on the unit box.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "axis_nodes", "grid_mesh", "gaussian_sum", "cinf_bump", "paper_bump",
    "radial_gaussian", "Workload", "config1", "config2", "config3",
    "batch_config", "serving_trace", "ServeRequest", "small_case", "wide_plane",
    "slab_config", "example6_data", "example7_config",
]


def axis_nodes(n: int, lo: float, hi: float) -> np.ndarray:
    """Cell-centred nodes ``lo + (i + 1/2) h``, ``h = (hi - lo)/n``."""
    h = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * h


def grid_mesh(n: Sequence[int], lo: Sequence[float], hi: Sequence[float]):
    """Return broadcastable coordinate arrays ``(Z, Y, X)`` of shapes
    ``(nz,1,1)``, ``(1,ny,1)``, ``(1,1,nx)``; ``n``/``lo``/``hi`` are (x, y, z)."""
    x = axis_nodes(n[0], lo[0], hi[0])
    y = axis_nodes(n[1], lo[1], hi[1])
    z = axis_nodes(n[2], lo[2], hi[2])
    return z[:, None, None], y[None, :, None], x[None, None, :]


def gaussian_sum(n: Sequence[int], lo: Sequence[float], hi: Sequence[float],
                 seed: int, nbumps: int = 8, amp=(-1.0, 1.0), width=(0.5, 2.0),
                 centre=(-8.0, 8.0)) -> np.ndarray:
    """Seeded sum of ``nbumps`` isotropic Gaussians on the cell-centred grid.

    Each bump is evaluated as the product of three 1-D factors (the Gaussian
    is separable), which keeps 256^3+ grids cheap on the host.
    """
    rng = np.random.default_rng(seed)
    Z, Y, X = grid_mesh(n, lo, hi)
    out = np.zeros((n[2], n[1], n[0]), dtype=np.float64)
    for _ in range(nbumps):
        a = rng.uniform(*amp)
        w = rng.uniform(*width)
        c = rng.uniform(centre[0], centre[1], size=3)
        s = 1.0 / (2.0 * w * w)
        ex = np.exp(-s * (X - c[0]) ** 2)
        ey = np.exp(-s * (Y - c[1]) ** 2)
        ez = np.exp(-s * (Z - c[2]) ** 2)
        out += a * (ez * ey * ex)
    return out


def _radius2(n, lo, hi, centre):
    Z, Y, X = grid_mesh(n, lo, hi)
    return (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2


def radial_gaussian(n, lo, hi, amp: float = 0.5, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """``amp * exp(-|x - centre|^2 / 2)``."""
    r2 = _radius2(n, lo, hi, centre)
    return amp * np.exp(-0.5 * r2)


def cinf_bump(n, lo, hi, amp: float, R: float, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Scale-invariant C-infinity bump ``A exp(1 - 1/(1 - r^2/R^2))`` for
    ``r < R``, else 0."""
    r2 = _radius2(n, lo, hi, centre)
    q = r2 / (R * R)
    out = np.zeros(q.shape, dtype=np.float64)
    m = q < 1.0
    out[m] = amp * np.exp(1.0 - 1.0 / (1.0 - q[m]))
    return out


def paper_bump(n, lo, hi, C, R: float) -> np.ndarray:
    """The paper's bump (section 3, eq. (bump)):
    ``exp(1/R^2 - 1/(R^2 - |x - C|^2))`` for ``|x - C| < R``, else 0."""
    r2 = _radius2(n, lo, hi, C)
    out = np.zeros(r2.shape, dtype=np.float64)
    m = r2 < R * R
    out[m] = np.exp(1.0 / (R * R) - 1.0 / (R * R - r2[m]))
    return out


def example6_data(n: int, C, C2, R: float, a0: float, a1: float):
    """Section 3, Example 6, on the unit box with ``n`` cells per axis:
    ``phi0 = a0 B(x; C, R) B(x; C2, R) sin(2 pi x_1)`` (``x_1`` the first
    coordinate) and ``phi1 = a1 B(x; C, R)``."""
    nn, lo, hi = (n, n, n), (0.0,) * 3, (1.0,) * 3
    _, _, X = grid_mesh(nn, lo, hi)
    b1 = paper_bump(nn, lo, hi, C, R)
    b2 = paper_bump(nn, lo, hi, C2, R)
    return a0 * b1 * b2 * np.sin(2.0 * np.pi * X), a1 * b1


def example7_config(n: int = 500, steps: int = 200):
    """Section 3, Example 7 at the section's default grid (``n``^3 cells on the
    unit box, dt = 1e-4, L = 5): ``phi0 = B(x; (0.4,)*3, 0.2) + B(x; (0.6,)*3,
    0.2)``, ``phi1 = -5 phi0``, ``lambda = mu^2 = 0.1`` -- the paper's longest
    run (to t = 50)."""
    nn, lo, hi = (n, n, n), (0.0,) * 3, (1.0,) * 3

    cache = {}

    def bumps():  # evaluated once per workload (500^3 takes seconds)
        if "b" not in cache:
            cache["b"] = paper_bump(nn, lo, hi, (0.4,) * 3, 0.2) + paper_bump(nn, lo, hi, (0.6,) * 3, 0.2)
        return cache["b"]

    def phi0():
        return bumps().copy()

    def phi1():
        return -5.0 * bumps()

    return Workload(f"paper_example7_{n}", nn, lo, hi, mu2=0.1, lam=0.1, dt=1e-4, steps=steps,
                    inv_L2=1.0 / 25.0, phi0=phi0, phi1=phi1)


@dataclasses.dataclass
class Workload:
    """One solve: grid, coefficients, time stepping and initial data."""
    name: str
    n: Tuple[int, int, int]          # points per axis (x, y, z)
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    mu2: float
    lam: float
    dt: float
    steps: int
    t0: float = 0.0
    inv_L2: float = 1.0
    phi0: Optional[Callable[[], np.ndarray]] = None
    phi1: Optional[Callable[[], np.ndarray]] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(3))

    @property
    def points(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def initial(self) -> Tuple[np.ndarray, np.ndarray]:
        shape = (self.n[2], self.n[1], self.n[0])
        p0 = self.phi0() if self.phi0 else np.zeros(shape)
        p1 = self.phi1() if self.phi1 else np.zeros(shape)
        return np.ascontiguousarray(p0, np.float64), np.ascontiguousarray(p1, np.float64)


def _zeros(n):
    return lambda: np.zeros((n[2], n[1], n[0]), dtype=np.float64)


def config1() -> Workload:
    """32^3 on [-8,8]^3, mu=1, lambda=1, phi0 = 0.5 exp(-|x|^2/2), phi1 = 0,
    dt = 0.01, 100 steps."""
    n, lo, hi = (32, 32, 32), (-8.0,) * 3, (8.0,) * 3
    return Workload("cube32_gauss", n, lo, hi, mu2=1.0, lam=1.0, dt=0.01, steps=100,
                    phi0=lambda: radial_gaussian(n, lo, hi, 0.5), phi1=_zeros(n))


def config2(n: int = 256, steps: int = 2000, seed: int = 0) -> Workload:
    """256^3 on [-16,16]^3, mu = sqrt(2) (mu^2 = 2 exactly), lambda = 1,
    phi0 = 8 seeded Gaussians, phi1 = 0, dt = 0.005, 2000 steps."""
    nn, lo, hi = (n, n, n), (-16.0,) * 3, (16.0,) * 3
    return Workload(f"cube{n}_gauss8", nn, lo, hi, mu2=2.0, lam=1.0, dt=0.005, steps=steps,
                    phi0=lambda: gaussian_sum(nn, lo, hi, seed), phi1=_zeros(nn),
                    meta={"seed": seed})


def config3(n: int = 512, steps: int = 1000, L: float = 32.0) -> Workload:
    """512^3 on [-32,32]^3 (h = 0.125), mu^2 = 2, lambda = 1, dt = 0.005,
    phi0 = 0.8 exp(1 - 1/(1 - r^2/100)) for r < 10, phi1 = 0, 1000 steps."""
    nn, lo, hi = (n, n, n), (-L,) * 3, (L,) * 3
    return Workload(f"cube{n}_cinfbump", nn, lo, hi, mu2=2.0, lam=1.0, dt=0.005, steps=steps,
                    phi0=lambda: cinf_bump(nn, lo, hi, 0.8, 10.0), phi1=_zeros(nn))


def slab_config(steps: int = 200) -> Workload:
    """One GPU's share of the 512^3 workload under an 8-way z-slab split: the
    middle slab z in [-4, 4] (64 planes) of config3's box and initial data,
    512 x 512 x 64 points."""
    w = config3()
    n, lo, hi = (512, 512, 64), (w.lo[0], w.lo[1], -4.0), (w.hi[0], w.hi[1], 4.0)
    return Workload("slab512x512x64", n, lo, hi, mu2=w.mu2, lam=w.lam, dt=w.dt, steps=steps,
                    phi0=lambda: cinf_bump(n, lo, hi, 0.8, 10.0), phi1=_zeros(n))


def small_case(nx: int, ny: int, nz: int, seed: int = 7, steps: int = 10, dt: float = 0.005,
               L: float = 16.0, mu2: float = 2.0, lam: float = 1.0, nbumps: int = 8,
               t0: float = 0.0, inv_L2: float = 1.0, with_velocity: bool = True) -> Workload:
    """A small (possibly non-cubic, ragged) seeded case with the h = 0.125-like
    resolution of the large configurations scaled to the box.  ``phi1`` is a
    second seeded Gaussian sum when ``with_velocity``."""
    n = (nx, ny, nz)
    hx = 2 * L / max(n)
    lo = tuple(-0.5 * hx * k for k in n)
    hi = tuple(0.5 * hx * k for k in n)
    span = 0.5 * hx * min(n)
    cen = (-0.6 * span, 0.6 * span)
    wid = (0.25 * span / 4, span / 4)
    p0 = lambda: gaussian_sum(n, lo, hi, seed, nbumps, centre=cen, width=wid)
    p1 = (lambda: 0.5 * gaussian_sum(n, lo, hi, seed + 1000, nbumps, centre=cen, width=wid)) \
        if with_velocity else _zeros(n)
    return Workload(f"small{nx}x{ny}x{nz}_s{seed}", n, lo, hi, mu2=mu2, lam=lam, dt=dt,
                    steps=steps, t0=t0, inv_L2=inv_L2, phi0=p0, phi1=p1, meta={"seed": seed})


def batch_config(count: int = 64, steps: int = 500, nmin: int = 64, nmax: int = 192,
                 batch_seed: int = 4, dt: float = 0.005) -> List[Workload]:
    """64 independent solves: cubic N ~ U{64..192}, box [-16,16]^3,
    mu ~ U[0.5,2] (mu^2 = mu*mu), lambda ~ U[0.5,4], 8-Gaussian phi0 with data
    seed 1+i, phi1 = 0, dt = 0.005.  N, mu, lambda are drawn in that order per
    solve from ``default_rng(batch_seed)``."""
    rng = np.random.default_rng(batch_seed)
    out = []
    for i in range(count):
        N = int(rng.integers(nmin, nmax + 1))
        mu = float(rng.uniform(0.5, 2.0))
        lam = float(rng.uniform(0.5, 4.0))
        nn, lo, hi = (N, N, N), (-16.0,) * 3, (16.0,) * 3
        out.append(Workload(f"batch{i}_n{N}", nn, lo, hi, mu2=mu * mu, lam=lam, dt=dt,
                            steps=steps,
                            phi0=(lambda nn=nn, lo=lo, hi=hi, s=1 + i: gaussian_sum(nn, lo, hi, s)),
                            phi1=_zeros(nn), meta={"seed": 1 + i, "mu": mu}))
    return out


@dataclasses.dataclass
class ServeRequest:
    index: int
    arrival: float          # seconds since the start of the trace
    workload: Workload
    precision: str          # "f64" or "f32c"


def serving_trace(count: int = 300, rate: float = 50.0, seed: int = 12345,
                  sizes=(48, 96, 128, 192, 256, 384), steps=(200, 2000),
                  precisions=("f64", "f32c")) -> List[ServeRequest]:
    """Poisson arrivals at ``rate``/s.  Per request j, drawn in this order from
    ``default_rng(seed)``: the exponential inter-arrival gap, N from ``sizes``,
    the step count ~ U{steps}, and the precision (50/50).  mu^2 = 2, lambda = 1,
    box [-16,16]^3, dt = 0.005, phi0 = 8 Gaussians with data seed 10000+j."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(count):
        t += float(rng.exponential(1.0 / rate))
        N = int(sizes[int(rng.integers(0, len(sizes)))])
        st = int(rng.integers(steps[0], steps[1] + 1))
        prec = precisions[int(rng.integers(0, len(precisions)))]
        nn, lo, hi = (N, N, N), (-16.0,) * 3, (16.0,) * 3
        w = Workload(f"req{j}_n{N}", nn, lo, hi, mu2=2.0, lam=1.0, dt=0.005, steps=st,
                     phi0=(lambda nn=nn, lo=lo, hi=hi, s=10000 + j: gaussian_sum(nn, lo, hi, s)),
                     phi1=_zeros(nn), meta={"seed": 10000 + j})
        out.append(ServeRequest(j, t, w, prec))
    return out


def radial_sweep(count: int = 4096, m: int = 1000, dr: float = 5e-4, R: float = 0.3,
                 seed: int = 7):
    """A parameter sweep of radial solves (the section 2.2 form of Example 3):
    phi0 = A b(r), phi1 = a A b(r) with b the paper's bump of radius R on the
    nodes r_i = i dr; per solve A ~ U[0.5, 2], a ~ U[-8, 0], mu2 ~ U[1, 9],
    lambda ~ U[0.5, 4], drawn in that order from ``default_rng(seed)``.
    Returns (phi0, phi1, params): the solves back to back (count * m values
    each) and a list of (mu2, lambda) pairs."""
    rng = np.random.default_rng(seed)
    r = np.arange(m) * dr
    b = np.zeros(m)
    inside = r < R
    b[inside] = np.exp(1.0 / (R * R) - 1.0 / (R * R - r[inside] ** 2))
    phi0 = np.empty(count * m)
    phi1 = np.empty(count * m)
    params = []
    for i in range(count):
        A = rng.uniform(0.5, 2.0)
        a = rng.uniform(-8.0, 0.0)
        mu2 = rng.uniform(1.0, 9.0)
        lam = rng.uniform(0.5, 4.0)
        phi0[i * m:(i + 1) * m] = A * b
        phi1[i * m:(i + 1) * m] = a * A * b
        params.append((mu2, lam))
    return phi0, phi1, params


def wide_plane(nx: int, ny: int, seed: int = 3, h: float = 0.125, steps: int = 2) -> Workload:
    """One x-y plane of nx x ny points at spacing h (the box centred on 0,
    one cell thick), mu^2 = 2, lambda = 1, dt = 0.005, phi1 = 0, and
    phi0 = f1(x) g1(y) + f2(x) g2(y), each factor a sum of two sinusoids
    a sin(k s + p) with a ~ U(0.2, 0.6), k ~ U(0.5, 3), p ~ U(0, 2 pi), drawn
    in that order per sinusoid (f1, g1, f2, g2) from ``default_rng(seed)``.
    Separable, so planes of 10^8-10^9 points cost little to build."""
    rng = np.random.default_rng(seed)
    n = (nx, ny, 1)
    lo = (-nx * h / 2, -ny * h / 2, -h / 2)
    hi = (nx * h / 2, ny * h / 2, h / 2)
    x = axis_nodes(nx, lo[0], hi[0])
    y = axis_nodes(ny, lo[1], hi[1])

    def factor(s):
        out = np.zeros_like(s)
        for _ in range(2):
            a, k, p = rng.uniform(0.2, 0.6), rng.uniform(0.5, 3.0), rng.uniform(0.0, 2 * np.pi)
            out += a * np.sin(k * s + p)
        return out

    f1, g1, f2, g2 = factor(x), factor(y), factor(x), factor(y)

    def phi0():
        out = np.empty((1, ny, nx))
        for y0 in range(0, ny, 2048):
            y1 = min(ny, y0 + 2048)
            out[0, y0:y1] = g1[y0:y1, None] * f1[None, :] + g2[y0:y1, None] * f2[None, :]
        return out

    return Workload(f"plane{nx}x{ny}", n, lo, hi, mu2=2.0, lam=1.0, dt=0.005, steps=steps,
                    phi0=phi0, phi1=_zeros(n))

