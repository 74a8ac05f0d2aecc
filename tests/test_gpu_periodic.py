"""Periodic boundaries (HB_BC_PERIODIC, whole-step scheme) against the
oracle's periodic mode: every node, on grids with axes shorter than the
stencil's reach (the wrap then goes round more than once), ragged tiles and
both precisions; constant data follows the damped Duffing ODE at every node
alike; the diagnostics use the wrapped Laplacian."""
import math

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu
TOL64, TOL32C = 1e-12, 1e-5


def periodic_case(n, seed, steps, mu2=2.0, lam=1.0, inv_L2=1.0, t0=0.0):
    """Seeded data that do not vanish at the faces (uniform in [-1, 1]), on a
    box with h = 0.25 per axis, dt at 40% of the RK4 stability limit."""
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    p0 = rng.uniform(-1.0, 1.0, shape)
    p1 = 0.5 * rng.uniform(-1.0, 1.0, shape)
    h = 0.25
    lo = tuple(0.0 for _ in n)
    hi = tuple(h * k for k in n)
    rho = 3 * 16.0 / (3.0 * h * h)
    dt = 0.4 * 2.0 * math.sqrt(2.0) / math.sqrt(inv_L2 * math.exp(-2.0 * t0) * rho)
    return si.Workload(f"periodic{n}", n, lo, hi, mu2=mu2, lam=lam, dt=dt, steps=steps, t0=t0,
                       inv_L2=inv_L2, phi0=lambda: p0, phi1=lambda: p1)


def gpu_solve(hb, w, prec=0, tiling=None):
    return hb.solve_host(w, precision=prec, flags=hb.HB_BC_PERIODIC, tiling=tiling)


def oracle_solve(w):
    p0, p1 = w.initial()
    return oracle.solve(p0, p1, w.h, w.mu2, w.lam, w.dt, w.steps, t0=w.t0, inv_L2=w.inv_L2,
                        bc=oracle.BC_PERIODIC)


@pytest.mark.parametrize("n,tiling", [
    ((70, 21, 13), None),        # ragged tiles in x and y
    ((130, 25, 19), (11, 6)),    # 64 x 11 tiles, z-marches of 6
    ((64, 16, 9), (16, 4)),      # 60 x 12 tiles
    ((40, 35, 10), (20, 3)),     # 32 x 16 tiles, ragged in x and y
    ((5, 3, 7), None),           # axes shorter than the reach of one step
    ((1, 2, 6), (8, 0)),         # one- and two-cell axes: every neighbour wraps onto itself
    ((33, 1, 1), None),
])
def test_periodic_vs_oracle(hb, oracle_mod, n, tiling):
    w = periodic_case(n, seed=sum(n), steps=7)
    ref = oracle_solve(w)
    g = gpu_solve(hb, w, 0, tiling)
    err = oracle.rel_maxnorm(*g, *ref)
    g32 = gpu_solve(hb, w, 1, tiling)
    err32 = oracle.rel_maxnorm(*g32, *ref)
    print(f"periodic {n} tiling {tiling}: FP64 {err:.3e}, FP32c {err32:.3e}")
    assert err <= TOL64 and err32 <= TOL32C


def test_periodic_differs_from_zero_halo(hb):
    """The flag changes the boundary (the data reach the faces)."""
    w = periodic_case((40, 20, 10), seed=4, steps=3)
    per = gpu_solve(hb, w)
    zero = hb.solve_host(w)
    assert np.max(np.abs(per[0] - zero[0])) > 1e-3


def test_constant_data_follow_the_duffing_ode(hb, oracle_mod):
    """Spatially constant data on a periodic grid: every node follows the
    damped Duffing ODE phi'' + 3 phi' = mu^2 phi - lambda phi^3 (the
    Laplacian of a constant vanishes), identically at every node, as the
    oracle's one-node periodic solve does."""
    n = (37, 23, 11)
    shape = (n[2], n[1], n[0])
    p0, p1 = np.full(shape, 0.3), np.full(shape, -0.2)
    w = si.Workload("const", n, (0.0,) * 3, tuple(0.25 * k for k in n), mu2=9.0, lam=2.0,
                    dt=0.01, steps=400, inv_L2=1 / 25, phi0=lambda: p0, phi1=lambda: p1)
    phi, psi = gpu_solve(hb, w)
    assert np.ptp(phi) == 0.0 and np.ptp(psi) == 0.0
    r = oracle.solve(p0[:1, :1, :1], p1[:1, :1, :1], (0.25,) * 3, 9.0, 2.0, 0.01, 400,
                     inv_L2=1 / 25, bc=oracle.BC_PERIODIC)
    err = max(abs(phi.flat[0] - r[0].flat[0]), abs(psi.flat[0] - r[1].flat[0]))
    print(f"constant data, 400 steps: phi {phi.flat[0]:.12f}, |GPU - oracle| {err:.3e}")
    assert err <= 1e-12 * max(abs(r[0].flat[0]), abs(r[1].flat[0]))


def test_periodic_diagnostics(hb, oracle_mod):
    from oracle import laplacian
    from oracle.diagnostics import diagnostics
    w = periodic_case((40, 21, 9), seed=11, steps=4)
    p0, p1 = w.initial()
    h = hb.hb_create(hb.config_from_workload(w, flags=hb.HB_BC_PERIODIC))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, w.steps)
        d = hb.hb_diagnostics(h)
        phi, psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, phi, psi)
    finally:
        hb.hb_destroy(h)
    t = w.t0 + w.steps * w.dt
    ref = diagnostics(phi, psi, w.h, w.mu2, w.lam, t, w.inv_L2)  # zero-halo terms
    lap = laplacian(np.pad(phi, 2, mode="wrap"), w.h)             # the wrapped Laplacian
    c = math.exp(-2.0 * t) * w.inv_L2
    vol = w.h[0] * w.h[1] * w.h[2]
    energy = vol * np.sum(0.5 * psi * psi + 0.5 * c * phi * (-lap) - 0.5 * w.mu2 * phi * phi
                          + 0.25 * w.lam * phi ** 4)
    assert d["lap_max"] == pytest.approx(c * np.max(np.abs(lap)), rel=1e-12)
    assert d["energy"] == pytest.approx(energy, rel=1e-11)
    assert d["integral"] == pytest.approx(ref["integral"], rel=1e-12, abs=1e-12)
    assert d["linf_phi"] == ref["linf_phi"]


def test_periodic_needs_the_whole_step_scheme(hb):
    w = periodic_case((16, 16, 16), seed=1, steps=1)
    for flags in (hb.HB_PAIRWISE, hb.HB_STAGEWISE):
        with pytest.raises(hb.HBError) as e:
            hb.hb_create(hb.config_from_workload(w, flags=hb.HB_BC_PERIODIC | flags))
        assert e.value.code == hb.HB_E_ARG


def test_batch_mixes_periodic_and_zero_halo(hb):
    """Solves of one batch keep their own boundary (a descriptor field): each
    equals the same solve alone, bitwise."""
    ws = [periodic_case((30, 20, 12), seed=2, steps=5), periodic_case((21, 9, 14), seed=3, steps=5)]
    flags = [hb.HB_BC_PERIODIC, 0]
    b = hb.hb_batch_create([hb.config_from_workload(w, 0, f) for w, f in zip(ws, flags)])
    try:
        for i, w in enumerate(ws):
            hb.hb_batch_set_initial(b, i, *w.initial())
        hb.hb_batch_step(b, 5)
        for i, (w, f) in enumerate(zip(ws, flags)):
            phi = np.empty(w.n[::-1])
            hb.hb_batch_read(b, i, phi, None)
            alone = hb.solve_host(w, flags=f)
            np.testing.assert_array_equal(phi, alone[0])
    finally:
        hb.hb_batch_destroy(b)
