"""Pins of the oracle's time integration (section 2.1 classical RK4) against
closed forms and an independent ODE solver.

* Spatially constant data, periodic halo, lambda = 0: the Laplacian vanishes
  and classical RK4 on the linear system v' = A v, A = [[0, 1], [mu2, -3]], is
  multiplication by the stability polynomial R(dt A) = sum_{j<=4} (dt A)^j / j!.
* Spatially constant data, lambda != 0: the reduction to the damped unforced
  Duffing equation (section 3, eq. (duffing)); fourth-order convergence
  against a DOP853 reference, and the paper's printed equilibria.
* One Fourier mode on a periodic grid, lambda = 0, time-dependent c(t): the
  exact semi-discrete solution is e^{-3t/2} [A J_nu(k e^{-t}) + B Y_nu(k e^{-t})]
  with nu = sqrt(mu2 + 9/4) (the paper's M for n = 3) and the discrete symbol
  k^2 = inv_L2 sum_d (1 - cos th_d)(7 - cos th_d) / (3 h_d^2); RK4 must converge
  to it at fourth order (this pins the stage times of c(t)).
* A tiny zero-halo grid, nonlinear and time dependent: fourth-order
  convergence to a DOP853 solve of the Kronecker-assembled system.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import jv, jvp, yv, yvp

import oracle
from test_oracle_stencil import kron_laplacian


def const_fields(shape, a0, a1):
    return np.full(shape, a0, np.float64), np.full(shape, a1, np.float64)


def test_linear_constant_data_is_rk4_stability_polynomial(oracle_mod):
    mu2, dt, nsteps = 2.0, 0.05, 40
    a0, a1 = 0.7, -0.3
    phi, psi = const_fields((2, 3, 2), a0, a1)
    # h large so the rounding residue of the constant's Laplacian is negligible
    p, q = oracle_mod.solve(phi, psi, (10.0, 10.0, 10.0), mu2, 0.0, dt, nsteps,
                            bc=oracle.BC_PERIODIC)
    A = np.array([[0.0, 1.0], [mu2, -3.0]])
    Z = dt * A
    R = np.eye(2) + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    y = np.linalg.matrix_power(R, nsteps) @ np.array([a0, a1])
    assert np.max(np.abs(p - y[0])) < 1e-13 * abs(y[0])
    assert np.max(np.abs(q - y[1])) < 1e-13 * max(abs(y[1]), abs(y[0]))


def duffing_reference(mu2, lam, a0, a1, T):
    sol = solve_ivp(lambda t, y: [y[1], -3 * y[1] + mu2 * y[0] - lam * y[0] ** 3], (0, T),
                    [a0, a1], method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[:, -1]


def test_duffing_reduction_fourth_order(oracle_mod):
    mu2, lam, a0, a1, T = 9.0, 2.0, 0.3, 1.0, 1.0
    ref = duffing_reference(mu2, lam, a0, a1, T)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        phi, psi = const_fields((1, 1, 1), a0, a1)
        p, q = oracle_mod.solve(phi, psi, (1.0, 1.0, 1.0), mu2, lam, dt, int(round(T / dt)),
                                bc=oracle.BC_PERIODIC)
        errs.append(max(abs(p[0, 0, 0] - ref[0]), abs(q[0, 0, 0] - ref[1])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def bessel_mode(T, a0, a1, kappa2, mu2):
    nu = math.sqrt(mu2 + 9.0 / 4.0)
    s0 = math.sqrt(kappa2)
    # a(0) = A J(s0) + B Y(s0);  a'(0) = -3/2 a(0) - s0 (A J'(s0) + B Y'(s0))
    M = np.array([[jv(nu, s0), yv(nu, s0)], [-s0 * jvp(nu, s0), -s0 * yvp(nu, s0)]])
    A, B = np.linalg.solve(M, [a0, a1 + 1.5 * a0])
    s = s0 * math.exp(-T)
    return math.exp(-1.5 * T) * (A * jv(nu, s) + B * yv(nu, s))


@pytest.mark.parametrize("inv_L2", [1.0, 1.0 / 25.0])
def test_fourier_mode_matches_bessel_closed_form(oracle_mod, inv_L2):
    n = (16, 8, 4)
    h = (0.25, 0.3, 0.5)
    m = (1, 2, 1)
    mu2, T, a1 = 2.0, 1.0, 0.4
    k = [2 * math.pi * m[d] / (n[d] * h[d]) for d in range(3)]
    th = [k[d] * h[d] for d in range(3)]
    kappa2 = inv_L2 * sum((1 - math.cos(t)) * (7 - math.cos(t)) / (3 * h[d] ** 2)
                          for d, t in enumerate(th))
    x = (np.arange(n[0]) + 0.5) * h[0]
    y = (np.arange(n[1]) + 0.5) * h[1]
    z = (np.arange(n[2]) + 0.5) * h[2]
    mode = np.cos(k[0] * x[None, None, :] + k[1] * y[None, :, None] + k[2] * z[:, None, None])
    want = bessel_mode(T, 1.0, a1, kappa2, mu2)
    errs = []
    for dt in (0.04, 0.02, 0.01):
        p, _ = oracle_mod.solve(mode, a1 * mode, h, mu2, 0.0, dt, int(round(T / dt)),
                                inv_L2=inv_L2, bc=oracle.BC_PERIODIC)
        errs.append(np.max(np.abs(p - want * mode)))
    # observed order log2(e(dt)/e(dt/2)) must be about 4 (a wrong stage time
    # of c(t) drops it to 2 or less)
    orders = [math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])]
    assert all(3.6 < o < 4.9 for o in orders), (errs, orders)
    # a wrong stencil symbol would leave an O(1e-2) gap here
    assert errs[-1] < 1e-6 * abs(want)


def test_kronecker_system_fourth_order_nonlinear(oracle_mod):
    rng = np.random.default_rng(11)
    n = (5, 4, 3)
    h = (0.5, 0.45, 0.6)
    mu2, lam, invL2, t0, T = 2.0, 1.0, 1.0, 0.2, 0.5
    phi0 = 0.8 * rng.normal(size=(n[2], n[1], n[0]))
    psi0 = 0.5 * rng.normal(size=(n[2], n[1], n[0]))
    L = kron_laplacian(n, h)
    N = phi0.size

    def f(t, y):
        p, q = y[:N], y[N:]
        return np.concatenate([q, -3 * q + invL2 * math.exp(-2 * t) * (L @ p) + mu2 * p - lam * p ** 3])

    ref = solve_ivp(f, (t0, t0 + T), np.concatenate([phi0.ravel(), psi0.ravel()]),
                    method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    errs = []
    for dt in (0.02, 0.01, 0.005):
        p, q = oracle_mod.solve(phi0, psi0, h, mu2, lam, dt, int(round(T / dt)), t0=t0, inv_L2=invL2)
        errs.append(np.max(np.abs(np.concatenate([p.ravel(), q.ravel()]) - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_step_offset_equals_t0_shift(oracle_mod):
    # t_n = t0 + n dt: starting at step0 = k is the same as t0 + k dt (checkpoint restart)
    rng = np.random.default_rng(3)
    phi0 = rng.normal(size=(4, 5, 6))
    psi0 = rng.normal(size=(4, 5, 6))
    a = oracle_mod.solve(phi0, psi0, (0.5, 0.5, 0.5), 2.0, 1.0, 0.01, 7, t0=0.1, step0=3)
    b = oracle_mod.solve(phi0, psi0, (0.5, 0.5, 0.5), 2.0, 1.0, 0.01, 7, t0=0.1 + 3 * 0.01)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-13, atol=1e-13)
