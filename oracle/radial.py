"""Radial 1-D form of the Higgs boson equation -- TEST INFRASTRUCTURE ONLY.

Section 2.2, eq. (radial):
    phi_tt - c(t) (2/r phi_r + phi_rr) + 3 phi_t = mu2 phi - lambda phi^3,
    r in (0, R), phi_r(0, t) = 0, phi(R, t) = 0,   c(t) = inv_L2 exp(-2t).

Discretisation (section 2.2 and the section 2.1 stencil):
* nodes r_i = i dr, i = 0 .. m-1; r_m = R carries the zero boundary value;
* phi_rr: the fourth-order central second difference of section 2.1;
* phi_r:  the fourth-order central first difference
  (u[i-2] - 8u[i-1] + 8u[i+1] - u[i+2]) / (12 dr)  -- the paper does not print
  its first-derivative stencil; this is the matching fourth-order choice;
* even symmetry at r = 0: u[-1] = u[1], u[-2] = u[2] (the symmetric ghost of
  section 2.2), and zeros beyond r = R;
* r = 0: L'Hospital, phi_r / r -> phi_rr(0), so the radial operator there is
  3 phi_rr(0) with phi_rr(0) = (-5/2 u0 + 8/3 u1 - 1/6 u2) / dr^2 (section 2.2);
* time: classical RK4 as in section 2.1; c(t) at each stage time is the C
  library's FP64 exp (``math.exp``), the values the 3-D oracle uses.
"""
from __future__ import annotations

import math

import numpy as np


def _padded(u: np.ndarray) -> np.ndarray:
    """u[0..m-1] -> [u2, u1, u0 .. u_{m-1}, 0, 0]: even ghosts at r = 0, zero at/after R."""
    m = u.shape[0]
    p = np.zeros(m + 4, dtype=np.float64)
    p[2:m + 2] = u
    p[1] = u[1] if m > 1 else 0.0
    p[0] = u[2] if m > 2 else 0.0
    return p


def radial_operator(u: np.ndarray, dr: float) -> np.ndarray:
    """(2/r) u_r + u_rr on the nodes r_i = i dr, with 3 u_rr at r = 0."""
    m = u.shape[0]
    p = _padded(u)
    um2, um1, u0, up1, up2 = p[0:m], p[1:m + 1], p[2:m + 2], p[3:m + 3], p[4:m + 4]
    urr = (-1.0 / 12.0 * um2 + 4.0 / 3.0 * um1 - 5.0 / 2.0 * u0 + 4.0 / 3.0 * up1
           - 1.0 / 12.0 * up2) / (dr * dr)
    ur = (um2 - 8.0 * um1 + 8.0 * up1 - up2) / (12.0 * dr)
    out = np.empty(m, dtype=np.float64)
    r = np.arange(1, m, dtype=np.float64) * dr
    out[1:] = 2.0 / r * ur[1:] + urr[1:]
    out[0] = 3.0 * urr[0]
    return out


def radial_rhs(t: float, phi: np.ndarray, psi: np.ndarray, dr: float, mu2: float, lam: float,
               inv_L2: float):
    c = math.exp(-2.0 * t) * inv_L2
    return psi, -3.0 * psi + c * radial_operator(phi, dr) + mu2 * phi - lam * phi * phi * phi


def radial_solve(phi0: np.ndarray, psi0: np.ndarray, dr: float, mu2: float, lam: float,
                 dt: float, nsteps: int, t0: float = 0.0, inv_L2: float = 1.0,
                 callback=None):
    """Classical RK4 of the radial system.  ``callback(n, t, phi, psi)`` is
    called after each step when given (for time series such as sign changes)."""
    y1 = np.array(phi0, dtype=np.float64, copy=True)
    y2 = np.array(psi0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        t = t0 + n * dt
        k1a, k1b = radial_rhs(t, y1, y2, dr, mu2, lam, inv_L2)
        k2a, k2b = radial_rhs(t + dt / 2.0, y1 + dt / 2.0 * k1a, y2 + dt / 2.0 * k1b, dr, mu2, lam, inv_L2)
        k3a, k3b = radial_rhs(t + dt / 2.0, y1 + dt / 2.0 * k2a, y2 + dt / 2.0 * k2b, dr, mu2, lam, inv_L2)
        k4a, k4b = radial_rhs(t + dt, y1 + dt * k3a, y2 + dt * k3b, dr, mu2, lam, inv_L2)
        y1 = y1 + dt / 6.0 * (k1a + 2.0 * k2a + 2.0 * k3a + k4a)
        y2 = y2 + dt / 6.0 * (k1b + 2.0 * k2b + 2.0 * k3b + k4b)
        if callback is not None:
            callback(n + 1, t0 + (n + 1) * dt, y1, y2)
    return y1, y2
