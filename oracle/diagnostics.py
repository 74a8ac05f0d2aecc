"""Plain FP64 definitions of the solver's observables -- TEST INFRASTRUCTURE ONLY.

* integral   h^3 sum phi               (the paper's integral of phi, Example 2)
* linf       max |phi|, max |psi|
* l2         sqrt(h^3 sum phi^2), same for psi
* lap_max    P(t) = c(t) max |Lap_h phi|   (the paper's P(t), Example 4)
* energy     E_h = h^3 sum [ psi^2/2 + c phi (-Lap_h phi)/2 - mu2 phi^2/2 + lambda phi^4/4 ]
             (the discrete energy of the damped equation; with the zero halo
             -Lap_h is symmetric positive semi-definite and c' = -2c, so the
             semi-discrete E_h does not increase)
* nonfinite  number of NaN/Inf entries in phi and psi
* negative   number of interior points with phi < 0 (sign-change probe for
             the paper's bubbles, section 1)
* bubbles    the paper's bubbles (section 1: maximal connected sets where the
             solution changes sign): the number of face-connected node sets
             of {phi < -eps} and of {phi > eps} (``components`` in the C part)
"""
from __future__ import annotations

import math

import numpy as np

from . import BC_PERIODIC, BC_ZERO, components, laplacian


def _lap_zero_halo(phi: np.ndarray, h) -> np.ndarray:
    pad = np.zeros(tuple(s + 4 for s in phi.shape), np.float64)
    pad[2:-2, 2:-2, 2:-2] = phi
    return laplacian(pad, h)


def diagnostics(phi: np.ndarray, psi: np.ndarray, h, mu2: float, lam: float, t: float,
                inv_L2: float = 1.0) -> dict:
    vol = h[0] * h[1] * h[2]
    c = math.exp(-2.0 * t) * inv_L2
    lap = _lap_zero_halo(phi, h)
    e = vol * np.sum(0.5 * psi * psi + 0.5 * c * phi * (-lap) - 0.5 * mu2 * phi * phi
                     + 0.25 * lam * phi ** 4)
    return {
        "integral": float(vol * np.sum(phi)),
        "linf_phi": float(np.max(np.abs(phi))),
        "linf_psi": float(np.max(np.abs(psi))),
        "l2_phi": float(math.sqrt(vol * np.sum(phi * phi))),
        "l2_psi": float(math.sqrt(vol * np.sum(psi * psi))),
        "lap_max": float(c * np.max(np.abs(lap))),
        "energy": float(e),
        "nonfinite": int(np.count_nonzero(~np.isfinite(phi)) + np.count_nonzero(~np.isfinite(psi))),
        "negative": int(np.count_nonzero(phi < 0)),
    }


def bubbles(phi: np.ndarray, eps: float = 0.0, periodic: bool = False) -> tuple:
    """(negative sets, positive sets): face-connected components of
    {phi < -eps} and {phi > eps} over the interior nodes."""
    return components(phi, eps, BC_PERIODIC if periodic else BC_ZERO)
