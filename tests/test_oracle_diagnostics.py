"""Pins of the oracle's observables (oracle/diagnostics.py) against
mathematics, not against the formulas they are written with.

* integral and L2 norms: closed-form Gaussian integrals (the midpoint rule on
  a Gaussian well inside the box is exact to rounding), exact sums of
  constant fields; anisotropic spacings, so a cell volume built from the
  wrong axes fails;
* linf: the largest node value of a centred Gaussian on the cell-centred
  grid, in closed form;
* lap_max (the paper's P(t) of Example 4, section 3): a single spike, whose
  Laplacian is largest at the spike with the centre weight 5/2 sum 1/h_d^2 of
  the section 2.1 stencil; random fields against the Kronecker-sum assembly
  of the operator; the time factor e^{-2t}/L^2 of eq. (higgs-boson-rescalled);
* energy: phi = 0 with constant psi, a spike with psi = 0, and random fields
  against the Kronecker assembly;
* negative and nonfinite: planted counts (signed zeros, NaN, +-Inf);
* bubbles (section 1: maximal connected sets where the solution changes
  sign): constructed fields with known counts and random fields against
  scipy.ndimage.label with face connectivity.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle.diagnostics import bubbles, diagnostics

from test_oracle_stencil import kron_laplacian


def cell_nodes(n, lo, hi):
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h, h


def grid(n, lo, hi):
    (x, hx), (y, hy), (z, hz) = (cell_nodes(n[d], lo[d], hi[d]) for d in range(3))
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z, (hx, hy, hz)


# anisotropic box and spacings: hx = 0.25, hy = 0.375, hz = 0.175
N3 = (64, 48, 80)
LO = (-8.0, -9.0, -7.0)
HI = (8.0, 9.0, 7.0)


def test_gaussian_integral_l2_linf_closed_forms():
    X, Y, Z, h = grid(N3, LO, HI)
    A, w = 0.7, 0.9
    B, v = -1.3, 0.8
    r2 = X * X + Y * Y + Z * Z
    phi = A * np.exp(-r2 / (2 * w * w))
    psi = B * np.exp(-r2 / (2 * v * v))
    d = diagnostics(phi, psi, h, mu2=2.0, lam=1.0, t=0.0)
    # int A e^{-r^2/(2w^2)} dx = A (2 pi w^2)^{3/2};  int phi^2 = A^2 (pi w^2)^{3/2}
    assert d["integral"] == pytest.approx(A * (2 * math.pi * w * w) ** 1.5, rel=1e-10)
    assert d["l2_phi"] == pytest.approx(abs(A) * (math.pi * w * w) ** 0.75, rel=1e-10)
    assert d["l2_psi"] == pytest.approx(abs(B) * (math.pi * v * v) ** 0.75, rel=1e-10)
    # the nodes nearest the centre sit at (+-hx/2, +-hy/2, +-hz/2)
    rmin2 = sum((hd / 2) ** 2 for hd in h)
    assert d["linf_phi"] == pytest.approx(A * math.exp(-rmin2 / (2 * w * w)), rel=1e-14)
    assert d["linf_psi"] == pytest.approx(abs(B) * math.exp(-rmin2 / (2 * v * v)), rel=1e-14)
    assert d["nonfinite"] == 0 and d["negative"] == 0


def test_constant_fields_exact_sums():
    n = (5, 7, 3)
    h = (0.5, 0.25, 2.0)
    a, b = -0.75, 1.5
    phi = np.full((n[2], n[1], n[0]), a)
    psi = np.full_like(phi, b)
    vol_box = n[0] * h[0] * n[1] * h[1] * n[2] * h[2]   # 26.25, exact in binary
    d = diagnostics(phi, psi, h, mu2=0.0, lam=0.0, t=0.0)
    assert d["integral"] == pytest.approx(a * vol_box, rel=1e-14)
    assert d["l2_phi"] == pytest.approx(abs(a) * math.sqrt(vol_box), rel=1e-14)
    assert d["l2_psi"] == pytest.approx(abs(b) * math.sqrt(vol_box), rel=1e-14)
    assert d["linf_phi"] == abs(a) and d["linf_psi"] == abs(b)
    assert d["negative"] == phi.size


def spike_field(n, at, s):
    phi = np.zeros((n[2], n[1], n[0]))
    phi[at[2], at[1], at[0]] = s
    return phi


@pytest.mark.parametrize("t,L", [(0.0, 1.0), (0.3, 5.0), (1.7, 2.0)])
def test_lap_max_of_a_spike(t, L):
    # Lap_h of a spike s: the centre weight -5/2 sum_d 1/h_d^2 times s at the
    # spike, 4/3 / h_d^2 and -1/12 / h_d^2 times s at its neighbours, zero
    # elsewhere; the largest magnitude is at the spike
    n = (9, 8, 10)
    h = (0.5, 0.3, 0.7)
    s = -1.25
    phi = spike_field(n, (4, 3, 5), s)
    d = diagnostics(phi, np.zeros_like(phi), h, mu2=1.0, lam=1.0, t=t, inv_L2=1.0 / L ** 2)
    coeff = math.e ** (-2 * t) / L ** 2   # e^{-2t}/L^2 of eq. (higgs-boson-rescalled)
    want = coeff * 2.5 * sum(1 / hd ** 2 for hd in h) * abs(s)
    assert d["lap_max"] == pytest.approx(want, rel=1e-14)


def test_lap_max_and_energy_against_kronecker_operator():
    rng = np.random.default_rng(11)
    n = (7, 6, 5)
    h = (0.4, 0.55, 0.3)
    phi = rng.normal(size=(n[2], n[1], n[0]))
    psi = rng.normal(size=phi.shape)
    mu2, lam, t, L = 1.7, 0.9, 0.45, 3.0
    coeff = math.e ** (-2 * t) / L ** 2
    K = kron_laplacian(n, h)
    lap = K @ phi.ravel()
    vol = h[0] * h[1] * h[2]
    f = phi.ravel()
    energy = vol * (0.5 * psi.ravel() @ psi.ravel() + 0.5 * coeff * (f @ (-lap))
                    - 0.5 * mu2 * (f @ f) + 0.25 * lam * np.sum(f ** 4))
    d = diagnostics(phi, psi, h, mu2=mu2, lam=lam, t=t, inv_L2=1.0 / L ** 2)
    assert d["lap_max"] == pytest.approx(coeff * np.max(np.abs(lap)), rel=1e-13)
    assert d["energy"] == pytest.approx(energy, rel=1e-12)


def test_energy_closed_forms():
    n = (6, 5, 7)
    h = (0.5, 0.25, 0.4)
    vol = h[0] * h[1] * h[2]
    # phi = 0, psi = b: kinetic part only, b^2/2 over the box
    b = 0.6
    zero = np.zeros((n[2], n[1], n[0]))
    d = diagnostics(zero, np.full_like(zero, b), h, mu2=3.0, lam=2.0, t=0.2, inv_L2=0.5)
    assert d["energy"] == pytest.approx(0.5 * b * b * vol * zero.size, rel=1e-14)
    # a spike s with psi = 0: one node of c s (5/2 sum 1/h^2) s / 2 - mu2 s^2/2 + lambda s^4/4
    s, mu2, lam, t, L = 0.8, 3.0, 2.0, 0.2, 5.0
    phi = spike_field(n, (2, 2, 3), s)
    coeff = math.e ** (-2 * t) / L ** 2
    want = vol * (0.5 * coeff * s * s * 2.5 * sum(1 / hd ** 2 for hd in h)
                  - 0.5 * mu2 * s * s + 0.25 * lam * s ** 4)
    d = diagnostics(phi, zero, h, mu2=mu2, lam=lam, t=t, inv_L2=1 / L ** 2)
    assert d["energy"] == pytest.approx(want, rel=1e-14)


def test_negative_and_nonfinite_planted_counts():
    rng = np.random.default_rng(3)
    shape = (6, 7, 8)
    phi = np.abs(rng.normal(size=shape)) + 0.1
    idx = rng.choice(phi.size, size=37, replace=False)
    phi.ravel()[idx] *= -1.0
    # signed zeros are not negative values
    free = np.setdiff1d(np.arange(phi.size), idx)[:5]
    phi.ravel()[free[:3]] = -0.0
    phi.ravel()[free[3:]] = 0.0
    psi = rng.normal(size=shape)
    d = diagnostics(phi, psi, (0.3, 0.3, 0.3), mu2=1.0, lam=1.0, t=0.0)
    assert d["negative"] == 37
    assert d["nonfinite"] == 0
    # NaN and +-Inf in both fields
    phi2, psi2 = phi.copy(), psi.copy()
    phi2.ravel()[[0, 5]] = [np.nan, np.inf]
    psi2.ravel()[[1, 2, 3]] = [-np.inf, np.nan, np.nan]
    with np.errstate(invalid="ignore"):  # the other sums turn NaN, as they should
        d = diagnostics(phi2, psi2, (0.3, 0.3, 0.3), mu2=1.0, lam=1.0, t=0.0)
    assert d["nonfinite"] == 5


# ---- bubbles ---------------------------------------------------------------------

def ball_field(n, centres, radius, inside=-1.0, outside=1.0):
    z, y, x = np.meshgrid(*(np.arange(k, dtype=float) for k in (n[2], n[1], n[0])), indexing="ij")
    phi = np.full((n[2], n[1], n[0]), outside)
    for c in centres:
        phi[(x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= radius ** 2] = inside
    return phi, (x, y, z)


def test_bubbles_separate_and_touching_balls():
    n = (40, 30, 30)
    phi, _ = ball_field(n, [(10, 15, 15), (28, 15, 15)], 5.0)
    assert bubbles(phi) == (2, 1)
    phi, _ = ball_field(n, [(12, 15, 15), (21, 15, 15)], 5.0)   # overlap: one set
    assert bubbles(phi) == (1, 1)


def test_bubbles_face_connectivity_only():
    phi = np.ones((5, 5, 5))
    phi[2, 2, 2] = -1.0
    phi[2, 3, 3] = -1.0        # shares an edge only
    phi[3, 3, 3] = -1.0        # face neighbour of the second
    assert bubbles(phi) == (2, 1)
    phi[1, 1, 1] = -1.0        # a corner neighbour of the first: separate
    assert bubbles(phi) == (3, 1)


def test_bubbles_shell_and_nested_ball():
    n = (33, 33, 33)
    _, (x, y, z) = ball_field(n, [], 1.0)
    r = np.sqrt((x - 16) ** 2 + (y - 16) ** 2 + (z - 16) ** 2)
    phi = np.where((r >= 9) & (r <= 12), -1.0, 1.0)
    assert bubbles(phi) == (1, 2)          # the inside is cut off from the outside
    phi[r <= 4] = -1.0
    assert bubbles(phi) == (2, 2)


def test_bubbles_torus_is_one_set():
    n = (48, 48, 24)
    _, (x, y, z) = ball_field(n, [], 1.0)
    rho = np.sqrt((x - 24) ** 2 + (y - 24) ** 2)
    phi = np.where((rho - 12) ** 2 + (z - 12) ** 2 <= 16.0, -1.0, 1.0)
    # a solid torus: one negative set; the hole connects to the outside
    assert bubbles(phi) == (1, 1)


def test_bubbles_periodic_wrap():
    phi = np.ones((6, 7, 20))
    phi[:, :, :2] = -1.0
    phi[:, :, 18:] = -1.0
    assert bubbles(phi) == (2, 1)
    assert bubbles(phi, periodic=True) == (1, 1)


def test_bubbles_threshold():
    phi = np.full((8, 8, 8), 1.0)
    phi[1, 1, 1] = -0.5
    phi[6, 6, 6] = -1e-9      # dust below the threshold
    phi[3, 3, 3] = 0.0
    assert bubbles(phi) == (2, 1)
    assert bubbles(phi, eps=1e-6) == (1, 1)
    # a node at exactly eps belongs to neither class
    assert bubbles(phi, eps=0.5) == (0, 1)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_bubbles_random_fields_against_scipy_label(seed):
    rng = np.random.default_rng(seed)
    shape = (9, 12, 15)
    phi = rng.normal(size=shape)
    eps = [0.0, 0.3, 0.0, 1.0][seed]
    face = ndimage.generate_binary_structure(3, 1)
    _, nneg = ndimage.label(phi < -eps, structure=face)
    _, npos = ndimage.label(phi > eps, structure=face)
    assert bubbles(phi, eps) == (nneg, npos)
