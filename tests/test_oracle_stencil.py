"""Pins of the oracle's spatial operator (section 2.1 fourth-order central
difference; section 2.2 radial form) against mathematics, not against itself.

* The 5-point symmetric second-difference weights are re-derived here from the
  moment (Taylor) conditions, not copied, and the oracle must be exact on every
  polynomial of per-axis degree <= 5.
* Degree 6 pins the truncation constant: for x^6 the stencil returns
  30 x^4 - 8 h^4 exactly (error -h^4/90 f^(6)).
* A Kronecker-sum assembly of the 3-D operator on a tiny grid (independent
  index bookkeeping and boundary handling) must reproduce the oracle's f(t, v).
* The radial operator must be exact on even polynomials r^2, r^4.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.radial import radial_operator


def derived_weights():
    """Weights w_{-2..2} of the symmetric 5-point second difference, from the
    moment conditions sum_k w_k k^p = p! [p == 2], p = 0..4."""
    ks = np.arange(-2, 3, dtype=np.float64)
    A = np.vstack([ks ** p for p in range(5)])
    b = np.array([0.0, 0.0, 2.0, 0.0, 0.0])
    return np.linalg.solve(A, b)


def padded_coords(n, h):
    # centred cell-centred coordinates of padded nodes i = -2 .. n+1
    i = np.arange(-2, n + 2, dtype=np.float64)
    return (i + 0.5 - n / 2.0) * h


def test_derived_weights_match_paper_print():
    # the paper prints (-1/12, 4/3, -5/2, 4/3, -1/12)/dx^2 (section 2.1);
    # the moment conditions give the same numbers
    w = derived_weights()
    np.testing.assert_allclose(w, [-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12], rtol=1e-12)


@pytest.mark.parametrize("seed", [1, 2])
def test_laplacian_exact_on_per_axis_degree5(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = (9, 7, 8)
    h = (0.3, 0.25, 0.35)
    x = padded_coords(n[0], h[0])[None, None, :]
    y = padded_coords(n[1], h[1])[None, :, None]
    z = padded_coords(n[2], h[2])[:, None, None]
    u = np.zeros((n[2] + 4, n[1] + 4, n[0] + 4))
    lap = np.zeros_like(u)
    for a in range(6):
        for b in range(6):
            for c in range(6):
                co = rng.normal() / math.factorial(a + b + c)
                u += co * x ** a * y ** b * z ** c
                if a >= 2:
                    lap += co * a * (a - 1) * x ** (a - 2) * y ** b * z ** c
                if b >= 2:
                    lap += co * b * (b - 1) * x ** a * y ** (b - 2) * z ** c
                if c >= 2:
                    lap += co * c * (c - 1) * x ** a * y ** b * z ** (c - 2)
    got = oracle_mod.laplacian(u, h)
    want = lap[2:-2, 2:-2, 2:-2]
    scale = 16.0 / min(h) ** 2 * np.max(np.abs(u)) * 1e-13
    assert np.max(np.abs(got - want)) < scale


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laplacian_degree6_truncation_constant(oracle_mod, axis):
    n = (8, 9, 10)
    h = (0.2, 0.3, 0.4)
    coords = [padded_coords(n[d], h[d]) for d in range(3)]
    shape = (n[2] + 4, n[1] + 4, n[0] + 4)
    q = np.broadcast_to(
        [coords[0][None, None, :], coords[1][None, :, None], coords[2][:, None, None]][axis], shape)
    u = np.ascontiguousarray(q ** 6)
    got = oracle_mod.laplacian(u, h)
    want = 30.0 * q[2:-2, 2:-2, 2:-2] ** 4 - 8.0 * h[axis] ** 4
    assert np.max(np.abs(got - want)) < 1e-9


def kron_laplacian(n, h):
    """3-D operator as a Kronecker sum of 1-D banded matrices with the 2-cell
    zero halo (rows truncated), C-order [z][y][x] flattening."""
    w = derived_weights()
    mats = []
    for d in range(3):
        m = n[d]
        diags = [np.full(m - abs(k), w[k + 2]) for k in range(-2, 3) if m - abs(k) > 0]
        offs = [k for k in range(-2, 3) if m - abs(k) > 0]
        mats.append(sp.diags(diags, offs, shape=(m, m), format="csr") / h[d] ** 2)
    Ix, Iy, Iz = (sp.identity(n[d], format="csr") for d in range(3))
    return (sp.kron(Iz, sp.kron(Iy, mats[0])) + sp.kron(Iz, sp.kron(mats[1], Ix))
            + sp.kron(mats[2], sp.kron(Iy, Ix))).tocsr()


def test_rhs_matches_kronecker_assembly(oracle_mod):
    rng = np.random.default_rng(5)
    n = (5, 4, 3)
    h = (0.5, 0.4, 0.7)
    phi = rng.normal(size=(n[2], n[1], n[0]))
    psi = rng.normal(size=(n[2], n[1], n[0]))
    mu2, lam, invL2, t = 2.0, 1.5, 0.3, 0.37
    L = kron_laplacian(n, h)
    c = math.exp(-2 * t) * invL2
    lap = (L @ phi.ravel()).reshape(phi.shape)
    f1, f2 = oracle_mod.rhs(phi, psi, h, mu2, lam, invL2, t)
    np.testing.assert_array_equal(f1, psi)
    want = -3 * psi + c * lap + mu2 * phi - lam * phi ** 3
    assert np.max(np.abs(f2 - want)) < 1e-12 * np.max(np.abs(want))


def test_laplacian_zero_halo_matches_kronecker(oracle_mod):
    rng = np.random.default_rng(6)
    n = (7, 6, 5)
    h = (0.25, 0.5, 0.3)
    u = rng.normal(size=(n[2], n[1], n[0]))
    pad = np.zeros((n[2] + 4, n[1] + 4, n[0] + 4))
    pad[2:-2, 2:-2, 2:-2] = u
    got = oracle_mod.laplacian(pad, h)
    want = (kron_laplacian(n, h) @ u.ravel()).reshape(u.shape)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_radial_operator_exact_on_even_polynomials():
    dr = 0.05
    m = 60
    r = np.arange(m) * dr
    # r^2 -> 6 and r^4 -> 20 r^2 (3-D radial Laplacian), away from r = R
    for p, lap in ((2, lambda r: 6.0 + 0 * r), (4, lambda r: 20.0 * r ** 2)):
        got = radial_operator(r ** p, dr)
        np.testing.assert_allclose(got[: m - 3], lap(r)[: m - 3], rtol=1e-10, atol=1e-9)


def test_radial_operator_origin_uses_symmetric_ghost():
    # at r = 0 the section 2.2 formula (-5/2 u0 + 8/3 u1 - 1/6 u2)/dr^2 times 3
    dr = 0.1
    u = np.array([1.0, 0.7, 0.2, 0.05, 0.0, 0.0])
    got = radial_operator(u, dr)[0]
    assert got == pytest.approx(3 * (-2.5 * 1.0 + 8 / 3 * 0.7 - 1 / 6 * 0.2) / dr ** 2, rel=1e-14)
