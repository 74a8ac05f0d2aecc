"""The window construction used for single-node oracle values on planes too
large for the oracle: on a plane the oracle runs whole, every sampled node's
window value equals the whole-grid value bitwise (domain of dependence of the
RK4 step with the 13-point stencil), including nodes at corners and edges."""
import numpy as np

import oracle
import synth_inputs as si
from windows import sample_nodes, window_solve


def test_window_values_equal_whole_grid(oracle_mod):
    w = si.wide_plane(300, 200, steps=2)
    p0 = w.phi0()
    P, S = oracle.solve(p0, np.zeros_like(p0), w.h, w.mu2, w.lam, w.dt, 2)
    for (y, x) in sample_nodes(200, 300):
        p, s = window_solve(oracle, p0, y, x, w, 2)
        assert p == P[0, y, x] and s == S[0, y, x], (y, x)


def test_dependence_radius_is_four_cells_per_step(oracle_mod):
    """Two steps: a window of radius 8 = 4 x 2 already gives the whole-grid
    value bitwise, radius 7 does not (so the check above is not vacuous, and
    the reach of one step is exactly 4 cells per axis)."""
    w = si.wide_plane(300, 200, steps=2)
    p0 = w.phi0()
    P, S = oracle.solve(p0, np.zeros_like(p0), w.h, w.mu2, w.lam, w.dt, 2)
    y, x = 100, 150
    p, s = window_solve(oracle, p0, y, x, w, 2, R=8)
    assert p == P[0, y, x] and s == S[0, y, x]
    p, s = window_solve(oracle, p0, y, x, w, 2, R=7)
    assert (p, s) != (P[0, y, x], S[0, y, x])
