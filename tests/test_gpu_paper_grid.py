"""The paper's default grid (section 3: 500^3 cells of the unit box,
dt = 1e-4, L = 5) with Example 7's data, the benchmark's `paper_grid` leg:
both precisions in the launch configuration the benchmark times (the
library's default region shape for this grid), 20 steps, then sampled nodes
against the oracle run on a window around each node (tests/windows.py: a
window reaching 4 cells per step beyond the node gives the node its
whole-grid value).  Nodes: the two bump centres and the box centre, where
the solution is largest, points on the bumps' rims, the corners and edges
(next to the zero halo), and seeded random nodes."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from windows import window_solve3

pytestmark = pytest.mark.gpu

STEPS = 20


@pytest.fixture(scope="module")
def example7_500():
    w = si.example7_config(500, STEPS)
    p0, p1 = w.initial()
    n = 500
    nodes = [(200, 200, 200), (300, 300, 300), (250, 250, 250), (200, 200, 290), (250, 210, 300),
             (0, 0, 0), (499, 499, 499), (0, 250, 499), (499, 0, 250), (1, 498, 2)]
    rng = np.random.default_rng(5)
    nodes += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(3)]
    refs = {}
    scale = 0.0
    for (z, y, x) in nodes:
        p, s, m = window_solve3(oracle, p0, p1, z, y, x, w, STEPS)
        refs[(z, y, x)] = (p, s)
        scale = max(scale, m)
    return w, p0, p1, refs, scale


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)], ids=["f64", "f32c"])
def test_paper_grid_sampled_vs_oracle(hb, oracle_mod, example7_500, prec, tol):
    w, p0, p1, refs, scale = example7_500
    h = hb.hb_create(hb.config_from_workload(w, prec))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, STEPS)
        phi, psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, phi, psi)
    finally:
        hb.hb_destroy(h)
    err = max(max(abs(phi[k] - p), abs(psi[k] - s)) for k, (p, s) in refs.items())
    print(f"500^3 Example 7, precision {prec}, {STEPS} steps: {len(refs)} sampled nodes, "
          f"relative max-norm error {err / scale:.3e} (scale {scale:.3f})", flush=True)
    assert np.isfinite(phi).all() and np.isfinite(psi).all()
    assert err / scale <= tol
