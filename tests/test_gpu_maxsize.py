"""Parity at the largest x-y planes the library accepts.  The whole-step
kernel addresses a plane with 32-bit byte offsets, so a padded plane of
16-byte cells must stay under 2 GiB; the largest square
one-plane grids are found from hb_footprint
(host-only) and the next size up must be rejected.  Two steps on the GPU, then
sampled nodes (corners, edges, the far end of the plane where the offsets are
largest, random nodes) against the oracle run on a window around each node
(tests/windows.py: bitwise the whole-grid value)."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from windows import sample_nodes, window_solve

pytestmark = pytest.mark.gpu


def largest_square_plane(hb, prec):
    ok, bad = 1024, 1 << 16
    assert hb.hb_footprint(hb.config_from_workload(si.wide_plane(ok, ok), prec)) > 0
    assert hb.hb_footprint(hb.config_from_workload(si.wide_plane(bad, bad), prec)) == 0
    while bad - ok > 1:
        mid = (ok + bad) // 2
        if hb.hb_footprint(hb.config_from_workload(si.wide_plane(mid, mid), prec)) > 0:
            ok = mid
        else:
            bad = mid
    return ok


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)], ids=["f64", "f32c"])
def test_largest_plane_vs_oracle_windows(hb, oracle_mod, prec, tol):
    n = largest_square_plane(hb, prec)
    cell = 16  # a cell's state slot: (phi, psi) FP64 or (phi hi, psi hi, phi lo, psi lo) FP32c
    line = 128 // cell
    pitch = (n + 4 + line - 1) // line * line
    assert pitch * (n + 4) * cell < 2 ** 31 <= ((n + 5 + line - 1) // line * line) * (n + 5) * cell
    print(f"largest accepted plane, precision {prec}: {n} x {n} "
          f"({pitch * (n + 4) * cell} bytes padded)", flush=True)
    steps = 2
    w = si.wide_plane(n, n, steps=steps)
    p0 = w.phi0()
    h = hb.hb_create(hb.config_from_workload(w, prec))
    try:
        hb.hb_set_initial(h, p0, None)
        hb.hb_step(h, steps)
        phi, psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, phi, psi)
    finally:
        hb.hb_destroy(h)
    refs = {(y, x): window_solve(oracle, p0, y, x, w, steps) for (y, x) in sample_nodes(n, n)}
    scale = max(max(abs(p), abs(s)) for p, s in refs.values())
    err = max(max(abs(phi[0, y, x] - p), abs(psi[0, y, x] - s)) for (y, x), (p, s) in refs.items())
    print(f"  {len(refs)} sampled nodes: relative max-norm error {err / scale:.3e}", flush=True)
    assert np.isfinite(phi).all() and np.isfinite(psi).all()
    assert err / scale <= tol
