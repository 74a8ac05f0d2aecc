"""The paper's bubbles (section 1: maximal connected sets on which the
solution has changed sign) counted on the GPU (hb_bubbles, a union-find over
the interior nodes) against the oracle's breadth-first flood fill
(oracle.components) on the very state the GPU holds (hb_read; FP32c states
are classed on hi + lo in FP64 on both sides).  Counts are integers: the bar
is equality."""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu


def random_state(hb, n, prec, seed, flags=0, scale=1.0):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    phi = rng.uniform(-1.0, 1.0, size=(nz, ny, nx)) * scale
    cfg = hb.make_config(n, (0.0,) * 3, (1.0,) * 3, 1.0, 1.0, 1e-4, precision=prec, flags=flags)
    h = hb.hb_create(cfg)
    hb.hb_set_initial(h, phi, None)
    return h, phi


def gpu_and_oracle(hb, h, shape, eps, periodic):
    got = hb.hb_bubbles(h, eps)
    phi = np.empty(shape)
    hb.hb_read(h, phi, None)
    want = oracle.components(phi, eps, oracle.BC_PERIODIC if periodic else oracle.BC_ZERO)
    return got, want


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32c"])
@pytest.mark.parametrize("periodic", [False, True], ids=["zero", "periodic"])
@pytest.mark.parametrize("n", [(37, 23, 19), (1, 1, 1), (64, 3, 2), (2, 70, 5), (1, 1, 300)])
def test_random_fields(hb, n, prec, periodic):
    """Uniform noise: thousands of small sets, all three axes, ragged and
    degenerate grids; several thresholds (eps = 0 is the sign itself)."""
    flags = hb.HB_BC_PERIODIC if periodic else 0
    h, phi = random_state(hb, n, prec, seed=sum(n) + 7 * prec, flags=flags)
    try:
        for eps in (0.0, 0.3, 0.9, 2.0):
            got, want = gpu_and_oracle(hb, h, phi.shape, eps, periodic)
            print(f"{n} prec {prec} periodic {periodic} eps {eps}: GPU {got}, oracle {want}")
            assert got == want
        # the count after stepping (the state of the other parity)
        hb.hb_step(h, 3)
        got, want = gpu_and_oracle(hb, h, phi.shape, 0.0, periodic)
        assert got == want
    finally:
        hb.hb_destroy(h)


def test_large_grid_many_sets(hb):
    """256^3 of noise (about a million sets of each sign at eps = 0.5): one
    launch set of the union-find over 16.7M nodes."""
    h, phi = random_state(hb, (256, 256, 256), 0, seed=3)
    try:
        got, want = gpu_and_oracle(hb, h, phi.shape, 0.5, False)
        print(f"256^3 noise, eps 0.5: GPU {got}, oracle {want}")
        assert got == want and got[0] > 100000
    finally:
        hb.hb_destroy(h)


def test_constructed_sets(hb):
    """Known counts: two separate negative balls in a positive sea -> (2, 1);
    touching balls -> (1, 1); a negative shell holding a positive core with a
    negative centre -> (2, 2)."""
    n = 48
    z, y, x = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")

    def ball(c, r):
        return (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 < r * r

    cases = []
    f = np.ones((n, n, n))
    f[ball((14, 14, 14), 6)] = -1
    f[ball((34, 34, 34), 6)] = -1
    cases.append((f, (2, 1)))
    g = np.ones((n, n, n))
    g[ball((18, 24, 24), 7)] = -1
    g[ball((31, 24, 24), 7)] = -1
    cases.append((g, (1, 1)))
    s = np.ones((n, n, n))
    r2 = (x - 24) ** 2 + (y - 24) ** 2 + (z - 24) ** 2
    s[(r2 < 18 ** 2) & (r2 >= 12 ** 2)] = -1
    s[r2 < 4 ** 2] = -1
    cases.append((s, (2, 2)))
    for field, want in cases:
        cfg = hb.make_config((n, n, n), (0.0,) * 3, (1.0,) * 3, 1.0, 1.0, 1e-4)
        h = hb.hb_create(cfg)
        try:
            hb.hb_set_initial(h, field, None)
            got = hb.hb_bubbles(h, 0.0)
            assert got == want == oracle.components(field, 0.0)
        finally:
            hb.hb_destroy(h)


def sets_at(hb, h, shape, rel_eps):
    """GPU and oracle counts of the current state, the sets counted above
    rel_eps x max|phi| (the far field beyond the data's support carries
    sign-alternating values many orders of magnitude below the peak)."""
    eps = rel_eps * hb.hb_diagnostics(h)["linf_phi"]
    return gpu_and_oracle(hb, h, shape, eps, False)


def run_marks(hb, cfg, phi0, phi1, dt, marks, rel_eps):
    h = hb.hb_create(cfg)
    out = []
    try:
        hb.hb_set_initial(h, phi0, phi1)
        done = 0
        for t in marks:
            k = int(round(t / dt)) - done
            hb.hb_step(h, k)
            done += k
            got, want = sets_at(hb, h, phi0.shape, rel_eps)
            assert got == want
            out.append(got)
    finally:
        hb.hb_destroy(h)
    return out


def test_example3_one_bubble(hb):
    """Section 3, Example 3 at 64^3 (dt = 1e-3): one positive set and no
    negative one at t = 0.21; the sign change by t = 0.22 is one bubble (one
    negative set inside the positive one), which persists."""
    nn, lo, hi = (64,) * 3, (0.0,) * 3, (1.0,) * 3
    b = si.paper_bump(nn, lo, hi, (0.5, 0.5, 0.5), 0.3)
    cfg = hb.make_config(nn, lo, hi, 9.0, 2.0, 1e-3, inv_L2=1 / 25)
    counts = run_marks(hb, cfg, b, -5.0 * b, 1e-3, [0.21, 0.22, 0.3, 0.5], 1e-2)
    print("Example 3 (64^3) sets (negative, positive) at t = 0.21, 0.22, 0.3, 0.5:", counts)
    assert counts == [(0, 1), (1, 1), (1, 1), (1, 1)]


def test_example7_two_bubbles_merge(hb):
    """Section 3, Example 7 at 64^3 (dt = 1e-3), sets above 1% of the peak:
    two positive sets and no bubble at first; two bubbles (negative sets)
    once the sign changes; the positive sets join, then the two bubbles join
    into one.  The paper's order of events, later in time under this
    reading (bubbles by t = 0.12-0.15 instead of 0.08, joined by t = 2
    instead of 0.69)."""
    w = si.example7_config(64, 0)
    cfg = hb.config_from_workload(w)
    cfg.dt = 1e-3
    p0, p1 = w.initial()
    marks = [0.1, 0.15, 0.3, 0.8, 1.5, 2.0, 3.0]
    counts = run_marks(hb, cfg, p0, p1, 1e-3, marks, 1e-2)
    print("Example 7 (64^3) sets (negative, positive) at t =", marks, ":", counts)
    assert counts[0] == (0, 2)
    assert counts[1] == counts[2] == (2, 2)
    assert counts[3] == counts[4] == (2, 1)
    assert counts[5] == counts[6] == (1, 1)
