"""The paper's section 3 examples on the GPU path at reduced resolution
(Examples 1, 3, 4, 5, 6 and 7).

Unit box [0,1]^3 (cell-centred), L = 5 (inv_L2 = 1/25), the paper's bump
B(x; C, R) = exp(1/R^2 - 1/(R^2 - |x-C|^2)) with C the box centre (Example
6 multiplies two bumps and a sine, and is not radial).  Each run
is checked against the oracle at the same resolution (same discrete
problem) and against the facts the paper prints (tests/golden/
paper_facts.json).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu
FACTS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def unit_box_case(n, amp0, amp1, R, mu2, lam, dt):
    nn, lo, hi = (n, n, n), (0.0,) * 3, (1.0,) * 3
    b = si.paper_bump(nn, lo, hi, (0.5, 0.5, 0.5), R)
    w = si.Workload(f"paper_unit{n}", nn, lo, hi, mu2=mu2, lam=lam, dt=dt, steps=0,
                    inv_L2=1.0 / 25.0, phi0=lambda: amp0 * b, phi1=lambda: amp1 * b)
    return w


def run_segments(hb, w, segments):
    """Advance through the given step counts; return the states after each."""
    p0, p1 = w.initial()
    h = hb.hb_create(hb.config_from_workload(w))
    out = []
    try:
        hb.hb_set_initial(h, p0, p1)
        for k in segments:
            hb.hb_step(h, k)
            phi, psi = np.empty_like(p0), np.empty_like(p0)
            hb.hb_read(h, phi, psi)
            out.append((phi, psi, hb.hb_diagnostics(h)))
    finally:
        hb.hb_destroy(h)
    return out


def test_example3_bubble_onset(hb, oracle_mod):
    f = FACTS["example3_bubble_onset"]
    dt = 1e-3
    w = unit_box_case(96, 1.0, f["phi1_factor"], f["bump_radius"], f["mu2"], f["lambda"], dt)
    n1 = int(round(f["positive_at"] / dt))
    n2 = int(round(f["sign_change_at"] / dt)) - n1
    (a, sa, da), (b, sb, db) = run_segments(hb, w, [n1, n2])
    # same discrete problem on the oracle
    r = oracle.solve_workload(w, nsteps=n1 + n2)
    assert oracle.rel_maxnorm(b, sb, *r) <= 1e-12
    scale = np.max(np.abs(b))
    print(f"Example 3 (96^3): min phi {a.min():.3e} at t={f['positive_at']}, "
          f"{b.min():.3e} at t={f['sign_change_at']} (max {scale:.3e})")
    assert a.min() > -1e-4 * scale          # still positive (up to the stencil's far-field dust)
    assert b.min() < -0.1 * scale           # sign change: a bubble wall has formed
    assert db["negative"] > 0


def test_example5_no_bubble(hb):
    f = FACTS["example5_no_bubble"]
    dt = 2e-3
    w = unit_box_case(64, f["amp"], 0.0, f["bump_radius"], f["mu2"], f["lambda"], dt)
    segs = [50] * int(round(f["until"] / dt / 50))
    worst = 0.0
    for phi, psi, d in run_segments(hb, w, segs):
        worst = min(worst, phi.min() / np.max(np.abs(phi)))
    print(f"Example 5 (64^3): most negative phi / max phi over t <= {f['until']}: {worst:.3e}")
    assert worst > -1e-4


def test_example4_plateau_and_P(hb):
    f = FACTS["example4_long_time_plateau"]
    dt = 2e-3
    n = 64
    w = unit_box_case(n, 1.0, f["phi1_factor"], f["bump_radius"], f["mu2"], f["lambda"], dt)
    k = int(round(1.0 / dt))
    states = run_segments(hb, w, [k] * int(round(f["t"])))
    phi, psi, d = states[-1]
    c = n // 2
    centre = phi[c - 1:c + 1, c - 1:c + 1, c - 1:c + 1].mean()  # the 8 nodes around the centre
    P = [s[2]["lap_max"] for s in states]
    print(f"Example 4 (64^3): bubble-centre phi at t={f['t']}: {centre:.5f}; "
          f"P(t) at t=1..{int(f['t'])}: " + " ".join(f"{p:.2e}" for p in P))
    assert round(centre, f["decimals"]) == f["value"]
    assert abs(centre + math.sqrt(f["mu2"] / f["lambda"])) < 5e-3
    # P(t) = c(t) max|Lap_h phi| goes to zero; once the step function has
    # formed, max|Lap_h phi| settles and P falls like c(t) ~ e^{-2t}
    ratios = [P[i + 1] / P[i] for i in range(4, len(P) - 1)]
    assert all(r < 0.2 for r in ratios), ratios
    assert P[-1] < 1e-5 * P[0]


def example6_case(n, dt):
    f = FACTS["example6_positive_limit"]
    p0, p1 = si.example6_data(n, f["bump_centre"], f["second_centre"], f["bump_radius"],
                              f["phi0_amp"], f["phi1_amp"])
    nn, lo, hi = (n, n, n), (0.0,) * 3, (1.0,) * 3
    return si.Workload(f"paper_example6_{n}", nn, lo, hi, mu2=f["mu2"], lam=f["lambda"], dt=dt,
                       steps=0, inv_L2=1.0 / f["L"] ** 2, phi0=lambda: p0, phi1=lambda: p1)


def test_example6_parity(hb, oracle_mod):
    """Example 6's non-radial, sign-changing data: GPU against the oracle at
    48^3 over t in [0, 1] (500 steps), every node."""
    w = example6_case(48, 2e-3)
    (phi, psi, _), = run_segments(hb, w, [500])
    err = oracle.rel_maxnorm(phi, psi, *oracle.solve_workload(w, nsteps=500))
    print(f"Example 6 (48^3 x 500): relative max-norm error {err:.3e}")
    assert err <= 1e-12


def test_example6_positive_limit(hb):
    """At 96^3: the negative lobe of phi0 is gone from t = 1 on (what stays
    below zero is far-field rounding dust), and at t = 4 the positive region
    sits at sqrt(9/2), printed as 2.12."""
    f = FACTS["example6_positive_limit"]
    dt, n = 2e-3, 96
    w = example6_case(n, dt)
    k = int(round(1.0 / dt))
    states = run_segments(hb, w, [k] * int(round(f["t"])))
    for i, (phi, _, d) in enumerate(states):
        print(f"Example 6 (96^3) t={i + 1}: min {phi.min():.3e}, max {phi.max():.5f}")
        assert phi.min() > -1e-4 * phi.max()
        assert d["nonfinite"] == 0
    phi = states[-1][0]
    c = n // 2
    centre = phi[c - 1:c + 1, c - 1:c + 1, c - 1:c + 1].mean()
    median = float(np.median(phi[phi > 1.0]))
    print(f"Example 6 (96^3) t={f['t']}: median over phi > 1 {median:.5f}, centre {centre:.5f}")
    assert round(median, f["decimals"]) == f["value"]
    assert round(centre, f["decimals"]) == f["value"]
    assert abs(median - math.sqrt(f["mu2"] / f["lambda"])) < 5e-3


def test_example1_grid_convergence_and_precision(hb):
    """Example 1 (phi0 = 3 B(x; C, 0.3), phi1 = 0, mu^2 = 9, lambda = 2): the
    paper compares coarser grids with a finer one at t = 1 and t = 2 and sees
    the differences shrink, and finds single against double precision close
    and not growing in time.  Here n = 60 and 180 against 540 on the nodes the
    three cell-centred grids share (ratio 3): the differences shrink, and by
    the factor 3^p + 1 that a method of spatial order p gives, with p = 4
    (section 2: the fourth-order stencil; dt = 1e-3 keeps the RK4 error far
    below).  FP32c against FP64 at n = 180 stays below 1e-6 relative at both
    times and does not grow."""
    dt = 1e-3
    ns = (60, 180, 540)

    def run(n, prec):
        w = unit_box_case(n, 3.0, 0.0, 0.3, 9.0, 2.0, dt)
        k = int(round(1.0 / dt))
        p0, p1 = w.initial()
        h = hb.hb_create(hb.config_from_workload(w, prec))
        out = []
        try:
            hb.hb_set_initial(h, p0, p1)
            for _ in range(2):
                hb.hb_step(h, k)
                phi = np.empty_like(p0)
                hb.hb_read(h, phi, None)
                out.append(phi)
        finally:
            hb.hb_destroy(h)
        return out

    res = {n: run(n, 0) for n in ns}
    for ti in range(2):
        fine = res[540][ti]
        # the nodes of the 60^3 grid, as they sit in each finer grid
        on60 = {n: res[n][ti][(n // 60) // 2::n // 60, (n // 60) // 2::n // 60, (n // 60) // 2::n // 60]
                for n in ns}
        d60 = np.abs(on60[60] - on60[540]).max()
        d180 = np.abs(on60[180] - on60[540]).max()
        order = math.log(d60 / d180 - 1.0, 3.0)
        print(f"Example 1, t={ti + 1}: max |phi_n - phi_540| on the 60^3 nodes: n=60 {d60:.3e}, "
              f"n=180 {d180:.3e}; observed spatial order {order:.2f} (max |phi| {np.abs(fine).max():.3f})")
        assert d180 < d60 < 1e-2 * np.abs(fine).max()
        assert 3.7 < order < 4.3
    a32 = run(180, 1)
    diff = [np.abs(a32[i] - res[180][i]).max() / np.abs(res[180][i]).max() for i in range(2)]
    print(f"Example 1 (180^3): FP32c vs FP64 relative max difference at t=1, 2: "
          f"{diff[0]:.3e}, {diff[1]:.3e}")
    assert max(diff) < 1e-6
    assert diff[1] < 2 * diff[0]


def test_example7_parity(hb, oracle_mod):
    """Example 7's two-bump data (the paper's longest run, benchmarked at its
    500^3 grid): GPU against the oracle at 64^3, dt = 1e-3, 150 steps (past
    the sign changes near t = 0.12), every node."""
    w = si.example7_config(64, 150)
    w.dt = 1e-3
    (phi, psi, d), = run_segments(hb, w, [150])
    err = oracle.rel_maxnorm(phi, psi, *oracle.solve_workload(w, nsteps=150))
    print(f"Example 7 (64^3 x 150): relative max-norm error {err:.3e}, negative nodes {d['negative']}")
    assert err <= 1e-12
    assert phi.min() < -0.01 * phi.max()   # the bubbles have formed


def example2_workload(n, reading, steps=0):
    """Section 3, Example 2 on the unit box (L = 5): mu^2 = 1, lambda = -1,
    phi0 = 2 B, phi1 = 10 B, B of radius 0.2 at the centre; `reading` picks
    the bump: "literal" = the printed exp(1/R^2 - 1/(R^2 - r^2)),
    "scale_invariant" = exp(1 - 1/(1 - r^2/R^2)) (both equal 1 at the
    centre; the literal one is much narrower)."""
    nn, lo, hi = (n,) * 3, (0.0,) * 3, (1.0,) * 3
    C = (0.5,) * 3
    b = si.paper_bump(nn, lo, hi, C, 0.2) if reading == "literal" else si.cinf_bump(nn, lo, hi, 1.0, 0.2, C)
    return si.Workload(f"example2_{reading}_{n}", nn, lo, hi, mu2=1.0, lam=-1.0, dt=1e-3, steps=steps,
                       inv_L2=1.0 / 25.0, phi0=lambda: 2.0 * b, phi1=lambda: 10.0 * b)


@pytest.mark.parametrize("reading", ["literal", "scale_invariant"])
def test_example2_parity(hb, oracle_mod, reading):
    """Example 2's data under both bump readings: GPU against the oracle at
    48^3, dt = 1e-3, 300 steps (before any blow-up), every node."""
    w = example2_workload(48, reading, 300)
    (phi, psi, d), = run_segments(hb, w, [300])
    err = oracle.rel_maxnorm(phi, psi, *oracle.solve_workload(w))
    print(f"Example 2 ({reading}, 48^3 x 300): relative max-norm error {err:.3e}, max|phi| {d['linf_phi']:.3f}")
    assert err <= 1e-12


def test_example2_both_readings(hb):
    """What each reading gives at 64^3 against the paper's account (max|phi|
    about 2 up to t = 2, about 130 at t = 2.97, the integral of phi blowing
    up shortly after; neither reading reproduces it):
    * scale-invariant bump: max|phi| passes 100 by t = 0.7 and the state
      turns non-finite before t = 1, which hb_diagnostics reports as
      HB_E_NONFINITE (overflow of the solution, not a device fault);
    * literal bump: the narrow pulse disperses, max|phi| falls below 0.2 by
      t = 1 and stays below 0.2 to t = 4, while the integral of phi grows
      throughout (the zero state is unstable for lambda < 0)."""
    w = example2_workload(64, "scale_invariant")
    p0, p1 = w.initial()
    h = hb.hb_create(hb.config_from_workload(w))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, 700)
        d = hb.hb_diagnostics(h)
        print(f"Example 2 scale-invariant: max|phi| {d['linf_phi']:.1f} at t = 0.7")
        assert d["linf_phi"] > 100
        hb.hb_step(h, 300)
        with pytest.raises(hb.HBError) as e:
            hb.hb_diagnostics(h)
        assert e.value.code == hb.HB_E_NONFINITE
        assert hb.hb_diagnostics(h, allow_nonfinite=True)["nonfinite"] > 0
    finally:
        hb.hb_destroy(h)
    w = example2_workload(64, "literal")
    segs = [100] * 40  # t = 0.1 .. 4.0
    series = [(k + 1) * 0.1 for k in range(40)]
    states = run_segments(hb, w, segs)
    lin = [d["linf_phi"] for _, _, d in states]
    integ = [d["integral"] for _, _, d in states]
    print("Example 2 literal: max|phi| at t = 0.5, 1, 2, 2.97, 4:",
          [round(lin[int(round(t * 10)) - 1], 4) for t in (0.5, 1.0, 2.0, 3.0, 4.0)])
    assert lin[0] > 1.0 and max(lin[9:]) < 0.2
    assert all(b > a for a, b in zip(integ, integ[1:]))
    assert len(series) == len(lin)


def test_example2_pool_evicts_blowup(hb):
    """The scale-invariant Example 2 solve and a healthy one (Example 3's
    data) share a pool: hb_pool_check stops the first once its state turns
    non-finite (before t = 1), and the second runs to its end bitwise as it
    does alone."""
    bad = example2_workload(48, "scale_invariant")
    good = unit_box_case(48, 1.0, -5.0, 0.3, 9.0, 2.0, 1e-3)
    pool = hb.hb_pool_create(1 << 32, 4)
    try:
        sb = hb.hb_pool_admit(pool, hb.config_from_workload(bad), *bad.initial(), 1000)
        sg = hb.hb_pool_admit(pool, hb.config_from_workload(good), *good.initial(), 1000)
        failed_at = None
        for k in range(20):
            hb.hb_pool_advance(pool, 50)
            f = hb.hb_pool_check(pool)
            if f:
                assert f == [sb] and failed_at is None
                failed_at = 50 * (k + 1)
        print(f"Example 2 (scale-invariant) stopped by hb_pool_check after {failed_at} steps")
        assert failed_at is not None and failed_at <= 1000
        assert sorted(hb.hb_pool_poll(pool)) == sorted([sb, sg])
        phi = np.empty(good.n[::-1])
        hb.hb_pool_read(pool, sg, phi, None)
        good.steps = 1000
        np.testing.assert_array_equal(phi, hb.solve_host(good, 1000)[0])
    finally:
        hb.hb_pool_destroy(pool)
