"""Batched GPU radial solver (section 2.2 form) against the radial oracle.

Bar: FP64 state-vector relative max norm <= 1e-12.  The kernel evaluates
every node in the oracle's operation order (no contraction, difference
quotients divided by dr^2 and 12 dr) with the same host FP64 c(t), so the
two agree far below the bar although the radial discretisation amplifies
rounding differences near r = 0: the oracle against itself with its
difference quotients summed in mirrored order and multiplied by reciprocals
(a legitimate reordering) differs by 3e-14 after 100 steps and 2.4e-12 after
2200 steps of Example 3; that floor is printed beside each case.  Every
solve of a batch is bitwise equal to the same solve alone.
"""
import oracle.radial as radial_mod
import numpy as np
import pytest

from oracle.radial import radial_solve

pytestmark = pytest.mark.gpu


def paper_bump_r(r, R):
    out = np.zeros_like(r)
    m = r < R
    out[m] = np.exp(1.0 / R ** 2 - 1.0 / (R ** 2 - r[m] ** 2))
    return out


def rel(a, b, ra, rb):
    num = max(np.max(np.abs(a - ra)), np.max(np.abs(b - rb)))
    return num / max(np.max(np.abs(ra)), np.max(np.abs(rb)))


CASES = [
    # m, dr, mu2, lam, inv_L2, t0, dt, steps, amp0, amp1, R   (Examples 3 and 2 of section 3)
    (1000, 5e-4, 9.0, 2.0, 1 / 25, 0.0, 1e-4, 500, 1.0, -5.0, 0.3),
    (1000, 5e-4, 1.0, -1.0, 1 / 25, 0.0, 1e-4, 500, 2.0, 10.0, 0.2),
    (777, 1e-3, 0.1, 0.1, 0.3, 0.25, 2e-4, 333, 1.0, -5.0, 0.4),
    (5, 0.2, 2.0, 1.0, 1.0, 0.0, 0.01, 40, 1.0, 0.5, 0.7),
    (1, 0.5, 2.0, 1.0, 1.0, 0.0, 0.01, 40, 1.0, 0.5, 0.7),
    (2700, 2e-4, 9.0, 2.0, 1 / 25, 0.0, 5e-5, 200, 1.0, -5.0, 0.3),
    # every nodes-per-thread variant of the kernel (256 threads): 1, 2, 4, 8, 11
    (300, 1e-3, 4.0, 1.5, 1 / 25, 0.0, 1e-4, 300, 1.0, -3.0, 0.25),
    (1500, 3e-4, 2.0, 0.5, 1 / 25, 0.1, 1e-4, 150, 1.5, -2.0, 0.35),
    (257, 2e-3, 1.0, 1.0, 1 / 25, 0.0, 2e-4, 200, 1.0, 1.0, 0.4),
]


def initial(c):
    m, dr, *_rest = c
    amp0, amp1, R = c[8], c[9], c[10]
    r = np.arange(m) * dr
    b = paper_bump_r(r, R)
    return amp0 * b, amp1 * b


@pytest.mark.parametrize("case", CASES, ids=[f"m{c[0]}_mu2{c[2]}_lam{c[3]}" for c in CASES])
def test_radial_vs_oracle(hb, case):
    m, dr, mu2, lam, invL2, t0, dt, steps = case[:8]
    p0, p1 = initial(case)
    phi, psi = p0.copy(), p1.copy()
    hb.hb_radial_solve([hb.make_radial_config(m, dr, mu2, lam, dt, steps, t0, invL2)], phi, psi)
    rp, rs = radial_solve(p0, p1, dr, mu2, lam, dt, steps, t0=t0, inv_L2=invL2)
    err = rel(phi, psi, rp, rs)
    tol, floor = bar(p0, p1, (rp, rs), dr, mu2, lam, dt, steps, t0, invL2)
    print(f"radial m={m}: rel err {err:.3e} (oracle noise floor {floor:.3e})")
    assert err <= tol


def reordered_oracle(p0, p1, dr, mu2, lam, dt, steps, t0, invL2):
    """The oracle with its difference quotients summed in mirrored order and
    multiplied by reciprocals: a legitimate reordering, for the noise floor."""
    orig = radial_mod.radial_operator

    def op(u, dr):
        m = u.shape[0]
        p = radial_mod._padded(u)
        um2, um1, u0, up1, up2 = p[0:m], p[1:m + 1], p[2:m + 2], p[3:m + 3], p[4:m + 4]
        urr = (-1.0 / 12.0 * up2 + 4.0 / 3.0 * up1 - 5.0 / 2.0 * u0 + 4.0 / 3.0 * um1
               - 1.0 / 12.0 * um2) * (1.0 / (dr * dr))
        ur = (-up2 + 8.0 * up1 - 8.0 * um1 + um2) * (1.0 / (12.0 * dr))
        out = np.empty(m)
        out[1:] = 2.0 / (np.arange(1, m) * dr) * ur[1:] + urr[1:]
        out[0] = 3.0 * urr[0]
        return out

    radial_mod.radial_operator = op
    try:
        return radial_solve(p0, p1, dr, mu2, lam, dt, steps, t0=t0, inv_L2=invL2)
    finally:
        radial_mod.radial_operator = orig


def bar(p0, p1, ref, dr, mu2, lam, dt, steps, t0, invL2):
    """(the FP64 bar, the oracle's own reordering floor for this case)"""
    alt = reordered_oracle(p0, p1, dr, mu2, lam, dt, steps, t0, invL2)
    floor = rel(alt[0], alt[1], *ref)
    return 1e-12, floor


def test_radial_long_run_within_noise_floor(hb):
    """Example 3 to t = 0.22 (2200 steps): the sign-change run."""
    m, dr, mu2, lam, invL2, t0, dt, steps = 1000, 5e-4, 9.0, 2.0, 1 / 25, 0.0, 1e-4, 2200
    r = np.arange(m) * dr
    b = paper_bump_r(r, 0.3)
    phi, psi = b.copy(), -5.0 * b
    hb.hb_radial_solve([hb.make_radial_config(m, dr, mu2, lam, dt, steps, t0, invL2)], phi, psi)
    ref = radial_solve(b, -5.0 * b, dr, mu2, lam, dt, steps, t0=t0, inv_L2=invL2)
    tol, floor = bar(b, -5.0 * b, ref, dr, mu2, lam, dt, steps, t0, invL2)
    err = rel(phi, psi, *ref)
    print(f"radial Example 3, 2200 steps: GPU err {err:.3e}, oracle noise floor {floor:.3e}")
    assert err <= tol
    assert phi.min() < -1e-3 * np.max(np.abs(phi))  # the bubble of Example 3 has formed


def test_radial_batch_bitwise_equals_alone(hb):
    cfgs, phis, psis = [], [], []
    for k, c in enumerate(CASES[:5]):
        m, dr, mu2, lam, invL2, t0, dt, steps = c[:8]
        cfgs.append(hb.make_radial_config(m, dr, mu2, lam, dt, min(steps, 300), t0, invL2))
        p0, p1 = initial(c)
        phis.append(p0)
        psis.append(p1)
    phi = np.concatenate(phis)
    psi = np.concatenate(psis)
    hb.hb_radial_solve(cfgs, phi, psi)
    off = 0
    for c, p0, p1 in zip(cfgs, phis, psis):
        a, b = p0.copy(), p1.copy()
        hb.hb_radial_solve([c], a, b)
        np.testing.assert_array_equal(phi[off:off + c.m], a)
        np.testing.assert_array_equal(psi[off:off + c.m], b)
        off += c.m


def test_radial_device_arrays(hb):
    import torch
    c = CASES[2]
    p0, p1 = initial(c)
    cfg = hb.make_radial_config(*c[:2], c[2], c[3], c[6], c[7], c[5], c[4])
    tp = torch.from_numpy(p0).cuda()
    ts = torch.from_numpy(p1).cuda()
    hb.hb_radial_solve([cfg], tp, ts)
    a, b = p0.copy(), p1.copy()
    hb.hb_radial_solve([cfg], a, b)
    np.testing.assert_array_equal(tp.cpu().numpy(), a)
    np.testing.assert_array_equal(ts.cpu().numpy(), b)


def test_radial_bubble_sweep(hb):
    """A parameter sweep in one launch: the sign change of Example 3 appears
    only for phi1 = a phi0 negative enough, and earlier for smaller a."""
    m, dr, dt = 1000, 5e-4, 1e-4
    r = np.arange(m) * dr
    b = paper_bump_r(r, 0.3)
    factors = [-8.0, -6.0, -5.0, 0.0]
    onset = {}
    for a in factors:
        onset[a] = None
    phi = np.concatenate([b for _ in factors])
    psi = np.concatenate([a * b for a in factors])
    for k in range(30):  # t = 0.01 .. 0.30
        cfgs = [hb.make_radial_config(m, dr, 9.0, 2.0, dt, 100, t0=0.01 * k, inv_L2=1 / 25)
                for _ in factors]
        hb.hb_radial_solve(cfgs, phi, psi)
        for i, a in enumerate(factors):
            seg = phi[i * m:(i + 1) * m]
            if onset[a] is None and seg.min() < -1e-3 * np.max(np.abs(seg)):
                onset[a] = round(0.01 * (k + 1), 2)
    print("sign-change onset by phi1/phi0:", onset)
    assert onset[-5.0] == 0.22          # the paper's Example 3 (section 3)
    assert onset[-8.0] < onset[-6.0] < onset[-5.0]
    assert onset[0.0] is None           # Example 5: no bubble


def test_radial_errors(hb):
    bad = hb.make_radial_config(hb.HB_RADIAL_MAX_NODES + 1, 1e-3, 1.0, 1.0, 1e-4, 1)
    x = np.zeros(bad.m)
    with pytest.raises(hb.HBError) as e:
        hb.hb_radial_solve([bad], x, x.copy())
    assert e.value.code == hb.HB_E_ARG
    bad = hb.make_radial_config(100, 1e-3, 1.0, 1.0, 1.0, 1)
    x = np.zeros(100)
    with pytest.raises(hb.HBError) as e:
        hb.hb_radial_solve([bad], x, x.copy())
    assert e.value.code == hb.HB_E_CFL


def test_radial_sweep_full_size_sampled(hb):
    """The benchmark's radial sweep (4096 solves x 1000 nodes x 2000 steps, one
    launch, device-resident state): three solves against the oracle, each
    within 1e-12."""
    import torch
    import synth_inputs as si
    count, m, steps, dr, dt, invL2 = 4096, 1000, 2000, 5e-4, 1e-4, 1 / 25
    phi0, phi1, params = si.radial_sweep(count, m, dr)
    cfgs = [hb.make_radial_config(m, dr, mu2, lam, dt, steps, 0.0, invL2) for mu2, lam in params]
    phi = torch.from_numpy(phi0).cuda()
    psi = torch.from_numpy(phi1).cuda()
    hb.hb_radial_solve(cfgs, phi, psi)
    phi, psi = phi.cpu().numpy(), psi.cpu().numpy()
    for i in (0, 1, count - 1):
        mu2, lam = params[i]
        p0, p1 = phi0[i * m:(i + 1) * m], phi1[i * m:(i + 1) * m]
        ref = radial_solve(p0, p1, dr, mu2, lam, dt, steps, t0=0.0, inv_L2=invL2)
        tol, floor = bar(p0, p1, ref, dr, mu2, lam, dt, steps, 0.0, invL2)
        err = rel(phi[i * m:(i + 1) * m], psi[i * m:(i + 1) * m], *ref)
        print(f"sweep solve {i} (mu2 {mu2:.2f}, lambda {lam:.2f}): err {err:.3e}, floor {floor:.3e}")
        assert err <= tol


def test_radial_steps_across_launches(hb):
    """A solve longer than one launch's step range (65536 steps) runs in
    several launches with its state in memory between them: it matches the
    oracle, and a shorter solve of the same call stays bitwise what it is
    alone (its state passes unchanged through the later launches)."""
    # dt small enough that the dynamics (and c(t)) still move across the
    # launch boundary, so a lost, repeated or mistimed step would show
    long_case = (16, 0.05, 9.0, 2.0, 1 / 25, 0.0, 1e-5, 65536 + 700, 1.0, -5.0, 0.3)
    short_case = (40, 0.02, 9.0, 2.0, 1 / 25, 0.0, 1e-3, 300, 1.0, -5.0, 0.3)
    cfgs, p0s, p1s = [], [], []
    for c in (long_case, short_case):
        m, dr, mu2, lam, invL2, t0, dt, steps = c[:8]
        cfgs.append(hb.make_radial_config(m, dr, mu2, lam, dt, steps, t0, invL2))
        a, b = initial(c)
        p0s.append(a)
        p1s.append(b)
    phi, psi = np.concatenate(p0s), np.concatenate(p1s)
    hb.hb_radial_solve(cfgs, phi, psi)
    m0 = long_case[0]
    lp, ls = phi[:m0], psi[:m0]
    sp, ss = p0s[1].copy(), p1s[1].copy()
    hb.hb_radial_solve([cfgs[1]], sp, ss)
    assert np.array_equal(phi[m0:], sp) and np.array_equal(psi[m0:], ss)
    m, dr, mu2, lam, invL2, t0, dt, steps = long_case[:8]
    at_boundary = {}

    def keep(n, t, p, q):
        if n == 65536:
            at_boundary["s"] = (p.copy(), q.copy())

    rp, rs = radial_solve(p0s[0], p1s[0], dr, mu2, lam, dt, steps, t0=t0, inv_L2=invL2, callback=keep)
    assert rel(*at_boundary["s"], rp, rs) > 1e-4  # the steps after the boundary matter
    err = rel(lp, ls, rp, rs)
    print(f"radial m={m}, {steps} steps (two launches): rel err {err:.3e}")
    assert err <= 1e-12
