"""GPU path (libhb through its C ABI) against the FP64 CPU oracle.

Bar: FP64 state-vector relative max norm <= 1e-12 (elementwise comparison);
FP32c (FP32 storage/stencil, compensated state) <= 1e-5 against the FP64
oracle.  Sizes span several tiles of every scheme's shapes, ragged x/y/z
tails and z-chunks.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32C = 1e-5


def run_gpu(hb, w, nsteps=None, precision=0, flags=0, tiling=None):
    return hb.solve_host(w, nsteps, precision=precision, flags=flags, tiling=tiling)


def test_config1_full(hb, oracle_mod):
    w = si.config1()
    g = run_gpu(hb, w)
    r = oracle.solve_workload(w)
    err = oracle.rel_maxnorm(*g, *r)
    print(f"cube32 100 steps: rel err {err:.3e}")
    assert err <= TOL64


# Whole-step kernel tiles (the default scheme): 32 x 24 (by 8), 60 x 12
# (by 16), 64 x 11 (by 11) and 32 x 16 (by 20); tiling (by, zc), zc = 0 for
# the library's z-march length.
@pytest.mark.parametrize("shape,tiling", [
    ((70, 21, 13), None),          # 3 x-tiles (32 + 32 + 6), one ragged y-tile
    ((130, 17, 40), (8, 7)),       # 5 x-tiles (ragged 2), z-marches of 7 (ragged 5)
    ((64, 32, 24), (16, 5)),       # 2 x-tiles of 60 (ragged 4), 3 y-tiles (ragged 8)
    ((200, 9, 11), (16, 0)),       # a y extent below one tile
    ((5, 3, 30), (8, 4)),          # narrower than one tile
    ((97, 53, 41), (8, 0)),        # 4 x 3 tiles, every axis ragged (1, 5, z)
    ((125, 50, 29), (16, 9)),      # 3 x 5 tiles of 60 x 12, ragged in all axes
    ((130, 25, 19), (11, 6)),      # 3 x 3 tiles of 64 x 11 (ragged 2, 3), z ragged 1
    ((64, 11, 7), (11, 0)),        # exactly one 64 x 11 tile
    ((256, 23, 12), (11, 5)),      # 4 whole 64-column tiles, y ragged 1
    ((70, 37, 15), (20, 4)),       # 3 x 3 tiles of 32 x 16 (ragged 6, 5), z ragged 3
    ((32, 16, 9), (20, 0)),        # exactly one 32 x 16 tile
])
def test_ragged_shapes(hb, oracle_mod, shape, tiling):
    w = si.small_case(*shape, seed=sum(shape), steps=12)
    g = run_gpu(hb, w, tiling=tiling)
    r = oracle.solve_workload(w)
    err = oracle.rel_maxnorm(*g, *r)
    print(f"{shape} tiling {tiling}: rel err {err:.3e}")
    assert err <= TOL64


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 3), (1, 40, 1), (3, 3, 70)])
def test_degenerate_shapes(hb, oracle_mod, shape):
    w = si.small_case(*shape, seed=3, steps=6)
    g = run_gpu(hb, w)
    r = oracle.solve_workload(w)
    assert oracle.rel_maxnorm(*g, *r) <= TOL64


def test_zero_data_stays_zero(hb):
    w = si.small_case(40, 10, 10, steps=5)
    w.phi0 = w.phi1 = None
    phi, psi = run_gpu(hb, w)
    assert not np.any(phi) and not np.any(psi)


@pytest.mark.parametrize("mu2,lam,t0,inv_L2", [(9.0, 2.0, 0.0, 1 / 25), (1.0, -1.0, 0.3, 1.0),
                                               (0.1, 0.1, -0.2, 0.5), (-1.0, 0.0, 1.0, 2.0)])
def test_coefficients(hb, oracle_mod, mu2, lam, t0, inv_L2):
    w = si.small_case(66, 12, 10, seed=11, steps=10, mu2=mu2, lam=lam, t0=t0, inv_L2=inv_L2)
    g = run_gpu(hb, w)
    r = oracle.solve_workload(w)
    assert oracle.rel_maxnorm(*g, *r) <= TOL64


def test_anisotropic_spacing(hb, oracle_mod):
    w = si.small_case(40, 20, 12, seed=2, steps=8)
    w.hi = (w.hi[0], w.hi[1] * 1.7, w.hi[2] * 0.6)
    g = run_gpu(hb, w)
    r = oracle.solve_workload(w)
    assert oracle.rel_maxnorm(*g, *r) <= TOL64


def test_fp32c_against_fp64_oracle(hb, oracle_mod):
    w = si.small_case(96, 40, 24, seed=5, steps=40)
    g = run_gpu(hb, w, precision=hb.HB_F32C)
    r = oracle.solve_workload(w)
    err = oracle.rel_maxnorm(*g, *r)
    print(f"fp32c rel err {err:.3e}")
    assert err <= TOL32C


def test_graph_replay_bitwise(hb):
    w = si.small_case(70, 20, 18, seed=8, steps=37)
    a = run_gpu(hb, w)
    b = run_gpu(hb, w, flags=hb.HB_USE_GRAPH)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape", [(75, 22, 19), (121, 25, 7), (3, 14, 30)])
def test_schemes_bitwise_equal(hb, precision, shape):
    """whole-step (default), stage-pair and per-stage kernels: same bits"""
    w = si.small_case(*shape, seed=15, steps=11)
    a = run_gpu(hb, w, precision=precision)
    b = run_gpu(hb, w, precision=precision, flags=hb.HB_PAIRWISE)
    c = run_gpu(hb, w, precision=precision, flags=hb.HB_STAGEWISE)
    for x in (b, c):
        np.testing.assert_array_equal(a[0], x[0])
        np.testing.assert_array_equal(a[1], x[1])


@pytest.mark.parametrize("flags", ["HB_PAIRWISE", "HB_STAGEWISE"])
def test_other_schemes_vs_oracle(hb, oracle_mod, flags):
    w = si.small_case(70, 21, 13, seed=16, steps=9)
    g = run_gpu(hb, w, flags=getattr(hb, flags))
    r = oracle.solve_workload(w)
    assert oracle.rel_maxnorm(*g, *r) <= TOL64


@pytest.mark.parametrize("flags", [0, 8])
def test_tiling_does_not_change_results(hb, flags):
    w = si.small_case(90, 30, 33, seed=9, steps=6)
    ref = run_gpu(hb, w, tiling=(8, 0), flags=flags)
    shapes = [(16, 0), (8, 5), (16, 11), (8, 1), (16, 2)]
    if flags == 0:  # the 64 x 11 and 32 x 16 tiles of the whole-step kernel
        shapes += [(11, 0), (11, 4), (11, 1), (20, 0), (20, 5), (20, 1)]
    for t in shapes:
        got = run_gpu(hb, w, tiling=t, flags=flags)
        np.testing.assert_array_equal(ref[0], got[0])
        np.testing.assert_array_equal(ref[1], got[1])


def test_repeatable_bitwise(hb):
    w = si.small_case(80, 24, 20, seed=10, steps=9)
    a = run_gpu(hb, w)
    b = run_gpu(hb, w)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("precision", [0, 1])
def test_checkpoint_resume_bitwise(hb, precision):
    w = si.small_case(70, 16, 12, seed=12, steps=10)
    p0, p1 = w.initial()
    cfg = hb.config_from_workload(w, precision)
    h = hb.hb_create(cfg)
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, 10)
        full_phi, full_psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, full_phi, full_psi)
    finally:
        hb.hb_destroy(h)
    h = hb.hb_create(cfg)
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, 4)
        if precision == 0:
            a, b = np.empty_like(p0), np.empty_like(p0)
            hb.hb_read(h, a, b)
            hb.hb_destroy(h)
            h = hb.hb_create(cfg)
            hb.hb_set_state(h, a, b, 4)
        hb.hb_step(h, 3)
        hb.hb_step(h, 3)
        assert hb.hb_time(h)[1] == 10
        phi, psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, phi, psi)
    finally:
        hb.hb_destroy(h)
    np.testing.assert_array_equal(phi, full_phi)
    np.testing.assert_array_equal(psi, full_psi)


def test_device_pointers_torch(hb, oracle_mod):
    import torch
    w = si.small_case(68, 10, 9, seed=13, steps=7)
    p0, p1 = w.initial()
    dev = torch.device("cuda:0")
    t0 = torch.from_numpy(p0).to(dev)
    t1 = torch.from_numpy(p1).to(dev)
    s = torch.cuda.current_stream()
    h = hb.hb_create(hb.config_from_workload(w, stream=s.cuda_stream or None))
    try:
        hb.hb_set_initial(h, t0, t1)
        hb.hb_step(h, w.steps)
        o0 = torch.empty_like(t0)
        o1 = torch.empty(t0.shape, dtype=torch.float32, device=dev)
        hb.hb_read(h, o0, None)
        hb.hb_read(h, None, o1)
        torch.cuda.synchronize()
    finally:
        hb.hb_destroy(h)
    r = oracle.solve_workload(w)
    assert np.max(np.abs(o0.cpu().numpy() - r[0])) <= TOL64 * np.max(np.abs(r[0]))
    np.testing.assert_allclose(o1.cpu().numpy(), r[1].astype(np.float32), rtol=1e-6, atol=1e-7)


def test_diagnostics_match_oracle(hb, oracle_mod):
    from oracle.diagnostics import diagnostics
    w = si.small_case(50, 30, 20, seed=14, steps=5, inv_L2=0.7, t0=0.1)
    p0, p1 = w.initial()
    h = hb.hb_create(hb.config_from_workload(w))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, w.steps)
        d = hb.hb_diagnostics(h)
        phi, psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, phi, psi)
    finally:
        hb.hb_destroy(h)
    ref = diagnostics(phi, psi, w.h, w.mu2, w.lam, w.t0 + w.steps * w.dt, w.inv_L2)
    for k in ("integral", "linf_phi", "linf_psi", "l2_phi", "l2_psi", "lap_max", "energy"):
        assert d[k] == pytest.approx(ref[k], rel=1e-12, abs=1e-14), k
    assert d["nonfinite"] == 0 and d["negative"] == ref["negative"]


def test_errors(hb):
    w = si.small_case(16, 16, 16, steps=1)
    h = hb.hb_create(hb.config_from_workload(w))
    try:
        with pytest.raises(hb.HBError) as e:
            hb.hb_step(h, 1)
        assert e.value.code == hb.HB_E_STATE
        p0, p1 = w.initial()
        # step counts and indices are capped at 2^40 (no overflow, no huge table)
        with pytest.raises(hb.HBError) as e:
            hb.hb_set_state(h, p0, p1, 2 ** 41)
        assert e.value.code == hb.HB_E_ARG
        hb.hb_set_initial(h, p0, p1)
        with pytest.raises(hb.HBError) as e:
            hb.hb_step(h, 2 ** 41)
        assert e.value.code == hb.HB_E_ARG
        hb.hb_step(h, 1)  # still usable
        assert hb.hb_time(h)[1] == 1
        for by in (0, 12, 32):
            with pytest.raises(hb.HBError) as e:
                hb.hb_set_tiling(h, by, 0)
            assert e.value.code == hb.HB_E_ARG
    finally:
        hb.hb_destroy(h)
    # 64 x 11 and 32 x 16 tiles exist for the whole-step kernel only
    h = hb.hb_create(hb.config_from_workload(w, flags=hb.HB_PAIRWISE))
    try:
        for by in (11, 20):
            with pytest.raises(hb.HBError) as e:
                hb.hb_set_tiling(h, by, 0)
            assert e.value.code == hb.HB_E_ARG
    finally:
        hb.hb_destroy(h)
    bad = hb.config_from_workload(w)
    bad.dt = 10.0
    with pytest.raises(hb.HBError) as e:
        hb.hb_create(bad)
    assert e.value.code == hb.HB_E_CFL
    bad = hb.config_from_workload(w)
    bad.n[1] = 0
    with pytest.raises(hb.HBError) as e:
        hb.hb_create(bad)
    assert e.value.code == hb.HB_E_ARG


def test_nonfinite_detected(hb):
    w = si.small_case(20, 20, 20, steps=2)
    p0, p1 = w.initial()
    p0[3, 4, 5] = np.nan
    h = hb.hb_create(hb.config_from_workload(w))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, 1)
        with pytest.raises(hb.HBError) as e:
            hb.hb_diagnostics(h)
        assert e.value.code == hb.HB_E_NONFINITE
        assert hb.hb_diagnostics(h, allow_nonfinite=True)["nonfinite"] > 1
    finally:
        hb.hb_destroy(h)


def random_cases(count=16, seed=2024):
    """Seeded random configurations: shape, box aspect (anisotropic h),
    coefficients (lambda of both signs), start time, c(t) scale, dt inside the
    stability limit, steps, precision, scheme and tiling."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(count):
        n = tuple(int(v) for v in rng.integers(1, 90, size=3))
        L = float(rng.uniform(4.0, 20.0))
        mu2 = float(rng.uniform(0.0, 9.0))
        lam = float(rng.choice([-1.0, 1.0]) * rng.uniform(0.1, 4.0))
        t0 = float(rng.uniform(0.0, 1.0))
        inv_L2 = float(rng.uniform(0.05, 1.0))
        steps = int(rng.integers(1, 14))
        prec = int(rng.integers(0, 2))
        flags = [0, 0, 8, 4][int(rng.integers(0, 4))]          # whole-step (x2), pairs, stages
        tiling = (int(rng.choice([8, 16])), int(rng.choice([0, 1, 3, 7, 32])))
        cases.append((k, n, L, mu2, lam, t0, inv_L2, steps, prec, flags, tiling))
    return cases


def random_dt(w, inv_L2, t0):
    """dt at 40% of the RK4 stability limit of the stencil part (section 2.1
    symbol), and at most 0.02 so that the few steps stay far from the
    finite-time blow-up of the focusing (lambda < 0) cases."""
    rho = sum(16.0 / (3.0 * hd * hd) for hd in w.h)
    return min(0.02, 0.4 * 2.0 * np.sqrt(2.0) / np.sqrt(inv_L2 * np.exp(-2.0 * t0) * rho))


@pytest.mark.parametrize("case", random_cases(), ids=lambda c: f"r{c[0]}_{c[1][0]}x{c[1][1]}x{c[1][2]}")
def test_random_configurations(hb, oracle_mod, case):
    k, n, L, mu2, lam, t0, inv_L2, steps, prec, flags, tiling = case
    w = si.small_case(*n, seed=100 + k, steps=steps, L=L, mu2=mu2, lam=lam, t0=t0,
                      inv_L2=inv_L2)
    w.dt = random_dt(w, inv_L2, t0)
    g = run_gpu(hb, w, precision=prec, flags=flags, tiling=tiling)
    r = oracle.solve_workload(w)
    assert np.all(np.isfinite(r[0])) and np.all(np.isfinite(r[1]))
    err = oracle.rel_maxnorm(*g, *r)
    print(f"case {case}: rel err {err:.3e}")
    assert err <= (TOL32C if prec else TOL64)


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32c"])
@pytest.mark.parametrize("flags", ["step", "HB_PAIRWISE", "HB_STAGEWISE", "HB_BC_PERIODIC"])
def test_padding_is_never_read(hb, prec, flags):
    """HB_DEBUG_POISON fills every stored cell outside the interior and its
    2-cell halo with NaN: no kernel reads one, so results stay bitwise those
    of a clean run and the diagnostics find no NaN."""
    f = 0 if flags == "step" else getattr(hb, flags)
    wide = (11, 6) if f in (0, hb.HB_BC_PERIODIC) else (16, 6)
    for shape, tiling in [((70, 21, 13), None), ((5, 3, 7), (8, 0)), ((130, 25, 19), wide),
                          ((1, 2, 6), None)]:
        w = si.small_case(*shape, seed=sum(shape) + 3, steps=5)
        clean = run_gpu(hb, w, precision=prec, flags=f, tiling=tiling)
        p0, p1 = w.initial()
        h = hb.hb_create(hb.config_from_workload(w, prec, f | hb.HB_DEBUG_POISON))
        try:
            if tiling is not None:
                hb.hb_set_tiling(h, *tiling)
            hb.hb_set_initial(h, p0, p1)
            hb.hb_step(h, w.steps)
            phi, psi = np.empty_like(p0), np.empty_like(p0)
            hb.hb_read(h, phi, psi)
            d = hb.hb_diagnostics(h)
        finally:
            hb.hb_destroy(h)
        np.testing.assert_array_equal(phi, clean[0])
        np.testing.assert_array_equal(psi, clean[1])
        assert d["nonfinite"] == 0


def test_poison_marks_exactly_the_padding(hb):
    """The check above is not vacuous: the raw state allocation of a poisoned
    whole-step solve (caught through the allocator hook) holds NaN in every
    cell outside the interior and its halo, and zeros in the rest."""
    import torch
    held = {}

    def alloc(nbytes, stream):
        t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        held[t.data_ptr()] = t
        return t.data_ptr()

    def release(ptr, nbytes):
        held.pop(ptr)

    nx, ny, nz = 13, 9, 5
    w = si.small_case(nx, ny, nz, seed=1, steps=1)
    hb.hb_set_allocator(alloc, release)
    try:
        h = hb.hb_create(hb.config_from_workload(w, 0, hb.HB_DEBUG_POISON))
    finally:
        hb.hb_set_allocator()
    try:
        hb.hb_sync(h)
        # layout of the whole-step state: 16-byte cells, 8 to a 128-byte line,
        # row pitch nx + 4 rounded up to a line, cell (0, y, z) on a line,
        # fields rounded up to 256 bytes, one field per step parity
        ru = lambda v, m: (v + m - 1) // m * m
        sy = ru(nx + 4, 8)
        sz = sy * (ny + 4)
        origin = 2 * sz + 2 * sy + 8
        cells = ru(origin + (nz + 1) * sz + (ny + 1) * sy + nx + 2, 16)
        state = [t for t in held.values() if t.numel() == 2 * cells * 16]
        assert len(state) == 1
        raw = state[0].cpu().numpy().view(np.float64).reshape(2, cells, 2)
    finally:
        hb.hb_destroy(h)
    keep = np.zeros(cells, bool)
    for z in range(-2, nz + 2):
        for y in range(-2, ny + 2):
            keep[origin + z * sz + y * sy + np.arange(-2, nx + 2)] = True
    assert np.isnan(raw[:, ~keep, :]).all()
    assert (raw[:, keep, :] == 0).all()
    assert held == {}


def test_trace_prints_one_line_per_step():
    """HB_TRACE=1: hb_step times each launch and prints a line per step (run
    in a child process, since the setting is read once per process)."""
    import os
    import subprocess
    import sys
    code = ("import synth_inputs as si\n"
            "from paper_1803_01291_amd import hb\n"
            "w = si.small_case(40, 20, 10, seed=5, steps=3)\n"
            "hb.solve_host(w)\n"
            "hb.solve_host(w, flags=hb.HB_PAIRWISE)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, HB_TRACE="1", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=240, cwd=root)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stderr.splitlines() if l.startswith("hb_trace")]
    assert len(lines) == 6
    assert all(l.count(" ms") == 1 for l in lines[:3]) and all(l.count(" ms") == 2 for l in lines[3:])
