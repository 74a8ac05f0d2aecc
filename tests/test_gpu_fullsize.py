"""Full-size parity in the launch configuration bench.py times (library
default tiling, whole-step kernel).

* 256^3 x 2000 steps (the benchmark workload): GPU vs oracle reference values
  stored by tests/golden/make_golden.py (an oracle-only script) at sampled
  nodes, relative to the whole-grid max norm; whole-grid max norms and the
  integral of phi via the GPU's FP64 diagnostics.
* 256^3 x 10 steps and x 2000 steps (FP64 and FP32c): every node against
  the oracle run here.
* 512 x 512 x 64 (the benchmark's shard slab) x 10 steps: every node, FP64
  and FP32c, against the oracle run here.
* 512^3 x 1000 steps: FP64 vs the stored oracle samples; FP32c against FP64
  (max and L2 error over the whole grid, and at the samples vs the oracle).
* 64 uneven solves x 500 steps in one batched launch (graph replay, as timed):
  solves 0, 1, 2 vs the stored oracle samples; FP32c batch vs FP64 batch.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_gold(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"reference {name} not generated (tests/golden/make_golden.py)")
    return json.load(open(path))


def gpu_run(hb, w, steps, precision=0):
    p0, p1 = w.initial()
    h = hb.hb_create(hb.config_from_workload(w, precision))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, steps)
        phi, psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, phi, psi)
        d = hb.hb_diagnostics(h)
    finally:
        hb.hb_destroy(h)
    return phi, psi, d


def sampled_error(g, phi, psi):
    pts = np.array(g["points_zyx"])
    idx = (pts[:, 0], pts[:, 1], pts[:, 2])
    num = max(np.max(np.abs(phi[idx] - np.array(g["phi"]))),
              np.max(np.abs(psi[idx] - np.array(g["psi"]))))
    return num / max(g["max_abs_phi"], g["max_abs_psi"])


def test_cube256_2000_steps_vs_oracle_samples(hb):
    g = load_gold("cube256_gauss8_oracle.json")
    w = si.config2()
    assert list(w.n) == g["n"] and w.dt == g["dt"] and w.mu2 == g["mu2"]
    phi, psi, d = gpu_run(hb, w, g["steps"])
    err = sampled_error(g, phi, psi)
    print(f"256^3 x {g['steps']}: sampled relative max-norm error {err:.3e} "
          f"({len(g['points_zyx'])} nodes)")
    assert err <= 1e-12
    assert abs(np.max(np.abs(phi)) - g["max_abs_phi"]) <= 1e-12 * g["max_abs_phi"]
    assert abs(np.max(np.abs(psi)) - g["max_abs_psi"]) <= 1e-12 * g["max_abs_psi"]
    assert d["linf_phi"] == pytest.approx(g["max_abs_phi"], rel=1e-12)
    scale = np.sqrt(g["sum_phi2"] * 8 * 16 ** 3)  # |integral| <= sqrt(V * int phi^2)
    assert abs(d["integral"] - g["integral"]) <= 1e-11 * scale


def test_cube256_2000_steps_fp32c_vs_oracle_samples(hb):
    """The FP32c form of the benchmark workload (its FP32-storage default
    tiling) against the FP64 oracle samples: within 1e-5 relative."""
    g = load_gold("cube256_gauss8_oracle.json")
    w = si.config2()
    phi, psi, d = gpu_run(hb, w, g["steps"], precision=1)
    err = sampled_error(g, phi, psi)
    print(f"256^3 x {g['steps']} FP32c: sampled relative max-norm error {err:.3e}")
    assert err <= 1e-5
    assert d["nonfinite"] == 0


def test_cube256_10_steps_every_node(hb, oracle_mod):
    w = si.config2()
    phi, psi, _ = gpu_run(hb, w, 10)
    r = oracle.solve_workload(w, nsteps=10)
    err = oracle.rel_maxnorm(phi, psi, *r)
    print(f"256^3 x 10 every node: relative max-norm error {err:.3e}")
    assert err <= 1e-12


def test_cube256_2000_steps_every_node(hb, oracle_mod):
    """The benchmark's whole horizon on every node: 2000 steps (t = 10) of
    the benchmark workload in its benchmark tiling, FP64 and FP32c, against
    the oracle run here (3.4e10 point-updates on the host, about 1.5 minutes
    on 16 threads)."""
    w = si.config2()
    print("oracle: 256^3 x 2000 steps on the host", flush=True)
    r = oracle.solve_workload(w, nsteps=2000)
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        phi, psi, _ = gpu_run(hb, w, 2000, precision=prec)
        err = oracle.rel_maxnorm(phi, psi, *r)
        print(f"256^3 x 2000 every node, precision {prec}: relative max-norm error {err:.3e}")
        assert err <= tol


def test_slab512x512x64_10_steps_every_node(hb, oracle_mod):
    """The benchmark's shard leg (one GPU's z-slab of the 512^3 workload, its
    own default tiling: 64 x 11 tiles, 32-plane marches), every node."""
    w = si.slab_config()
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        phi, psi, _ = gpu_run(hb, w, 10, precision=prec)
        if prec == 0:
            r = oracle.solve_workload(w, nsteps=10)
        err = oracle.rel_maxnorm(phi, psi, *r)
        print(f"512x512x64 x 10, precision {prec}, every node: relative max-norm error {err:.3e}")
        assert err <= tol


def test_cube512_fp64_and_fp32c(hb):
    g = load_gold("cube512_cinfbump_oracle.json")
    w = si.config3()
    phi64, psi64, _ = gpu_run(hb, w, g["steps"], precision=0)
    e64 = sampled_error(g, phi64, psi64)
    phi32, psi32, _ = gpu_run(hb, w, g["steps"], precision=1)
    e32 = sampled_error(g, phi32, psi32)
    den = max(np.max(np.abs(phi64)), np.max(np.abs(psi64)))
    dmax = max(np.max(np.abs(phi32 - phi64)), np.max(np.abs(psi32 - psi64))) / den
    vol = 0.125 ** 3
    l2 = np.sqrt(vol * (np.sum((phi32 - phi64) ** 2) + np.sum((psi32 - psi64) ** 2)))
    l2ref = np.sqrt(vol * (np.sum(phi64 ** 2) + np.sum(psi64 ** 2)))
    print(f"512^3 x {g['steps']}: FP64 sampled error {e64:.3e}; FP32c sampled error vs oracle "
          f"{e32:.3e}; FP32c vs FP64 whole grid: max {dmax:.3e}, relative L2 {l2 / l2ref:.3e}")
    assert e64 <= 1e-12
    assert e32 <= 1e-5 and dmax <= 1e-5 and l2 / l2ref <= 1e-5


def test_batch64_500_steps_vs_oracle_samples(hb):
    g = load_gold("batch64_oracle.json")
    ws = si.batch_config()
    steps = ws[0].steps
    outs = {}
    for prec in (0, 1):
        cfgs = [hb.config_from_workload(w, prec, hb.HB_USE_GRAPH) for w in ws]
        b = hb.hb_batch_create(cfgs)
        try:
            for i, w in enumerate(ws):
                hb.hb_batch_set_initial(b, i, w.initial()[0], None)
            hb.hb_batch_step(b, steps)
            for i in g["solves"]:
                p0 = np.empty(ws[i].n[::-1], np.float64)
                phi, psi = np.empty_like(p0), np.empty_like(p0)
                hb.hb_batch_read(b, i, phi, psi)
                outs[(prec, i)] = (phi, psi)
        finally:
            hb.hb_batch_destroy(b)
    for i, rec in zip(g["solves"], g["records"]):
        assert ws[i].name == rec["workload"] and rec["steps"] == steps
        e64 = sampled_error(rec, *outs[(0, i)])
        e32 = sampled_error(rec, *outs[(1, i)])
        print(f"batch solve {i} ({rec['workload']}): FP64 sampled error {e64:.3e}, "
              f"FP32c {e32:.3e}")
        assert e64 <= 1e-12
        assert e32 <= 1e-5
