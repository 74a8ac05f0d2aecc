"""Benchmark: RK4 grid-point updates/s of the FP64 whole-step kernel.

Workload: 256^3 interior points on [-16,16]^3 (h = 0.125), mu^2 = 2,
lambda = 1, phi0 = 8 seeded Gaussians (seed 0), phi1 = 0, dt = 0.005 (the
2000-step single-solve configuration).  A "step" is one full RK4 step (one
whole-step kernel + the step-counter tick) over the whole grid; inputs are
resident in HBM before timing starts.

Prints ONE JSON line.  Extra objects:
  roofline      -- the whole-step kernel (one launch per RK4 step): its
                   algorithmic bytes, 32 B per interior point (the state slot
                   of every point read once and written once: the floor for
                   a method that reads and writes the state once per step) x
                   points / the kernel's mean duration from HIP events on the
                   solver's stream, against 8 TB/s (frac must stay <= 1).
                   The one-pass-per-stage figure of 152 B/point (19 field
                   passes) is kept as contract_19pass_equiv_GBps: the rate a
                   stage-by-stage design would need to match this kernel;
                   traffic is the PMC-measured bytes per launch and
                   traffic_over_alg its ratio to the 32 B/point;
  cpu_baseline  -- the FP64 CPU oracle on a bounded number of steps of the
                   same grid, on all of this host's cores (OpenMP), with a
                   one-thread run of fewer steps beside it (single_thread);
  forms         -- the same step rate for the FP32c form (same grid);
  hbm_probe     -- the streamed-bandwidth ceiling measured by the library's
                   copy and 5-read/2-write probe kernels;
  batched       -- 64 uneven solves (N ~ U{64..192}^3, 500 steps), one
                   whole-step launch per step and precision over all of them,
                   FP64 and FP32c, tiles from the batch autotuner (default
                   tiles timed beside), vs the same solves run one by one;
  served        -- the first 300 arrivals of a Poisson request stream (50/s,
                   N in {48..384}^3, 200-2000 steps, FP64/FP32c) through the
                   continuous-batching pool: p50/p99 latency and solves/s
                   (offered load is far above capacity, so latency is mostly
                   queueing);
  serve_sweep   -- 12-arrival traces at 0.5, 1, 2, 4 and 8 requests/s: the
                   latency knee;
  shard         -- a 512 x 512 x 64 FP64 slab (one GPU's share of 512^3 over
                   eight), timed like the main leg;
  radial        -- the batched radial parameter sweep (4096 solves) against
                   the FP64 vector peak (the kernel is bound by FP64 issue);
  paper_grid    -- the paper's longest run (section 3, Example 7) at its
                   default grid, 500^3 cells, dt = 1e-4, FP64 and FP32c: step
                   rate and the projected hours to t = 50 (5e5 steps) beside
                   the paper's 27 h;
  precision_c3  -- the precision form's own workload (512^3 C-infinity bump,
                   1000 steps): FP64 and FP32c run times, FP32c against FP64
                   over the grid (max and L2) and both against the oracle's
                   stored sample nodes;
  accuracy      -- after the workload's 2000 steps, FP64 and FP32c: relative
                   max error at the oracle's stored sample nodes, and FP32c
                   against FP64 over the whole grid (max and L2);
  paper_context -- the paper's own K40c rate (context, not a baseline);
  system        -- device name, CUs, HBM, host CPU count and model.
"""
import argparse
import json
import math

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per interior point for each kernel of one RK4 step
# (field passes x element size).  Stage-pair scheme: kernel A (stages 1+2)
# reads Y_phi, Y_psi and writes G1, G2 (4 passes); kernel B (stages 3+4)
# reads Y_phi, Y_psi, G1, G2 and writes Y'_phi, Y'_psi (6 passes); FP32c adds
# the read and write of the two FP32 low parts in kernel B (16 B).
KERNEL_BYTES = {0: [32, 48], 1: [16, 40]}  # stage-pair kernels (HB_PAIRWISE)
# whole-step kernel: Y_phi, Y_psi in, Y'_phi, Y'_psi out (+ FP32c low parts
# read and written: 16 B)
STEP_BYTES = {0: 32, 1: 32}
# the per-stage (19-pass) scheme: 3, 4, 5, 7 passes; FP32c + 16 B in stage 4
STAGEWISE_BYTES = {0: [24, 32, 40, 56], 1: [12, 16, 20, 44]}

# HBM bytes per launch of the FP64 whole-step kernel on the 256^3 workload,
# from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs (profiles/
# step_kernel_cube256.md), each scaled by the counter's reading for the plain
# copy probe of known size (FETCH x 2.0, WRITE x 1.0).  Valid only for the
# kernel and runtime code they were measured on (the runtime picks the
# tiling; source_sha() below); any other code reports null.
TRAFFIC_SOURCE_SHA = "23bf8311d98de432"
TRAFFIC_KERNEL = "step_kernel<double, false, 36, 20, false>"  # the 256^3 default region shape
TRAFFIC_BYTES_F64 = 562.8 * 2 ** 20


def source_sha():
    """Hash of the code that decides the whole-step kernel's traffic: the
    kernels and the runtime that tiles them, with comments and whitespace
    taken out (a comment edit does not invalidate a measurement; any code
    edit does)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("hb_kernels.hip", "hb_runtime.cpp", "hb_internal.h"):
        text = open(os.path.join(ROOT, "paper_1803_01291_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


class GpuRun:
    """Timings of one single-solve leg: `elapsed` (s, host clock around the
    timed steps), `region_ms` (ms per step from HIP events recorded on the
    solver's stream before and after the timed steps: with one launch per
    step, the average launch duration over the timed region), `stage_ms`
    (mean per-kernel device time of separately timed single-step launches),
    `diag`, and the ms per step of the repeat runs."""

    def __init__(self, elapsed, region_ms, stage_ms, diag, rep_ms):
        self.elapsed, self.region_ms, self.stage_ms = elapsed, region_ms, stage_ms
        self.diag, self.rep_ms = diag, rep_ms


def run_gpu(w, precision, steps, warmup, timed_stage_steps, flags=0, repeats=None):
    """Time `steps` RK4 steps after `warmup` on a stream of torch's (so HIP
    events can bracket them on the stream the kernels run on), then the
    per-kernel device time of `timed_stage_steps` single-step launches.  With
    repeats = (r, k), r further timed runs of k steps each follow the timed
    steps."""
    import numpy as np
    import torch
    from paper_1803_01291_amd import hb

    p0, p1 = w.initial()
    stream = torch.cuda.Stream()  # default priority
    h = hb.hb_create(hb.config_from_workload(w, precision, flags, stream=stream.cuda_stream))
    rep_ms = []
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, warmup)
        hb.hb_sync(h)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        hb.hb_step(h, steps)
        e1.record(stream)
        hb.hb_sync(h)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        region_ms = e0.elapsed_time(e1) / steps
        if repeats:
            r, k = repeats
            for _ in range(r):
                t1 = time.perf_counter()
                hb.hb_step(h, k)
                hb.hb_sync(h)
                rep_ms.append((time.perf_counter() - t1) * 1e3 / k)
        stage_ms = hb.hb_step_timed(h, timed_stage_steps)
        d = hb.hb_diagnostics(h, allow_nonfinite=True)
    finally:
        hb.hb_destroy(h)
    return GpuRun(elapsed, region_ms, [m / timed_stage_steps for m in stage_ms], d, rep_ms)


def run_batch(count, steps, warmup, tune_steps=3):
    """64 uneven solves (N ~ U{64..192}^3) advanced together: one whole-step
    launch per step and precision over a tile table spanning all solves, hipGraph
    replay of 16-step chunks, tiles chosen by the library's autotuner
    (hb_batch_autotune; the default tiles are timed first, for comparison).
    Baseline: the same solves one after another through the single-solve path
    (also graph-replayed), same GPU."""
    import torch
    import synth_inputs as si
    from paper_1803_01291_amd import hb
    ws = si.batch_config(count=count, steps=steps)
    data = [w.initial()[0] for w in ws]
    pts = sum(w.points for w in ws)
    out = {"solves": count, "steps": steps, "grid_points": pts,
           "sizes": [w.n[0] for w in ws]}
    for prec, name in ((0, "f64"), (1, "f32c")):
        cfgs = [hb.config_from_workload(w, prec, hb.HB_USE_GRAPH) for w in ws]
        b = hb.hb_batch_create(cfgs)
        try:
            for i in range(count):
                hb.hb_batch_set_initial(b, i, data[i], None)
            hb.hb_batch_step(b, warmup)
            hb.hb_batch_sync(b)
            t0 = time.perf_counter()
            hb.hb_batch_step(b, steps)
            hb.hb_batch_sync(b)
            tdef = time.perf_counter() - t0
            # the library's autotuner picks this group's tiles (states are
            # restored), then the same number of steps is timed again
            choice = hb.hb_batch_autotune(b, tune_steps)[prec]
            hb.hb_batch_step(b, warmup)
            hb.hb_batch_sync(b)
            t0 = time.perf_counter()
            hb.hb_batch_step(b, steps)
            hb.hb_batch_sync(b)
            tb = time.perf_counter() - t0
        finally:
            hb.hb_batch_destroy(b)
        handles = []
        try:
            for i, w in enumerate(ws):
                h = hb.hb_create(hb.config_from_workload(w, prec, hb.HB_USE_GRAPH))
                handles.append(h)
                hb.hb_set_initial(h, data[i], None)
                hb.hb_step(h, warmup)
                hb.hb_sync(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for h in handles:
                hb.hb_step(h, steps)
                hb.hb_sync(h)
            ts = time.perf_counter() - t0
        finally:
            for h in handles:
                hb.hb_destroy(h)
        out[name] = {"seconds": tb, "solves_per_s": count / tb, "pt_updates_per_s": pts * steps / tb,
                     "tiles": {"by": choice[0], "zc": choice[1], "chosen_by": "hb_batch_autotune"},
                     "default_tiles_seconds": tdef, "tuned_speedup_vs_default": tdef / tb,
                     "sequential_seconds": ts, "speedup_vs_sequential": ts / tb}
    out["f32c_speedup_vs_f64"] = out["f64"]["seconds"] / out["f32c"]["seconds"]
    return out


def run_serve(count, rate, budget_gb):
    """Poisson stream of parameter-sweep requests through the continuous-
    batching pool; payloads (phi0) are generated before the clock starts."""
    import synth_inputs as si
    from paper_1803_01291_amd import hb, serve
    trace = si.serving_trace(count=count, rate=rate)
    reqs = []
    for r in trace:
        prec = hb.HB_F64 if r.precision == "f64" else hb.HB_F32C
        reqs.append(serve.Request(r.index, r.arrival, hb.config_from_workload(r.workload, prec),
                                  r.workload.steps, r.workload.phi0(), None))
    res = serve.serve(reqs, budget_bytes=int(budget_gb * (1 << 30)), max_slots=64, advance_k=25,
                      keep_results=False)
    offered = sum(int(np.prod(q.phi0.shape)) * q.steps for q in reqs) / max(trace[-1].arrival, 1e-9)
    return {"requests": count, "rate_per_s": rate, "budget_GiB": budget_gb,
            "p50_latency_s": res["p50_latency_s"], "p99_latency_s": res["p99_latency_s"],
            "solves_per_s": res["solves_per_s"], "pt_updates_per_s": res["pt_updates_per_s"],
            "offered_pt_updates_per_s": offered, "max_active": res["max_active"],
            "span_s": res["span_s"]}


def run_shard(steps, warmup):
    """One GPU's share of the 512^3 workload under an 8-way z-slab split:
    512 x 512 x 64 (FP64), timed like the main leg; the slab's own zero halo
    stands in for the planes a neighbour would send."""
    import synth_inputs as si
    sw = si.slab_config(steps)
    g = run_gpu(sw, 0, steps, warmup, 20)
    return {"grid": [512, 512, 64], "steps": steps,
            "pt_updates_per_s": sw.points * steps / g.elapsed,
            "ms_per_step": g.elapsed / steps * 1e3, "kernel_ms": g.region_ms,
            "kernel_ms_single": sum(g.stage_ms),
            "GBps": STEP_BYTES[0] * sw.points / (g.region_ms * 1e-3) / 1e9,
            "frac": STEP_BYTES[0] * sw.points / (g.region_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def run_precision_c3(steps):
    """The precision form on its own workload: 512^3 on [-32,32]^3, the
    C-infinity bump (A = 0.8, R = 10), mu^2 = 2, lambda = 1, dt = 0.005,
    `steps` steps from the initial data, FP64 and FP32c on the GPU.  Reports
    each run's time and, after the last step, the FP32c error against FP64
    over the whole grid (state-vector relative max norm and relative L2) and
    both against the oracle's values at the nodes stored by
    tests/golden/make_golden.py (when the stored run has this many steps)."""
    import torch
    import synth_inputs as si
    from paper_1803_01291_amd import hb
    w = si.config3(steps=steps)
    p0, p1 = w.initial()
    dev = torch.device("cuda")
    out = {"grid": list(w.n), "steps": steps, "dt": w.dt}
    st = {}
    for prec, name in ((0, "f64"), (1, "f32c")):
        h = hb.hb_create(hb.config_from_workload(w, prec))
        try:
            hb.hb_set_initial(h, p0, p1)
            hb.hb_sync(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hb.hb_step(h, steps)
            hb.hb_sync(h)
            el = time.perf_counter() - t0
            phi = torch.empty(tuple(w.n[::-1]), dtype=torch.float64, device=dev)
            psi = torch.empty_like(phi)
            hb.hb_read(h, phi, psi)
        finally:
            hb.hb_destroy(h)
        st[name] = (phi, psi)
        out[name] = {"seconds": el, "ms_per_step": el / steps * 1e3,
                     "pt_updates_per_s": w.points * steps / el}
    out["f32c_speedup_vs_f64"] = out["f64"]["seconds"] / out["f32c"]["seconds"]
    (a, b), (c, d) = st["f64"], st["f32c"]
    den = max(a.abs().max().item(), b.abs().max().item())
    out["f32c_vs_f64_rel_max"] = max((c - a).abs().max().item(), (d - b).abs().max().item()) / den
    out["f32c_vs_f64_rel_l2"] = (math.sqrt(((c - a) ** 2).sum().item() + ((d - b) ** 2).sum().item())
                                 / math.sqrt((a ** 2).sum().item() + (b ** 2).sum().item()))
    path = os.path.join(ROOT, "tests", "golden", "cube512_cinfbump_oracle.json")
    if os.path.exists(path):
        g = json.load(open(path))
        if g["steps"] == steps and list(w.n) == g["n"]:
            pts = torch.tensor(g["points_zyx"], device=dev)
            gp = torch.tensor(g["phi"], dtype=torch.float64, device=dev)
            gs = torch.tensor(g["psi"], dtype=torch.float64, device=dev)
            gden = max(g["max_abs_phi"], g["max_abs_psi"])
            for name, (p, q) in st.items():
                vp = p[pts[:, 0], pts[:, 1], pts[:, 2]]
                vq = q[pts[:, 0], pts[:, 1], pts[:, 2]]
                out[name]["vs_oracle_sampled_rel_max"] = max((vp - gp).abs().max().item(),
                                                             (vq - gs).abs().max().item()) / gden
            out["oracle_nodes"] = len(g["points_zyx"])
            # the oracle's own run of this workload (the one that stored the
            # samples), timed by tests/golden/make_golden.py on its host
            if "oracle_seconds" in g:
                out["oracle_run"] = {"seconds": g["oracle_seconds"], "threads": g.get("oracle_threads"),
                                     "pt_updates_per_s": w.points * steps / g["oracle_seconds"]}
    return out


def run_paper_grid(steps, warmup):
    """The paper's longest run at its default grid: Example 7 on 500^3 cells
    of the unit box, dt = 1e-4 (section 3), FP64 and FP32c, `steps` steps
    timed like the main leg.  The hours to t = 50 (5e5 steps) are projected
    from the measured step time, beside the paper's 27 h on one Tesla K40c."""
    import synth_inputs as si
    w = si.example7_config(500, steps)
    out = {"grid": list(w.n), "dt": w.dt, "steps": steps, "paper_hours_to_t50": 27.0}
    for prec, name in ((0, "f64"), (1, "f32c")):
        g = run_gpu(w, prec, steps, warmup, 10)
        ms = g.elapsed / steps * 1e3
        out[name] = {"pt_updates_per_s": w.points * steps / g.elapsed, "ms_per_step": ms,
                     "kernel_ms": g.region_ms, "kernel_ms_single": sum(g.stage_ms),
                     "projected_hours_to_t50": 5e5 * ms / 3.6e6,
                     "nonfinite": g.diag["nonfinite"]}
    return out


# radial batch kernel: FP64 arithmetic per node-step of the kernel's main
# loop (gfx950 code of radial_kernel<4>: 266 multiplies, 260 adds and 64
# fused multiply-adds per thread and step for 4 nodes), as flops (a fused
# multiply-add counts 2) and as instructions (each occupies a SIMD lane for
# one of the issue slots behind the 78.6 TFLOP/s FP64 vector peak: 256 CUs x
# 64 lanes x 2.4 GHz = 39.3e12 operations/s)
RADIAL_FLOPS_PER_NODE_STEP = (266 + 260 + 2 * 64) / 4
RADIAL_FP64_OPS_PER_NODE_STEP = (266 + 260 + 64) / 4
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP64_OPS_PEAK = 256 * 64 * 2.4e9


def run_radial(count, m, steps, cpu_sample):
    """A radial parameter sweep (section 2.2 form): `count` solves of `m`
    nodes advanced `steps` RK4 steps in one launch, state resident in HBM;
    the radial oracle timed on `cpu_sample` of the same solves."""
    import torch
    import synth_inputs as si
    from paper_1803_01291_amd import hb
    dr, dt, inv_L2 = 5e-4, 1e-4, 1 / 25
    phi0, phi1, params = si.radial_sweep(count, m, dr)
    cfgs = [hb.make_radial_config(m, dr, mu2, lam, dt, steps, 0.0, inv_L2) for mu2, lam in params]
    dev = torch.device("cuda")
    phi = torch.from_numpy(phi0).to(dev)
    psi = torch.from_numpy(phi1).to(dev)
    warm = [hb.make_radial_config(m, dr, mu2, lam, dt, 10, 0.0, inv_L2) for mu2, lam in params]
    hb.hb_radial_solve(warm, phi.clone(), psi.clone())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hb.hb_radial_solve(cfgs, phi, psi)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    node_steps = count * m * steps
    rate = node_steps / sec
    achieved = RADIAL_FLOPS_PER_NODE_STEP * rate / 1e12
    cpu = None
    if cpu_sample > 0:
        from oracle.radial import radial_solve
        t1 = time.perf_counter()
        for i in range(cpu_sample):
            mu2, lam = params[i]
            radial_solve(phi0[i * m:(i + 1) * m], phi1[i * m:(i + 1) * m], dr, mu2, lam, dt,
                         steps, t0=0.0, inv_L2=inv_L2)
        cpu_sec = time.perf_counter() - t1
        cpu = {"value": cpu_sample * m * steps / cpu_sec, "unit": "node-updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{cpu_sample} of the solves, NumPy radial oracle, {cpu_sec:.1f} s"}
    return {"solves": count, "nodes": m, "steps": steps, "seconds": sec,
            "solves_per_s": count / sec, "node_updates_per_s": rate,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                         "flops_per_node_step": RADIAL_FLOPS_PER_NODE_STEP,
                         "fp64_ops_per_node_step": RADIAL_FP64_OPS_PER_NODE_STEP,
                         "issue_frac": RADIAL_FP64_OPS_PER_NODE_STEP * rate / FP64_OPS_PEAK},
            "cpu_baseline": cpu}


def system_info():
    """The device and host the run used."""
    import torch
    p = torch.cuda.get_device_properties(0)
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"device": p.name, "arch": getattr(p, "gcnArchName", ""), "cus": p.multi_processor_count,
            "hbm_GiB": round(p.total_memory / 2 ** 30, 1), "host_cpus": os.cpu_count(), "host_cpu": cpu}


def run_accuracy(w):
    """Errors of the benchmark workload after its 2000 steps, FP64 and FP32c
    from the same initial data: against the oracle's values at the sampled
    nodes stored by tests/golden/make_golden.py (relative to the oracle's
    whole-grid max norm), and FP32c against FP64 over the whole grid (max
    and L2, relative)."""
    import numpy as np
    from paper_1803_01291_amd import hb
    path = os.path.join(ROOT, "tests", "golden", "cube256_gauss8_oracle.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    if list(w.n) != g["n"] or w.dt != g["dt"] or w.mu2 != g["mu2"]:
        return None
    steps = g["steps"]
    p0, p1 = w.initial()
    out = {}
    for prec in (0, 1):
        h = hb.hb_create(hb.config_from_workload(w, prec))
        try:
            hb.hb_set_initial(h, p0, p1)
            hb.hb_step(h, steps)
            phi, psi = np.empty_like(p0), np.empty_like(p0)
            hb.hb_read(h, phi, psi)
        finally:
            hb.hb_destroy(h)
        out[prec] = (phi, psi)
    pts = np.array(g["points_zyx"])
    idx = (pts[:, 0], pts[:, 1], pts[:, 2])
    den = max(g["max_abs_phi"], g["max_abs_psi"])

    def sampled(phi, psi):
        return max(np.max(np.abs(phi[idx] - np.array(g["phi"]))),
                   np.max(np.abs(psi[idx] - np.array(g["psi"])))) / den

    (a, b), (c, d) = out[0], out[1]
    den64 = max(np.max(np.abs(a)), np.max(np.abs(b)))
    l2 = np.sqrt(np.sum((c - a) ** 2) + np.sum((d - b) ** 2))
    l2ref = np.sqrt(np.sum(a ** 2) + np.sum(b ** 2))
    return {"steps": steps, "oracle_nodes": len(pts),
            "f64_vs_oracle_sampled_rel_max": float(sampled(a, b)),
            "f32c_vs_oracle_sampled_rel_max": float(sampled(c, d)),
            "f32c_vs_f64_rel_max": float(max(np.max(np.abs(c - a)), np.max(np.abs(d - b))) / den64),
            "f32c_vs_f64_rel_l2": float(l2 / l2ref)}


def cpu_baseline(w, steps, steps_1t):
    """The FP64 C oracle on `steps` RK4 steps of the workload's grid on all
    host threads (OpenMP over z-planes), and on `steps_1t` steps with one
    thread; its results do not depend on the thread count."""
    import oracle
    p0, p1 = w.initial()
    nthr = oracle.get_threads()
    t0 = time.perf_counter()
    oracle.solve(p0, p1, w.h, w.mu2, w.lam, w.dt, steps, t0=w.t0, inv_L2=w.inv_L2)
    dt = time.perf_counter() - t0
    out = {"value": w.points * steps / dt, "unit": "grid-point-updates/s",
           "cores": nthr, "kind": "oracle",
           "sample": f"{steps} RK4 steps of the same {w.n[0]}^3 grid (FP64 C oracle, OpenMP, "
                     f"{nthr} threads), {dt:.1f} s"}
    if steps_1t > 0:
        oracle.set_threads(1)
        try:
            t0 = time.perf_counter()
            oracle.solve(p0, p1, w.h, w.mu2, w.lam, w.dt, steps_1t, t0=w.t0, inv_L2=w.inv_L2)
            d1 = time.perf_counter() - t0
        finally:
            oracle.set_threads(nthr)
        out["single_thread"] = {"value": w.points * steps_1t / d1, "cores": 1,
                                "sample": f"{steps_1t} RK4 steps of the same grid, one thread, "
                                          f"{d1:.1f} s"}
    return out


def progress(leg):
    """One line on stderr as each leg starts (the JSON line stays alone on stdout)."""
    print(f"bench: {leg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--stage-steps", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--cpu-steps-1t", type=int, default=20,
                    help="steps of the one-thread oracle run (0 skips it)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-count", type=int, default=300,
                    help="arrivals of the served leg's trace (the first N of the 50/s stream)")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-sweep", type=str, default="0.5,1,2,4,8",
                    help="comma-separated arrival rates (req/s): a trace of --serve-sweep-count "
                         "arrivals at each (the latency knee); empty to skip")
    ap.add_argument("--serve-sweep-count", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-radial", action="store_true")
    ap.add_argument("--no-shard", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the error check of the workload against the stored oracle samples")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the precision form's own workload (512^3, 1000 steps, FP64 vs FP32c)")
    ap.add_argument("--c3-steps", type=int, default=1000)
    ap.add_argument("--no-paper-grid", action="store_true",
                    help="skip the paper's default-grid leg (Example 7, 500^3, dt 1e-4)")
    ap.add_argument("--scheme", choices=("step", "pairs", "stages"), default="step",
                    help="3-D scheme of the single-solve legs: the whole-step kernel (default) "
                         "or, for comparison, the stage-pair or per-stage kernels")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of the main leg after the timed steps (median and min reported)")
    ap.add_argument("--repeat-steps", type=int, default=200)
    ap.add_argument("--radial-count", type=int, default=4096)
    ap.add_argument("--radial-steps", type=int, default=2000)
    ap.add_argument("--forms", action="store_true", help="(on by default)")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32c form of the main leg")
    ap.add_argument("--probe", action="store_true", help="(on by default)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the streamed-HBM ceiling (copy and 5-read/2-write probes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import synth_inputs as si
    w = si.config2(n=args.n)
    N = w.points
    from paper_1803_01291_amd import hb as _hb
    flags = {"step": 0, "pairs": _hb.HB_PAIRWISE, "stages": _hb.HB_STAGEWISE}[args.scheme]
    g = run_gpu(w, 0, args.steps, args.warmup, args.stage_steps, flags,
                repeats=(args.repeats, args.repeat_steps))
    elapsed, diag, rep_ms = g.elapsed, g.diag, g.rep_ms
    # the dominant kernel's average launch duration: HIP events on the
    # solver's stream around the timed steps, one launch per step (the
    # comparison schemes: their kernels summed over the step); the
    # separately timed single launches are reported beside it
    kernel_ms = g.region_ms
    kernel_ms_single = sum(g.stage_ms)
    rate = N * args.steps / elapsed
    # algorithmic bytes per launch of the timed scheme: the whole-step kernel
    # reads and writes each point's 16-byte state slot once (32 B/point), the
    # stage-pair kernels move 80 B, the per-stage kernels 152 B
    own_b = {"step": STEP_BYTES[0], "pairs": 80, "stages": sum(STAGEWISE_BYTES[0])}[args.scheme]
    achieved = own_b * N / (kernel_ms * 1e-3) / 1e9
    frac = achieved / HBM_PEAK_GBS
    if not frac <= 1.0:
        raise SystemExit(f"roofline fraction {frac:.3f} > 1: the kernel time or the byte count is wrong")
    # the one-pass-per-stage contract (152 B FP64 = 19 field passes) priced on
    # the same kernel time: the rate a stage-by-stage design would need
    contract = sum(STAGEWISE_BYTES[0]) * N / (kernel_ms * 1e-3) / 1e9
    traffic = (TRAFFIC_BYTES_F64 if source_sha() == TRAFFIC_SOURCE_SHA and args.n == 256
               and args.scheme == "step" else None)
    out = {
        "metric": "RK4 grid-point updates/s + % HBM roofline; batched solves/s, p50/p99 latency",
        "value": rate,
        "unit": "grid-point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single solve {args.n}^3 on [-16,16]^3, mu^2=2, lambda=1, "
                               f"8 seeded Gaussians, dt=0.005, FP64",
                   "grid": [args.n] * 3, "dt": w.dt, "precision": "f64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": frac, "traffic": traffic,
                     "traffic_over_alg": traffic / (own_b * N) if traffic else None,
                     # the kernel and sources the traffic was measured on
                     # (profiles/step_kernel_cube256.md); null traffic otherwise
                     "traffic_kernel": TRAFFIC_KERNEL, "source_sha": source_sha(),
                     "kernel": {"step": "step_kernel (whole RK4 step)",
                                "pairs": "pair_kernel x 2 (sum per step)",
                                "stages": "stage_kernel x 4 (sum per step)"}[args.scheme],
                     "kernel_ms": kernel_ms, "kernel_ms_timing": "HIP events around the timed steps",
                     "kernel_ms_single": kernel_ms_single,
                     "bytes_per_point": own_b,
                     "contract_19pass_bytes_per_point": sum(STAGEWISE_BYTES[0]),
                     "contract_19pass_equiv_GBps": contract,
                     "step_frac": own_b * N / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS},
        "state_check": {"linf_phi": diag["linf_phi"], "nonfinite": diag["nonfinite"]},
        # the same solve timed again in short runs after the timed region:
        # the spread of ms per step on this device (not part of `value`)
        "repeats": ({"runs": len(rep_ms), "steps_each": args.repeat_steps, "ms_per_step": rep_ms,
                     "median_ms": sorted(rep_ms)[len(rep_ms) // 2], "min_ms": min(rep_ms)}
                    if rep_ms else None),
        # the paper's only timing (section 2.1): 27 h to reach t = 50 on one
        # Tesla K40c, with the default grid and step of section 3 (500^3
        # points, dt 1e-4: 5e5 RK4 steps), i.e. about 6.4e8 point-updates/s;
        # another machine and workload, quoted as context only
        "paper_context": {"value": 500 ** 3 * 5e5 / (27 * 3600.0), "unit": "grid-point-updates/s",
                          "hardware": "1x Tesla K40c (CUDA Fortran)",
                          "workload": "500^3, dt 1e-4, 5e5 steps to t = 50 (27 h)",
                          "f64_over_f32_time": 1.8},
    }
    if not args.no_forms:
        progress("forms")
        g32 = run_gpu(w, 1, args.steps, args.warmup, args.stage_steps, flags)
        e32, k32 = g32.elapsed, g32.region_ms
        out["forms"] = {"f32c": {"value": N * args.steps / e32, "speedup_vs_f64": elapsed / e32,
                                 "kernel_ms": k32, "kernel_ms_single": sum(g32.stage_ms),
                                 "GBps": STEP_BYTES[1] * N / (k32 * 1e-3) / 1e9,
                                 "frac": STEP_BYTES[1] * N / (k32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "contract_19pass_equiv_GBps":
                                     sum(STAGEWISE_BYTES[1]) * N / (k32 * 1e-3) / 1e9}}
    if not args.no_probe:
        progress("hbm_probe")
        from paper_1803_01291_amd import hb
        gib = 1 << 30
        copy = hb.hb_probe_bandwidth(0, gib, 20)
        out["hbm_probe"] = {"copy_GBps": copy,
                            "read5_write2_GBps": hb.hb_probe_bandwidth(2, gib // 2, 20),
                            "bytes_per_array": [gib, gib // 2]}
        # the kernel's own bytes against the measured streaming ceiling
        out["roofline"]["frac_of_copy"] = achieved / copy
    if not args.no_batch:
        progress("batched")
        out["batched"] = run_batch(args.batch_count, args.batch_steps, 16)
    if not args.no_serve:
        progress("served")
        out["served"] = run_serve(args.serve_count, args.serve_rate, 192.0)
    if args.serve_sweep:
        progress("serve_sweep")
        out["serve_sweep"] = []
        for rate in (float(r) for r in args.serve_sweep.split(",")):
            out["serve_sweep"].append(run_serve(args.serve_sweep_count, rate, 192.0))
            r = out["serve_sweep"][-1]
            print(f"serve sweep: {rate} req/s: p50 {r['p50_latency_s']:.3f} s, "
                  f"p99 {r['p99_latency_s']:.3f} s, {r['solves_per_s']:.2f} solves/s",
                  file=sys.stderr, flush=True)
    out["system"] = system_info()
    if not args.no_accuracy and args.n == 256:
        progress("accuracy")
        out["accuracy"] = run_accuracy(w)
    if not args.no_shard:
        progress("shard")
        out["shard"] = run_shard(200, 10)
    if not args.no_c3:
        progress("precision_c3")
        out["precision_c3"] = run_precision_c3(args.c3_steps)
    if not args.no_paper_grid:
        progress("paper_grid")
        out["paper_grid"] = run_paper_grid(200, 10)
    if not args.no_radial:
        progress("radial")
        out["radial"] = run_radial(args.radial_count, 1000, args.radial_steps,
                                   0 if args.no_cpu else 4)
    if not args.no_cpu:
        progress("cpu_baseline")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, args.cpu_steps_1t)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
