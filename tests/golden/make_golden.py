"""Write oracle reference values for the full-size parity tests.

Calls only the CPU oracle (oracle/) and the seeded input generators
(synth_inputs/); nothing here touches the GPU path.  For a workload it runs
the FP64 oracle to the given step count and stores:
  * sampled points: the 192 largest |phi| and 192 largest |psi| nodes, 192
    random nodes where |phi| or |psi| exceeds 1e-3 of its maximum, 64
    uniformly random nodes (seeded), with phi and psi at each;
  * whole-grid max |phi|, max |psi| (the relative-norm denominators), and
    h^3 sum phi, h^3 sum phi^2.
Usage:  python tests/golden/make_golden.py cube256 [cube512] [batch]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth_inputs as si  # noqa: E402


def sample_points(phi, psi, seed):
    rng = np.random.default_rng(seed)
    flat_p = np.abs(phi).ravel()
    flat_s = np.abs(psi).ravel()
    pick = set(np.argpartition(flat_p, -192)[-192:].tolist())
    pick |= set(np.argpartition(flat_s, -192)[-192:].tolist())
    active = np.nonzero((flat_p > 1e-3 * flat_p.max()) | (flat_s > 1e-3 * flat_s.max()))[0]
    if active.size:
        pick |= set(rng.choice(active, size=min(192, active.size), replace=False).tolist())
    pick |= set(rng.integers(0, flat_p.size, size=64).tolist())
    idx = np.array(sorted(pick))
    return np.stack(np.unravel_index(idx, phi.shape), axis=1)


def record(w, phi, psi, steps, seconds, seed):
    pts = sample_points(phi, psi, seed)
    vol = w.h[0] * w.h[1] * w.h[2]
    return {
        "workload": w.name, "n": list(w.n), "lo": list(w.lo), "hi": list(w.hi), "mu2": w.mu2,
        "lambda": w.lam, "dt": w.dt, "t0": w.t0, "inv_L2": w.inv_L2, "steps": steps,
        "max_abs_phi": float(np.max(np.abs(phi))), "max_abs_psi": float(np.max(np.abs(psi))),
        "integral": float(vol * np.sum(phi)), "sum_phi2": float(vol * np.sum(phi * phi)),
        "points_zyx": pts.tolist(),
        "phi": [float(phi[tuple(p)]) for p in pts], "psi": [float(psi[tuple(p)]) for p in pts],
        "oracle_seconds": seconds, "oracle_threads": oracle.get_threads(),
    }


def run(w, steps, seed, out):
    t = time.time()
    phi, psi = oracle.solve_workload(w, nsteps=steps)
    rec = record(w, phi, psi, steps, time.time() - t, seed)
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=0)
    print(f"{out}: {w.name} {steps} steps in {rec['oracle_seconds']:.0f} s", flush=True)


def main(which):
    if "cube256" in which:
        run(si.config2(), 2000, 1, "cube256_gauss8_oracle.json")
    if "cube512" in which:
        run(si.config3(), 1000, 2, "cube512_cinfbump_oracle.json")
    if "batch" in which:
        ws = si.batch_config()
        recs = []
        for i in (0, 1, 2):
            t = time.time()
            phi, psi = oracle.solve_workload(ws[i])
            recs.append(record(ws[i], phi, psi, ws[i].steps, time.time() - t, 10 + i))
            print(f"batch solve {i}: {ws[i].name}", flush=True)
        with open(os.path.join(HERE, "batch64_oracle.json"), "w") as f:
            json.dump({"solves": [0, 1, 2], "records": recs}, f, indent=0)


if __name__ == "__main__":
    main(sys.argv[1:] or ["cube256"])
