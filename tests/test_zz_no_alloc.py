"""hb_radial_solve_noalloc: the radial batch for callers that cannot
allocate device memory.  Called through the C ABI with device arrays; its
results must equal hb_radial_solve's on the same solves (bitwise: both run
the same kernels on the same host FP64 c(t) values), on two calls in a row,
the second with a smaller batch, so the second reads a scratch array the
first has filled with other descriptors and tables."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def paper_bump_r(r, R):
    out = np.zeros_like(r)
    m = r < R
    out[m] = np.exp(1.0 / R ** 2 - 1.0 / (R ** 2 - r[m] ** 2))
    return out


def batch(hb, count, seed, steps):
    rng = np.random.default_rng(seed)
    cfgs, p0, p1 = [], [], []
    for i in range(count):
        m = int(rng.integers(1, 1200))
        dr = float(rng.uniform(4e-4, 2e-3))
        dt = float(rng.choice([1e-4, 5e-5]))
        t0 = float(rng.choice([0.0, 0.1]))
        mu2, lam = float(rng.uniform(1, 9)), float(rng.uniform(0.5, 4))
        cfgs.append(hb.make_radial_config(m, dr, mu2, lam, dt, int(steps[i % len(steps)]), t0, 1 / 25))
        r = np.arange(m) * dr
        b = float(rng.uniform(0.5, 2)) * paper_bump_r(r, 0.3 * m * dr)
        p0.append(b)
        p1.append(float(rng.uniform(-6, 0)) * b)
    return cfgs, np.concatenate(p0), np.concatenate(p1)


def noalloc(hb, cfgs, phi, psi):
    """The entry point through the C ABI (the binding only marshals: torch
    device tensors become device pointers)."""
    hb.hb_radial_solve_noalloc(cfgs, phi, psi)


def test_noalloc_equals_allocating_entry_point_twice(hb):
    import torch
    for count, seed, steps in ((300, 1, (700, 1500, 33)), (7, 2, (900, 5))):
        cfgs, p0, p1 = batch(hb, count, seed, steps)
        ref_phi, ref_psi = p0.copy(), p1.copy()
        hb.hb_radial_solve(cfgs, ref_phi, ref_psi)
        phi = torch.from_numpy(p0).cuda()
        psi = torch.from_numpy(p1).cuda()
        noalloc(hb, cfgs, phi, psi)
        np.testing.assert_array_equal(phi.cpu().numpy(), ref_phi)
        np.testing.assert_array_equal(psi.cpu().numpy(), ref_psi)
        print(f"noalloc radial batch of {count} solves: bitwise equal to hb_radial_solve")


def test_noalloc_rejects_oversized_batch(hb):
    """More descriptors than the 8 MiB scratch holds: a clear HB_E_ARG, and
    nothing is launched (the arrays stay as they were)."""
    import torch
    n = 110000   # 80-byte descriptors: 8.8 MB
    cfgs = [hb.make_radial_config(1, 1e-3, 1.0, 1.0, 1e-4, 1, 0.0, 1.0)] * n
    phi = torch.zeros(n, dtype=torch.float64, device="cuda")
    psi = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(hb.HBError) as e:
        noalloc(hb, cfgs, phi, psi)
    assert e.value.code == hb.HB_E_ARG and "scratch" in str(e.value)
    assert float(psi.min()) == 1.0 and float(phi.abs().max()) == 0.0
