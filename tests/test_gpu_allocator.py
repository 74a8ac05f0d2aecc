"""The device-allocator hook (hb_set_allocator): with torch's caching
allocator owning the library's memory, every entry point gives the same bits
as with hipMalloc, every block goes back through the allocator that made it
(also after the hook is removed), and nothing is left allocated."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


class CountingTorchAllocator:
    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}
        self.allocs = 0

    def alloc(self, nbytes, stream):
        p = self.torch.cuda.caching_allocator_alloc(nbytes, self.torch.cuda.current_device(), stream)
        self.live[p] = nbytes
        self.allocs += 1
        return p

    def release(self, ptr, nbytes):
        assert self.live.pop(ptr) == nbytes
        self.torch.cuda.caching_allocator_delete(ptr)


def run_all(hb):
    """Single solve (with diagnostics and the autotuner), a batch, a pool and
    a radial batch; returns their results."""
    out = []
    w = si.small_case(70, 21, 13, seed=16, steps=6)
    p0, p1 = w.initial()
    h = hb.hb_create(hb.config_from_workload(w))
    try:
        hb.hb_set_initial(h, p0, p1)
        hb.hb_step(h, 3)
        hb.hb_autotune(h, 1)
        hb.hb_step(h, 3)
        phi, psi = np.empty_like(p0), np.empty_like(p0)
        hb.hb_read(h, phi, psi)
        out += [phi, psi, np.array(list(hb.hb_diagnostics(h).values()), dtype=float)]
    finally:
        hb.hb_destroy(h)
    ws = [si.small_case(40, 30, 20, seed=5, steps=4), si.small_case(33, 17, 9, seed=6, steps=4)]
    b = hb.hb_batch_create([hb.config_from_workload(x, k) for k, x in enumerate(ws)])
    try:
        for i, x in enumerate(ws):
            hb.hb_batch_set_initial(b, i, *x.initial())
        hb.hb_batch_step(b, 4)
        for i, x in enumerate(ws):
            a = np.empty(x.n[::-1])
            hb.hb_batch_read(b, i, a, None)
            out.append(a)
    finally:
        hb.hb_batch_destroy(b)
    pool = hb.hb_pool_create(1 << 30, 4)
    try:
        slot = hb.hb_pool_admit(pool, hb.config_from_workload(ws[0]), *ws[0].initial(), 5)
        for _ in range(5):
            hb.hb_pool_advance(pool, 1)
        a = np.empty(ws[0].n[::-1])
        hb.hb_pool_read(pool, slot, a, None)
        out.append(a)
        hb.hb_pool_release(pool, slot)
    finally:
        hb.hb_pool_destroy(pool)
    r = np.arange(64) * 0.02
    b0 = np.exp(-r ** 2 / 0.05)
    phi, psi = b0.copy(), -b0
    hb.hb_radial_solve([hb.make_radial_config(64, 0.02, 2.0, 1.0, 1e-3, 50, 0.0, 1 / 25)], phi, psi)
    out += [phi, psi]
    return out


def test_torch_allocator_same_bits_nothing_leaked(hb):
    ref = run_all(hb)
    counting = CountingTorchAllocator()
    hb.hb_set_allocator(counting.alloc, counting.release)
    try:
        got = run_all(hb)
    finally:
        hb.hb_set_allocator()
    assert counting.allocs > 10
    assert counting.live == {}
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)


def test_blocks_return_to_their_allocator(hb):
    """A solver created under the hook and destroyed after the hook is removed
    still returns its blocks to the hook's allocator."""
    counting = CountingTorchAllocator()
    w = si.small_case(24, 24, 24, seed=2, steps=2)
    hb.hb_set_allocator(counting.alloc, counting.release)
    try:
        h = hb.hb_create(hb.config_from_workload(w))
    finally:
        hb.hb_set_allocator()
    try:
        hb.hb_set_initial(h, *w.initial())  # staging now from hipMalloc
        hb.hb_step(h, 2)
        assert counting.live  # the state and table are the hook's
    finally:
        hb.hb_destroy(h)
    assert counting.live == {}


def test_allocator_failure_is_nomem(hb):
    w = si.small_case(24, 24, 24, seed=2, steps=2)
    hb.hb_set_allocator(lambda n, s: 0, lambda p, n: None)
    try:
        with pytest.raises(hb.HBError) as e:
            hb.hb_create(hb.config_from_workload(w))
        assert e.value.code == hb.HB_E_NOMEM
    finally:
        hb.hb_set_allocator()
    h = hb.hb_create(hb.config_from_workload(w))  # hipMalloc again
    hb.hb_destroy(h)
