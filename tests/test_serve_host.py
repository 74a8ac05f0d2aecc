"""Host logic of the serving loop (paper_1803_01291_amd/serve.py), on the CPU:
the hb_pool_* calls are replaced by a small in-process pool with the same
contract (admission by footprint against the budget and by free slots, a step
count per solve, poll / read / release), and time by a fake clock."""
import types

import numpy as np
import pytest

from paper_1803_01291_amd import serve


class FakePool:
    def __init__(self, budget, slots):
        self.budget, self.slots = budget, slots
        self.active = {}          # slot -> [index, bytes, steps left, released?]
        self.max_active = 0
        self.next = 0

    def used(self):
        return sum(v[1] for v in self.active.values())


def install(monkeypatch, clock_box):
    pools = []
    fake = types.SimpleNamespace()

    def create(budget, slots):
        p = FakePool(budget, slots)
        pools.append(p)
        return p

    def admit(p, cfg, phi0, phi1, steps):
        if len(p.active) >= p.slots or p.used() + cfg.bytes > p.budget:
            return None
        s = p.next
        p.next += 1
        p.active[s] = [cfg.index, cfg.bytes, steps]
        p.max_active = max(p.max_active, len(p.active))
        return s

    def advance(p, k):
        clock_box[0] += 0.01 * k           # device time per advance
        for v in p.active.values():
            v[2] = max(0, v[2] - k)

    def stats(p):
        return len(p.active), p.used()

    def poll(p):
        return [s for s, v in sorted(p.active.items()) if v[2] == 0]

    def read(p, s, phi, psi):
        phi[...] = p.active[s][0]
        psi[...] = -p.active[s][0]

    def release(p, s):
        del p.active[s]

    def destroy(p):
        pass

    fake.hb_pool_create, fake.hb_pool_admit, fake.hb_pool_advance = create, admit, advance
    fake.hb_pool_stats, fake.hb_pool_poll, fake.hb_pool_read = stats, poll, read
    fake.hb_pool_release, fake.hb_pool_destroy = release, destroy
    monkeypatch.setattr(serve, "hb", fake)

    def sleep(dt):
        clock_box[0] += max(0.0, dt)

    monkeypatch.setattr(serve.time, "sleep", sleep)
    return pools


def request(i, arrival, nbytes, steps):
    cfg = types.SimpleNamespace(index=i, bytes=nbytes)
    return serve.Request(i, arrival, cfg, steps, np.zeros((2, 2, 2)))


def run(monkeypatch, reqs, budget, slots, lookahead=8, advance_k=5):
    clock = [0.0]
    pools = install(monkeypatch, clock)
    out = serve.serve(reqs, budget_bytes=budget, max_slots=slots, advance_k=advance_k,
                      lookahead=lookahead, clock=lambda: clock[0])
    return out, pools[0]


def test_every_request_completes_with_its_own_result(monkeypatch):
    reqs = [request(i, 0.05 * i, 10, 10 + 5 * i) for i in range(12)]
    out, pool = run(monkeypatch, reqs, budget=30, slots=8)
    assert sorted(c.index for c in out["completions"]) == list(range(12))
    for c in out["completions"]:
        assert np.all(c.phi == c.index) and np.all(c.psi == -c.index)
        assert c.done >= c.admitted >= c.arrival
    assert pool.max_active <= 3                  # 3 x 10 bytes fit the budget
    assert out["max_active"] <= 3
    assert out["p99_latency_s"] >= out["p50_latency_s"] > 0


def test_slot_limit(monkeypatch):
    reqs = [request(i, 0.0, 1, 20) for i in range(10)]
    out, pool = run(monkeypatch, reqs, budget=1000, slots=2)
    assert pool.max_active == 2
    assert len(out["completions"]) == 10


def test_lookahead_lets_small_requests_pass_a_blocked_head(monkeypatch):
    # a long small solve occupies the pool; the big head request waits for
    # the whole budget, the small ones behind it fit alongside and go first
    reqs = [request(0, 0.0, 40, 200), request(1, 0.001, 80, 5)] + \
           [request(i, 0.002, 10, 5) for i in range(2, 6)]
    out, _ = run(monkeypatch, reqs, budget=100, slots=8, lookahead=8)
    order = [c.index for c in sorted(out["completions"], key=lambda c: c.done)]
    assert order.index(1) > max(order.index(i) for i in range(2, 6))
    out_fifo, _ = run(monkeypatch, reqs, budget=100, slots=8, lookahead=1)
    order = [c.index for c in sorted(out_fifo["completions"], key=lambda c: c.admitted)]
    assert order[:2] == [0, 1]                   # strict FIFO: nothing passes the head


def test_request_that_can_never_fit_raises(monkeypatch):
    with pytest.raises(RuntimeError):
        run(monkeypatch, [request(0, 0.0, 500, 5)], budget=100, slots=4)
