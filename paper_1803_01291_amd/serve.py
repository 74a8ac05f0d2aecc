"""Continuous-batching request loop over the hb_pool C ABI.

Requests (a configuration, initial data, a step count, an arrival time) are
admitted into the device-resident pool as slots and HBM budget free up; every
admitted solve advances in the same whole-step launches as the others, new
ones join at step boundaries while others are mid-flight, and finished ones
are read back and released.  The loop itself is host orchestration: all
arithmetic runs in libhb's kernels.

Admission is FIFO with a bounded size-aware skip: when the head of the queue
does not fit the unused budget, up to ``lookahead`` later requests that do fit
may go first.  The solves that finished in one advance are read back after
the next advance has been enqueued, so their copies (on the pool's copy
stream) overlap the device's work on the others.  Latency of a request =
completion (its state copied back to the host) - arrival.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import hb


@dataclasses.dataclass
class Request:
    index: int
    arrival: float             # seconds after the start of the run
    cfg: "hb.hb_config"
    steps: int
    phi0: np.ndarray
    phi1: Optional[np.ndarray] = None


@dataclasses.dataclass
class Completion:
    index: int
    arrival: float
    admitted: float
    done: float
    phi: np.ndarray
    psi: np.ndarray
    failed: bool = False       # its state turned non-finite (stopped early)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def serve(requests: List[Request], budget_bytes: int, max_slots: int = 64, advance_k: int = 25,
          lookahead: int = 8, keep_results: bool = True, check_every: int = 0,
          clock: Callable[[], float] = time.perf_counter) -> Dict:
    """Run the request stream to completion; returns completions and stats.
    With ``check_every`` > 0 the pool is checked for non-finite states every
    that many advances; such a solve stops, completes with ``failed`` set,
    and the others continue."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue: collections.deque = collections.deque()
    pool = hb.hb_pool_create(budget_bytes, max_slots)
    inflight: Dict[int, tuple] = {}
    done: List[Completion] = []
    advances = 0
    max_active = 0
    failed_slots = set()
    t0 = clock()
    to_read: List[int] = []  # slots that finished in the previous advance

    def collect(slot):
        r, t_adm = inflight.pop(slot)
        shape = r.phi0.shape
        phi = np.empty(shape, np.float64)
        psi = np.empty(shape, np.float64)
        hb.hb_pool_read(pool, slot, phi, psi)
        hb.hb_pool_release(pool, slot)
        t_done = clock() - t0
        done.append(Completion(r.index, r.arrival, t_adm, t_done,
                               phi if keep_results else None, psi if keep_results else None,
                               failed=slot in failed_slots))
        failed_slots.discard(slot)

    try:
        while pending or queue or inflight:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admission
            tried = 0
            i = 0
            while i < len(queue) and tried < lookahead:
                r = queue[i]
                slot = hb.hb_pool_admit(pool, r.cfg, r.phi0, r.phi1, r.steps)
                tried += 1
                if slot is None:
                    i += 1
                    continue
                inflight[slot] = (r, clock() - t0)
                del queue[i]
            active, _ = hb.hb_pool_stats(pool)
            if active == 0 and not to_read:
                if inflight:  # admitted with nothing to step: collect at once
                    to_read = hb.hb_pool_poll(pool)
                    for slot in to_read:
                        collect(slot)
                    to_read = []
                    continue
                if pending:  # idle: wait for the next arrival
                    time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                    continue
                if queue:
                    raise RuntimeError("a queued request can never fit the pool budget")
                break
            if active:
                hb.hb_pool_advance(pool, advance_k)
                advances += 1
                if check_every and advances % check_every == 0:
                    failed_slots.update(hb.hb_pool_check(pool))
            max_active = max(max_active, active)
            # results of the previous advance are copied out on the pool's copy
            # stream while this advance runs
            for slot in to_read:
                collect(slot)
            to_read = hb.hb_pool_poll(pool)
            if not active:
                for slot in to_read:
                    collect(slot)
                to_read = []
    finally:
        hb.hb_pool_destroy(pool)
    lat = np.array([c.latency for c in done]) if done else np.zeros(1)
    span = max(c.done for c in done) - min(c.arrival for c in done) if done else 0.0
    pts = sum(int(np.prod(r.phi0.shape)) * r.steps for r in requests)
    return {
        "completions": done,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "solves_per_s": len(done) / span if span > 0 else 0.0,
        "pt_updates_per_s": pts / span if span > 0 else 0.0,
        "span_s": span,
        "advances": advances,
        "failed": sum(1 for c in done if c.failed),
        "max_active": max_active,
    }
