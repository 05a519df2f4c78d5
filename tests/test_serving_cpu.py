"""Scheduler policy of the serving loop on the CPU: a fake executor with
deterministic costs and results and a virtual clock.  Admission by footprint
never exceeds the budget, oversized and malformed requests fail alone,
requests of one class are served in arrival order, arrivals during a batch
join the next one (continuous batching), and every request completes."""
import math

import numpy as np
import pytest

import workloads as W
from paper_2401_06861_amd.serving import Server, summarize, sv_footprint, dm_footprint


class VClock:
    def __init__(self):
        self.t = 0.0

    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Deterministic stand-in for the GPU executor.  Each SV class (n, L)
    has a context whose per-vector buffers grow to the largest batch it has
    served (as the library's do); `device_bytes()` is what the fake device
    holds now: every live context plus every running DM job."""

    BASE = 1000      # bytes of a context's tables

    def __init__(self, clk, sv_cost=lambda key, b: 1e-3 * (1 + 0.01 * b), dm_cost=lambda n: 2e-3):
        self.clk, self.sv_cost, self.dm_cost = clk, sv_cost, dm_cost
        self.launched = []
        self.cap = {}              # class -> vector capacity of its context
        self.dm_running = {}       # token id -> bytes
        self.released = []

    def footprint(self, r):
        return sv_footprint(r.n) + self.BASE if r.kind == "sv_vqe" else dm_footprint(r.n)

    def validate(self, r):
        if r.n < 1:
            return "bad n"
        return None

    def class_key(self, r):
        return (r.n, r.L)

    def classes(self):
        return list(self.cap)

    def class_bytes(self, key, count):
        self.cap.setdefault(key, 0)
        return self.BASE + max(self.cap[key], count) * sv_footprint(key[0])

    def release(self, key):
        self.released.append(key)
        del self.cap[key]

    def device_bytes(self):
        return sum(self.BASE + c * sv_footprint(k[0]) for k, c in self.cap.items()) + sum(self.dm_running.values())

    def thetas(self, r):
        return W.request_thetas(r, 2 * r.n * r.L)

    def start_sv(self, key, items, want_grad):
        assert key in self.cap, "batch on a released context"
        self.cap[key] = max(self.cap[key], len(items))
        self.launched.append((self.clk.t, key, [r.rid for r, _ in items], want_grad))
        outs = [(float(np.sum(th)) + r.h, np.full(2, r.h) if want_grad else None) for r, th in items]
        return ("sv", self.clk.t + self.sv_cost(key, len(items)), outs)

    def start_dm(self, r):
        tok = ("dm", self.clk.t + self.dm_cost(r.n), {"purity": 1.0 / (1 + r.n)}, len(self.dm_running) + 1e-9 * r.rid)
        self.dm_running[tok[3]] = dm_footprint(r.n)
        return tok

    def ready(self, token):
        return self.clk.t >= token[1]

    def collect(self, token):
        if token[0] == "dm":
            self.dm_running.pop(token[3], None)
        return token[2]

    def drain(self):
        pass


def trace(num=120, rate=400.0, seed=3):
    return W.serving_trace(num=num, rate=rate, seed=seed, sv_n=(4, 9), dm_n=(3, 6), L_range=(1, 3), opt_steps=(1, 4))


def test_all_complete_within_budget():
    clk = VClock()
    ex = FakeExecutor(clk)
    reqs = trace()
    budget = 6 * sv_footprint(9) + 2 * dm_footprint(6)
    peak = []
    srv = Server(ex, budget, clock=clk.clock, sleep=clk.sleep,
                 on_tick=lambda s: peak.append((ex.device_bytes(), s.in_use)))
    res = srv.run(reqs)
    assert all(r.error is None for r in res)
    assert all(r.finished is not None and r.finished >= r.arrival for r in res)
    assert srv.max_in_use <= budget
    # what the (fake) device holds never exceeds the charge, nor the budget
    assert all(dev <= charged <= budget for dev, charged in peak)
    # after the run only the contexts kept for reuse are charged
    assert srv.in_use == sum(ex.class_bytes(k, 0) for k in ex.classes())
    assert len(ex.released) == srv.released
    for q, r in zip(sorted(reqs, key=lambda x: (x.arrival, x.rid)), res):
        assert len(r.outputs) == (q.steps if q.kind == "sv_vqe" else 1)
    s = summarize(res)
    assert s["completed"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0


def test_oversized_and_malformed_fail_alone():
    clk = VClock()
    ex = FakeExecutor(clk)
    reqs = trace(num=40)
    big = W.Request(1000, 0.01, "sv_vqe", 20, L=2, want_grad=True, steps=2, seed=1)     # 2 x 16 x 2^20 B
    bad = W.Request(1001, 0.02, "sv_vqe", 0, L=2, steps=1, seed=2)
    budget = 4 * sv_footprint(9) + dm_footprint(6)
    res = Server(ex, budget, clock=clk.clock, sleep=clk.sleep).run(reqs + [big, bad])
    by = {r.rid: r for r in res}
    assert "exceeds the budget" in by[1000].error
    assert by[1001].error == "bad n"
    assert all(by[q.rid].error is None for q in reqs)


def test_fifo_within_class_and_continuous_batching():
    clk = VClock()
    ex = FakeExecutor(clk, sv_cost=lambda key, b: 5e-3)   # long batches
    reqs = [W.Request(i, 1e-3 * i, "sv_vqe", 5, L=2, want_grad=False, steps=3, seed=i, h=1.0) for i in range(12)]
    res = Server(ex, 1 << 40, clock=clk.clock, sleep=clk.sleep).run(reqs)
    # first launch holds only the first arrival; later arrivals join the next batch
    first = ex.launched[0]
    assert first[2] == [0]
    assert any(len(l[2]) > 1 for l in ex.launched[1:])
    # within the class, no batch serves a request before an earlier admitted one that is still waiting
    seen_first = {}
    for t, key, rids, _ in ex.launched:
        for rid in rids:
            seen_first.setdefault(rid, t)
    order = [seen_first[i] for i in range(12)]
    assert order == sorted(order)
    assert all(r.error is None for r in res)


def test_energy_and_gradient_requests_share_a_class():
    """Energy-only and gradient requests of one (n, L) go into the same
    batches; a batch computes gradients when any member asked, and members
    that did not ask get the energy only."""
    clk = VClock()
    ex = FakeExecutor(clk, sv_cost=lambda key, b: 5e-3)
    reqs = [W.Request(i, 1e-3 * i, "sv_vqe", 6, L=2, want_grad=bool(i % 2), steps=3, seed=i, h=1.0)
            for i in range(10)]
    res = Server(ex, 1 << 40, clock=clk.clock, sleep=clk.sleep).run(reqs)
    assert {k for _, k, _, _ in ex.launched} == {(6, 2)}
    mixed = [l for l in ex.launched if len(l[2]) > 1]
    assert mixed and all(l[3] for l in mixed if any(i % 2 for i in l[2]))
    for r in res:
        assert r.error is None and len(r.outputs) == 3
        for e, g in r.outputs:
            assert (g is not None) == bool(r.rid % 2)


def test_idle_contexts_freed_for_new_classes():
    """With room for about two classes' contexts, a sequence of requests of
    ever new classes is served by freeing idle contexts (least recently used
    first), and the device never holds more than the budget."""
    clk = VClock()
    ex = FakeExecutor(clk, sv_cost=lambda key, b: 1e-3)
    reqs = [W.Request(i, 0.01 * i, "sv_vqe", 8, L=1 + i, want_grad=False, steps=2, seed=i) for i in range(8)]
    budget = 2 * (sv_footprint(8) + FakeExecutor.BASE) + 10
    seen = []
    srv = Server(ex, budget, clock=clk.clock, sleep=clk.sleep, on_tick=lambda s: seen.append(ex.device_bytes()))
    res = srv.run(reqs)
    assert all(r.error is None for r in res)
    assert max(seen) <= budget
    assert ex.released[:2] == [(8, 1), (8, 2)]
    assert len(ex.classes()) <= 2


def test_admission_waits_for_memory_in_arrival_order():
    clk = VClock()
    ex = FakeExecutor(clk, sv_cost=lambda key, b: 1e-2)
    fp = sv_footprint(8, True)
    reqs = [W.Request(i, 0.0 + 1e-4 * i, "sv_vqe", 8, L=1, want_grad=True, steps=2, seed=i) for i in range(6)]
    srv = Server(ex, 2 * fp, clock=clk.clock, sleep=clk.sleep)
    res = srv.run(reqs)
    adm = [r.admitted for r in res]
    assert adm == sorted(adm)
    assert srv.max_in_use <= 2 * fp
    assert all(r.error is None for r in res)
