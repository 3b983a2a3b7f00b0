"""Host logic of the continuous-batching server and the autotuner, on the
CPU with fake device pools (no GPU): admission by HBM budget and free slots,
continuous admission while others run, per-job accounting, failure
isolation, latency summary, autotune caching."""
import json
import os

import pytest

import workloads as W
from paper_1608_04904_amd import autotune
from paper_1608_04904_amd.serve import Server, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakePool:
    """Stands in for a GPU pool: a tick costs `tick_s` of fake time."""

    def __init__(self, precision, n_slots, clock, tick_s=0.01, fail_seeds=(), barrier_fail=None):
        self.barrier_fail = dict(barrier_fail or {})   # seed -> admissions that time out
        self.admissions = {}
        self.precision = precision
        self.n_slots = n_slots
        self.clock = clock
        self.tick_s = tick_s
        self.slots = {}
        self.log = []
        self.fail_seeds = set(fail_seeds)
        self.max_occupied = 0

    def workspace_bytes(self, p):
        return 100 * int(p["n_solvent"])

    def admit(self, slot, p, seed, n_md):
        assert slot not in self.slots
        k = self.admissions.get(seed, 0)
        self.admissions[seed] = k + 1
        self.slots[slot] = dict(seed=seed, ticks=0, barrier=k < self.barrier_fail.get(seed, 0))
        self.log.append(("admit", slot, seed, self.clock()))
        self.max_occupied = max(self.max_occupied, len(self.slots))

    def retire(self, slot):
        del self.slots[slot]
        self.log.append(("retire", slot, self.clock()))

    def tick(self):
        for s in self.slots.values():
            s["ticks"] += 1
        self.clock.t += self.tick_s

    def observables(self, slot):
        s = self.slots[slot]
        f = (16 if s["seed"] in self.fail_seeds else 0) | (32 if s["barrier"] else 0)
        return dict(flags=f, coll_step=s["ticks"])

    def state(self, slot):
        return dict(ticks=self.slots[slot]["ticks"])


def _job(arr, n, nc, prec=64, seed=0, n_md=10):
    p = W.base_params(L=(8, 8, 8), rho=1, n_md=n_md, precision=prec)
    p["n_solvent"] = n
    return dict(arrival=arr, params=p, seed=seed, n_collide=nc)


def test_admission_respects_budget_and_slots():
    clock = FakeClock()
    pools = {64: FakePool(64, 2, clock), 32: FakePool(32, 4, clock)}
    srv = Server(hbm_budget=100 * 3000, pools=pools, clock=clock)
    jobs = [_job(0.0, 1000, 5, 64, seed=i) for i in range(5)] + \
           [_job(0.0, 1000, 3, 32, seed=10 + i) for i in range(3)]
    res = srv.run(jobs, realtime=True)
    assert len(res) == 8 and all(r.error is None for r in res)
    assert pools[64].max_occupied <= 2
    assert srv.peak_used <= srv.hbm_budget
    assert srv.used == 0
    for r in res:
        assert r.observables["coll_step"] == r.n_collide
        assert r.finished >= r.admitted >= r.arrival


def test_continuous_admission_while_others_run():
    """A job arriving while the only slot is busy is admitted the tick after
    the running job retires, not at the end of a batch."""
    clock = FakeClock()
    pool = FakePool(64, 1, clock, tick_s=0.1)
    srv = Server(hbm_budget=10**9, pools={64: pool}, clock=clock)
    jobs = [_job(0.0, 100, 10, seed=1), _job(0.35, 100, 2, seed=2), _job(0.0, 100, 1, seed=3)]
    res = {r.job_id: r for r in srv.run(jobs, realtime=True)}
    # job 0 runs ticks 0..9 (t = 0 .. 1.0); jobs 2 (t=0) and 1 (t=0.35) wait
    assert res[0].admitted == pytest.approx(0.0)
    assert res[2].admitted == pytest.approx(1.0)
    assert res[1].admitted == pytest.approx(1.1)
    assert res[1].latency == pytest.approx(1.3 - 0.35)


def test_small_job_passes_a_blocked_large_one():
    clock = FakeClock()
    pool = FakePool(64, 4, clock)
    srv = Server(hbm_budget=100 * 1500, pools={64: pool}, clock=clock)
    jobs = [_job(0.0, 1000, 20, seed=1), _job(0.0, 1000, 5, seed=2), _job(0.0, 400, 5, seed=3)]
    res = {r.job_id: r for r in srv.run(jobs, realtime=True)}
    assert res[2].admitted == pytest.approx(0.0)    # fits beside job 0
    assert res[1].admitted > res[2].admitted        # waits for memory


def test_device_failure_is_isolated():
    clock = FakeClock()
    pool = FakePool(64, 4, clock, fail_seeds={7})
    srv = Server(hbm_budget=10**9, pools={64: pool}, clock=clock)
    jobs = [_job(0.0, 100, 3, seed=s) for s in (5, 6, 7, 8)]
    res = {r.job_id: r for r in srv.run(jobs, realtime=True)}
    assert res[2].error is not None
    assert all(res[j].error is None for j in (0, 1, 3))
    s = summarize(list(res.values()))
    assert s["n_jobs"] == 3 and s["errors"] == 1


def test_job_larger_than_budget_is_rejected():
    clock = FakeClock()
    srv = Server(hbm_budget=1000, pools={64: FakePool(64, 2, clock)}, clock=clock)
    with pytest.raises(ValueError):
        srv.run([_job(0.0, 1000, 1)])


def test_summary_percentiles():
    clock = FakeClock()
    pool = FakePool(64, 8, clock, tick_s=0.01)
    srv = Server(hbm_budget=10**9, pools={64: pool}, clock=clock)
    jobs = [_job(0.0, 100, n, seed=n) for n in range(1, 101)]
    res = srv.run(jobs, realtime=False)
    s = summarize(res)
    assert s["n_jobs"] == 100
    assert s["p50_latency_s"] <= s["p99_latency_s"]
    assert s["particle_steps"] == sum(100 * 10 * n for n in range(1, 101))


def test_autotune_caches_best_per_box_class(tmp_path):
    cache = str(tmp_path / "tune.json")
    p = W.dimer_system(L=16, rho=5, n_md=10, seed=1)
    calls = []

    def fake_timer(params, cfg, seed, intervals):
        calls.append(cfg)
        return 1.0 + cfg["chain_k"] + (cfg["collide_cells"] == 32) * -0.5 + (cfg["stream_ppt"] == 1) * 0.1

    best = autotune.tune(p, cache_path=cache, timer=fake_timer)
    assert best == dict(chain_k=1, collide_cells=32, stream_ppt=2)
    npts = 1
    for v in autotune.GRID.values():
        npts *= len(v)
    assert len(calls) == npts
    again = autotune.tune(p, cache_path=cache, timer=fake_timer)
    assert again == best and len(calls) == npts            # cached
    assert autotune.lookup(p, cache_path=cache) == best
    q = W.dimer_system(L=20, rho=5, n_md=10, seed=1)
    assert autotune.box_class(q) != autotune.box_class(p)
    assert autotune.lookup(q, cache_path=cache) == autotune.DEFAULT
    data = json.load(open(cache))
    assert autotune.box_class(p) in data and len(data[autotune.box_class(p)]["points"]) == npts


def test_barrier_timeout_restarts_the_job_once():
    """A job flagged with RMP_FLAG_BARRIER is rerun once from its initial
    state (admitted again, ahead of the queue); a second time-out is
    reported as its error, and the other jobs are unaffected."""
    clock = FakeClock()
    pool = FakePool(64, 2, clock, barrier_fail={1: 1, 2: 2})
    srv = Server(hbm_budget=10**9, pools={64: pool}, clock=clock)
    jobs = [_job(0.0, 1000, 4, 64, seed=i) for i in range(4)]
    res = {r.job_id: r for r in srv.run(jobs, realtime=True)}
    assert len(res) == 4
    assert res[0].error is None and res[0].restarts == 0
    assert res[1].error is None and res[1].restarts == 1
    assert res[1].observables["coll_step"] == 4
    assert res[2].error is not None and "0x20" in res[2].error and res[2].restarts == 1
    assert res[3].error is None
    assert pool.admissions == {0: 1, 1: 2, 2: 2, 3: 1}
    assert srv.used == 0
