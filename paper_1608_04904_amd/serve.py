"""Continuous batching of simulation jobs on one GPU.

Jobs (a parameter set, a seed and a number of collisions) arrive over time.
Each is admitted into a replica slot of the FP32 or FP64 pool as soon as a
slot is free and its workspace fits the HBM budget; its state then stays
resident in device memory until it finishes.  Every tick advances each
occupied slot by one interval (its own n_md MD steps and one collision); the
two pools run on separate streams so their kernels overlap on the device.
Finished jobs are retired between ticks, which frees their slot and memory
for waiting jobs (requests that arrive while others run are admitted as soon
as capacity frees up, not at batch boundaries).

Replicas never interact and every kernel is deterministic, so a job's final
state does not depend on what else shares the batch.

A job whose interval lost an inter-workgroup exchange of the MD chain (the
RMP_FLAG_BARRIER device flag: a bounded wait for other workgroups expired,
so that interval's results are not to be trusted) is restarted once from its
own initial state, which reproduces the run it would have had; only a second
such failure is reported as the job's error.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

FLAG_BARRIER = 32          # rmpmd.h RMP_FLAG_BARRIER
MAX_RESTARTS = 1


@dataclass
class JobResult:
    job_id: int
    precision: int
    n_solvent: int
    n_md: int
    n_collide: int
    arrival: float
    admitted: float = -1.0
    finished: float = -1.0
    observables: dict | None = None
    state: dict | None = None
    error: str | None = None
    restarts: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def particle_steps(self) -> int:
        return self.n_solvent * self.n_md * self.n_collide


class GpuPool:
    """One precision pool: a replica batch on its own stream."""

    def __init__(self, precision: int, n_slots: int, device="cuda:0"):
        import torch
        import paper_1608_04904_amd as rm
        self.precision = precision
        self.stream = torch.cuda.Stream(device=device)
        self.batch = rm.Batch(n_slots, precision=precision, device=device, stream=self.stream)
        self.n_slots = n_slots
        self._rm = rm

    def workspace_bytes(self, params: dict) -> int:
        return self._rm.workspace_bytes(params)

    def admit(self, slot: int, params: dict, seed: int, n_md: int):
        self.batch.set_slot(slot, params, seed, n_md)

    def retire(self, slot: int):
        self.batch.clear_slot(slot)

    def tick(self):
        self.batch.step(1)

    def observables(self, slot: int) -> dict:
        return self.batch.observables(slot, raise_on_flags=False)

    def state(self, slot: int) -> dict:
        return self.batch.get_state(slot)

    def tune(self, **kw):
        self.batch.set_tuning(**kw)

    def synchronize(self):
        self.stream.synchronize()


@dataclass
class _Active:
    res: JobResult
    slot: int
    need: int
    ticks: int = 0


@dataclass
class Server:
    """Admission by HBM budget and free slots, one pool per precision."""
    hbm_budget: int
    pools: dict = field(default_factory=dict)      # precision -> pool
    keep_state: bool = False
    clock: object = time.perf_counter

    def __post_init__(self):
        self.used = 0
        self.active = {p: {} for p in self.pools}   # precision -> slot -> _Active
        self.peak_used = 0

    @classmethod
    def on_gpu(cls, hbm_budget: int, slots_per_pool: int = 32, device="cuda:0",
               precisions=(32, 64), keep_state=False):
        pools = {p: GpuPool(p, slots_per_pool, device) for p in precisions}
        return cls(hbm_budget=hbm_budget, pools=pools, keep_state=keep_state)

    def _free_slot(self, prec):
        used = self.active[prec]
        for s in range(self.pools[prec].n_slots):
            if s not in used:
                return s
        return None

    def _try_admit(self, job, jid, now) -> bool:
        p = job["params"]
        prec = int(p.get("precision", 64))
        pool = self.pools[prec]
        need = pool.workspace_bytes(p)
        if need > self.hbm_budget:
            raise ValueError(f"job {jid} needs {need} bytes, more than the whole budget")
        if self.used + need > self.hbm_budget:
            return False
        slot = self._free_slot(prec)
        if slot is None:
            return False
        res = JobResult(job_id=jid, precision=prec, n_solvent=int(p["n_solvent"]),
                        n_md=int(p["n_md"]), n_collide=int(job["n_collide"]),
                        arrival=float(job["arrival"]) if self._realtime else 0.0,
                        restarts=self._restarts.get(jid, 0))
        pool.admit(slot, p, int(job["seed"]), res.n_md)
        res.admitted = now
        self.active[prec][slot] = _Active(res=res, slot=slot, need=need)
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        return True

    def run(self, jobs, realtime: bool = True, max_wall: float | None = None):
        """Serve a trace.  jobs: dicts with arrival (s), params, seed,
        n_collide.  realtime: arrivals follow the wall clock from the start;
        otherwise every job is available at once (arrival = 0).  Returns the
        JobResults in completion order."""
        self._realtime = realtime
        self._restarts = {}
        order = sorted(range(len(jobs)), key=lambda j: jobs[j]["arrival"])
        pending = deque(order)
        queue: list[int] = []
        done: list[JobResult] = []
        t0 = self.clock()
        while pending or queue or any(self.active[p] for p in self.pools):
            now = self.clock() - t0
            if max_wall is not None and now > max_wall:
                break
            while pending and (not realtime or jobs[pending[0]]["arrival"] <= now):
                queue.append(pending.popleft())
            # first fit over the waiting queue, in arrival order
            still = []
            for jid in queue:
                if not self._try_admit(jobs[jid], jid, now):
                    still.append(jid)
            queue = still
            busy = [p for p in self.pools if self.active[p]]
            if not busy:
                if pending:
                    wait = jobs[pending[0]]["arrival"] - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            for p in busy:
                self.pools[p].tick()
            for p in busy:
                finished = []
                for slot, a in self.active[p].items():
                    a.ticks += 1
                    if a.ticks >= a.res.n_collide:
                        finished.append(slot)
                for slot in finished:
                    a = self.active[p].pop(slot)
                    pool = self.pools[p]
                    restart = False
                    try:
                        a.res.observables = pool.observables(slot)
                        flags = a.res.observables.get("flags", 0)
                        if flags & FLAG_BARRIER and a.res.restarts < MAX_RESTARTS:
                            restart = True
                        elif flags:
                            a.res.error = f"device flags {flags:#x}"
                        if self.keep_state and not restart:
                            a.res.state = pool.state(slot)
                    except Exception as e:        # reported per job; others continue
                        a.res.error = str(e)
                    pool.retire(slot)
                    self.used -= a.need
                    if restart:
                        # rerun from the job's initial state, ahead of the queue
                        self._restarts[a.res.job_id] = a.res.restarts + 1
                        queue.insert(0, a.res.job_id)
                        continue
                    a.res.finished = self.clock() - t0
                    done.append(a.res)
        return done


def summarize(results, makespan: float | None = None) -> dict:
    """p50/p99 completion latency and aggregate throughput of a served trace."""
    import numpy as np
    ok = [r for r in results if r.error is None and r.finished >= 0]
    if not ok:
        return dict(n_jobs=0)
    lat = np.array([r.latency for r in ok])
    steps = sum(r.particle_steps for r in ok)
    end = makespan if makespan is not None else max(r.finished for r in ok)
    start = min(r.arrival for r in ok)
    errs = [(r.job_id, r.error) for r in results if r.error is not None]
    return dict(n_jobs=len(ok), p50_latency_s=float(np.percentile(lat, 50)),
                p99_latency_s=float(np.percentile(lat, 99)),
                mean_latency_s=float(lat.mean()), makespan_s=float(end - start),
                particle_steps=int(steps),
                particle_steps_per_s=float(steps / max(end - start, 1e-9)),
                errors=len(results) - len(ok), error_jobs=errs[:10])
