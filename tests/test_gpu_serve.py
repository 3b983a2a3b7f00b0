"""Served and batched forms on the GPU: a job's result is the same alone and
in a continuously batched mix (bit-identical: replicas never interact and
every kernel is deterministic; FP64 jobs also equal the oracle), per-slot
tuning does not change results, and the autotuner picks a shape from real
timings."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _rm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_04904_amd as rm
    return rm


def _jobs():
    jobs = []
    specs = [(12, 6, 10, 64, "sphere", 4), (16, 5, 7, 32, "dimer", 3), (14, 8, 5, 64, "dimer", 5),
             (12, 5, 10, 32, "sphere", 2), (18, 4, 6, 64, "dimer", 3), (13, 7, 9, 32, "dimer", 4)]
    for j, (L, rho, n_md, prec, kind, ncoll) in enumerate(specs):
        if kind == "dimer":
            p = W.dimer_system(L=L, rho=rho, n_md=n_md, precision=prec, seed=50 + j, bulk_rate=0.04)
        else:
            p = W.base_params(L=(L, L, L), rho=rho, n_md=n_md, precision=prec)
            W.add_colloid(p, (L / 2.0, L / 2.0, L / 2.0), sigma=2.0)
        jobs.append(dict(arrival=0.002 * j, params=p, seed=900 + j, n_collide=ncoll))
    return jobs


def _alone(rm, job):
    s = rm.System(job["params"], job["seed"])
    s.step(job["params"]["n_md"], job["n_collide"])
    return s.get_state()


def test_served_results_equal_alone_results():
    rm = _rm()
    from paper_1608_04904_amd.serve import Server, summarize
    jobs = _jobs()
    srv = Server.on_gpu(hbm_budget=1 << 30, slots_per_pool=3, keep_state=True)
    res = srv.run(jobs, realtime=True)
    assert len(res) == len(jobs)
    assert all(r.error is None for r in res), [r.error for r in res]
    s = summarize(res)
    assert s["n_jobs"] == len(jobs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0
    for r in res:
        job = jobs[r.job_id]
        print(f"[serve] job {r.job_id} precision {r.precision} N={r.n_solvent}", flush=True)
        a = _alone(rm, job)
        for k in ("x", "v", "id", "state", "X", "V"):
            assert np.array_equal(a[k], r.state[k]), (r.job_id, k)
        if r.precision == 64:
            o = oracle.Oracle(job["params"], job["seed"], init=False)
            o.set_state(rm.System(job["params"], job["seed"]).get_state())
            o.run(job["params"]["n_md"], job["n_collide"])
            os_ = o.get_state()
            for k in ("x", "v", "id", "state", "X", "V"):
                assert np.array_equal(os_[k], r.state[k]), (r.job_id, k)


def test_per_slot_tile_size_does_not_change_results():
    rm = _rm()
    ps = [W.dimer_system(L=16, rho=5, n_md=8, seed=60, bulk_rate=0.03),
          W.dimer_system(L=20, rho=5, n_md=6, seed=61, bulk_rate=0.03)]
    outs = []
    for cells in ((0, 0), (8, 64)):
        b = rm.Batch(2, precision=64)
        for i, p in enumerate(ps):
            b.set_slot(i, p, 70 + i, p["n_md"])
            if cells[i]:
                b.set_slot_tuning(i, cells[i])
        b.step(3)
        outs.append([b.get_state(i) for i in range(2)])
    for i in range(2):
        for k in ("x", "v", "id", "state", "X", "V"):
            assert np.array_equal(outs[0][i][k], outs[1][i][k]), (i, k)


def test_autotune_on_device(tmp_path):
    _rm()
    from paper_1608_04904_amd import autotune
    p = W.dimer_system(L=16, rho=5, n_md=10, seed=62)
    best = autotune.tune(p, intervals=3, cache_path=str(tmp_path / "t.json"),
                         grid=dict(chain_k=(1, 2), collide_cells=(16, 32), stream_block=(256,)))
    assert best["chain_k"] in (1, 2) and best["collide_cells"] in (16, 32)
