"""On-device dimer analysis (directed velocity, centre-of-mass series and
MSD, cylindrical shell species histogram) against the FP64 oracle.

The device takes the same IEEE operations in the same order as the oracle's
definitions (contraction off), on a state that is itself bit-identical to
the oracle's, so series records and MSD values are compared bit for bit and
histogram counts exactly.  FP32 systems: the histogram and record of one
sample are compared with the oracle's evaluation of the same (uploaded)
state, again exactly.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

AN = dict(every=1, series_cap=16, hist_nz=16, hist_nr=8, hist_zmax=6.0, hist_rmax=5.0)


def _rm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_04904_amd as rm
    return rm


def _multi_dimer(L=24, n=3, seed=8):
    p = W.base_params(L=(L, L, L), rho=4, dt=0.01, n_md=10)
    p["bulk_rate"] = 0.02
    W.place_dimers(p, n, np.random.default_rng(seed))
    return p


CASES = {
    "one_dimer": (lambda: W.dimer_system(L=16, rho=5, n_md=20, seed=3, bulk_rate=0.05), AN, [2, 4]),
    "every2_capped": (lambda: W.dimer_system(L=14, rho=6, n_md=10, seed=4, bulk_rate=0.02),
                      dict(AN, every=2, series_cap=2, hist_nz=5, hist_nr=3), [7]),
    "three_dimers": (_multi_dimer, dict(AN, hist_nz=12, hist_nr=6, hist_zmax=7.0, hist_rmax=6.5), [3, 2]),
    "ragged_bins": (lambda: W.scaled(W.dimer_system(L=16, rho=4, n_md=8, seed=9, bulk_rate=0.05),
                                     L=(17, 14, 16)),
                    dict(AN, hist_nz=7, hist_nr=13, hist_zmax=7.3, hist_rmax=6.1), [5]),
}


def _compare(res, acc, what):
    k = len(acc["series"])
    assert res["n_samples"] == k and res["n_dropped"] == acc["n_dropped"], what
    assert res["md_step"].tolist() == acc["md_step"], what
    if k:
        want = np.stack(acc["series"])
        assert np.array_equal(res["series"], want), (
            what, np.argwhere(res["series"] != want)[:4].tolist())
    diff = np.argwhere(res["hist"] != acc["hist"])
    assert diff.size == 0, (what, diff[:4].tolist(), int(res["hist"].sum()), int(acc["hist"].sum()))


@pytest.mark.parametrize("graph", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_analysis_matches_oracle(case, graph):
    rm = _rm()
    make, an, calls = CASES[case]
    p = make()
    n_md = p["n_md"]
    s0 = W.random_state(p, 11, species_B_fraction=0.3, flag_fraction=0.05)
    print(f"[analysis] {case} graph={graph} L={p['L']} N={p['n_solvent']} bonds={len(p['bonds'])} "
          f"an={an} calls={calls}", flush=True)
    g = rm.System(p, 21)
    g.set_tuning(use_graph=graph)
    g.set_state(s0)
    g.analysis_attach(**an)
    o = oracle.Oracle(p, 21, init=False)
    o.set_state(s0)
    acc = None
    for k in calls:
        g.step(n_md, k)
        acc = o.run_analysed(n_md, k, an, acc)
        _compare(g.analysis_read(), acc, case)
    assert g.observables()["flags"] == 0
    # MSD of the stored series, on the device, against the oracle's
    T = len(acc["series"])
    max_lag = an["series_cap"] - 1
    m = g.analysis_msd(max_lag)
    for b in range(len(p["bonds"])):
        R = np.stack([acc["series"][t][b, 0:3] for t in range(T)]) if T else np.zeros((0, 3))
        want = oracle.msd(R, max_lag)
        assert np.array_equal(m[b], want), (b, m[b], want)


def test_reattach_clears_and_detach_stops():
    rm = _rm()
    p = W.dimer_system(L=12, rho=4, n_md=5, seed=5)
    s0 = W.random_state(p, 12, species_B_fraction=0.5)
    g = rm.System(p, 3)
    g.set_state(s0)
    g.analysis_attach(**AN)
    g.step(5, 3)
    r1 = g.analysis_read()
    assert r1["n_samples"] == 3 and r1["hist"].sum() > 0
    g.analysis_attach(**AN)                   # restart: counts cleared
    assert g.analysis_read()["n_samples"] == 0
    g.step(5, 1)
    r2 = g.analysis_read()
    assert r2["n_samples"] == 1 and r2["md_step"].tolist() == [20]
    g.analysis_detach()
    g.step(5, 2)                              # runs without the analysis
    o = oracle.Oracle(p, 3, init=False)
    o.set_state(s0)
    o.run(5, 6)
    assert np.array_equal(g.get_state()["x"], o.get_state()["x"])
    with pytest.raises(rm.RmpError):
        g.analysis_read()
    with pytest.raises(rm.RmpError):
        g.analysis_msd(0)


def test_fp32_sample_matches_oracle_on_the_same_state():
    rm = _rm()
    p = W.dimer_system(L=16, rho=5, n_md=10, seed=7, bulk_rate=0.05, precision=32)
    s0 = W.random_state(p, 13, species_B_fraction=0.3, float32=True)
    g = rm.System(p, 9)
    g.set_state(s0)
    g.step(10, 2)
    g.analysis_attach(**AN)
    g.step(10, 1)
    res = g.analysis_read()
    st = g.get_state()
    p64 = dict(p, precision=64)
    o = oracle.Oracle(p64, 9, init=False)
    o.set_state(st)
    assert np.array_equal(res["series"][0, 0], o.dimer_sample(0))
    assert np.array_equal(res["hist"][0], o.cyl_hist(0, AN["hist_nz"], AN["hist_nr"],
                                                     AN["hist_zmax"], AN["hist_rmax"]))


def test_batch_slot_analysis_equals_alone():
    rm = _rm()
    pa = W.dimer_system(L=16, rho=5, n_md=10, seed=3, bulk_rate=0.05)
    pb = W.dimer_system(L=12, rho=6, n_md=6, seed=4, bulk_rate=0.02)
    sa, sb = W.random_state(pa, 14, species_B_fraction=0.2), W.random_state(pb, 15)
    b = rm.Batch(2, 64)
    b.set_slot(0, pa, 31, 10)
    b.set_slot(1, pb, 32, 6)
    b.set_state(0, sa)
    b.set_state(1, sb)
    b.analysis_attach(1, **AN)
    b.step(4)
    rb = b.analysis_read(1)
    g = rm.System(pb, 32)
    g.set_state(sb)
    g.analysis_attach(**AN)
    g.step(6, 4)
    rg = g.analysis_read()
    assert rb["n_samples"] == rg["n_samples"] == 4
    assert np.array_equal(rb["series"], rg["series"]) and np.array_equal(rb["hist"], rg["hist"])
    assert np.array_equal(b.analysis_msd(1, 3), g.analysis_msd(3))
    with pytest.raises(rm.RmpError):
        b.analysis_read(0)                     # slot 0 has no analysis


def test_bench_workload_three_intervals_match_oracle():
    """The 32^3 dimer at rho = 10 (327,680 particles), 50 MD steps per
    collision, in the launch configuration the benchmark uses."""
    rm = _rm()
    p = W.dimer32()
    an = dict(every=1, series_cap=8, hist_nz=40, hist_nr=20, hist_zmax=10.0, hist_rmax=10.0)
    # the same uploaded state on both sides (the method's own initial
    # velocities use log/cos/sin, whose last bits differ between libraries)
    s0 = W.random_state(p, 16, species_B_fraction=0.2)
    g = rm.System(p, 5)
    g.set_state(s0)
    o = oracle.Oracle(p, 5, init=False)
    o.set_state(s0)
    g.analysis_attach(**an)
    g.step(50, 3)
    acc = o.run_analysed(50, 3, an)
    _compare(g.analysis_read(), acc, "dimer32")
    assert acc["hist"].sum() > 100000
