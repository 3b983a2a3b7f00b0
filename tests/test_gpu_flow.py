"""Flows on the GPU against the FP64 oracle: constant acceleration of the
solvent, plates at z = 0 and z = L_z with the bounce-back rule, and virtual
particles in the cells the plates cut.

A constant acceleration adds no transcendental function, so periodic
accelerated systems are compared bit for bit.  The virtual particles' summed
momentum is a Box-Muller normal vector (log, cos, sin, whose last bits differ
between the GPU math library and glibc), so systems with plates match the
oracle to 1e-12 in positions and velocities, with identical ids, species and
cell order."""
import math

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


def _flow(L, rho, g, walls, n_md=5, dt=0.01, **kw):
    p = W.base_params(L=L, rho=rho, dt=dt, n_md=n_md, **kw)
    p["walls"] = walls
    p["wall_density"] = rho if walls else 0
    p["accel"] = tuple(float(x) for x in g)
    return p


def _run(p, s0, seed, calls, tuning=None):
    rm = _rm()
    print(f"[flow] L={p['L']} N={p['n_solvent']} walls={p['walls']} g={p['accel']} "
          f"n_md={p['n_md']} calls={calls} tuning={tuning}", flush=True)
    g = rm.System(p, seed)
    if tuning:
        g.set_tuning(**tuning)
    g.set_state(s0)
    o = oracle.Oracle(p, seed, init=False)
    o.set_state(s0)
    for k in calls:
        g.step(p["n_md"], k)
        o.run(p["n_md"], k)
    return g, o


def _scale(s):
    return max(np.abs(s["v"]).max(), 1.0)


BITWISE = {
    "accel_periodic": lambda: dict(_flow((9, 7, 8), 5, (0.05, -0.02, 0.01), 0), bulk_rate=0.03),
    "accel_ragged": lambda: _flow((7, 5, 9), 6, (0.2, 0.0, -0.1), 0, n_md=3),
}


@pytest.mark.parametrize("case", sorted(BITWISE))
def test_accelerated_periodic_bitwise(case):
    p = BITWISE[case]()
    s0 = W.random_state(p, 41, species_B_fraction=0.3)
    g, o = _run(p, s0, 7, [2, 3])
    gs, os_ = g.get_state(), o.get_state()
    for k in ("id", "state", "x", "v"):
        assert np.array_equal(gs[k], os_[k]), k
    go, oo = g.observables(), o.observables()
    for k in ("n_B", "n_bulk_flips", "md_step", "coll_step", "n_candidates", "n_cells_T"):
        assert go[k] == oo[k], k
    assert go["n_candidates"] == 0
    np.testing.assert_allclose(go["momentum"], oo["momentum"], rtol=1e-12, atol=1e-9)


PLATES = {
    "plates": (lambda: _flow((8, 6, 10), 6, (0.02, 0.0, 0.0), 1), None),
    "plates_ragged_tiles": (lambda: _flow((7, 5, 9), 4, (0.01, 0.005, 0.0), 1),
                            dict(collide_cells=8, stream_block=64, use_graph=0)),
    "plates_no_accel": (lambda: _flow((6, 6, 7), 5, (0.0, 0.0, 0.0), 1), None),
    # fast particles and a long step: many crossings of both plates
    "plates_many_bounces": (lambda: _flow((6, 6, 5), 5, (0.1, 0.0, 0.0), 1, n_md=4, dt=0.1), None),
    "plates_bulk_reaction": (lambda: dict(_flow((8, 8, 8), 8, (0.03, 0.0, 0.0), 1), bulk_rate=0.05),
                             dict(use_graph=1)),
    # virtual particles at kT/m = 0.25: their summed momentum scales with
    # sqrt((n0 - n) kT / m)
    "plates_m2_kT05": (lambda: _flow((8, 6, 10), 6, (0.02, 0.0, 0.0), 1, kT=0.5, mass=2.0), None),
}


@pytest.mark.parametrize("case", sorted(PLATES))
def test_plates_match_oracle(case):
    make, tun = PLATES[case]
    p = make()
    vs = 3.0 if case == "plates_many_bounces" else None
    s0 = W.random_state(p, 42, species_B_fraction=0.2, velocity_scale=vs)
    g, o = _run(p, s0, 8, [1, 3], tuning=tun)
    gs, os_ = g.get_state(), o.get_state()
    assert np.array_equal(gs["id"], os_["id"])
    assert np.array_equal(gs["state"], os_["state"])
    sc = _scale(os_)
    assert np.abs(gs["v"] - os_["v"]).max() <= 1e-12 * sc
    assert np.abs(gs["x"] - os_["x"]).max() <= 1e-12 * max(p["L"])
    assert np.all(gs["x"][2] >= 0) and np.all(gs["x"][2] < p["L"][2])
    go, oo = g.observables(), o.observables()
    for k in ("n_B", "n_bulk_flips", "md_step", "coll_step", "n_candidates", "n_cells_T"):
        assert go[k] == oo[k], k
    assert go["temperature"] == pytest.approx(oo["temperature"], rel=1e-11)
    np.testing.assert_allclose(go["momentum"], oo["momentum"], rtol=1e-11, atol=1e-9)


def test_plates_fp32_one_interval_close_to_fp64_oracle():
    p = _flow((10, 8, 12), 6, (0.02, 0.0, 0.0), 1, precision=32)
    s0 = W.random_state(p, 43, float32=True)
    g, o = _run(p, s0, 9, [1])
    gs, os_ = g.get_state(), o.get_state()
    gi, oi = np.argsort(gs["id"]), np.argsort(os_["id"])
    L = np.array(p["L"], dtype=float)[:, None]
    dx = gs["x"][:, gi] - os_["x"][:, oi]
    dx[:2] -= L[:2] * np.round(dx[:2] / L[:2])
    assert np.abs(dx).max() <= 1e-5 * L.max()
    dv = gs["v"][:, gi] - os_["v"][:, oi]
    assert np.abs(dv).max() <= 1e-5 * np.abs(os_["v"]).max()


def test_flow_batch_slot_equals_alone():
    rm = _rm()
    pf = _flow((8, 6, 10), 6, (0.02, 0.0, 0.0), 1)
    pd = W.dimer_system(L=12, rho=5, n_md=5, seed=3, bulk_rate=0.02)
    sf, sd = W.random_state(pf, 44), W.random_state(pd, 45)
    b = rm.Batch(2, 64)
    b.set_slot(0, pd, 51, 5)
    b.set_slot(1, pf, 52, 5)
    b.set_state(0, sd)
    b.set_state(1, sf)
    b.step(3)
    a = rm.System(pf, 52)
    a.set_state(sf)
    a.step(5, 3)
    bs, as_ = b.get_state(1), a.get_state()
    for k in ("id", "state", "x", "v"):
        assert np.array_equal(bs[k], as_[k]), k
    o = oracle.Oracle(pd, 51, init=False)
    o.set_state(sd)
    o.run(5, 3)
    od, bd = o.get_state(), b.get_state(0)
    for k in ("id", "state", "x", "v", "X", "V"):
        assert np.array_equal(bd[k], od[k]), k


def test_poiseuille_workload_two_intervals_match_oracle():
    """The channel the benchmark times: 64 x 64 x 32 cells between plates,
    rho 10 (1,310,720 particles), g = 0.001 along x, 10 steps per collision."""
    p = W.poiseuille()
    s0 = W.random_state(p, 46)
    g, o = _run(p, s0, 10, [2])
    gs, os_ = g.get_state(), o.get_state()
    assert np.array_equal(gs["id"], os_["id"])
    assert np.abs(gs["v"] - os_["v"]).max() <= 1e-12 * _scale(os_)
    assert np.abs(gs["x"] - os_["x"]).max() <= 1e-12 * 64
