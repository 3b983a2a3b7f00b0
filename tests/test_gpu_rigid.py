"""Rigid bodies of several colloids on the GPU (iterative RATTLE: a composite
Janus particle of 13 beads and 42 bonds, a 24-bead chain with 66 bonds)
against the FP64 oracle, bit for bit: one lane of the MD chain performs the same sweeps over the bonds, in
the same order and arithmetic, as the oracle."""
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


def _rigid_state(p, seed):
    s = W.random_state(p, seed, species_B_fraction=0.2, flag_fraction=0.05)
    rng = np.random.default_rng(seed + 1)
    X = np.array([c["x"] for c in p["colloids"]])
    R = X.mean(axis=0)
    v0, w = rng.normal(0, 0.05, 3), rng.normal(0, 0.05, 3)
    s["V"] = np.array([v0 + np.cross(w, x - R) for x in X])
    return s


def _compare(g, o, what):
    gs, os_ = g.get_state(), o.get_state()
    for k in ("id", "state", "x", "v", "X", "V"):
        a, b = np.asarray(gs[k]), np.asarray(os_[k])
        assert np.array_equal(a, b), (what, k, np.argwhere(a != b)[:3].tolist())
    go, oo = g.observables(), o.observables()
    for k in ("n_B", "n_cat_flips", "n_bulk_flips", "md_step", "coll_step", "n_candidates", "flags"):
        assert go[k] == oo[k], (what, k)
    assert go["potential"] == pytest.approx(oo["potential"], rel=1e-12, abs=1e-12)


def _tetrahelix(n=24, tol=1e-9, L=16, rho=5, n_md=10):
    """A rigid chain of n beads on a helix, held by the bonds (i, i+1),
    (i, i+2) and (i, i+3): 3n - 6 bonds (66 for 24 beads, more than the 64
    lanes of a wave; 90 for 32, the most colloids a system holds), in layers
    of disjoint bonds as the workloads order them."""
    p = W.base_params(L=(L, L, L), rho=rho, dt=0.01, n_md=n_md)
    c = np.full(3, L / 2.0)
    X = [c + np.array([1.6 * np.cos(1.9 * i), 1.6 * np.sin(1.9 * i), 0.4 * (i - (n - 1) / 2.0)])
         for i in range(n)]
    for i, x in enumerate(X):
        cat = i < n // 2
        W.add_colloid(p, x, 1.0, 1.0, 1.0 if cat else 0.5, catalytic=cat,
                      ctype=W.TYPE_C if cat else W.TYPE_N)
    bonds = [(i, i + k, float(np.linalg.norm(X[i] - X[i + k]))) for k in (1, 2, 3) for i in range(n - k)]
    while bonds:
        used, layer = set(), []
        for bd in bonds:
            if bd[0] not in used and bd[1] not in used:
                layer.append(bd)
                used |= {bd[0], bd[1]}
        bonds = [bd for bd in bonds if bd not in layer]
        p["bonds"].extend(layer)
    p.update(rattle_tol=tol, rattle_maxit=2000, bulk_rate=0.02, name="tetrahelix")
    return p


CASES = {
    "tetrahelix66": _tetrahelix,
    "tetrahelix90_max_colloids": lambda: _tetrahelix(n=32, tol=1e-6),
    "janus": lambda: W.janus_system(L=16, rho=5, n_md=10, seed=3, bulk_rate=0.03),
    "janus_p05": lambda: W.janus_system(L=18, rho=4, n_md=8, seed=5, bulk_rate=0.0, cat_prob=0.5),
    "dimer_forced_iterative": lambda: dict(W.dimer_system(L=14, rho=5, n_md=10, seed=4, bulk_rate=0.02),
                                           rattle_iterative=1, rattle_tol=1e-12, rattle_maxit=1000),
}


@pytest.mark.parametrize("graph", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_rigid_body_trajectory_bitwise(case, graph):
    rm = _rm()
    p = CASES[case]()
    s0 = _rigid_state(p, 61)
    print(f"[rigid] {case} graph={graph} L={p['L']} N={p['n_solvent']} nc={len(p['colloids'])} "
          f"bonds={len(p['bonds'])}", flush=True)
    g = rm.System(p, 23)
    g.set_tuning(use_graph=graph)
    g.set_state(s0)
    o = oracle.Oracle(p, 23, init=False)
    o.set_state(s0)
    for k in (1, 2):
        g.step(p["n_md"], k)
        o.run(p["n_md"], k)
    _compare(g, o, case)
    # the body stays rigid
    st = g.get_state()
    for a, b, d in p["bonds"]:
        r = st["X"][a] - st["X"][b]
        assert abs(r @ r - d * d) <= 2.1 * p.get("rattle_tol", 1e-10) * d * d


def test_janus_fp32_close_to_fp64():
    rm = _rm()
    p = W.janus_system(L=16, rho=5, n_md=10, seed=3, bulk_rate=0.0, precision=32)
    s0 = _rigid_state(dict(p, precision=64), 62)
    s0["x"] = s0["x"].astype(np.float32).astype(np.float64)
    s0["x"] = np.where(s0["x"] >= 16.0, 0.0, s0["x"])
    s0["v"] = s0["v"].astype(np.float32).astype(np.float64)
    g = rm.System(p, 24)
    g.set_state(s0)
    g.step(10, 1)
    o = oracle.Oracle(dict(p, precision=64), 24, init=False)
    o.set_state(s0)
    o.run(10, 1)
    gs, os_ = g.get_state(), o.get_state()
    assert np.allclose(gs["X"], os_["X"], rtol=0, atol=1e-5)
    assert np.allclose(gs["V"], os_["V"], rtol=0, atol=1e-5)
    gi, oi = np.argsort(gs["id"]), np.argsort(os_["id"])
    assert np.abs(gs["v"][:, gi] - os_["v"][:, oi]).max() <= 1e-5 * np.abs(os_["v"]).max()


def test_janus_in_a_batch_equals_alone():
    rm = _rm()
    pj = W.janus_system(L=16, rho=5, n_md=10, seed=3, bulk_rate=0.03)
    pd = W.dimer_system(L=12, rho=5, n_md=6, seed=4, bulk_rate=0.02)
    sj, sd = _rigid_state(pj, 63), W.random_state(pd, 64)
    b = rm.Batch(2, 64)
    b.set_slot(0, pd, 71, 6)
    b.set_slot(1, pj, 72, 10)
    b.set_state(0, sd)
    b.set_state(1, sj)
    b.step(3)
    a = rm.System(pj, 72)
    a.set_state(sj)
    a.step(10, 3)
    bs, as_ = b.get_state(1), a.get_state()
    for k in ("id", "state", "x", "v", "X", "V"):
        assert np.array_equal(bs[k], as_[k]), k
    o = oracle.Oracle(pd, 71, init=False)
    o.set_state(sd)
    o.run(6, 3)
    od, bd = o.get_state(), b.get_state(0)
    for k in ("id", "state", "x", "v", "X", "V"):
        assert np.array_equal(bd[k], od[k]), k
