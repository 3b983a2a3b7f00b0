"""Pins of the FP64 CPU oracle against facts fixed outside the oracle itself:
a library implementation of the RNG, brute force on tiny inputs, a library
stable sort, exact conservation laws of the collision, analytic special cases
of rotations and ballistic motion, closed forms of MPCD transport theory and
statistical laws of the reactions.

Each test names the passage of the paper (section / equation) whose
statement it pins.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

ALPHA = math.radians(130.0)


# --------------------------------------------------------------------------
# Philox4x64-10 ("Algorithms": counter-based RNG) vs numpy's implementation.
# numpy's generator increments the counter before producing a block, so its
# first block for counter c-1 is the Philox function at counter c.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ctr,key", [
    ([1, 0, 0, 0], [0, 0]),
    ([5, 17, 3, 0], [0x524D50434D44, 2]),
    ([2**63 + 11, 2**40, 99, 7], [2**64 - 1, 12345]),
    ([123456789, 2**32 - 1, 0, 0], [42, 7]),
])
def test_philox_matches_numpy(ctr, key):
    c = list(ctr)
    c[0] -= 1
    ref = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                           key=np.array(key, dtype=np.uint64)).random_raw(4)
    got = oracle.philox(ctr, key)
    assert np.array_equal(np.asarray(ref, dtype=np.uint64), got)


# --------------------------------------------------------------------------
# WCA potential ("Algorithms", cut-off 12-6 LJ equation)
# --------------------------------------------------------------------------
def test_wca_known_values_and_cutoff():
    for sigma, eps in [(1.0, 1.0), (2.0, 0.5), (4.0, 1.0)]:
        coef, pot = oracle.wca(sigma * sigma, sigma, eps)
        # at r = sigma: V = eps and |F| = 24 eps / sigma (textbook LJ values)
        assert pot == pytest.approx(eps, rel=1e-15)
        assert coef * sigma == pytest.approx(24.0 * eps / sigma, rel=1e-14)
        rc = 2.0 ** (1.0 / 6.0) * sigma
        coef, pot = oracle.wca(rc * rc, sigma, eps)
        assert abs(pot) < 1e-13 * eps and abs(coef) < 1e-12 * eps


def test_wca_force_is_minus_gradient():
    sigma, eps = 4.0, 0.7
    for r in np.linspace(3.2, 4.45, 17):
        h = 1e-6
        _, vp = oracle.wca((r + h) ** 2, sigma, eps)
        _, vm = oracle.wca((r - h) ** 2, sigma, eps)
        coef, _ = oracle.wca(r * r, sigma, eps)
        dvdr = (vp - vm) / (2 * h)
        assert coef * r == pytest.approx(-dvdr, rel=2e-6, abs=1e-8)


# --------------------------------------------------------------------------
# Fixed reduction tree (reading: pairwise over list positions, zero padded)
# --------------------------------------------------------------------------
def _tree_py(a):
    a = list(a)
    if not a:
        return 0.0
    p = 1
    while p < len(a):
        p *= 2
    a += [0.0] * (p - len(a))
    while len(a) > 1:
        a = [a[2 * i] + a[2 * i + 1] for i in range(len(a) // 2)]
    return a[0]


def test_tree_sum_order():
    rng = np.random.default_rng(3)
    for n in [1, 2, 3, 5, 63, 64, 65, 1000]:
        a = rng.normal(size=n) * 10.0 ** rng.integers(-8, 8, size=n)
        assert oracle.tree_sum(a) == _tree_py(a)
    # order matters: pairwise != sequential for this input
    a = [1e16, 1.0, -1e16, 1.0]
    assert oracle.tree_sum(a) == (1e16 + 1.0) + (-1e16 + 1.0)
    assert oracle.tree_sum(a) != ((1e16 + 1.0) - 1e16) + 1.0
    ints = rng.integers(-1000, 1000, size=777).astype(float)
    assert oracle.tree_sum(ints) == math.fsum(ints)


# --------------------------------------------------------------------------
# Rotation and axis ("Algorithms": original MPCD collision rule)
# --------------------------------------------------------------------------
def test_marsaglia_axis_unit_and_isotropic():
    ns = np.array([oracle.marsaglia(77, 3, c) for c in range(20000)])
    assert np.allclose((ns ** 2).sum(1), 1.0, atol=4e-16)
    assert np.all(np.abs(ns.mean(0)) < 0.02)
    assert np.allclose((ns ** 2).mean(0), 1.0 / 3.0, atol=0.01)


def test_rotation_properties():
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        w = rng.normal(size=3)
        rw = oracle.rotate(n, ALPHA, w)
        assert np.linalg.norm(rw) == pytest.approx(np.linalg.norm(w), rel=1e-14)
        assert np.dot(rw, n) == pytest.approx(np.dot(w, n), abs=1e-14 * np.linalg.norm(w))
        wp = w - np.dot(w, n) * n
        rp = rw - np.dot(rw, n) * n
        # right-handed rotation by +alpha about n
        ang = math.atan2(np.dot(np.cross(wp, rp), n), np.dot(wp, rp))
        assert ang == pytest.approx(ALPHA, abs=1e-12)
        assert np.allclose(oracle.rotate(n, ALPHA, n), n, atol=1e-15)
        assert np.allclose(oracle.rotate(n, 0.0, w), w, rtol=0, atol=1e-15 * np.abs(w).max())
        # alpha = pi: reflection through the axis
        assert np.allclose(oracle.rotate(n, math.pi, w), 2 * np.dot(n, w) * n - w, atol=1e-14)


# --------------------------------------------------------------------------
# Binning and the stable counting sort ("Algorithms": sorting of solvent
# particles in cells, shared by collision and cell lists; Table 1's
# particle_system sorting routine)
# --------------------------------------------------------------------------
def _no_colloid(L=(6, 5, 4), rho=7, **kw):
    p = W.base_params(L=L, rho=rho, dt=0.01, n_md=3, **kw)
    return p


def test_cell_keys_contain_particle():
    p = _no_colloid()
    o = oracle.Oracle(p, 11)
    s = o.get_state()
    L = np.array(p["L"], dtype=float)
    for step in range(5):
        sh = o.shift(step)
        assert np.all((sh >= 0) & (sh < 1))
        keys = o.cell_keys(sh)
        cx = keys % p["L"][0]
        cy = (keys // p["L"][0]) % p["L"][1]
        cz = keys // (p["L"][0] * p["L"][1])
        c = np.stack([cx, cy, cz]).astype(float)
        rel = np.mod(s["x"] - sh[:, None] - c, L[:, None])
        assert np.all((rel >= 0) & (rel < 1))


@pytest.mark.parametrize("order", ["row", "hilbert"])
def test_sort_is_stable_argsort(order):
    """The collision's sort is numpy's stable argsort of the cells' ranks
    (row-major: the rank is the cell index)."""
    p = _no_colloid()
    p["cell_order"] = order
    o = oracle.Oracle(p, 12)
    if order == "row":
        assert np.array_equal(o.cell_ranks(), np.arange(int(np.prod(p["L"]))))
    s0 = o.get_state()
    sh = o.shift(0)
    rank = o.cell_ranks()[o.cell_keys(sh)]
    o.collide(3)
    s1 = o.get_state()
    perm = np.argsort(rank, kind="stable")
    assert np.array_equal(s1["id"], s0["id"][perm])
    assert np.array_equal(s1["x"], s0["x"][:, perm])
    start = o.last_cells()
    ncell = int(np.prod(p["L"]))
    assert np.array_equal(start, np.concatenate([[0], np.cumsum(np.bincount(rank, minlength=ncell))]))


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_hilbert_curve_invariants(bits):
    """The cell order's curve is a Hilbert curve of the 2^bits cube: a
    bijection onto [0, 8^bits) starting at the origin, consecutive indices
    are face neighbours, and every aligned run of 8^k indices fills an
    aligned 2^k cube (k = 1 .. bits)."""
    n = 1 << bits
    pts = np.array([(x, y, z) for z in range(n) for y in range(n) for x in range(n)])
    h = np.array([oracle.hilbert(x, y, z, bits) for x, y, z in pts])
    assert sorted(h.tolist()) == list(range(n ** 3))
    walk = pts[np.argsort(h)]
    assert tuple(walk[0]) == (0, 0, 0)
    assert np.all(np.abs(np.diff(walk, axis=0)).sum(axis=1) == 1)
    for k in range(1, bits + 1):
        m = 1 << k
        for blk in walk.reshape(-1, m ** 3, 3):
            lo = blk.min(axis=0)
            assert np.all(lo % m == 0) and np.all(blk.max(axis=0) - lo == m - 1)


@pytest.mark.parametrize("L", [(8, 8, 8), (7, 5, 9), (12, 12, 12), (1, 1, 1)])
def test_cell_ranks_follow_the_curve(L):
    """Cells are ranked by their curve index in the smallest power-of-two
    cube holding the box: a permutation of the cells, increasing along the
    curve; for a power-of-two cube the rank is the curve index itself."""
    p = W.base_params(L=L, rho=1, dt=0.01, n_md=1)
    p["cell_order"] = "hilbert"
    o = oracle.Oracle(p, 3)
    r = o.cell_ranks()
    ncell = L[0] * L[1] * L[2]
    assert sorted(r.tolist()) == list(range(ncell))
    bits = max(1, int(np.ceil(np.log2(max(L))))) if max(L) > 1 else 0
    c = np.arange(ncell)
    xyz = np.stack([c % L[0], (c // L[0]) % L[1], c // (L[0] * L[1])], axis=1)
    h = np.array([oracle.hilbert(x, y, z, bits) for x, y, z in xyz])
    assert np.all(np.diff(h[np.argsort(r)]) > 0)
    if L[0] == L[1] == L[2] and (L[0] & (L[0] - 1)) == 0 and L[0] > 1:
        assert np.array_equal(r, h)


# --------------------------------------------------------------------------
# Collision conservation laws and special cases
# --------------------------------------------------------------------------
def _cells_by_id(o, s_before):
    s1 = o.get_state()
    start = o.last_cells()
    inv = np.empty_like(s_before["id"], dtype=np.int64)
    inv[s_before["id"]] = np.arange(s_before["id"].size)
    before_v = s_before["v"][:, inv[s1["id"]]]
    return s1, start, before_v


@pytest.mark.parametrize("rule", ["srd", "at"])
def test_collision_conserves_cell_momentum_and_energy(rule):
    p = _no_colloid(rule=rule)
    o = oracle.Oracle(p, 13)
    s0 = o.get_state()
    o.collide(3)
    s1, start, vb = _cells_by_id(o, s0)
    va = s1["v"]
    for c in range(start.size - 1):
        b, e = start[c], start[c + 1]
        if e - b == 0:
            continue
        scale = np.abs(vb[:, b:e]).sum() + 1.0
        assert np.allclose(va[:, b:e].sum(1), vb[:, b:e].sum(1), atol=64 * 2.2e-16 * scale)
        if rule == "srd":
            assert (va[:, b:e] ** 2).sum() == pytest.approx((vb[:, b:e] ** 2).sum(), rel=1e-13)
            u = vb[:, b:e].mean(1, keepdims=True)
            assert np.allclose(np.linalg.norm(va[:, b:e] - u, axis=0),
                               np.linalg.norm(vb[:, b:e] - u, axis=0), rtol=1e-12, atol=1e-13)


def test_collision_single_particle_cells_unchanged_and_two_particle_rotation():
    p = W.base_params(L=(3, 3, 3), rho=1, dt=0.01, n_md=1)
    p["n_solvent"] = 3
    o = oracle.Oracle(p, 14, init=False)
    # two particles at the same point (same cell for any shift), one alone
    x = np.array([[0.5, 0.5, 2.5], [0.5, 0.5, 2.5], [0.5, 0.5, 2.5]])
    v = np.array([[1.0, -0.5, 0.3], [0.2, 0.7, -1.1], [0.0, 0.4, 2.0]])
    o.set_state(dict(x=x, v=v, id=np.arange(3, dtype=np.uint32),
                     state=np.zeros(3, np.uint8), X=np.zeros((0, 3)), V=np.zeros((0, 3))))
    sh = o.shift(0)
    keys = o.cell_keys(sh)
    o.collide(1)
    s = o.get_state()
    order = np.argsort(s["id"])
    va = s["v"][:, order]
    assert np.array_equal(va[:, 2], v[:, 2])                 # alone: unchanged
    n = oracle.marsaglia(14, 0, int(keys[0]))
    rel_b = v[:, 0] - v[:, 1]
    rel_a = va[:, 0] - va[:, 1]
    assert np.linalg.norm(rel_a) == pytest.approx(np.linalg.norm(rel_b), rel=1e-14)
    wp = rel_b - np.dot(rel_b, n) * n
    rp = rel_a - np.dot(rel_a, n) * n
    ang = math.atan2(np.dot(np.cross(wp, rp), n), np.dot(wp, rp))
    assert ang == pytest.approx(ALPHA, abs=1e-12)
    assert np.allclose(va[:, :2].sum(1), v[:, :2].sum(1), atol=1e-15)
    obs = o.observables()
    # T = (1/(3 N_c)) * sum |v - u|^2 / (N - 1) with one cell of two particles
    assert obs["n_cells_T"] == 1
    assert obs["temperature"] == pytest.approx(np.dot(rel_b, rel_b) / 2.0 / 3.0, rel=1e-14)


def test_collision_alpha_zero_and_pi():
    for alpha, check in [(0.0, "identity"), (math.pi, "reflect")]:
        p = _no_colloid()
        p["alpha"] = alpha
        o = oracle.Oracle(p, 15)
        s0 = o.get_state()
        sh = o.shift(0)
        keys0 = o.cell_keys(sh)
        o.collide(3)
        s1, start, vb = _cells_by_id(o, s0)
        if check == "identity":
            assert np.allclose(s1["v"], vb, rtol=0, atol=1e-14)
        else:
            inv = np.empty(s0["id"].size, np.int64)
            inv[s0["id"]] = np.arange(s0["id"].size)
            keys = keys0[inv[s1["id"]]]
            for c in range(start.size - 1):
                b, e = start[c], start[c + 1]
                if e - b < 2:
                    continue
                n = oracle.marsaglia(15, 0, int(keys[b]))
                u = vb[:, b:e].mean(1, keepdims=True)
                w = vb[:, b:e] - u
                ref = u + 2 * (n[:, None] * (n @ w)[None, :]) - w
                assert np.allclose(s1["v"][:, b:e], ref, atol=1e-13)


def test_collision_galilean_invariance():
    p = _no_colloid()
    o1 = oracle.Oracle(p, 16)
    s = o1.get_state()
    U = np.array([0.375, -1.25, 0.5])       # exactly representable boost
    s2 = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in s.items()}
    s2["v"] = s["v"] + U[:, None]
    o2 = oracle.Oracle(p, 16, init=False)
    o2.set_state(s2)
    o1.collide(3); o2.collide(3)
    a, b = o1.get_state(), o2.get_state()
    assert np.array_equal(a["id"], b["id"])
    assert np.allclose(b["v"] - U[:, None], a["v"], atol=1e-13)


# --------------------------------------------------------------------------
# Colloid-solvent forces over the Verlet list vs brute force
# --------------------------------------------------------------------------
def _brute_forces(s, p):
    L = np.array(p["L"], dtype=float)[:, None]
    f = np.zeros_like(s["x"])
    F = np.zeros((len(p["colloids"]), 3))
    for c, col in enumerate(p["colloids"]):
        Xw = np.mod(np.asarray(s["X"][c]), L[:, 0])[:, None]
        d = s["x"] - Xw
        d -= L * np.round(d / L)
        r = np.sqrt((d * d).sum(0))
        eps = np.where(s["state"] & 1, col["eps_B"], col["eps_A"])
        sig = col["sigma"]
        rc = 2 ** (1 / 6) * sig
        inside = r < rc
        # -dV/dr for V = 4 eps ((s/r)^12 - (s/r)^6 + 1/4)
        mag = np.where(inside, 4 * eps * (12 * sig ** 12 / r ** 13 - 6 * sig ** 6 / r ** 7), 0.0)
        g = mag * d / np.where(inside, r, 1.0)
        f += g
        F[c] -= g.sum(1)
    return f, F


@pytest.mark.parametrize("where", ["centre", "corner"])
def test_forces_match_brute_force_and_list_is_sound(where):
    p = W.dimer_system(L=16, rho=6, n_md=25, seed=3)
    if where == "corner":
        # dimer straddling the periodic boundary in every direction
        # (unwrapped coordinates: the bond vector is unchanged)
        for c in p["colloids"]:
            c["x"] = tuple(np.asarray(c["x"]) - 7.7)
    o = oracle.Oracle(p, 17)
    s = W.random_state(p, 18, species_B_fraction=0.4)
    o.set_state(s)
    for it in range(4):
        o.build_list(25)
        st = o.get_state()
        f = o.forces()
        fb, Fb = _brute_forces(st, p)
        scale = np.abs(fb).max()
        assert np.allclose(f, fb, rtol=1e-11, atol=1e-12 * scale)
        assert np.allclose(st["F"], Fb, rtol=1e-9, atol=1e-10 * np.abs(fb).sum())
        # list soundness: every interaction during the interval is in the list
        cand = set(o.candidates().tolist())
        o.interval(25, collide=False)
        fa, _ = o.forces_allpairs()
        nonzero = np.nonzero(np.abs(fa).sum(0))[0]
        assert set(nonzero.tolist()) <= cand
        o.interval(25, collide=True)
    assert o.observables()["flags"] == 0


# --------------------------------------------------------------------------
# Velocity-Verlet + exact RATTLE ("Algorithms": velocity-Verlet; RATTLE
# exact for the dimer)
# --------------------------------------------------------------------------
def test_rattle_holds_bond_and_velocity_constraint():
    p = W.dimer_system(L=16, rho=6, n_md=10, seed=4)
    p["bulk_rate"] = 0.0
    o = oracle.Oracle(p, 19)
    d = p["bonds"][0][2]
    for _ in range(30):
        o.interval(10, collide=True)
        s = o.get_state()
        r = s["X"][0] - s["X"][1]
        assert np.linalg.norm(r) == pytest.approx(d, rel=1e-13)
        dv = s["V"][0] - s["V"][1]
        assert abs(np.dot(dv, r)) < 1e-12 * np.linalg.norm(dv) * d + 1e-15


def _energy(o):
    ob = o.observables()
    return ob["ke_solvent"] + ob["ke_colloid"] + ob["potential"]


def test_velocity_verlet_energy_error_scales_dt2():
    base = W.dimer_system(L=16, rho=6, n_md=1, seed=5, bulk_rate=0.0, cat_prob=0.0)
    s0 = W.random_state(base, 20)
    amps = []
    for dt in (0.01, 0.005):
        p = dict(base); p["dt"] = dt
        o = oracle.Oracle(p, 21, init=False)
        o.set_state(s0)
        o.build_list(1)
        e0 = _energy(o)
        es = []
        nsteps = int(round(1.0 / dt))
        for _ in range(nsteps):
            o.interval(1, collide=False)
            es.append(_energy(o) - e0)
        amps.append(np.abs(es).max())
    ratio = amps[0] / amps[1]
    assert 3.0 < ratio < 5.0


@pytest.mark.parametrize("rule", ["srd", "at"])
def test_total_momentum_conserved_and_energy_bounded(rule):
    p = W.dimer_system(L=16, rho=6, n_md=20, seed=6, bulk_rate=0.0, cat_prob=0.0)
    p["rule"] = rule
    o = oracle.Oracle(p, 22)
    o.build_list(20)
    P0 = o.observables()["momentum"]
    e0 = _energy(o)
    for _ in range(20):
        o.run(20, 1)
    ob = o.observables()
    scale = np.sqrt(2 * ob["ke_solvent"] * p["n_solvent"])
    assert np.allclose(ob["momentum"], P0, atol=1e-11 * scale)
    if rule == "srd":
        assert abs(_energy(o) - e0) < 2e-4 * e0


# --------------------------------------------------------------------------
# Equilibrium and transport ("Implementation": validation by the velocity
# distribution and the viscosity); closed forms of MPCD kinetic theory
# (Kikuchi et al. 2003) for the rotation rule.
# --------------------------------------------------------------------------
def test_maxwell_boltzmann_from_non_gaussian_start():
    from scipy import stats
    p = _no_colloid(L=(10, 10, 10), rho=10)
    o = oracle.Oracle(p, 23)
    s = o.get_state()
    rng = np.random.default_rng(1)
    dirs = rng.normal(size=s["v"].shape)
    dirs /= np.linalg.norm(dirs, axis=0)
    s["v"] = dirs * math.sqrt(3.0)              # fixed speed, kT = 1
    s["v"] -= s["v"].mean(1, keepdims=True)
    o.set_state(s)
    o.run(10, 30)
    v = o.get_state()["v"]
    T = (v ** 2).mean()
    for d in range(3):
        assert stats.kstest(v[d] / math.sqrt(T), "norm").pvalue > 1e-3
    assert o.observables()["temperature"] == pytest.approx(T, rel=0.02)


def _closed_forms(tau, M=10, alpha=ALPHA):
    g = M - 1 + math.exp(-M)
    ca, c2 = math.cos(alpha), math.cos(2 * alpha)
    D = tau / 2 * (3 * M / ((1 - ca) * g) - 1)
    nu = tau / 2 * (5 * M / (g * (2 - ca - c2)) - 1) + (1 / (18 * tau)) * (g / M) * (1 - ca)
    return D, nu


@pytest.mark.slow
def test_self_diffusion_closed_form():
    tau = 0.5
    p = W.base_params(L=(10, 10, 10), rho=10, dt=tau, n_md=1)
    o = oracle.Oracle(p, 24)
    L = 10.0
    prev = o.get_state()["x"][:, np.argsort(o.get_state()["id"])]
    disp = np.zeros_like(prev)
    msd = []
    for _ in range(300):
        o.run(1, 1)
        s = o.get_state()
        cur = s["x"][:, np.argsort(s["id"])]
        d = cur - prev
        d -= L * np.round(d / L)
        disp += d
        prev = cur
        msd.append((disp ** 2).sum(0).mean())
    t = tau * np.arange(1, 301)
    slope = np.polyfit(t[100:], np.array(msd)[100:], 1)[0]
    D, _ = _closed_forms(tau)
    assert slope / 6 == pytest.approx(D, rel=0.05)


@pytest.mark.slow
def test_shear_viscosity_closed_form():
    tau, Lz = 0.5, 16
    k = 2 * math.pi / Lz
    nus = []
    for seed in range(6):
        p = W.base_params(L=(24, 24, Lz), rho=10, dt=tau, n_md=1)
        o = oracle.Oracle(p, 200 + seed)
        s = o.get_state()
        s["v"][0] += 0.5 * np.sin(k * s["x"][2])
        o.set_state(s)
        ts, amps = [], []
        for c in range(50):
            o.run(1, 1)
            s = o.get_state()
            amps.append(2 * np.mean(s["v"][0] * np.sin(k * s["x"][2])))
            ts.append((c + 1) * tau)
        ts, amps = np.array(ts), np.array(amps)
        m = (amps > 0.04) & (ts > 2)
        nus.append(-np.polyfit(ts[m], np.log(amps[m]), 1)[0] / k ** 2)
    _, nu = _closed_forms(tau)
    assert np.mean(nus) == pytest.approx(nu, rel=0.06)


# --------------------------------------------------------------------------
# Reactions: RMPCD bulk B->A (Overview: bulk kinetics) and catalytic A->B
# ("Applications": dimer motor chemistry; configuration `probability`)
# --------------------------------------------------------------------------
def test_bulk_reaction_statistics():
    p = _no_colloid(L=(12, 12, 12), rho=10)
    p["bulk_rate"] = 0.05
    n_md = 10
    tau = n_md * p["dt"]
    o = oracle.Oracle(p, 25)
    s = o.get_state()
    s["state"][:] = 1
    o.set_state(s)
    expected, var, got = 0.0, 0.0, 0
    for step in range(40):
        st = o.get_state()
        keys = o.cell_keys(o.shift(st["coll_step"]))
        nB = np.bincount(keys[(st["state"] & 1) == 1], minlength=int(np.prod(p["L"])))
        P = -np.expm1(-p["bulk_rate"] * tau * nB)
        expected += P.sum(); var += (P * (1 - P)).sum()
        before = o.observables()["n_B"]
        o.collide(n_md)
        got += before - o.observables()["n_B"]
    assert abs(got - expected) < 4 * math.sqrt(var)
    assert o.observables()["n_bulk_flips"] == got
    t = 40 * tau
    # weak-reaction limit: N_B(t) ~ N_B(0) exp(-k t)
    assert o.observables()["n_B"] / p["n_solvent"] == pytest.approx(math.exp(-p["bulk_rate"] * t), rel=0.02)
    tab = oracle.ptable(p["bulk_rate"], tau)
    assert np.allclose(tab[:50], 1 - np.exp(-p["bulk_rate"] * tau * np.arange(50)), rtol=1e-14, atol=1e-17)


def test_catalysis_ballistic_exit_times():
    """Frozen catalytic sphere with eps = 0 (no force): particles move on
    straight lines; an A particle becomes B at the first MD step at which it is
    outside the cut-off sphere after having been inside."""
    L = 20
    p = W.base_params(L=(L, L, L), rho=1, dt=0.01, n_md=1)
    W.add_colloid(p, (10.0, 10.0, 10.0), sigma=3.0, eps_A=0.0, eps_B=0.0,
                  catalytic=True, mass=1e30)
    rng = np.random.default_rng(7)
    n = 300
    p["n_solvent"] = n
    rc = 2 ** (1 / 6) * 3.0
    dirs = rng.normal(size=(3, n)); dirs /= np.linalg.norm(dirs, axis=0)
    r0 = rng.uniform(0.5 * rc, 1.6 * rc, size=n)
    x = 10.0 + dirs * r0
    v = rng.normal(size=(3, n))
    st = np.zeros(n, np.uint8)
    st[:20] = 1                               # some B: never converted
    o = oracle.Oracle(p, 26, init=False)
    o.set_state(dict(x=x, v=v, id=np.arange(n, dtype=np.uint32), state=st,
                     X=np.array([[10.0, 10.0, 10.0]]), V=np.zeros((1, 3))))
    nsteps = 400
    flip_step = np.full(n, -1)
    for k in range(nsteps):
        o.interval(1, collide=False)
        s = o.get_state()
        newly = (s["state"] & 1 == 1) & (flip_step < 0) & (np.arange(n) >= 20)
        flip_step[newly] = k
    # analytic: positions after k+1 steps are x0 + (k+1) dt v (straight line)
    t = (np.arange(nsteps) + 1) * p["dt"]
    pos = x[:, :, None] + v[:, :, None] * t[None, None, :]
    r = np.sqrt(((pos - 10.0) ** 2).sum(0))
    inside = r < rc
    for i in range(20, n):
        exp_step = -1
        was_in = False
        for k in range(nsteps):
            if inside[i, k]:
                was_in = True
            elif was_in:
                exp_step = k
                break
        margin = np.abs(r[i] - rc).min()
        if margin < 1e-9:
            continue                           # rounding-ambiguous crossing
        assert flip_step[i] == exp_step, i
    assert np.all(o.get_state()["state"][:20] & 1 == 1)
    assert (flip_step >= 0).sum() > 50


def test_catalysis_probability():
    L = 20
    p = W.base_params(L=(L, L, L), rho=1, dt=0.01, n_md=1)
    W.add_colloid(p, (10.0, 10.0, 10.0), sigma=3.0, eps_A=0.0, eps_B=0.0,
                  catalytic=True, mass=1e30)
    p["cat_prob"] = 0.3
    n = 4000
    p["n_solvent"] = n
    rng = np.random.default_rng(8)
    dirs = rng.normal(size=(3, n)); dirs /= np.linalg.norm(dirs, axis=0)
    x = 10.0 + dirs * 3.0
    v = dirs * 2.0                              # radially outward
    o = oracle.Oracle(p, 27, init=False)
    o.set_state(dict(x=x, v=v, id=np.arange(n, dtype=np.uint32),
                     state=np.zeros(n, np.uint8), X=np.array([[10.0] * 3]), V=np.zeros((1, 3))))
    for _ in range(60):
        o.interval(1, collide=False)
    s = o.get_state()
    frac = (s["state"] & 1).mean()
    assert frac == pytest.approx(0.3, abs=4 * math.sqrt(0.3 * 0.7 / n))
    assert np.all((s["state"] & 2) == 0)


# --------------------------------------------------------------------------
# Initialisation, determinism, resume
# --------------------------------------------------------------------------
def test_init_state():
    p = W.sphere10()
    o = oracle.Oracle(p, 28)
    s = o.get_state()
    assert np.array_equal(s["id"], np.arange(p["n_solvent"], dtype=np.uint32))
    assert np.all((s["x"] >= 0) & (s["x"] < 10))
    d = s["x"] - 5.0
    assert np.sqrt((d ** 2).sum(0)).min() >= 2.0
    assert np.allclose(s["v"].mean(1), 0, atol=1e-15)
    assert (s["v"] ** 2).mean() == pytest.approx(1.0, rel=0.03)
    assert o.observables()["flags"] == 0


def test_resume_is_bitwise():
    p = W.dimer_system(L=16, rho=6, n_md=10, seed=9)
    a = oracle.Oracle(p, 29)
    a.run(10, 5)
    b = oracle.Oracle(p, 29)
    b.run(10, 2)
    st = b.get_state()
    c = oracle.Oracle(p, 29, init=False)
    c.set_state(st)
    c.run(10, 3)
    sa, sc = a.get_state(), c.get_state()
    for k in ("x", "v", "id", "state", "X", "V"):
        assert np.array_equal(sa[k], sc[k]), k
    d = oracle.Oracle(p, 30)
    d.run(10, 5)
    assert not np.array_equal(sa["v"], d.get_state()["v"])


def test_paper_example_configuration_maps_to_params():
    """The appendix configuration file of the paper, parsed into a parameter
    set and run for a few steps (fixture: tests/golden/paper_example.parameters)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_example.parameters")
    cfg = W.parse_parameters(open(path).read())
    assert cfg["L"] == (32, 32, 32) and cfg["rho"] == 10 and cfg["N_MD"] == 100
    assert cfg["sigma_N"] == 3.0 and cfg["d"] == 6.5
    assert cfg["epsilon_N"] == (1.0, 0.2) and cfg["bulk_rmpcd"] is True
    p = W.params_from_config(cfg, L_override=(12, 12, 12))
    o = oracle.Oracle(p, 31)
    o.run(5, 2)
    s = o.get_state()
    assert np.linalg.norm(s["X"][0] - s["X"][1]) == pytest.approx(6.5, rel=1e-13)


# --------------------------------------------------------------------------
# Dimer analysis ("Applications of RMPCDMD": directed velocity, centre-of-mass
# MSD, cylindrical shell histogram of the product species)

def _analysis_system(L=16, rho=1, masses=None):
    p = W.base_params(L=(L, L, L), rho=rho, dt=0.01, n_md=5)
    W.add_dimer(p, (L / 2.0, L / 2.0, L / 2.0), (1.0, 0.0, 0.0))
    if masses is not None:
        for c, m in zip(p["colloids"], masses):
            c["mass"] = float(m)
    return p


def _set_colloids(o, p, X, V, seed=1):
    s = W.random_state(p, seed)
    s["X"] = np.asarray(X, dtype=float)
    s["V"] = np.asarray(V, dtype=float)
    o.set_state(s)
    return s


def test_dimer_sample_closed_form():
    p = _analysis_system(masses=(3.0, 1.0))
    o = oracle.Oracle(p, 1)
    a, b, _ = p["bonds"][0]
    # unwrapped positions far outside the box: the centre of mass is not wrapped
    Xa = np.array([-20.5, 40.25, 3.0])
    Xb = Xa + np.array([0.0, 3.0, 4.0])          # |Xb - Xa| = 5
    u = np.array([0.0, 3.0, 4.0]) / 5.0
    w = np.array([1.0, 0.0, 0.0])                # perpendicular to u
    Va = 0.7 * u + 0.25 * w
    Vb = 0.7 * u - 0.75 * w                      # COM velocity (3 Va + Vb) / 4 = 0.7 u
    X = np.zeros((2, 3)); V = np.zeros((2, 3))
    X[a], X[b], V[a], V[b] = Xa, Xb, Va, Vb
    _set_colloids(o, p, X, V)
    rec = o.dimer_sample(0)
    np.testing.assert_allclose(rec[0:3], (3.0 * Xa + Xb) / 4.0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(rec[3:6], 0.7 * u, rtol=0, atol=1e-15)
    np.testing.assert_allclose(rec[6:9], [0.0, 0.6, 0.8], rtol=0, atol=1e-16)
    assert abs(rec[9] - 0.7) < 1e-15
    # reversing the bond's direction reverses the axis and the directed velocity
    X[[a, b]] = X[[b, a]]; V[[a, b]] = V[[b, a]]
    _set_colloids(o, p, X, V)
    rec2 = o.dimer_sample(0)
    np.testing.assert_allclose(rec2[6:9], [0.0, -0.6, -0.8], rtol=0, atol=1e-16)
    # the masses stay with the indices: V_com = (3 Vb + Va) / 4 = 0.7 u - 0.5 w
    np.testing.assert_allclose(rec2[3:6], 0.7 * u - 0.5 * w, rtol=0, atol=1e-15)
    assert abs(rec2[9] + 0.7) < 1e-15
    with pytest.raises(ValueError):
        o.dimer_sample(1)


def test_dimer_sample_reversal_with_equal_masses():
    p = _analysis_system()
    o = oracle.Oracle(p, 1)
    a, b, _ = p["bonds"][0]
    Xa = np.array([2.0, 3.0, 4.0]); Xb = Xa + np.array([6.0, 0.0, 0.0])
    Vc = np.array([0.5, 0.125, -0.25])
    X = np.zeros((2, 3)); V = np.zeros((2, 3))
    X[a], X[b], V[a], V[b] = Xa, Xb, Vc, Vc
    _set_colloids(o, p, X, V)
    rec = o.dimer_sample(0)
    assert np.array_equal(rec[0:3], [5.0, 3.0, 4.0]) and np.array_equal(rec[3:6], Vc)
    assert np.array_equal(rec[6:9], [1.0, 0.0, 0.0]) and rec[9] == 0.5
    X[[a, b]] = X[[b, a]]
    _set_colloids(o, p, X, V)
    rec = o.dimer_sample(0)
    assert np.array_equal(rec[6:9], [-1.0, 0.0, 0.0]) and rec[9] == -0.5


def _perp_basis(u):
    u = np.asarray(u, dtype=float)
    t = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(u, t); e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    return e1, e2


@pytest.mark.parametrize("centre", [(8.3, 7.9, 8.1), (0.4, 15.7, 0.2)])
def test_cyl_hist_places_constructed_particles_in_their_bins(centre):
    """Particles put at the centre of chosen (z, rho) bins around a dimer with
    a tilted axis (and, for a centre near a corner, across the periodic
    boundaries) land in exactly those bins; particles just outside the
    cylinder and the far-away filler are not counted."""
    L, nz, nr, zmax, rmax = 16, 10, 8, 5.0, 4.0
    dz, dr = 2 * zmax / nz, rmax / nr
    p = _analysis_system(L=L, rho=1)
    o = oracle.Oracle(p, 2)
    a, b, _ = p["bonds"][0]
    u = np.array([1.0, 2.0, -2.0]) / 3.0
    R = np.asarray(centre) + np.array([3 * L, -L, 0.0])     # unwrapped centre of mass
    X = np.zeros((2, 3)); V = np.zeros((2, 3))
    X[a], X[b] = R - 3.35 * u, R + 3.35 * u
    s = _set_colloids(o, p, X, V)
    rec = o.dimer_sample(0)
    np.testing.assert_allclose(rec[6:9], u, atol=1e-15)
    n = p["n_solvent"]
    rng = np.random.default_rng(5)
    Rw = np.mod(rec[0:3], L)
    # filler: near the point of the box farthest from the centre
    x = np.mod(Rw[:, None] + 8.0 + rng.uniform(-0.5, 0.5, size=(3, n)), L)
    st = np.zeros(n, dtype=np.uint8)
    expect = np.zeros((2, nz, nr), dtype=np.uint64)
    e1, e2 = _perp_basis(u)
    m = 600
    for i in range(m):
        iz, ir, sp = rng.integers(nz), rng.integers(nr), rng.integers(2)
        z = -zmax + (iz + rng.uniform(0.1, 0.9)) * dz
        rho = (ir + rng.uniform(0.1, 0.9)) * dr
        phi = rng.uniform(0, 2 * np.pi)
        x[:, i] = np.mod(Rw + z * u + rho * (np.cos(phi) * e1 + np.sin(phi) * e2), L)
        st[i] = sp | (2 * rng.integers(2))       # the catalysis flag bit is not a species
        expect[sp, iz, ir] += 1
    # just outside: beyond either end cap, or beyond the radius
    for i in range(m, m + 60):
        kind = i % 3
        z = (zmax + 0.3 * dz) * (1 if kind == 0 else -1) if kind < 2 else 0.2
        rho = 0.5 if kind < 2 else rmax + 0.3 * dr
        x[:, i] = np.mod(Rw + z * u + rho * e1, L)
    x = np.where(x >= L, 0.0, x)
    s["x"], s["state"] = np.ascontiguousarray(x), st
    o.set_state(s)
    h = o.cyl_hist(0, nz, nr, zmax, rmax)
    assert np.array_equal(h, expect)


def test_cyl_hist_marginals_match_membership_counts():
    """Random state: per species, the number of particles with z below each
    bin edge and with rho below each shell edge (computed with a cross
    product, not by projection) equals the histogram's cumulative sums."""
    L, nz, nr, zmax, rmax = 12, 6, 5, 4.5, 3.5
    p = W.dimer_system(L=L, rho=5, n_md=5, seed=3)
    o = oracle.Oracle(p, 3)
    s = W.random_state(p, 9, species_B_fraction=0.4, flag_fraction=0.1)
    o.set_state(s)
    h = o.cyl_hist(0, nz, nr, zmax, rmax)
    a, b, _ = p["bonds"][0]
    X = s["X"]; M = np.array([c["mass"] for c in p["colloids"]])
    R = (M[a] * X[a] + M[b] * X[b]) / (M[a] + M[b])
    u = (X[b] - X[a]) / np.linalg.norm(X[b] - X[a])
    r = s["x"].T - np.mod(R, L)
    r -= L * np.round(r / L)
    z = r @ u
    rho = np.linalg.norm(np.cross(r, u), axis=1)
    inside = (z >= -zmax) & (z < zmax) & (rho < rmax)
    for sp in range(2):
        sel = inside & ((s["state"] & 1) == sp)
        assert h[sp].sum() == sel.sum() > 0
        for k in range(nz + 1):
            assert h[sp][:k].sum() == (sel & (z < -zmax + k * (2 * zmax / nz))).sum()
        for k in range(nr + 1):
            assert h[sp][:, :k].sum() == (sel & (rho < k * rmax / nr)).sum()


def test_msd_closed_forms():
    t = np.arange(41, dtype=float)[:, None]
    v = np.array([0.5, -0.25, 1.0])
    R = np.array([3.0, -7.5, 100.0]) + t * v           # exact in binary
    msd = oracle.msd(R, 45)
    lag = np.arange(46, dtype=float)
    want = np.where(lag < 41, (v @ v) * lag ** 2, 0.0)
    assert np.array_equal(msd, want)
    assert np.array_equal(oracle.msd(np.ones((7, 3)), 6), np.zeros(7))
    # two samples: lag 1 is the one squared displacement
    assert oracle.msd([[0, 0, 0], [1, 2, 2]], 1).tolist() == [0.0, 9.0]
    # alternating series: |d|^2 = 1 for odd lags, 0 for even lags
    alt = np.zeros((10, 3)); alt[1::2, 0] = 1.0
    m = oracle.msd(alt, 9)
    assert np.array_equal(m[1::2], np.ones(5)) and np.array_equal(m[0::2], np.zeros(5))


def test_analysis_schedule_and_series_cap():
    p = W.dimer_system(L=10, rho=3, n_md=4, seed=4)
    o = oracle.Oracle(p, 4)
    an = dict(every=2, series_cap=2, hist_nz=4, hist_nr=3, hist_zmax=4.0, hist_rmax=3.0)
    acc = o.run_analysed(4, 7, an)         # samples after collisions 2, 4, 6
    assert len(acc["series"]) == 2 and acc["n_dropped"] == 1
    assert acc["md_step"] == [8, 16]
    # histogram totals: three samples, each counting the cylinder's members
    assert acc["hist"].sum() > 0 and acc["hist"].dtype == np.uint64


# --------------------------------------------------------------------------
# Flows ("Algorithms": constant acceleration on the solvent; stick walls by
# bounce-back and virtual particles in the collision, Lamura et al. 2001)

def _flow(L=(6, 5, 8), rho=4, g=(0.0, 0.0, 0.0), walls=1, **kw):
    p = W.base_params(L=L, rho=rho, dt=0.01, n_md=5, **kw)
    p["walls"] = walls
    p["wall_density"] = rho
    p["accel"] = tuple(g)
    return p


def test_flow_validation():
    bad = [dict(_flow(), rule="at"), dict(_flow(), cell_order="hilbert"),
           dict(_flow(), wall_density=0), _flow(g=(0.0, 0.0, 0.1))]
    col = _flow(walls=0, g=(0.1, 0.0, 0.0))
    W.add_colloid(col, (3, 2.5, 4), sigma=1.0)
    bad.append(col)
    for p in bad:
        with pytest.raises(ValueError):
            oracle.Oracle(p, 1, init=False)


def test_constant_acceleration_free_flight():
    """Periodic box, no walls: velocity-Verlet with a constant force is exact
    for a parabola, so x(t) = x0 + v0 t + g t^2 / 2 (wrapped) and v = v0 + g t;
    collisions conserve momentum, so P grows by N m g per unit time."""
    g = np.array([0.25, -0.5, 0.125])
    p = _flow(walls=0, g=g)
    o = oracle.Oracle(p, 3, init=False)
    s = W.random_state(p, 4)
    o.set_state(s)
    n_md = 7
    o.interval(n_md, collide=False)
    t = n_md * p["dt"]
    st = o.get_state()
    L = np.array(p["L"], dtype=float)[:, None]
    want = np.mod(s["x"] + s["v"] * t + 0.5 * g[:, None] * t * t, L)
    d = st["x"] - want
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-12
    assert np.abs(st["v"] - (s["v"] + g[:, None] * t)).max() < 1e-13
    P0 = s["v"].sum(1)
    o.run(n_md, 3)
    P = o.observables()["momentum"]
    T = t + 3 * t
    np.testing.assert_allclose(P, P0 + p["n_solvent"] * g * T, rtol=0, atol=1e-9)


def test_bounce_back_at_both_plates():
    """A particle whose drift crosses a plate is reflected: z -> -z' below
    the bottom, 2 L_z - z' above the top, the velocity reversed, and the
    in-plane coordinates move back by the part of the step after the
    crossing: x -> x0 + v (2 t* - dt)."""
    p = _flow(L=(6, 5, 8), rho=1)
    n = p["n_solvent"]
    o = oracle.Oracle(p, 5, init=False)
    s = W.random_state(p, 6)
    rng = np.random.default_rng(7)
    dt = p["dt"]
    x, v = s["x"], s["v"]
    # half the particles just above the bottom plate moving down, half just
    # below the top moving up, each crossing within the step
    for i in range(n):
        vz = rng.uniform(0.5, 2.0)
        frac = rng.uniform(0.05, 0.95)
        if i % 2 == 0:
            v[2, i] = -vz
            x[2, i] = frac * vz * dt
        else:
            v[2, i] = vz
            x[2, i] = 8.0 - frac * vz * dt
    o.set_state(s)
    o.interval(1, collide=False)
    st = o.get_state()
    z1 = x[2] + v[2] * dt
    zw = np.where(v[2] < 0, 0.0, 8.0)
    ts = (zw - x[2]) / v[2]
    assert np.all((ts > 0) & (ts < dt))
    np.testing.assert_allclose(st["x"][2], 2 * zw - z1, rtol=0, atol=1e-13)
    L = np.array(p["L"], dtype=float)
    for d in range(2):
        want = np.mod(x[d] + v[d] * (2 * ts - dt), L[d])
        diff = st["x"][d] - want
        diff -= L[d] * np.round(diff / L[d])
        assert np.abs(diff).max() < 1e-13
    np.testing.assert_allclose(st["v"], -v, rtol=0, atol=0)
    assert np.all((st["x"][2] >= 0) & (st["x"][2] < 8.0))


def test_wall_cell_layers():
    """With plates the shifted grid has L_z + 1 layers: layer
    c_z = floor(z - s_z) + 1 holds z in [c_z - 1 + s_z, c_z + s_z)."""
    p = _flow(L=(6, 5, 7), rho=6)
    o = oracle.Oracle(p, 8)
    s = o.get_state()
    for step in range(4):
        sh = o.shift(step)
        keys = o.cell_keys(sh).astype(np.int64)
        cz = keys // (6 * 5)
        assert cz.min() >= 0 and cz.max() <= 7
        rel = s["x"][2] - sh[2] - (cz - 1)
        assert np.all((rel >= 0) & (rel < 1))
        # in-plane coordinates stay periodic
        cx = keys % 6
        relx = np.mod(s["x"][0] - sh[0] - cx, 6.0)
        assert np.all((relx >= 0) & (relx < 1))


def test_virtual_particles_in_cut_cells_at_zero_temperature():
    """kT = 0: the virtual particles of a cut cell carry no momentum, so a
    cut cell whose nn particles share one velocity V has mean u = nn V / n0
    and every particle leaves with the same velocity, |v' - u| = |V| (1 - nn/n0).
    Full cells with a common velocity are left unchanged."""
    p = _flow(L=(4, 4, 6), rho=5, kT=0.0)
    n0 = p["wall_density"]
    o = oracle.Oracle(p, 9, init=False)
    s = W.random_state(p, 10)
    V = np.array([0.3, -0.2, 0.1])
    s["v"][:] = V[:, None]
    o.set_state(s)
    sh = o.shift(0)
    keys = o.cell_keys(sh)
    o.collide(1)
    st = o.get_state()
    by_id = np.argsort(st["id"])
    v1 = st["v"][:, by_id]
    k0 = keys[np.argsort(s["id"])]
    cz = k0 // 16
    checked = 0
    for key in np.unique(k0):
        m = k0 == key
        nn = int(m.sum())
        vv = v1[:, m]
        assert np.abs(vv - vv[:, :1]).max() < 1e-15          # one common velocity
        cut = cz[m][0] in (0, 6)
        if cut and nn < n0:
            u = nn * V / n0
            assert np.linalg.norm(vv[:, 0] - u) == pytest.approx(np.linalg.norm(V) * (1 - nn / n0),
                                                                 rel=1e-12)
            assert np.abs(vv[:, 0] - V).max() > 1e-3
            checked += 1
        else:
            np.testing.assert_allclose(vv[:, 0], V, rtol=0, atol=1e-15)
    assert checked >= 4


def _poiseuille_profile(seed, wall_density=None, h=10, g=0.01, tau=0.1, Lxy=16):
    p = _flow(L=(Lxy, Lxy, h), rho=10, g=(g, 0.0, 0.0))
    p["dt"] = tau
    if wall_density is not None:
        p["wall_density"] = wall_density
    o = oracle.Oracle(p, seed)
    o.run(1, 600)                      # about 5 relaxation times h^2 / (pi^2 nu)
    prof = np.zeros(h)
    for _ in range(600):
        o.run(1, 5)
        s = o.get_state()
        k = np.minimum(s["x"][2].astype(int), h - 1)
        prof += np.bincount(k, weights=s["v"][0], minlength=h) / np.bincount(k, minlength=h)
    prof /= 600
    zc = np.arange(h) + 0.5
    c = np.polyfit(zc, prof, 2)        # slab means of a parabola: same curvature
    _, nu = _closed_forms(tau)
    vmax = g * h * h / (8 * nu)
    return c, nu, vmax, np.abs(np.polyval(c, zc) - prof).max()


@pytest.mark.slow
def test_poiseuille_profile_closed_form():
    """Steady flow between the plates driven by g along x: a parabola whose
    curvature is -g / (2 nu) (Stokes flow, with the MPCD kinematic viscosity
    of the closed form, Kikuchi et al. 2003), vanishing near both plates.
    The virtual particles are what keeps the slip small: without them (fill
    density 1, so no cell is ever filled) the wall velocity is a third of the
    centre's."""
    g = 0.01
    c, nu, vmax, resid = _poiseuille_profile(31)
    assert -c[0] == pytest.approx(g / (2 * nu), rel=0.08)
    assert resid < 0.04 * vmax
    slip = [np.polyval(c, 0.0) / vmax, np.polyval(c, 10.0) / vmax]
    assert max(abs(x) for x in slip) < 0.12, slip
    c0, _, _, _ = _poiseuille_profile(31, wall_density=1)
    slip0 = [np.polyval(c0, 0.0) / vmax, np.polyval(c0, 10.0) / vmax]
    assert min(slip0) > 0.25, slip0


# --------------------------------------------------------------------------
# Rigid bodies of several beads: RATTLE in its iterative form (Andersen
# 1983; "Algorithms": iterative for the Janus particle, exact for the dimer)

def _bond_errors(p, X, V):
    pos, vel = [], []
    for a, b, d in p["bonds"]:
        r = X[a] - X[b]
        pos.append(abs(r @ r - d * d) / (d * d))
        vel.append(abs(r @ (V[a] - V[b])) / (d * d))
    return max(pos), max(vel)


def _rigid_velocities(p, rng):
    """A rigid-body velocity field: V_c = v0 + w x (X_c - R)."""
    X = np.array([c["x"] for c in p["colloids"]])
    R = X.mean(axis=0)
    v0, w = rng.normal(0, 0.05, 3), rng.normal(0, 0.05, 3)
    return np.array([v0 + np.cross(w, x - R) for x in X])


def test_iterative_rattle_holds_janus_rigid_and_conserves_its_invariants():
    """An isolated composite Janus particle (13 beads, 42 bonds, no solvent)
    moves freely: every bond keeps its length within the tolerance and has
    no relative velocity along it, total momentum is conserved to rounding,
    and kinetic energy and angular momentum of the free rigid body stay
    constant to the integration error."""
    p = W.janus_system(L=16, rho=0, n_md=20, seed=3)
    assert p["n_solvent"] == 0 and len(p["bonds"]) == 42
    o = oracle.Oracle(p, 5, init=False)
    s = W.random_state(p, 6)
    s["V"] = _rigid_velocities(p, np.random.default_rng(7))
    o.set_state(s)
    M = np.array([c["mass"] for c in p["colloids"]])

    def invariants(st):
        X, V = st["X"], st["V"]
        P = (M[:, None] * V).sum(0)
        R = (M[:, None] * X).sum(0) / M.sum()
        Lm = (M[:, None] * np.cross(X - R, V)).sum(0)
        return P, 0.5 * (M * (V * V).sum(1)).sum(), Lm
    P0, K0, L0 = invariants(o.get_state())
    for _ in range(10):
        o.run(20, 1)
        st = o.get_state()
        ep, ev = _bond_errors(p, st["X"], st["V"])
        assert ep <= 2.1e-10 and ev <= 1e-10 / p["dt"] * 1.01
        P, K, Lm = invariants(st)
        assert np.abs(P - P0).max() < 1e-13
        assert abs(K - K0) / K0 < 1e-6
        assert np.abs(Lm - L0).max() < 1e-6 * np.abs(L0).max()
    assert o.observables()["flags"] == 0


def test_iterative_rattle_agrees_with_exact_for_the_dimer():
    """For a single bond the exact RATTLE has a closed form: the iterative
    one (forced) follows the same trajectory to within its tolerance."""
    p = W.dimer_system(L=14, rho=5, n_md=10, seed=4, bulk_rate=0.0)
    s0 = W.random_state(p, 8)
    outs = []
    for it in (0, 1):
        q = dict(p, rattle_iterative=it, rattle_tol=1e-12, rattle_maxit=1000)
        o = oracle.Oracle(q, 9, init=False)
        o.set_state(s0)
        o.interval(10, collide=False)
        outs.append(o.get_state())
    assert np.abs(outs[0]["X"] - outs[1]["X"]).max() < 1e-9
    assert np.abs(outs[0]["V"] - outs[1]["V"]).max() < 1e-7
    ep, ev = _bond_errors(p, outs[1]["X"], outs[1]["V"])
    assert ep < 3e-12


def test_iterative_rattle_flags_when_it_cannot_converge():
    p = dict(W.janus_system(L=16, rho=0, n_md=5, seed=3), rattle_maxit=1)
    o = oracle.Oracle(p, 5, init=False)
    s = W.random_state(p, 6)
    s["V"] = _rigid_velocities(p, np.random.default_rng(7)) * 40.0
    o.set_state(s)
    o.run(5, 1)
    assert o.observables()["flags"] & oracle.F_RATTLE


def test_rigid_body_validation_and_same_body_exclusion():
    base = W.janus_system(L=16, rho=2, n_md=5, seed=3)
    for bad in (dict(base, rattle_tol=0.0), dict(base, rattle_maxit=0),
                dict(base, bonds=base["bonds"] + [base["bonds"][0]])):
        with pytest.raises(ValueError):
            oracle.Oracle(bad, 1, init=False)
    # beads of one body overlap (spacing 2.5-2.6 < 2^(1/6) 4): no
    # colloid-colloid force acts inside the body, so a body at rest with no
    # solvent nearby stays at rest
    p = dict(base, n_solvent=0)
    o = oracle.Oracle(p, 2, init=False)
    s = W.random_state(p, 3)
    s["V"] = np.zeros_like(s["V"])
    o.set_state(s)
    o.run(5, 1)
    st = o.get_state()
    assert np.abs(st["V"]).max() == 0.0 and np.abs(st["X"] - s["X"]).max() == 0.0


# --------------------------------------------------------------------------
# Solvent mass m and temperature kT away from 1 ("Algorithms": Maxwellian
# initial velocities at kT, the velocity-Verlet kicks dt f / (2 m), the
# cell-frame temperature equation with its factor m, the Anderson thermostat
# drawing relative velocities from N(0, kT/m), and the virtual particles of
# cut wall cells, Lamura et al. 2001).  Every pin below runs at m = 2.5 and
# kT = 0.7 (kT/m = 0.28), so that a factor of m or kT dropped, inverted or
# taken under the wrong square root moves the checked quantity by far more
# than its statistical error.
# --------------------------------------------------------------------------
MASS, KT = 2.5, 0.7


def test_init_maxwellian_at_nonunit_mass_and_temperature():
    """Initial velocities: each component N(0, kT/m), mean removed; the
    kinetic energy is (m/2) sum v^2 = (3/2) N kT up to sampling error."""
    from scipy import stats
    p = _no_colloid(L=(12, 12, 12), rho=10, kT=KT, mass=MASS)
    o = oracle.Oracle(p, 101)
    v = o.get_state()["v"]
    n = p["n_solvent"]
    var = (v ** 2).mean()
    # the pooled variance of 3N normals has relative error sqrt(2 / 3N) ~ 0.6 %
    assert var == pytest.approx(KT / MASS, rel=0.03)
    for d in range(3):
        assert stats.kstest(v[d] / math.sqrt(KT / MASS), "norm").pvalue > 1e-3
    ke = o.observables()["ke_solvent"]
    assert ke == pytest.approx(1.5 * n * KT, rel=0.03)
    assert ke == pytest.approx(0.5 * MASS * (v ** 2).sum(), rel=1e-12)


@pytest.mark.parametrize("rule", ["srd", "at"])
def test_temperature_equation_returns_kT(rule):
    """The cell-frame estimator T = m sum |v - u|^2 / (3 sum (n_c - 1)) of a
    Maxwellian state at kT returns kT (not kT/m), for both collision rules."""
    p = _no_colloid(L=(12, 12, 12), rho=10, kT=KT, mass=MASS, rule=rule)
    o = oracle.Oracle(p, 102)
    o.collide(3)
    ob = o.observables()
    # about 3 * 15,800 degrees of freedom: relative error ~ 0.7 %
    assert ob["temperature"] == pytest.approx(KT, rel=0.03)
    assert ob["n_cells_T"] > 1500


def test_anderson_thermostat_draws_relative_velocities_at_kT():
    """MPC-AT from a state twice as fast (temperature 4 kT): after one
    collision each particle's velocity relative to its cell mean is
    g_i - <g>_cell with g_i ~ N(0, kT/m), so a component has variance
    (kT/m)(n_c - 1)/n_c whatever the state before (the thermostat's noise
    law), and the cell momenta are unchanged.  The temperature equation is
    evaluated on the velocities that arrive at the collision (before the
    rule), so it reads the hot state's 4 kT."""
    from scipy import stats
    p = _no_colloid(L=(12, 12, 12), rho=10, kT=KT, mass=MASS, rule="at")
    o = oracle.Oracle(p, 103)
    s0 = o.get_state()
    s0["v"] = s0["v"] * 2.0
    o.set_state(s0)
    o.collide(3)
    s1, start, vb = _cells_by_id(o, s0)
    va = s1["v"]
    z = []
    for c in range(start.size - 1):
        b, e = int(start[c]), int(start[c + 1])
        nn = e - b
        if nn < 2:
            continue
        np.testing.assert_allclose(va[:, b:e].sum(1), vb[:, b:e].sum(1), rtol=0,
                                   atol=1e-12 * (np.abs(vb[:, b:e]).sum() + 1))
        w = va[:, b:e] - va[:, b:e].mean(1, keepdims=True)
        z.append((w / math.sqrt(KT / MASS * (nn - 1) / nn)).ravel())
    z = np.concatenate(z)
    assert (z ** 2).mean() == pytest.approx(1.0, rel=0.03)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    assert o.observables()["temperature"] == pytest.approx(4.0 * KT, rel=0.03)


def test_momentum_and_energy_with_colloids_at_nonunit_mass():
    """Velocity-Verlet with the solvent kick dt f/(2m) and the colloid kick
    dt F/(2M): total momentum m sum v + sum M V is conserved to rounding
    through the colloid-solvent forces, and the energy error of the
    integrator still shrinks as dt^2."""
    base = W.dimer_system(L=16, rho=6, n_md=1, seed=5, bulk_rate=0.0, cat_prob=0.0)
    base["mass"], base["kT"] = MASS, KT
    s0 = W.random_state(base, 104)
    o = oracle.Oracle(base, 105, init=False)
    o.set_state(s0)
    o.build_list(1)
    P0 = o.observables()["momentum"]
    for _ in range(200):
        o.interval(1, collide=False)
    P1 = o.observables()["momentum"]
    pscale = math.sqrt(base["n_solvent"] * MASS * KT)
    assert np.abs(P1 - P0).max() < 1e-11 * pscale
    # the colloids did feel the solvent: the force was not zero throughout
    assert np.abs(o.get_state()["V"] - s0["V"]).max() > 1e-4
    amps = []
    for dt in (0.01, 0.005):
        p = dict(base); p["dt"] = dt
        q = oracle.Oracle(p, 106, init=False)
        q.set_state(s0)
        q.build_list(1)
        e0 = _energy(q)
        es = []
        for _ in range(int(round(1.0 / dt))):
            q.interval(1, collide=False)
            es.append(_energy(q) - e0)
        amps.append(np.abs(es).max())
    assert 3.0 < amps[0] / amps[1] < 5.0


def test_virtual_particles_carry_thermal_momentum_at_kT():
    """Cut wall cells with n < n0 particles, all at rest: the n0 - n virtual
    particles contribute a summed momentum of variance (n0 - n) kT/m per
    component, so u = sqrt(n0 - n) sqrt(kT/m) xi / n0 and every particle of
    the cell leaves with v' = u - R u.  Averaged over the random axis,
    E|v'|^2 = 4 (1 - cos alpha)(n0 - n) kT / (m n0^2).  Cells away from the
    plates (u = 0) stay at rest."""
    p = _flow(L=(16, 16, 4), rho=5, kT=KT, mass=MASS)
    n0 = 20
    p["wall_density"] = n0
    o = oracle.Oracle(p, 107, init=False)
    s = W.random_state(p, 108)
    s["v"][:] = 0.0
    ratio_num, ratio_den, cells = 0.0, 0.0, 0
    for coll in range(4):
        s["coll_step"] = coll
        o.set_state(s)
        keys = o.cell_keys(o.shift(coll))
        o.collide(1)
        st = o.get_state()
        order = np.argsort(st["id"])
        v1 = st["v"][:, order]
        k0 = keys[np.argsort(s["id"])]
        layer = k0 // (16 * 16)
        for key in np.unique(k0):
            m = k0 == key
            nn = int(m.sum())
            vv = v1[:, m]
            assert np.abs(vv - vv[:, :1]).max() < 1e-14 * (1 + np.abs(vv).max())
            if layer[m][0] in (0, 4) and nn < n0:
                ratio_num += float((vv[:, 0] ** 2).sum())
                ratio_den += 4.0 * (1.0 - math.cos(ALPHA)) * (n0 - nn) * KT / (MASS * n0 * n0)
                cells += 1
            else:
                assert np.abs(vv).max() == 0.0
    assert cells > 1500
    # about 2,000 cells: the ratio's relative error is about 3 %
    assert ratio_num / ratio_den == pytest.approx(1.0, rel=0.12)


def test_nonfinite_cell_velocity_is_flagged():
    """A cell whose centre-of-mass velocity is not finite (two velocities
    that overflow when summed) latches the non-finite flag at the collision;
    a finite state does not."""
    p = _no_colloid(L=(4, 4, 4), rho=3)
    o = oracle.Oracle(p, 109, init=False)
    s = W.random_state(p, 110)
    o.set_state(s)
    o.collide(1)
    assert o.observables()["flags"] & oracle.F_NONFINITE == 0
    s["x"][:, 1] = s["x"][:, 0]           # same cell for any shift? same point
    s["v"][0, 0] = s["v"][0, 1] = 1.5e308
    o.set_state(s)
    o.collide(1)
    assert o.observables()["flags"] & oracle.F_NONFINITE
