"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64 state: trajectories from identical uploaded states are compared element
by element and must be bit-identical (positions, velocities, ids, species and
flags, colloid positions and velocities), because both sides evaluate the
same defined sequence of IEEE operations (contraction off, explicit fma, the
same Philox streams, the same fixed reduction tree).  Observables that are
sums in a different order are compared to 1e-12 relative.  The Anderson
thermostat uses transcendental functions (log, cos, sin) whose last bits
differ between the GPU math library and glibc: compared to 1e-12.  FP32
state is compared with the FP64 oracle to 1e-5 (relative to the field's
scale), matched by particle id.
"""
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


def _run_both(p, state, seed, n_md, n_coll, tuning=None, per_call=None):
    rm = _rm()
    print(f"[parity] L={p['L']} N={p['n_solvent']} nc={len(p['colloids'])} n_md={n_md} "
          f"n_coll={n_coll} tuning={tuning}", flush=True)
    g = rm.System(p, seed)
    if tuning:
        g.set_tuning(**tuning)
    g.set_state(state)
    o = oracle.Oracle(p, seed, init=False)
    o.set_state(state)
    calls = per_call or [n_coll]
    for k in calls:
        g.step(n_md, k)
        o.run(n_md, k)
    return g, o


def _assert_bitwise(gs, os_, what=""):
    errs = []
    for k in ("id", "state", "x", "v", "X", "V"):
        a, b = np.asarray(gs[k]), np.asarray(os_[k])
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            first = [tuple(int(q) for q in i) for i in bad[:3]]
            vals = [(a[i].tolist(), b[i].tolist()) for i in first]
            msg = f"{k} differs at {len(bad)} entries, first {first} (gpu, oracle) {vals}"
            if a.dtype.kind == "f":
                msg += f", max abs diff {np.abs(a - b).max()}"
            errs.append(msg)
    if errs:
        raise AssertionError(f"{what}: " + "; ".join(errs))
    assert gs["md_step"] == os_["md_step"] and gs["coll_step"] == os_["coll_step"]


def _assert_obs(go, oo, rtol=1e-12):
    for k in ("ke_solvent", "ke_colloid", "potential", "temperature"):
        assert go[k] == pytest.approx(oo[k], rel=rtol, abs=1e-12), k
    for k in ("n_A", "n_B", "n_cat_flips", "n_bulk_flips", "md_step", "coll_step",
              "n_candidates", "n_cells_T"):
        assert go[k] == oo[k], k
    assert go["e_rxn"] == pytest.approx(oo["e_rxn"], rel=1e-9, abs=1e-9)
    scale = math.sqrt(2 * oo["ke_solvent"] + 1.0)
    assert np.allclose(go["momentum"], oo["momentum"], atol=1e-11 * scale)


# ---------------------------------------------------------------- FP64 ---

CASES = {
    "sphere_small": lambda: W.scaled(W.sphere10(), L=(10, 10, 10), rho=4),
    "dimer_react": lambda: W.dimer_system(L=16, rho=5, n_md=20, seed=3, bulk_rate=0.05),
    "dimer_p05": lambda: W.dimer_system(L=14, rho=6, n_md=10, seed=4, bulk_rate=0.02, cat_prob=0.5),
    "free_ragged": lambda: W.base_params(L=(7, 5, 9), rho=6, n_md=5),
    # compact-Hilbert cell order: a cubic power-of-two box (rank computed in
    # the kernels) and a ragged box (rank table)
    "dimer_hilbert_cube": lambda: dict(W.dimer_system(L=16, rho=5, n_md=10, seed=6, bulk_rate=0.03),
                                       cell_order="hilbert"),
    "ragged_hilbert": lambda: dict(W.base_params(L=(7, 5, 9), rho=6, n_md=5), cell_order="hilbert"),
    # solvent mass and temperature away from 1: the kicks dt f/(2m), the
    # velocity scale sqrt(kT/m) of the state and the factor m of the
    # temperature equation enter every step
    "dimer_react_m2_kT05": lambda: dict(W.dimer_system(L=16, rho=5, n_md=20, seed=3, bulk_rate=0.05),
                                        mass=2.0, kT=0.5),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fp64_trajectory_bitwise(case):
    p = CASES[case]()
    s0 = W.random_state(p, 101, species_B_fraction=0.3, flag_fraction=0.05)
    n_md = p["n_md"]
    g, o = _run_both(p, s0, 5150, n_md, 4)
    _assert_bitwise(g.get_state(), o.get_state(), case)
    _assert_obs(g.observables(), o.observables())


@pytest.mark.parametrize("mass,kT", [(1.0, 1.0), (2.0, 0.5)])
def test_fp64_gpu_init_matches_oracle_init(mass, kT):
    rm = _rm()
    p = dict(W.sphere10(), mass=mass, kT=kT)
    g = rm.System(p, 77)
    o = oracle.Oracle(p, 77)
    gs, os_ = g.get_state(), o.get_state()
    assert np.array_equal(gs["id"], os_["id"])
    assert np.array_equal(gs["x"], os_["x"])           # u01 * L: exact on both sides
    # Box-Muller uses log/cos/sin: last-bit differences, then the mean removal
    assert np.allclose(gs["v"], os_["v"], rtol=0, atol=1e-13)
    assert g.observables()["flags"] == 0


def test_fp64_chain_512_threads_two_entries_each():
    """A list capacity beyond 256 workgroups of 512 threads selects the
    512-thread shape with two entries per thread."""
    p = dict(W.dimer_system(L=16, rho=6, n_md=10, seed=11, bulk_rate=0.03), cand_capacity=140000)
    s0 = W.random_state(p, 109, species_B_fraction=0.3, flag_fraction=0.05)
    g, o = _run_both(p, s0, 17, 10, 3, tuning=dict(chain_block=512))
    _assert_bitwise(g.get_state(), o.get_state(), "512 x 2")
    _assert_obs(g.observables(), o.observables())


@pytest.mark.parametrize("tuning", [
    dict(chain_k=1, collide_cells=8, stream_block=64, use_graph=0),
    dict(chain_k=2, collide_cells=16, stream_block=128, use_graph=1),
    dict(chain_k=4, collide_cells=64, stream_block=256, use_graph=1),
    dict(chain_k=1, chain_block=512, collide_cells=32, stream_block=256, use_graph=0),
])
def test_fp64_launch_configuration_does_not_change_results(tuning):
    """Different tile sizes, list blockings (and hence numbers of chain
    workgroups and inter-workgroup barriers) and graph replay give the
    oracle's bits."""
    p = W.dimer_system(L=18, rho=8, n_md=12, seed=5, bulk_rate=0.03)
    s0 = W.random_state(p, 102, species_B_fraction=0.2)
    g, o = _run_both(p, s0, 99, 12, 3, tuning=tuning)
    _assert_bitwise(g.get_state(), o.get_state(), str(tuning))


def test_fp64_change_of_n_md_between_calls():
    p = W.dimer_system(L=14, rho=5, n_md=10, seed=6, bulk_rate=0.05)
    s0 = W.random_state(p, 103)
    rm = _rm()
    g = rm.System(p, 3)
    g.set_state(s0)
    o = oracle.Oracle(p, 3, init=False)
    o.set_state(s0)
    for n_md, k in [(10, 2), (7, 1), (13, 2), (10, 1)]:
        g.step(n_md, k)
        o.run(n_md, k)
    _assert_bitwise(g.get_state(), o.get_state())


def test_fp64_crowded_cells_and_oversized_cell():
    """A cell holding 1500 particles (beyond one LDS group: serial path) and
    one holding 300 (several groups per tile)."""
    p = W.base_params(L=(8, 8, 8), rho=6, n_md=3)
    s0 = W.random_state(p, 104)
    rng = np.random.default_rng(5)
    for d in range(3):
        s0["x"][d, :1500] = 2.0 + rng.uniform(0.3, 0.7, 1500)
        s0["x"][d, 1500:1800] = 5.0 + rng.uniform(0.3, 0.7, 300)
    g, o = _run_both(p, s0, 11, 3, 2)
    _assert_bitwise(g.get_state(), o.get_state(), "crowded")
    _assert_obs(g.observables(), o.observables())


def test_fp64_tiny_and_empty_systems():
    for L, n in [((1, 1, 1), 5), ((3, 2, 1), 0), ((2, 2, 2), 1)]:
        p = W.base_params(L=L, rho=1, n_md=2)
        p["n_solvent"] = n
        s0 = W.random_state(p, 105)
        g, o = _run_both(p, s0, 12, 2, 3)
        _assert_bitwise(g.get_state(), o.get_state(), f"L={L} n={n}")


@pytest.mark.parametrize("mass,kT", [(1.0, 1.0), (2.0, 0.5)])
def test_fp64_anderson_thermostat(mass, kT):
    p = dict(W.dimer_system(L=14, rho=6, n_md=10, seed=7, bulk_rate=0.0), mass=mass, kT=kT)
    p["rule"] = "at"
    s0 = W.random_state(p, 106)
    g, o = _run_both(p, s0, 13, 10, 1)
    gs, os_ = g.get_state(), o.get_state()
    assert np.array_equal(gs["id"], os_["id"])
    assert np.allclose(gs["v"], os_["v"], rtol=0, atol=1e-12)
    assert np.allclose(gs["x"], os_["x"], rtol=0, atol=1e-12)
    go, oo = g.observables(), o.observables()
    assert go["temperature"] == pytest.approx(oo["temperature"], rel=1e-12)
    assert go["n_cells_T"] == oo["n_cells_T"]


def test_fp64_many_list_workgroups():
    """Large colloids and K=1: the Verlet list spans many workgroups (the
    inter-workgroup barrier and the tree over workgroups are exercised)."""
    p = W.base_params(L=(24, 24, 24), rho=10, n_md=8)
    W.add_colloid(p, (12.0, 12.0, 12.0), sigma=6.0, eps_A=1.0, eps_B=0.7, catalytic=True)
    W.add_colloid(p, (12.0, 12.0, 1.0), sigma=3.0)
    s0 = W.random_state(p, 107, species_B_fraction=0.5)
    g, o = _run_both(p, s0, 14, 8, 3, tuning=dict(chain_k=1))
    ob = g.observables()
    assert ob["n_candidates"] > 8 * 256, ob["n_candidates"]
    _assert_bitwise(g.get_state(), o.get_state(), "many workgroups")
    _assert_obs(ob, o.observables())


@pytest.mark.parametrize("n_small", [1, 2])
def test_fp64_master_exchange_over_two_row_chunks(n_small):
    """More than 128 list workgroups (one entry per thread, 256 threads) around
    one large sphere: the master form of the exchange reads its rows in two
    chunks of 128 and sums each value over 256 rows.  With one small sphere
    the two-colloid variant runs (its 8-value table), with two the generic
    one."""
    p = W.base_params(L=(32, 32, 32), rho=10, n_md=4)
    W.add_colloid(p, (16.0, 16.0, 16.0), sigma=11.0, eps_A=1.0, eps_B=0.7, catalytic=True)
    for k in range(n_small):
        W.add_colloid(p, (3.0 + 4.0 * k, 3.0, 3.0), sigma=1.5)
    p["cand_capacity"] = 65536
    s0 = W.random_state(p, 131 + n_small, species_B_fraction=0.3)
    g, o = _run_both(p, s0, 18 + n_small, 4, 2, tuning=dict(chain_k=1, chain_block=256))
    ob = g.observables()
    assert ob["n_candidates"] > 128 * 256, ob["n_candidates"]
    _assert_bitwise(g.get_state(), o.get_state(), "two row chunks")
    _assert_obs(ob, o.observables())


def test_fp64_many_colloids_with_contacts():
    """Three dimers placed inside each other's colloid-colloid cut-off plus
    two free spheres: many colloids per list entry, colloid-colloid WCA."""
    p = W.base_params(L=(26, 26, 26), rho=5, n_md=10)
    p["bulk_rate"] = 0.03
    ex = np.array([1.0, 0.0, 0.0])
    W.add_dimer(p, (8.0, 8.0, 8.0), ex)                 # C at (11.35, 8, 8)
    W.add_dimer(p, (8.0, 16.6, 8.0), ex)                # C-C 8.6 apart (< 8.98)
    W.add_dimer(p, (20.0, 20.0, 19.0), np.array([0.0, 0.6, 0.8]))
    W.add_colloid(p, (17.85, 8.0, 8.0), sigma=2.0, catalytic=True)   # 6.5 from C (< 6.73)
    W.add_colloid(p, (3.0, 3.0, 20.0), sigma=2.5)
    s0 = W.random_state(p, 109, species_B_fraction=0.3)
    g, o = _run_both(p, s0, 16, 10, 3)
    _assert_bitwise(g.get_state(), o.get_state(), "many colloids")
    _assert_obs(g.observables(), o.observables())


def test_fp64_most_colloids_free_spheres():
    """32 free spheres, the most colloids a system holds (one lane and one
    bit of the pair masks each), half catalytic, eight pairs inside each
    other's colloid-colloid cut-off."""
    p = W.base_params(L=(22, 22, 22), rho=5, n_md=10)
    p["bulk_rate"] = 0.03
    rng = np.random.default_rng(77)
    k = 0
    for ix in range(4):
        for iy in range(4):
            for iz in range(2):
                x = np.array([2.5 + 5.0 * ix, 2.5 + 5.0 * iy, 5.0 + 11.0 * iz]) + rng.uniform(-0.3, 0.3, 3)
                if k % 4 == 1:
                    x = prev + np.array([2.1, 0.0, 0.0])     # 2.1 < 2^(1/6) * 2
                W.add_colloid(p, x, 1.0, 1.0, 0.5, catalytic=k % 2 == 0,
                              ctype=W.TYPE_C if k % 2 == 0 else W.TYPE_N)
                prev = x
                k += 1
    assert len(p["colloids"]) == 32
    s0 = W.random_state(p, 113, species_B_fraction=0.3)
    g, o = _run_both(p, s0, 16, 10, 3)
    _assert_bitwise(g.get_state(), o.get_state(), "32 colloids")
    _assert_obs(g.observables(), o.observables())


def test_fp64_resume_and_determinism():
    rm = _rm()
    p = W.dimer_system(L=14, rho=6, n_md=10, seed=8, bulk_rate=0.05)
    a = rm.System(p, 21)
    a.step(10, 5)
    b = rm.System(p, 21)
    b.step(10, 2)
    st = b.get_state()
    c = rm.System(p, 21)
    c.set_state(st)
    c.step(10, 3)
    sa, sc = a.get_state(), c.get_state()
    _assert_bitwise(sa, sc, "resume")
    d = rm.System(p, 21)
    d.step(10, 5)
    _assert_bitwise(sa, d.get_state(), "determinism")


def test_fp64_full_size_dimer32_one_interval():
    """The benchmark workload at full size (32^3 cells, 327,680 particles,
    N_MD = 50), in the launch configuration the benchmark times."""
    rm = _rm()
    p = W.dimer32()
    g = rm.System(p, W.BASE_SEED + 2)
    s0 = g.get_state()
    o = oracle.Oracle(p, W.BASE_SEED + 2, init=False)
    o.set_state(s0)
    g.step(50, 1)
    o.run(50, 1)
    _assert_bitwise(g.get_state(), o.get_state(), "dimer32")
    _assert_obs(g.observables(), o.observables())


def test_fp64_full_size_sphere10():
    """The single-sphere configuration at full size (10^3 cells, rho 10,
    10,000 particles, 10 MD steps per collision), five intervals."""
    rm = _rm()
    p = W.sphere10()
    s0 = W.random_state(p, 110, species_B_fraction=0.1)
    g, o = _run_both(p, s0, W.BASE_SEED + 1, 10, 5)
    _assert_bitwise(g.get_state(), o.get_state(), "sphere10")
    _assert_obs(g.observables(), o.observables())


def test_fp64_full_size_batch_of_64_sampled_slots():
    """The 64-replica ensemble at full size (box edges from {16, 20, 24, 32},
    8.47 M particles, per-replica seeds) in FP64, one tick: sampled slots
    equal the oracle run of that replica alone, bit for bit."""
    rm = _rm()
    reps = [dict(p, precision=64) for p in W.batch_replicas(n=64, precision=64)]
    b = rm.Batch(len(reps), precision=64)
    for i, p in enumerate(reps):
        b.set_slot(i, p, p["seed"], p["n_md"])
    states = {i: b.get_state(i) for i in (0, 17, 40, 63)}
    b.step(1)
    for i, s0 in states.items():
        p = reps[i]
        print(f"[parity] batch slot {i} L={p['L']}", flush=True)
        o = oracle.Oracle(p, p["seed"], init=False)
        o.set_state(s0)
        o.run(p["n_md"], 1)
        _assert_bitwise(b.get_state(i), o.get_state(), f"slot {i}")


def test_fp64_full_size_large128_one_interval():
    """The large single system at full size: 128^3 cells, 20,971,520
    particles, 8 dimers, N_MD = 50, default launch shape (the chain with
    512-thread workgroups over its 67 k-entry list), one interval against the
    oracle, every particle compared."""
    rm = _rm()
    p = W.large128()
    seed = W.BASE_SEED + 3
    print("[parity] large128 fp64 full size", flush=True)
    g = rm.System(p, seed)
    s0 = g.get_state()
    g.step(50, 1)
    gs = g.get_state()
    go = g.observables()
    g.close()
    del g
    o = oracle.Oracle(p, seed, init=False)
    o.set_state(s0)
    del s0
    o.run(50, 1)
    _assert_bitwise(gs, o.get_state(), "large128")
    _assert_obs(go, o.observables())
    assert go["n_candidates"] > 256 * 256


def test_fp32_full_size_large128_one_interval_close_to_fp64():
    """The FP32 form of the large system, one interval from the FP64 state
    rounded to FP32, against the FP64 oracle from the same rounded state,
    matched by id: positions within 1e-5 of the box.  Velocities leave the
    collision, where a particle whose FP32 position lies within rounding of
    a cell face (a few FP32 ulps of 128, some 10^-5, so a few thousand of
    the 2 x 10^7) joins a different cell, which changes the rotation of both
    cells involved and so the velocities of about 2 rho = 20 particles per
    such particle (measured: 0.4 %).  The 99th percentile of the velocity
    error is within 1e-5 of the velocity scale and the affected fraction
    below 1 %.  One by one: outside the cells that such particles touch,
    every particle that streamed freely and shares its cell with no particle
    of the colloids' list is within 1e-5; the list particles, whose FP32
    positions enter the steep colloid potential for 50 MD steps, and their
    cell mates within 2e-3 (measured 4.7e-4 at most, 3 % of the list beyond
    1e-5)."""
    rm = _rm()
    p = W.large128(precision=32)
    seed = W.BASE_SEED + 3
    print("[parity] large128 fp32 full size", flush=True)
    g = rm.System(p, seed)
    s0 = g.get_state()                      # FP32 values, exact in FP64
    s0_coll = s0["coll_step"]
    g.step(50, 1)
    gs = g.get_state()
    g.close()
    del g
    o = oracle.Oracle(dict(p, precision=64), seed, init=False)
    o.set_state(s0)
    o.build_list(50)                        # the interval below builds the same list
    listed_ids = s0["id"][o.candidates()]
    del s0
    o.run(50, 1)
    os_ = o.get_state()
    gi, oi = np.argsort(gs["id"]), np.argsort(os_["id"])
    L = np.array(p["L"], dtype=float)[:, None]
    vs = np.abs(os_["v"]).max()
    err = np.zeros(gi.size)
    for d in range(3):
        dx = gs["x"][d, gi] - os_["x"][d, oi]
        dx -= L[d] * np.round(dx / L[d])
        assert np.abs(dx).max() <= 1e-5 * L.max()
        err = np.maximum(err, np.abs(gs["v"][d, gi] - os_["v"][d, oi]))
    off = err > 1e-5 * vs
    print(f"[parity] large128 fp32: {int(off.sum())} velocities beyond 1e-5", flush=True)
    assert np.percentile(err, 99) <= 1e-5 * vs
    assert off.mean() < 1e-2
    # One by one: the collision is the interval's last step, so the final
    # positions fix each particle's cell on the shifted grid.  A particle
    # whose shifted coordinate lies within 1e-4 of a face on either side
    # (far beyond the FP32 rounding of a coordinate near 128, 7.6e-6) or
    # whose cell differs between the two sides marks its cells on both
    # sides; every particle outside the marked cells shares its cell's
    # members with the oracle.  A key that differs has a face between the
    # two positions, so the oracle's particle lies within its own position
    # error of that face.
    sh = o.shift(int(s0_coll))[:, None]
    Li = np.array(p["L"], dtype=np.int64)
    keys, cells, near = [], [], np.zeros(gi.size, dtype=bool)
    for xs in (gs["x"][:, gi], os_["x"][:, oi]):
        f = xs - sh
        near |= (np.abs(f - np.round(f)) < 1e-4).any(axis=0)
        c = np.floor(f).astype(np.int64) % Li[:, None]
        cells.append(c)
        keys.append(c[0] + Li[0] * (c[1] + Li[1] * c[2]))
    flip = keys[0] != keys[1]
    fo = os_["x"][:, oi[flip]] - sh
    dx = np.abs(gs["x"][:, gi[flip]] - os_["x"][:, oi[flip]])
    dx = np.minimum(dx, L - dx)
    cross = (cells[0][:, flip] != cells[1][:, flip]) & (np.abs(fo - np.round(fo)) <= dx + 1e-9)
    assert (cross == (cells[0][:, flip] != cells[1][:, flip])).all()
    print(f"[parity] large128 fp32: {int(flip.sum())} cell-face flips, "
          f"{int(near.sum())} particles within 1e-4 of a face", flush=True)

    def cells_of(sel):
        m = np.zeros(int(Li.prod()), dtype=bool)
        m[keys[0][sel]] = True
        m[keys[1][sel]] = True
        return m[keys[0]] | m[keys[1]]

    clean = ~cells_of(near | flip)
    listed = np.zeros(gi.size, dtype=bool)
    listed[listed_ids] = True               # ids are 0 .. N-1, gi sorts by id
    free = clean & ~cells_of(listed)
    mixed = clean & ~free
    print(f"[parity] large128 fp32: {int((~clean).sum())} particles in marked cells; "
          f"free {int(free.sum())}, max error {err[free].max() / vs:.2e}; list and cell mates "
          f"{int(mixed.sum())}, max error {err[mixed].max() / vs:.2e}, "
          f"{int((listed & off).sum())} of {int(listed.sum())} listed beyond 1e-5", flush=True)
    assert free.mean() > 0.9
    assert err[free].max() <= 1e-5 * vs
    assert err[mixed].max() <= 2e-3 * vs
    assert (listed & off).sum() <= 0.1 * listed.sum()
    assert np.allclose(gs["X"], os_["X"], rtol=1e-6, atol=1e-6)


# ---------------------------------------------------------------- errors ---

def test_errors_are_reported():
    rm = _rm()
    p = W.dimer_system(L=14, rho=6, n_md=10, seed=9)
    g = rm.System(p, 1)
    s = g.get_state()
    bad = dict(s)
    bad["x"] = s["x"].copy()
    bad["x"][0, 0] = 14.0                              # outside [0, L)
    with pytest.raises(rm.RmpError):
        g.set_state(bad)
    with pytest.raises(rm.RmpError):
        g.step(0, 1)
    q = dict(p)
    q["cand_capacity"] = 16                            # far too small
    h = rm.System(q, 1)
    h.step(10, 1)
    with pytest.raises(rm.RmpError) as e:
        h.observables()
    assert e.value.flags & 16
    # the entries beyond the capacity stream freely: every particle is still
    # binned exactly once
    hs = h.get_state()
    assert np.array_equal(np.sort(hs["id"]), np.arange(hs["id"].size))
    L = np.array(q["L"], dtype=float)[:, None]
    assert ((hs["x"] >= 0.0) & (hs["x"] < L)).all()
    assert np.isfinite(hs["v"]).all()


def test_set_state_rejects_invalid_states_and_nonfinite_cell_is_flagged():
    """set_state applies the library's state check before uploading (a NaN
    velocity, a duplicated id, a particle deep in a colloid core are
    rejected and the system keeps its state); a finite state whose cell
    velocity overflows in the collision latches the non-finite flag.  The
    overflowing particles leave the box in one step, so this is a GPU-side
    check of the flag (the kernels' cell index guards keep every access in
    bounds); the oracle's flag is pinned on the CPU."""
    rm = _rm()
    p = W.dimer_system(L=14, rho=6, n_md=10, seed=9)
    g = rm.System(p, 1)
    s = g.get_state()
    for what in ("v", "id", "core"):
        bad = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in s.items()}
        if what == "v":
            bad["v"][1, 3] = np.nan
        elif what == "id":
            bad["id"][4] = bad["id"][5]
        else:
            bad["x"][:, 4] = np.mod(s["X"][0], 14.0)
        with pytest.raises(rm.RmpError):
            g.set_state(bad)
    after = g.get_state()
    for k in ("x", "v", "id", "state"):
        assert np.array_equal(after[k], s[k]), k
    q = W.base_params(L=(6, 6, 6), rho=3, n_md=2)
    h = rm.System(q, 3)
    st = W.random_state(q, 4)
    st["x"][:, 1] = st["x"][:, 0]
    st["v"][:, 0] = st["v"][:, 1] = 1.5e308
    h.set_state(st)
    print("[parity] overflowing cell velocity: 6^3 cells, two particles at 1.5e308", flush=True)
    h.step(2, 1)
    assert h.observables(raise_on_flags=False)["flags"] & 4


def test_chain_wait_budget_exceeded_is_reported():
    """A chain workgroup that waits longer than its budget for the other
    workgroups' values gives up, raises RMP_FLAG_BARRIER and waits no more,
    so the launch ends.  Forced from the host with a budget of 1 us on a
    list of some thirty workgroups: the interval is then flagged, or (had
    every wait ended in time) equal to the oracle's.  A new system on the
    same device, with the default budget, then matches the oracle bit for
    bit.  Some 34 workgroups meet at more than 40 barriers per call and one
    exchange alone takes about 2 us, so under a 1 us budget some wait always
    expires: the flag is required."""
    rm = _rm()
    p = W.dimer_system(L=32, rho=10, n_md=10, seed=21, bulk_rate=0.01)
    s0 = W.random_state(p, 81)
    o = oracle.Oracle(p, 7, init=False)
    o.set_state(s0)
    o.run(p["n_md"], 2)
    g = rm.System(p, 7)
    with pytest.raises(rm.RmpError):
        g.set_tuning(barrier_budget_us=10_000_001)
    g.set_tuning(barrier_budget_us=1, use_graph=0)
    assert g.get_tuning()["barrier_budget_us"] == 1
    g.set_state(s0)
    print(f"[parity] budget 1 us: N={p['n_solvent']} n_md={p['n_md']}", flush=True)
    g.step(p["n_md"], 2)
    flags = g.observables(raise_on_flags=False)["flags"]
    print(f"[parity] budget 1 us: flags {flags} (time-out path {'taken' if flags & 32 else 'NOT taken'})",
          flush=True)
    assert flags & 32, "a 1 us wait budget expired nowhere: the budget is not honoured"
    with pytest.raises(rm.RmpError) as e:
        g.observables()
    assert e.value.flags & 32
    g.close()
    h = rm.System(p, 7)
    h.set_state(s0)
    h.step(p["n_md"], 2)
    assert h.observables()["flags"] == 0
    _assert_bitwise(h.get_state(), o.get_state(), "default budget")


def test_colloid_displacement_flag_matches_oracle():
    """A dimer driven across more than half the skin within one interval:
    the GPU and the oracle raise the displacement flag alike and their
    trajectories stay equal bit for bit."""
    rm = _rm()
    p = W.dimer_system(L=14, rho=5, n_md=10, seed=9, bulk_rate=0.0)
    s0 = W.random_state(p, 71)
    s0["V"] = np.tile(np.array([3.0, 0.0, 0.0]), (2, 1))   # 0.3 per interval > skin / 2
    g = rm.System(p, 5)
    g.set_state(s0)
    o = oracle.Oracle(p, 5, init=False)
    o.set_state(s0)
    g.step(p["n_md"], 1)
    o.run(p["n_md"], 1)
    go, oo = g.observables(raise_on_flags=False), o.observables()
    assert oo["flags"] & 1
    assert go["flags"] == oo["flags"]
    with pytest.raises(rm.RmpError) as e:
        g.observables()
    assert e.value.flags & 1
    _assert_bitwise(g.get_state(), o.get_state(), "displacement flag")


# ----------------------------------------------------------------- FP32 ---

def test_fp32_one_interval_close_to_fp64_oracle():
    p = W.dimer_system(L=16, rho=6, n_md=20, seed=10, bulk_rate=0.0, precision=32)
    s0 = W.random_state(p, 108, float32=True)
    g, o = _run_both(p, s0, 15, 20, 1)
    gs, os_ = g.get_state(), o.get_state()
    gi, oi = np.argsort(gs["id"]), np.argsort(os_["id"])
    L = np.array(p["L"], dtype=float)[:, None]
    dx = gs["x"][:, gi] - os_["x"][:, oi]
    dx -= L * np.round(dx / L)
    assert np.abs(dx).max() <= 1e-5 * L.max()
    dv = gs["v"][:, gi] - os_["v"][:, oi]
    assert np.abs(dv).max() <= 1e-5 * np.abs(os_["v"]).max()
    assert np.allclose(gs["X"], os_["X"], rtol=1e-6, atol=1e-6)


# ---------------------------------------------------------------- batch ---

def test_batch_replicas_match_alone_and_oracle():
    rm = _rm()
    ps = [W.dimer_system(L=L, rho=5, n_md=nmd, seed=20 + i, bulk_rate=0.03)
          for i, (L, nmd) in enumerate([(14, 10), (16, 7), (12, 10), (18, 5)])]
    ps.append(W.base_params(L=(9, 7, 5), rho=6, n_md=4))
    seeds = [31, 32, 33, 34, 35]
    b = rm.Batch(len(ps), precision=64)
    states = []
    for i, p in enumerate(ps):
        b.set_slot(i, p, seeds[i], p["n_md"])
        s0 = W.random_state(p, 200 + i, species_B_fraction=0.2)
        b.set_state(i, s0)
        states.append(s0)
    b.step(3)
    for i, p in enumerate(ps):
        o = oracle.Oracle(p, seeds[i], init=False)
        o.set_state(states[i])
        o.run(p["n_md"], 3)
        fl = b.observables(i, raise_on_flags=False)["flags"]
        _assert_bitwise(b.get_state(i), o.get_state(), f"replica {i} (flags {fl})")
        _assert_obs(b.observables(i), o.observables())
    # retire one, admit another, keep stepping: the others are unaffected
    b.clear_slot(1)
    q = W.dimer_system(L=15, rho=5, n_md=9, seed=40, bulk_rate=0.03)
    b.set_slot(1, q, 41, 9)
    sq = W.random_state(q, 300)
    b.set_state(1, sq)
    b.step(2)
    o = oracle.Oracle(q, 41, init=False)
    o.set_state(sq)
    o.run(9, 2)
    _assert_bitwise(b.get_state(1), o.get_state(), "admitted")
    o0 = oracle.Oracle(ps[0], seeds[0], init=False)
    o0.set_state(states[0])
    o0.run(ps[0]["n_md"], 5)
    _assert_bitwise(b.get_state(0), o0.get_state(), "replica 0 after 5 ticks")


def test_batch_chain_waves_match_resident_launch_and_oracle():
    """64 replicas with one list entry per chain thread and the K raise
    switched off: far more chain workgroups than the device holds at once,
    so they run in waves through the ticketed work list.  Every replica ends
    bit-identical to the launch shape that fits on the device, none reports a
    timed-out exchange wait, and two sampled replicas match the oracle."""
    rm = _rm()
    ps = W.batch_replicas(n=64, edges=(16, 20, 24), precision=64)
    for p in ps:
        p["n_md"] = 10
    states = [W.random_state(p, 500 + i, species_B_fraction=0.1) for i, p in enumerate(ps)]
    out = {}
    for name, tun in (("waves", dict(chain_k=1, chain_resident=1 << 30)), ("resident", {})):
        print(f"[parity] batch of {len(ps)} tuning={tun}", flush=True)
        b = rm.Batch(len(ps), precision=64)
        if tun:
            b.set_tuning(**tun)
        for i, p in enumerate(ps):
            b.set_slot(i, p, p["seed"], p["n_md"])
            b.set_state(i, states[i])
        b.step(1)
        out[name] = [b.get_state(i) for i in range(len(ps))]
        flags = [b.observables(i, raise_on_flags=False)["flags"] for i in range(len(ps))]
        assert not any(flags), f"{name}: flagged replicas {[i for i, f in enumerate(flags) if f]}"
        del b
    for i in range(len(ps)):
        _assert_bitwise(out["waves"][i], out["resident"][i], f"replica {i}")
    for i in (0, len(ps) - 1):
        o = oracle.Oracle(ps[i], ps[i]["seed"], init=False)
        o.set_state(states[i])
        o.run(ps[i]["n_md"], 1)
        _assert_bitwise(out["waves"][i], o.get_state(), f"replica {i} vs oracle")


def test_fp32_drift_against_fp64_is_bounded():
    """FP32 state against FP64 (the oracle's trajectory, bitwise) from one
    initial state, 20 intervals of a 16^3 dimer system: total momentum, which
    the method conserves exactly, drifts by rounding only (FP64 to 1e-12,
    FP32 to 1e-5 of the thermal momentum sqrt(N m kT)); the total energy
    KE + U - e_rxn of the two forms agrees to 1e-4 relative."""
    rm = _rm()
    p64 = W.dimer_system(L=16, rho=10, n_md=50, seed=5, bulk_rate=0.01)
    p32 = dict(p64, precision=32)
    st0 = W.random_state(p64, 91)
    out = {}
    for prec, p in ((64, p64), (32, p32)):
        s = rm.System(p, 17)
        s.set_state(st0)
        P, E = [], []
        for k in range(21):
            if k:
                s.step(p["n_md"], 1)
            o = s.observables()
            P.append(np.array(o["momentum"]))
            E.append(o["ke_solvent"] + o["ke_colloid"] + o["potential"] - o["e_rxn"])
        out[prec] = (np.array(P), np.array(E))
    scale = math.sqrt(p64["n_solvent"] * p64["mass"] * p64["kT"])
    P64, E64 = out[64]
    P32, E32 = out[32]
    assert np.max(np.linalg.norm(P64 - P64[0], axis=1)) / scale < 1e-12
    assert np.max(np.linalg.norm(P32 - P32[0], axis=1)) / scale < 1e-5
    assert np.max(np.abs(E32 - E64)) / abs(E64[0]) < 1e-4
