"""rmp_observables_noalloc (static device scratch, no allocation in the
call) against rmp_observables on the same systems: identical results, on two
calls in a row with the second system smaller than the first, in FP64 and
FP32, and a clear refusal of a system beyond the scratch's limit."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("momentum", "ke_solvent", "ke_colloid", "potential", "temperature", "n_cells_T", "e_rxn",
          "n_A", "n_B", "n_cat_flips", "n_bulk_flips", "md_step", "coll_step", "n_candidates", "flags",
          "colloid_X", "colloid_V")


def _rm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_04904_amd as rm
    return rm


def _same(a: dict, b: dict):
    for k in FIELDS:
        x, y = np.asarray(a[k], dtype=float), np.asarray(b[k], dtype=float)
        assert np.array_equal(x, y), (k, x, y)


@pytest.mark.parametrize("precision", [64, 32])
def test_noalloc_matches_observables_on_two_calls_second_smaller(precision):
    rm = _rm()
    big = W.dimer_system(24, precision=precision, seed=W.BASE_SEED + 41)
    small = W.sphere10(precision=precision)
    assert small["n_solvent"] < big["n_solvent"]
    for p, seed, n_md in ((big, W.BASE_SEED + 42, 50), (small, W.BASE_SEED + 43, 10)):
        print(f"[noalloc] precision={precision} L={p['L']} N={p['n_solvent']} n_md={n_md}", flush=True)
        s = rm.System(p, seed)
        s.step(n_md, 3)
        ref = s.observables()
        got = s.observables_noalloc()
        _same(ref, got)
        assert got["n_A"] + got["n_B"] == p["n_solvent"]
        assert math.isfinite(got["ke_solvent"]) and got["ke_solvent"] > 0
        # a second call on the same state gives the same result again
        _same(ref, s.observables_noalloc())
        s.close()


def test_noalloc_refuses_a_system_beyond_its_scratch():
    rm = _rm()
    from paper_1608_04904_amd import _capi
    # 34,560,000 particles: more than the 33,553,408 the scratch can sum
    p = W.base_params(L=(120, 120, 120), rho=20, dt=0.01, n_md=1, precision=32)
    print(f"[noalloc] oversized N={p['n_solvent']}", flush=True)
    s = rm.System(p, W.BASE_SEED + 44)
    with pytest.raises(rm.RmpError) as e:
        s.observables_noalloc()
    assert e.value.status == _capi.ENOMEM
    assert "static scratch" in str(e.value)
    # the allocating call still works on it, and a small system after it
    # gets its results from the scratch again
    assert s.observables()["n_A"] == p["n_solvent"]
    s.close()
    q = W.sphere10(precision=64)
    t = rm.System(q, W.BASE_SEED + 45)
    t.step(10, 1)
    _same(t.observables(), t.observables_noalloc())
    t.close()
