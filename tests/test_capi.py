"""The C-ABI library loads, exports every entry point include/rmpmd.h
declares, and the ctypes mirrors of its structs match the header's layout
(checked against the header compiled by gcc).  No compute calls: no GPU."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmpmd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rmp_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1608_04904_amd import _capi
    lib = _capi.lib()
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(_capi.SIGNATURES), set(declared) ^ set(_capi.SIGNATURES)


def test_struct_layout_matches_header():
    from paper_1608_04904_amd import _capi
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "rmpmd.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(rmp_params), sizeof(rmp_obs), sizeof(rmp_host_state), sizeof(rmp_tuning));
  printf("%zu %zu %zu %zu\n", offsetof(rmp_params, colloid_x), offsetof(rmp_params, bond_d),
         offsetof(rmp_obs, flags), offsetof(rmp_obs, colloid_V));
  printf("%zu %zu %zu %zu %d\n", sizeof(rmp_analysis_params), sizeof(rmp_analysis_out),
         offsetof(rmp_analysis_params, hist_rmax), offsetof(rmp_analysis_out, hist), RMP_SERIES_FIELDS);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    sizes = list(map(int, out))
    assert sizes[0] == C.sizeof(_capi.Params)
    assert sizes[1] == C.sizeof(_capi.Obs)
    assert sizes[2] == C.sizeof(_capi.HostState)
    assert sizes[3] == C.sizeof(_capi.Tuning)
    assert sizes[4] == _capi.Params.colloid_x.offset
    assert sizes[5] == _capi.Params.bond_d.offset
    assert sizes[6] == _capi.Obs.flags.offset
    assert sizes[7] == _capi.Obs.colloid_V.offset
    assert sizes[8] == C.sizeof(_capi.AnalysisParams)
    assert sizes[9] == C.sizeof(_capi.AnalysisOut)
    assert sizes[10] == _capi.AnalysisParams.hist_rmax.offset
    assert sizes[11] == _capi.AnalysisOut.hist.offset
    assert sizes[12] == _capi.SERIES_FIELDS


def test_workspace_bytes_and_validation_on_host():
    """rmp_workspace_bytes is a pure host function: usable without a GPU."""
    import workloads as W
    from paper_1608_04904_amd import _capi, workspace_bytes
    p = W.dimer32()
    n64 = workspace_bytes(p)
    p32 = dict(p); p32["precision"] = 32
    n32 = workspace_bytes(p32)
    # FP64: two x, v buffers (96 B), ids and states (10 B), key/rank (8 B), the
    # 64-byte staging record of the scatter, list flag, cell arrays
    assert 150 * p["n_solvent"] < n64 < 220 * p["n_solvent"]
    assert n32 < n64
    bad = dict(p); bad["L"] = (0, 32, 32)
    with pytest.raises(_capi.RmpError):
        workspace_bytes(bad)
    bad = dict(p); bad["precision"] = 16
    with pytest.raises(_capi.RmpError):
        workspace_bytes(bad)
    small = W.base_params(L=(6, 6, 6), rho=5)
    W.add_colloid(small, (3, 3, 3), sigma=4.0)      # reach beyond half the box
    with pytest.raises(_capi.RmpError):
        workspace_bytes(small)


def test_analysis_bytes_and_validation_on_host():
    import workloads as W
    from paper_1608_04904_amd import _capi, analysis_bytes
    p = W.dimer32()
    a = dict(every=1, series_cap=1000, hist_nz=64, hist_nr=32, hist_zmax=10.0, hist_rmax=8.0)
    n = analysis_bytes(p, a)
    assert n >= 2 * 64 * 32 * 8 + 1000 * 10 * 8 + 1000 * 8 + 1000 * 8
    assert analysis_bytes(p, dict(a, series_cap=2000)) > n
    for bad in (dict(every=0), dict(series_cap=0), dict(hist_nz=0), dict(hist_nr=-1),
                dict(hist_zmax=0.0), dict(hist_rmax=float("nan")), dict(hist_zmax=float("inf"))):
        with pytest.raises(_capi.RmpError):
            analysis_bytes(p, dict(a, **bad))
    nob = W.sphere10()                                   # no bond: no dimer to analyse
    with pytest.raises(_capi.RmpError):
        analysis_bytes(nob, a)


def test_flow_parameters_validated_on_host():
    import workloads as W
    from paper_1608_04904_amd import _capi, workspace_bytes

    def flow(walls=1, g=(0.0, 0.0, 0.0), **kw):
        p = W.base_params(L=(6, 6, 6), rho=5, **kw)
        p.update(walls=walls, wall_density=5, accel=g)
        return p
    assert workspace_bytes(flow()) > workspace_bytes(W.base_params(L=(6, 6, 6), rho=5))  # one layer more
    workspace_bytes(flow(walls=0, g=(0.1, 0.0, 0.2), rule="at"))   # periodic acceleration: any rule
    bad = [flow(rule="at"), dict(flow(), cell_order="hilbert"), flow(g=(0.0, 0.0, 0.1)),
           dict(flow(), wall_density=0), dict(flow(), wall_density=2000), dict(flow(), walls=2),
           flow(walls=0, g=(float("nan"), 0.0, 0.0))]
    col = flow(walls=0, g=(0.1, 0.0, 0.0))
    W.add_colloid(col, (3, 3, 3), sigma=1.0)
    bad.append(col)
    for p in bad:
        with pytest.raises(_capi.RmpError):
            workspace_bytes(p)


def test_rigid_body_parameters_validated_on_host():
    import workloads as W
    from paper_1608_04904_amd import _capi, workspace_bytes
    p = W.janus_system(L=16, rho=4, n_md=5, seed=3)
    assert len(p["bonds"]) == 42
    workspace_bytes(p)
    workspace_bytes(dict(W.dimer_system(L=14, rho=4), rattle_iterative=1))
    for bad in (dict(p, rattle_tol=0.0), dict(p, rattle_maxit=0), dict(p, rattle_maxit=200000),
                dict(p, bonds=p["bonds"] + [p["bonds"][3]]),
                dict(p, bonds=p["bonds"][:-1] + [(0, 0, 1.0)]),
                dict(W.dimer_system(L=14, rho=4), rattle_iterative=2)):
        with pytest.raises(_capi.RmpError):
            workspace_bytes(bad)


def test_product_package_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_1608_04904_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text, f
                assert "rmp_oracle" not in text, f


# --------------------------------------------------------------------------
# rmp_check_state: the host-side check every rmp_set_state applies before
# uploading (a pure host function, so it runs here without a GPU).
# --------------------------------------------------------------------------
def _state_case():
    import workloads as W
    p = W.dimer_system(L=16, rho=3, n_md=10, seed=3)
    return p, W.random_state(p, 5, species_B_fraction=0.3, flag_fraction=0.05)


def _status(p, s):
    import paper_1608_04904_amd as rm
    return rm.check_state(p, s)


def test_check_state_accepts_a_valid_state():
    p, s = _state_case()
    assert _status(p, s) == 0
    # FP32 system: a velocity that still rounds to a finite float is fine
    s["v"][1, 7] = 3.0e38
    assert _status(dict(p, precision=32), s) == 0


@pytest.mark.parametrize("what", [
    "x_above_L", "x_negative", "x_nan", "v_nan", "v_inf", "v_float_overflow",
    "id_duplicate", "id_out_of_range", "state_bits", "X_nan", "V_inf", "particle_in_core",
])
def test_check_state_rejects(what):
    import numpy as np
    from paper_1608_04904_amd import _capi
    p, s = _state_case()
    prec = 64
    if what == "x_above_L":
        s["x"][0, 3] = 16.0
    elif what == "x_negative":
        s["x"][2, 3] = -1e-12
    elif what == "x_nan":
        s["x"][1, 3] = np.nan
    elif what == "v_nan":
        s["v"][0, 10] = np.nan
    elif what == "v_inf":
        s["v"][2, 11] = -np.inf
    elif what == "v_float_overflow":
        s["v"][1, 7] = 1.0e39              # finite in FP64, infinite as a float
        prec = 32
    elif what == "id_duplicate":
        s["id"][5] = s["id"][6]
    elif what == "id_out_of_range":
        s["id"][5] = p["n_solvent"]
    elif what == "state_bits":
        s["state"][9] = 4
    elif what == "X_nan":
        s["X"][1, 0] = np.nan
    elif what == "V_inf":
        s["V"][0, 2] = np.inf
    elif what == "particle_in_core":
        X0 = np.mod(s["X"][0], 16.0)
        s["x"][:, 4] = X0 + np.array([0.3, -0.2, 0.1]) * p["colloids"][0]["sigma"] / 2
    assert _status(dict(p, precision=prec), s) == _capi.EINVAL


def test_check_state_core_boundary():
    """Inside sigma/2 of a colloid centre is rejected, just outside accepted
    (minimum image across the periodic boundary)."""
    import numpy as np
    from paper_1608_04904_amd import _capi
    p, s = _state_case()
    sig = p["colloids"][0]["sigma"]
    X0 = np.mod(s["X"][0], 16.0)
    ax = np.array([1.0, 0.0, 0.0])
    s["x"][:, 4] = np.mod(X0 + 0.501 * sig * ax, 16.0)
    assert _status(p, s) == 0
    s["x"][:, 4] = np.mod(X0 + 0.499 * sig * ax, 16.0)
    assert _status(p, s) == _capi.EINVAL
