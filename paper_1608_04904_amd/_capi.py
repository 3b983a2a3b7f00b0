"""ctypes declarations of the rmpmd C ABI (include/rmpmd.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``librmpmd.so``.  Importing this module raises if the library is missing;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmpmd.so")

MAX_COLLOIDS = 32
MAX_BONDS = 96
PTABLE = 1024

OK, EINVAL, ENOMEM, EHIP, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
FLAG_DISPLACEMENT, FLAG_RATTLE, FLAG_NONFINITE, FLAG_INIT, FLAG_LIST_OVERFLOW, FLAG_BARRIER = (
    1, 2, 4, 8, 16, 32)


class Params(C.Structure):
    _fields_ = [
        ("L", C.c_int32 * 3), ("precision", C.c_int32), ("n_solvent", C.c_int64),
        ("kT", C.c_double), ("mass", C.c_double), ("dt", C.c_double),
        ("alpha", C.c_double), ("skin", C.c_double), ("cat_prob", C.c_double),
        ("bulk_rate", C.c_double), ("rule", C.c_int32), ("n_colloids", C.c_int32),
        ("n_bonds", C.c_int32), ("cand_capacity", C.c_int32),
        ("colloid_x", (C.c_double * 3) * MAX_COLLOIDS),
        ("colloid_mass", C.c_double * MAX_COLLOIDS), ("sigma", C.c_double * MAX_COLLOIDS),
        ("eps_A", C.c_double * MAX_COLLOIDS), ("eps_B", C.c_double * MAX_COLLOIDS),
        ("catalytic", C.c_int32 * MAX_COLLOIDS), ("ctype", C.c_int32 * MAX_COLLOIDS),
        ("eps_cc", (C.c_double * 2) * 2), ("bond_a", C.c_int32 * MAX_BONDS),
        ("bond_b", C.c_int32 * MAX_BONDS), ("bond_d", C.c_double * MAX_BONDS),
        ("cell_order", C.c_int32), ("pad_order", C.c_int32),
        ("walls", C.c_int32), ("wall_density", C.c_int32), ("accel", C.c_double * 3),
        ("rattle_tol", C.c_double), ("rattle_maxit", C.c_int32), ("rattle_iterative", C.c_int32),
    ]

CELL_ORDERS = {"row": 0, "hilbert": 1}


class Obs(C.Structure):
    _fields_ = [
        ("momentum", C.c_double * 3), ("ke_solvent", C.c_double),
        ("ke_colloid", C.c_double), ("potential", C.c_double),
        ("temperature", C.c_double), ("e_rxn", C.c_double),
        ("n_A", C.c_int64), ("n_B", C.c_int64), ("n_cat_flips", C.c_int64),
        ("n_bulk_flips", C.c_int64), ("md_step", C.c_int64), ("coll_step", C.c_int64),
        ("n_candidates", C.c_int64), ("n_cells_T", C.c_int64), ("flags", C.c_uint32),
        ("pad", C.c_int32), ("colloid_X", (C.c_double * 3) * MAX_COLLOIDS),
        ("colloid_V", (C.c_double * 3) * MAX_COLLOIDS),
    ]


class HostState(C.Structure):
    _fields_ = [
        ("x", C.c_void_p), ("v", C.c_void_p), ("id", C.c_void_p), ("state", C.c_void_p),
        ("X", C.c_void_p), ("V", C.c_void_p), ("md_step", C.c_int64), ("coll_step", C.c_int64),
    ]


class Tuning(C.Structure):
    _fields_ = [
        ("stream_block", C.c_int32), ("stream_ppt", C.c_int32), ("collide_cells", C.c_int32),
        ("chain_k", C.c_int32), ("use_graph", C.c_int32), ("chain_resident", C.c_int32),
        ("chain_block", C.c_int32), ("barrier_budget_us", C.c_int32),
        ("collide_block", C.c_int32), ("collide_ppt", C.c_int32), ("collide_xcd", C.c_int32),
        ("chain_serial", C.c_int32),
    ]


SERIES_FIELDS = 10   # R_com[3], V_com[3], axis u[3], directed velocity


class AnalysisParams(C.Structure):
    _fields_ = [
        ("every", C.c_int32), ("series_cap", C.c_int32), ("hist_nz", C.c_int32),
        ("hist_nr", C.c_int32), ("hist_zmax", C.c_double), ("hist_rmax", C.c_double),
    ]


class AnalysisOut(C.Structure):
    _fields_ = [
        ("n_samples", C.c_int64), ("n_dropped", C.c_int64), ("md_step", C.c_void_p),
        ("series", C.c_void_p), ("hist", C.c_void_p),
    ]


# name -> (restype, argtypes); the full exported surface of include/rmpmd.h
P, I32, I64, U64, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
SIGNATURES = {
    "rmp_status_string": (C.c_char_p, [I32]),
    "rmp_last_error": (C.c_char_p, []),
    "rmp_workspace_bytes": (SZ, [C.POINTER(Params), C.POINTER(I32)]),
    "rmp_init_system": (I32, [C.POINTER(Params), U64, P, SZ, P, C.POINTER(P)]),
    "rmp_step": (I32, [P, I32, I32]),
    "rmp_observables": (I32, [P, C.POINTER(Obs)]),
    "rmp_observables_noalloc": (I32, [P, C.POINTER(Obs)]),
    "rmp_get_state": (I32, [P, C.POINTER(HostState)]),
    "rmp_set_state": (I32, [P, C.POINTER(HostState)]),
    "rmp_check_state": (I32, [C.POINTER(Params), C.POINTER(HostState)]),
    "rmp_destroy": (I32, [P]),
    "rmp_set_tuning": (I32, [P, C.POINTER(Tuning)]),
    "rmp_get_tuning": (I32, [P, C.POINTER(Tuning)]),
    "rmp_profile": (I32, [P, I32]),
    "rmp_profile_read": (I32, [P, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                               C.POINTER(I64), I32]),
    "rmp_batch_ctl_bytes": (SZ, [I32]),
    "rmp_batch_create": (I32, [I32, I32, P, SZ, P, C.POINTER(P)]),
    "rmp_batch_set_slot": (I32, [P, I32, C.POINTER(Params), U64, I32, P, SZ]),
    "rmp_batch_clear_slot": (I32, [P, I32]),
    "rmp_batch_step": (I32, [P, I32]),
    "rmp_batch_slot_observables": (I32, [P, I32, C.POINTER(Obs)]),
    "rmp_batch_get_state": (I32, [P, I32, C.POINTER(HostState)]),
    "rmp_batch_set_state": (I32, [P, I32, C.POINTER(HostState)]),
    "rmp_batch_set_tuning": (I32, [P, C.POINTER(Tuning)]),
    "rmp_batch_set_slot_tuning": (I32, [P, I32, C.POINTER(Tuning)]),
    "rmp_batch_destroy": (I32, [P]),
    "rmp_analysis_bytes": (SZ, [C.POINTER(Params), C.POINTER(AnalysisParams), C.POINTER(I32)]),
    "rmp_analysis_attach": (I32, [P, C.POINTER(AnalysisParams), P, SZ]),
    "rmp_analysis_detach": (I32, [P]),
    "rmp_analysis_read": (I32, [P, C.POINTER(AnalysisOut)]),
    "rmp_analysis_msd": (I32, [P, I32, P]),
    "rmp_batch_analysis_attach": (I32, [P, I32, C.POINTER(AnalysisParams), P, SZ]),
    "rmp_batch_analysis_detach": (I32, [P, I32]),
    "rmp_batch_analysis_read": (I32, [P, I32, C.POINTER(AnalysisOut)]),
    "rmp_batch_analysis_msd": (I32, [P, I32, I32, P]),
}

_lib = None


def lib():
    """Load librmpmd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class RmpError(RuntimeError):
    def __init__(self, status: int, what: str = "", flags: int = 0, detail: bool = False):
        msg = lib().rmp_status_string(status).decode()
        if status == EHIP or detail:
            msg += " [" + lib().rmp_last_error().decode() + "]"
        super().__init__(f"{what}: {msg} (status {status}, flags {flags:#x})")
        self.status = status
        self.flags = flags


def check(status: int, what: str = ""):
    if status != OK:
        raise RmpError(status, what)
    return status


def make_params(p: dict) -> Params:
    q = Params()
    for d in range(3):
        q.L[d] = int(p["L"][d])
    q.precision = int(p.get("precision", 64))
    q.n_solvent = int(p["n_solvent"])
    q.kT, q.mass, q.dt = float(p["kT"]), float(p["mass"]), float(p["dt"])
    q.alpha, q.skin = float(p["alpha"]), float(p["skin"])
    q.cat_prob, q.bulk_rate = float(p["cat_prob"]), float(p["bulk_rate"])
    q.rule = {"srd": 0, "at": 1}[p.get("rule", "srd")]
    q.cand_capacity = int(p.get("cand_capacity", 0))
    q.cell_order = CELL_ORDERS[p.get("cell_order", "row")]
    q.walls = int(p.get("walls", 0))
    q.wall_density = int(p.get("wall_density", 0))
    for d, g in enumerate(p.get("accel", (0.0, 0.0, 0.0))):
        q.accel[d] = float(g)
    cols = p["colloids"]
    if len(cols) > MAX_COLLOIDS:
        raise ValueError("too many colloids")
    q.n_colloids = len(cols)
    for c, col in enumerate(cols):
        for d in range(3):
            q.colloid_x[c][d] = float(col["x"][d])
        q.colloid_mass[c], q.sigma[c] = float(col["mass"]), float(col["sigma"])
        q.eps_A[c], q.eps_B[c] = float(col["eps_A"]), float(col["eps_B"])
        q.catalytic[c] = int(bool(col["catalytic"]))
        q.ctype[c] = int(col["type"])
    for a in range(2):
        for b in range(2):
            q.eps_cc[a][b] = float(p["eps_cc"][a][b])
    q.n_bonds = len(p["bonds"])
    if q.n_bonds > MAX_BONDS:
        raise ValueError("too many bonds")
    for k, (a, b, dd) in enumerate(p["bonds"]):
        q.bond_a[k], q.bond_b[k], q.bond_d[k] = int(a), int(b), float(dd)
    q.rattle_tol = float(p.get("rattle_tol", 1e-10))
    q.rattle_maxit = int(p.get("rattle_maxit", 500))
    q.rattle_iterative = int(p.get("rattle_iterative", 0))
    return q


def obs_dict(o: Obs, nc: int) -> dict:
    d = {k: getattr(o, k) for k, _ in Obs._fields_ if k not in ("pad", "colloid_X", "colloid_V")}
    d["momentum"] = [o.momentum[i] for i in range(3)]
    d["colloid_X"] = [[o.colloid_X[c][i] for i in range(3)] for c in range(nc)]
    d["colloid_V"] = [[o.colloid_V[c][i] for i in range(3)] for c in range(nc)]
    return d


def make_analysis_params(a: dict) -> AnalysisParams:
    q = AnalysisParams()
    q.every, q.series_cap = int(a.get("every", 1)), int(a["series_cap"])
    q.hist_nz, q.hist_nr = int(a["hist_nz"]), int(a["hist_nr"])
    q.hist_zmax, q.hist_rmax = float(a["hist_zmax"]), float(a["hist_rmax"])
    return q

