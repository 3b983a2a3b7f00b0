"""FP64 CPU oracle for the MPCD+MD solvent path -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product package never
imports it and shares no code with it.

The arithmetic lives in ``rmp_oracle.c`` (plain C, FP64, contraction off);
this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
MAXC = 32
MAXB = 96
PTABLE = 1024

F_DISPLACEMENT, F_RATTLE, F_NONFINITE, F_INIT = 1, 2, 4, 8


def build(verbose=False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           os.path.join(_HERE, "rmp_oracle.c"), "-o", _SO + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [
        ("L", C.c_int32 * 3), ("rule", C.c_int32), ("n_solvent", C.c_int64),
        ("kT", C.c_double), ("mass", C.c_double), ("dt", C.c_double),
        ("alpha", C.c_double), ("skin", C.c_double), ("cat_prob", C.c_double),
        ("bulk_rate", C.c_double), ("n_colloids", C.c_int32), ("n_bonds", C.c_int32),
        ("cx", (C.c_double * 3) * MAXC), ("cmass", C.c_double * MAXC),
        ("sigma", C.c_double * MAXC), ("epsA", C.c_double * MAXC),
        ("epsB", C.c_double * MAXC), ("catalytic", C.c_int32 * MAXC),
        ("ctype", C.c_int32 * MAXC), ("eps_cc", (C.c_double * 2) * 2),
        ("bond_a", C.c_int32 * MAXB), ("bond_b", C.c_int32 * MAXB),
        ("bond_d", C.c_double * MAXB), ("cell_order", C.c_int32), ("pad", C.c_int32),
        ("walls", C.c_int32), ("wall_density", C.c_int32), ("accel", C.c_double * 3),
        ("rattle_tol", C.c_double), ("rattle_maxit", C.c_int32), ("rattle_iterative", C.c_int32),
    ]


class Obs(C.Structure):
    _fields_ = [
        ("momentum", C.c_double * 3), ("ke_solvent", C.c_double),
        ("ke_colloid", C.c_double), ("potential", C.c_double),
        ("temperature", C.c_double), ("e_rxn", C.c_double),
        ("n_A", C.c_int64), ("n_B", C.c_int64), ("n_cat_flips", C.c_int64),
        ("n_bulk_flips", C.c_int64), ("md_step", C.c_int64),
        ("coll_step", C.c_int64), ("n_candidates", C.c_int64),
        ("n_cells_T", C.c_int64), ("flags", C.c_int32), ("pad", C.c_int32),
    ]


_lib = None


def _load(path: str):
    L = C.CDLL(path)
    P, D, I64, I32, U64 = C.c_void_p, C.c_double, C.c_int64, C.c_int32, C.c_uint64
    L.orc_create.restype = P
    L.orc_create.argtypes = [C.POINTER(Params), U64]
    L.orc_destroy.argtypes = [P]
    L.orc_init.argtypes = [P]
    L.orc_set_state.argtypes = [P, P, P, P, P, P, P, I64, I64]
    L.orc_get_state.argtypes = [P, P, P, P, P, P, P, P, P, P]
    L.orc_run.argtypes = [P, I32, I32]
    L.orc_interval.argtypes = [P, I32, I32]
    L.orc_collide.argtypes = [P, I32]
    L.orc_observables.argtypes = [P, C.POINTER(Obs)]
    L.orc_candidates.restype = I64
    L.orc_candidates.argtypes = [P, P, I64]
    L.orc_forces.argtypes = [P, P]
    L.orc_build_list.argtypes = [P, I32]
    L.orc_forces_allpairs.argtypes = [P, P, P]
    L.orc_cell_keys.argtypes = [P, P, P]
    L.orc_shift.argtypes = [P, I64, P]
    L.orc_last_cells.restype = I64
    L.orc_last_cells.argtypes = [P, P, I64]
    L.orc_cell_ranks.restype = I64
    L.orc_cell_ranks.argtypes = [P, P, I64]
    L.orc_hilbert.restype = U64
    L.orc_hilbert.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_int]
    L.orc_philox.argtypes = [P, P, P]
    L.orc_wca.argtypes = [D, D, D, C.POINTER(D), C.POINTER(D)]
    L.orc_tree_sum.restype = D
    L.orc_tree_sum.argtypes = [P, I64]
    L.orc_marsaglia.argtypes = [U64, I64, I64, P]
    L.orc_rotate.argtypes = [P, D, D, P, P]
    L.orc_ptable.argtypes = [D, D, P]
    L.orc_dimer_sample.restype = C.c_int
    L.orc_dimer_sample.argtypes = [P, I32, P]
    L.orc_cyl_hist.restype = C.c_int
    L.orc_cyl_hist.argtypes = [P, I32, I32, I32, D, D, P]
    L.orc_msd.argtypes = [P, I64, I32, P]
    return L


def lib():
    """The oracle library: the in-tree build, or the build named by the
    environment variable RMP_ORACLE_LIB (the sanitizer run of the pins)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("RMP_ORACLE_LIB")
        if alt:
            _lib = _load(alt)
        else:
            if not os.path.exists(_SO):
                build()
            _lib = _load(_SO)
    return _lib


@contextlib.contextmanager
def using(path: str):
    """Run the oracle from another build of its source while the block lasts
    (the mutation tests load copies with planted mistakes).  Oracle objects
    keep the build that created them."""
    global _lib
    saved = lib()
    _lib = _load(path)
    try:
        yield _lib
    finally:
        _lib = saved


def compile_variant(src_text: str, out_path: str, extra_flags=()) -> str:
    """Compile C source text of the oracle (a copy of rmp_oracle.c, possibly
    altered) into a shared library with the oracle's flags."""
    d = os.path.dirname(os.path.abspath(out_path))
    c_path = os.path.join(d, os.path.basename(out_path) + ".c")
    with open(c_path, "w") as f:
        f.write(src_text)
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", *extra_flags,
           "-I", _HERE, c_path, "-o", out_path, "-lm"]
    subprocess.check_call(cmd)
    return out_path


def source() -> str:
    with open(os.path.join(_HERE, "rmp_oracle.c")) as f:
        return f.read()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_params(p: dict) -> Params:
    q = Params()
    for d in range(3):
        q.L[d] = int(p["L"][d])
    q.rule = {"srd": 0, "at": 1}[p.get("rule", "srd")]
    q.cell_order = {"row": 0, "hilbert": 1}[p.get("cell_order", "row")]
    q.n_solvent = int(p["n_solvent"])
    q.kT, q.mass, q.dt = p["kT"], p["mass"], p["dt"]
    q.alpha, q.skin = p["alpha"], p["skin"]
    q.cat_prob, q.bulk_rate = p["cat_prob"], p["bulk_rate"]
    cols = p["colloids"]
    if len(cols) > MAXC:
        raise ValueError("too many colloids")
    q.n_colloids = len(cols)
    for c, col in enumerate(cols):
        for d in range(3):
            q.cx[c][d] = col["x"][d]
        q.cmass[c], q.sigma[c] = col["mass"], col["sigma"]
        q.epsA[c], q.epsB[c] = col["eps_A"], col["eps_B"]
        q.catalytic[c] = int(col["catalytic"])
        q.ctype[c] = int(col["type"])
    for a in range(2):
        for b in range(2):
            q.eps_cc[a][b] = p["eps_cc"][a][b]
    q.n_bonds = len(p["bonds"])
    if q.n_bonds > MAXB:
        raise ValueError("too many bonds")
    for k, (a, b, dd) in enumerate(p["bonds"]):
        q.bond_a[k], q.bond_b[k], q.bond_d[k] = a, b, dd
    q.rattle_tol = float(p.get("rattle_tol", 1e-10))
    q.rattle_maxit = int(p.get("rattle_maxit", 500))
    q.rattle_iterative = int(p.get("rattle_iterative", 0))
    q.walls = int(p.get("walls", 0))
    q.wall_density = int(p.get("wall_density", 0))
    for d, g in enumerate(p.get("accel", (0.0, 0.0, 0.0))):
        q.accel[d] = float(g)
    return q


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def wca(r2: float, sigma: float, eps: float):
    coef, pot = C.c_double(), C.c_double()
    lib().orc_wca(r2, sigma, eps, C.byref(coef), C.byref(pot))
    return coef.value, pot.value


def tree_sum(a) -> float:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return lib().orc_tree_sum(_ptr(a), a.size)


def marsaglia(seed: int, coll_step: int, cell: int) -> np.ndarray:
    n = np.zeros(3)
    lib().orc_marsaglia(seed, coll_step, cell, _ptr(n))
    return n


def hilbert(x: int, y: int, z: int, bits: int) -> int:
    """Index of (x, y, z) along the Hilbert curve of the 2^bits cube."""
    return int(lib().orc_hilbert(int(x), int(y), int(z), int(bits)))


def msd(R, max_lag: int) -> np.ndarray:
    """Mean-squared displacement of a [T][3] series for lags 0..max_lag
    (average over all time origins, summed in order)."""
    R = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(-1, 3))
    out = np.zeros(max_lag + 1)
    lib().orc_msd(_ptr(R), R.shape[0], int(max_lag), _ptr(out))
    return out


SERIES_FIELDS = 10   # R_com[3], V_com[3], axis u[3], directed velocity V_com.u


def rotate(n, alpha: float, w) -> np.ndarray:
    import math
    n = np.ascontiguousarray(np.asarray(n, dtype=np.float64))
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    out = np.zeros(3)
    lib().orc_rotate(_ptr(n), math.cos(alpha), math.sin(alpha), _ptr(w), _ptr(out))
    return out


def ptable(bulk_rate: float, tau: float) -> np.ndarray:
    t = np.zeros(PTABLE)
    lib().orc_ptable(bulk_rate, tau, _ptr(t))
    return t


class Oracle:
    """One simulated system in the FP64 oracle."""

    def __init__(self, params: dict, seed: int, init: bool = True):
        self.params = params
        self._p = make_params(params)
        self.seed = int(seed)
        self._L = lib()            # the build that owns the handle
        self.h = self._L.orc_create(C.byref(self._p), self.seed)
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.n = int(params["n_solvent"])
        self.nc = len(params["colloids"])
        if init:
            self._L.orc_init(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._L.orc_destroy(h)
            self.h = None

    def set_state(self, s: dict):
        x = np.ascontiguousarray(s["x"], dtype=np.float64).reshape(3, self.n)
        v = np.ascontiguousarray(s["v"], dtype=np.float64).reshape(3, self.n)
        ids = np.ascontiguousarray(s["id"], dtype=np.uint32)
        st = np.ascontiguousarray(s["state"], dtype=np.uint8)
        X = np.ascontiguousarray(s["X"], dtype=np.float64).reshape(self.nc, 3) if self.nc else np.zeros((0, 3))
        V = np.ascontiguousarray(s["V"], dtype=np.float64).reshape(self.nc, 3) if self.nc else np.zeros((0, 3))
        X = np.ascontiguousarray(X)
        V = np.ascontiguousarray(V)
        self._L.orc_set_state(self.h, _ptr(x), _ptr(v), _ptr(ids), _ptr(st), _ptr(X), _ptr(V),
                            int(s.get("md_step", 0)), int(s.get("coll_step", 0)))

    def get_state(self) -> dict:
        x = np.zeros((3, self.n)); v = np.zeros((3, self.n))
        ids = np.zeros(self.n, dtype=np.uint32); st = np.zeros(self.n, dtype=np.uint8)
        X = np.zeros((self.nc, 3)); V = np.zeros((self.nc, 3)); F = np.zeros((self.nc, 3))
        md, co = C.c_int64(), C.c_int64()
        self._L.orc_get_state(self.h, _ptr(x), _ptr(v), _ptr(ids), _ptr(st), _ptr(X), _ptr(V),
                            _ptr(F), C.cast(C.pointer(md), C.c_void_p),
                            C.cast(C.pointer(co), C.c_void_p))
        return dict(x=x, v=v, id=ids, state=st, X=X, V=V, F=F,
                    md_step=md.value, coll_step=co.value)

    def run(self, n_md: int, n_collide: int):
        if self._L.orc_run(self.h, int(n_md), int(n_collide)) != 0:
            raise ValueError("bad arguments")

    def interval(self, n_md: int, collide: bool = True):
        if self._L.orc_interval(self.h, int(n_md), int(bool(collide))) != 0:
            raise ValueError("bad arguments")

    def collide(self, n_md: int):
        if self._L.orc_collide(self.h, int(n_md)) != 0:
            raise ValueError("bad arguments")

    def build_list(self, n_md: int):
        self._L.orc_build_list(self.h, int(n_md))

    def observables(self) -> dict:
        o = Obs()
        self._L.orc_observables(self.h, C.byref(o))
        d = {k: getattr(o, k) for k, _ in Obs._fields_ if k != "pad"}
        d["momentum"] = np.array(list(o.momentum))
        return d

    def candidates(self) -> np.ndarray:
        n = self._L.orc_candidates(self.h, None, 0)
        idx = np.zeros(max(n, 1), dtype=np.int64)
        self._L.orc_candidates(self.h, _ptr(idx), n)
        return idx[:n]

    def forces(self) -> np.ndarray:
        f = np.zeros((3, self.n))
        self._L.orc_forces(self.h, _ptr(f))
        return f

    def forces_allpairs(self):
        f = np.zeros((3, self.n)); F = np.zeros((max(self.nc, 1), 3))
        self._L.orc_forces_allpairs(self.h, _ptr(f), _ptr(F))
        return f, F[: self.nc]

    def shift(self, coll_step: int) -> np.ndarray:
        s = np.zeros(3)
        self._L.orc_shift(self.h, int(coll_step), _ptr(s))
        return s

    def cell_keys(self, shift) -> np.ndarray:
        sh = np.ascontiguousarray(np.asarray(shift, dtype=np.float64))
        k = np.zeros(self.n, dtype=np.uint32)
        self._L.orc_cell_keys(self.h, _ptr(sh), _ptr(k))
        return k

    def cell_ranks(self) -> np.ndarray:
        """Sort rank of every cell (linear cell index -> position in the
        Hilbert cell order)."""
        m = self._L.orc_cell_ranks(self.h, None, 0)
        a = np.zeros(m, dtype=np.uint32)
        self._L.orc_cell_ranks(self.h, _ptr(a), m)
        return a

    def last_cells(self) -> np.ndarray:
        m = self._L.orc_last_cells(self.h, None, 0)
        a = np.zeros(m, dtype=np.uint32)
        self._L.orc_last_cells(self.h, _ptr(a), m)
        return a

    def dimer_sample(self, k: int) -> np.ndarray:
        """R_com[3], V_com[3], unit axis u[3] (bond_a -> bond_b) and V_com.u
        of bond k."""
        rec = np.zeros(SERIES_FIELDS)
        if self._L.orc_dimer_sample(self.h, int(k), _ptr(rec)) != 0:
            raise ValueError("no such bond")
        return rec

    def cyl_hist(self, k: int, nz: int, nr: int, zmax: float, rmax: float) -> np.ndarray:
        """Counts [species A/B][nz][nr] of the current state around bond k."""
        h = np.zeros((2, nz, nr), dtype=np.uint64)
        if self._L.orc_cyl_hist(self.h, int(k), int(nz), int(nr), float(zmax), float(rmax), _ptr(h)) != 0:
            raise ValueError("bad histogram arguments")
        return h

    def run_analysed(self, n_md: int, n_collide: int, an: dict, acc: dict | None = None) -> dict:
        """Intervals with the dimer analysis schedule: after every collision
        whose count is a multiple of an["every"], one sample of every bond
        (kept while fewer than an["series_cap"] are stored, else counted as
        dropped) and the species histogram added."""
        nb = len(self.params["bonds"])
        nz, nr = int(an["hist_nz"]), int(an["hist_nr"])
        if acc is None:
            acc = dict(series=[], md_step=[], n_dropped=0,
                       hist=np.zeros((nb, 2, nz, nr), dtype=np.uint64))
        for _ in range(n_collide):
            self.run(n_md, 1)
            st = self.observables()
            if st["coll_step"] % int(an["every"]):
                continue
            if len(acc["series"]) < int(an["series_cap"]):
                acc["series"].append(np.stack([self.dimer_sample(k) for k in range(nb)]))
                acc["md_step"].append(st["md_step"])
            else:
                acc["n_dropped"] += 1
            for k in range(nb):
                acc["hist"][k] += self.cyl_hist(k, nz, nr, an["hist_zmax"], an["hist_rmax"])
        return acc

