"""Seeded synthetic inputs for the MPCD+MD solvent path.

This module is the only code shared by the CPU oracle's tests, the GPU tests
and the benchmark.  It holds parameter sets and seeded random states and none
of the method's arithmetic: no streaming, binning, collision, force or
reaction step lives here.  Each side converts the plain dictionaries below
into its own C structure.

Units are the reduced MPCD units of the paper (cell size a = 1, solvent mass
m = 1, kT = 1); parameter names follow the paper's configuration file
(appendix "Example configuration file": T, L, rho, tau, N_MD, probability,
bulk_rate, sigma_*, epsilon_*, d).

Workloads (sizes as stated for the five benchmark cases):
  sphere10   10^3 cells, 10/cell, one WCA sphere (sigma 2, M = 4/3 pi sigma^3)
             at the centre, SRD angle 130 deg, dt 0.01, N_MD 10.
  dimer32    32^3 cells, 10/cell, catalytic C + non-catalytic N dimer
             (sigma 4, d 6.7), eps_A 1 / eps_B 0.5 on N, 1/1 on C, p = 1,
             bulk B->A rate 0.01, dt 0.01, N_MD 50 (tau 0.5).
  large128   128^3 cells, 10/cell, 8 such dimers at random non-overlapping
             sites.
  batch      64 replicas of dimer physics, box edge drawn from {16,20,24,32}.
  serve      Poisson job trace: sphere or dimer, edge 12..48, density 5..20,
             tau 0.1..0.5, 500..5000 collisions, FP32 or FP64.
"""
from __future__ import annotations

import math
import copy
import numpy as np

BASE_SEED = 0x524D50434D44          # per-workload seed = BASE_SEED + workload index

A, B = 0, 1                          # solvent species codes (bit 0 of the state byte)
TYPE_C, TYPE_N = 0, 1                # colloid types for the colloid-colloid epsilon table


def colloid_mass(sigma: float, density: float = 1.0) -> float:
    """Colloid mass convention M = (4/3) pi sigma^3 * density (M ~ 33.5 at sigma 2)."""
    return 4.0 / 3.0 * math.pi * sigma ** 3 * density


def base_params(L=(10, 10, 10), rho=10, dt=0.01, n_md=10, alpha_deg=130.0,
                kT=1.0, mass=1.0, skin=0.4, precision=64, rule="srd") -> dict:
    L = tuple(int(v) for v in L)
    return dict(
        L=L, n_solvent=int(rho * L[0] * L[1] * L[2]), rho=rho, kT=float(kT),
        mass=float(mass), dt=float(dt), n_md=int(n_md),
        alpha=math.radians(alpha_deg), rule=rule, skin=float(skin),
        cat_prob=1.0, bulk_rate=0.0, colloids=[], bonds=[],
        eps_cc=((1.0, 1.0), (1.0, 1.0)), precision=int(precision))


def add_colloid(p: dict, x, sigma, eps_A=1.0, eps_B=1.0, catalytic=False,
                ctype=TYPE_N, mass=None) -> int:
    p["colloids"].append(dict(
        x=tuple(float(c) for c in x), sigma=float(sigma), eps_A=float(eps_A),
        eps_B=float(eps_B), catalytic=bool(catalytic), type=int(ctype),
        mass=float(colloid_mass(sigma) if mass is None else mass)))
    return len(p["colloids"]) - 1


def random_axis(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def add_dimer(p: dict, centre, axis, sigma_C=4.0, sigma_N=4.0, d=6.7,
              eps_C=(1.0, 1.0), eps_N=(1.0, 0.5)):
    centre = np.asarray(centre, dtype=float)
    axis = np.asarray(axis, dtype=float)
    xc = centre + 0.5 * d * axis
    xn = centre - 0.5 * d * axis
    c = add_colloid(p, xc, sigma_C, eps_C[0], eps_C[1], catalytic=True, ctype=TYPE_C)
    n = add_colloid(p, xn, sigma_N, eps_N[0], eps_N[1], catalytic=False, ctype=TYPE_N)
    p["bonds"].append((c, n, float(d)))
    return c, n


def sphere10(precision=64, seed=None) -> dict:
    p = base_params(L=(10, 10, 10), rho=10, dt=0.01, n_md=10, precision=precision)
    add_colloid(p, (5.0, 5.0, 5.0), sigma=2.0, eps_A=1.0, eps_B=1.0)
    p["name"] = "sphere10"
    p["n_collide"] = 100
    return p


def dimer_system(L=32, rho=10, n_md=50, precision=64, seed=None, bulk_rate=0.01,
                 cat_prob=1.0) -> dict:
    p = base_params(L=(L, L, L), rho=rho, dt=0.01, n_md=n_md, precision=precision)
    rng = np.random.default_rng(BASE_SEED + 2 if seed is None else seed)
    add_dimer(p, (L / 2.0, L / 2.0, L / 2.0), random_axis(rng))
    p["cat_prob"] = float(cat_prob)
    p["bulk_rate"] = float(bulk_rate)
    return p


def dimer32(precision=64, seed=None) -> dict:
    p = dimer_system(32, precision=precision, seed=seed)
    p["name"] = "dimer32"
    p["n_collide"] = 10_000
    return p


def place_dimers(p: dict, n_dimers: int, rng: np.random.Generator, d=6.7,
                 sigma=4.0, gap=1.0, max_tries=100000):
    """Random non-overlapping dimers: sphere centres of different dimers at
    least sigma_i + sigma_j + gap apart (minimum image)."""
    L = np.asarray(p["L"], dtype=float)
    centres = []
    tries = 0
    while len(centres) < 2 * n_dimers:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place dimers")
        c = rng.uniform(0, 1, 3) * L
        ax = random_axis(rng)
        xc = c + 0.5 * d * ax
        xn = c - 0.5 * d * ax
        ok = True
        for y in centres:
            for x in (xc, xn):
                dd = x - y
                dd -= L * np.round(dd / L)
                if np.linalg.norm(dd) < 2 * sigma + gap:
                    ok = False
        if ok:
            centres.extend([xc, xn])
            add_dimer(p, c, ax, d=d)
    return p


def large128(precision=64, seed=None, L=128) -> dict:
    p = base_params(L=(L, L, L), rho=10, dt=0.01, n_md=50, precision=precision)
    p["bulk_rate"] = 0.01
    rng = np.random.default_rng(BASE_SEED + 3 if seed is None else seed)
    place_dimers(p, 8, rng)
    p["name"] = f"large{L}"
    p["n_collide"] = 1000
    return p


def icosahedron(radius: float) -> tuple[np.ndarray, list]:
    """Vertices of a regular icosahedron of the given circumradius (a vertex
    on +z) and its 30 edges."""
    v = [(0.0, 0.0, 1.0), (0.0, 0.0, -1.0)]
    zr = 1.0 / math.sqrt(5.0)
    rr = 2.0 / math.sqrt(5.0)
    for k in range(5):
        a = 2.0 * math.pi * k / 5.0
        v.append((rr * math.cos(a), rr * math.sin(a), zr))
    for k in range(5):
        a = 2.0 * math.pi * (k + 0.5) / 5.0
        v.append((rr * math.cos(a), rr * math.sin(a), -zr))
    V = np.array(v) * radius
    d = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=2)
    edge = d[d > 1e-9].min()
    edges = [(i, j) for i in range(12) for j in range(i + 1, 12) if abs(d[i, j] - edge) < 1e-6 * radius]
    assert len(edges) == 30
    return V, edges


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def add_janus(p: dict, centre, rng: np.random.Generator, shell=2.5, sigma=2.0,
              eps_cat=(1.0, 1.0), eps_non=(1.0, 0.5)):
    """A composite Janus particle: a central bead and 12 beads on the
    vertices of an icosahedron, held rigid by 42 bonds (12 spokes, 30 edges);
    the beads of the upper half (the +z vertex and its ring, in the body
    frame) are catalytic.  Returns the colloid indices."""
    V, edges = icosahedron(shell)
    R = random_rotation(rng)
    c0 = np.asarray(centre, dtype=float)
    first = len(p["colloids"])
    centre_i = add_colloid(p, c0, sigma, eps_non[0], eps_non[1], catalytic=False, ctype=TYPE_N)
    ids = []
    for k in range(12):
        cat = V[k, 2] > 0.0
        e = eps_cat if cat else eps_non
        ids.append(add_colloid(p, c0 + R @ V[k], sigma, e[0], e[1], catalytic=bool(cat),
                               ctype=TYPE_C if cat else TYPE_N))
    bonds = [(centre_i, ids[k], float(shell)) for k in range(12)]
    bonds += [(ids[i], ids[j], float(np.linalg.norm(V[i] - V[j]))) for i, j in edges]
    # order the bonds as successive sets with no colloid in common (greedy),
    # so that a sweep of the iterative RATTLE has few dependent steps
    while bonds:
        used, layer = set(), []
        for bd in bonds:
            if bd[0] not in used and bd[1] not in used:
                layer.append(bd)
                used |= {bd[0], bd[1]}
        bonds = [bd for bd in bonds if bd not in layer]
        p["bonds"].extend(layer)
    return list(range(first, first + 13))


def janus_system(L=24, rho=10, n_md=50, precision=64, seed=None, bulk_rate=0.01,
                 cat_prob=1.0) -> dict:
    """One composite Janus motor at the box centre (iterative RATTLE)."""
    p = base_params(L=(L, L, L), rho=rho, dt=0.01, n_md=n_md, precision=precision)
    rng = np.random.default_rng(BASE_SEED + 6 if seed is None else seed)
    add_janus(p, (L / 2.0, L / 2.0, L / 2.0), rng)
    p["cat_prob"] = float(cat_prob)
    p["bulk_rate"] = float(bulk_rate)
    p["rattle_tol"] = 1e-10
    p["rattle_maxit"] = 500
    p["name"] = f"janus{L}"
    return p


def poiseuille(L=(64, 64, 32), rho=10, g=0.001, dt=0.01, n_md=10, precision=64) -> dict:
    """Flow between plates at z = 0 and z = L_z driven by a constant
    acceleration g along x, no colloid (the paper's poiseuille_flow setup)."""
    p = base_params(L=L, rho=rho, dt=dt, n_md=n_md, precision=precision)
    p["walls"] = 1
    p["wall_density"] = int(rho)
    p["accel"] = (float(g), 0.0, 0.0)
    p["name"] = f"poiseuille{L[0]}x{L[1]}x{L[2]}"
    p["n_collide"] = 2000
    return p


def batch_replicas(n=64, edges=(16, 20, 24, 32), precision=32, seed=None):
    """Replica parameter list for the batched ensemble (per-replica seeds)."""
    rng = np.random.default_rng(BASE_SEED + 4 if seed is None else seed)
    out = []
    for r in range(n):
        L = int(rng.choice(edges))
        p = dimer_system(L, precision=precision, seed=BASE_SEED + 1000 * (r + 1))
        p["name"] = f"replica{r}_L{L}"
        p["seed"] = BASE_SEED + 1000 * (r + 1)
        p["n_collide"] = 2000
        out.append(p)
    return out


def serve_trace(n_jobs=200, rate=20.0, seed=None, edge=(12, 48), rho=(5, 20),
                n_collide=(500, 5000), taus=(0.1, 0.2, 0.3, 0.4, 0.5)):
    """Seeded Poisson trace of simulation jobs: list of dicts with an arrival
    time, a parameter dict and a collision count."""
    rng = np.random.default_rng(BASE_SEED + 5 if seed is None else seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        L = int(rng.integers(edge[0], edge[1] + 1))
        dens = int(rng.integers(rho[0], rho[1] + 1))
        tau = float(rng.choice(taus))
        n_md = int(round(tau / 0.01))
        prec = int(rng.choice((32, 64)))
        kind = "dimer" if (rng.random() < 0.5 and L >= 16) else "sphere"
        if kind == "dimer":
            p = dimer_system(L, rho=dens, n_md=n_md, precision=prec,
                             seed=BASE_SEED + 7 * j + 1)
        else:
            p = base_params(L=(L, L, L), rho=dens, dt=0.01, n_md=n_md, precision=prec)
            add_colloid(p, (L / 2.0, L / 2.0, L / 2.0), sigma=2.0)
        # Verlet-list skin: at least twice a generous colloid displacement per
        # interval (4 thermal speeds sqrt(3 kT / M) times tau)
        m_min = min(c["mass"] for c in p["colloids"])
        p["skin"] = max(p["skin"], round(2 * 4 * math.sqrt(3 * p["kT"] / m_min) * tau, 2))
        p["name"] = f"job{j}_{kind}_L{L}_rho{dens}"
        jobs.append(dict(arrival=t, params=p, seed=BASE_SEED + 100000 + j,
                         n_collide=int(rng.integers(n_collide[0], n_collide[1] + 1))))
    return jobs


def scaled(p: dict, **kw) -> dict:
    q = copy.deepcopy(p)
    q.update(kw)
    if "L" in kw or "rho" in kw:
        L = q["L"]
        q["n_solvent"] = int(q["rho"] * L[0] * L[1] * L[2])
    return q


# ----------------------------------------------------------------------------
# Seeded solvent states for parity tests (independent of the method's own
# initialisation; any state with x in [0, L) is a valid starting point).
# ----------------------------------------------------------------------------

def random_state(p: dict, seed: int, species_B_fraction=0.0, flag_fraction=0.0,
                 exclude_cores=True, float32=False, velocity_scale=None):
    """Return a dict of SoA numpy arrays x[3,N], v[3,N], id[N], state[N] plus
    colloid X[nc,3], V[nc,3] for parameter set p."""
    rng = np.random.default_rng(seed)
    L = np.asarray(p["L"], dtype=float)
    n = int(p["n_solvent"])
    cols = p["colloids"]
    x = rng.uniform(0.0, 1.0, size=(n, 3)) * L
    if exclude_cores and cols:
        for _ in range(1000):
            bad = np.zeros(n, dtype=bool)
            for c in cols:
                dd = x - np.asarray(c["x"])
                dd -= L * np.round(dd / L)
                bad |= (dd * dd).sum(axis=1) < c["sigma"] ** 2
            if not bad.any():
                break
            x[bad] = rng.uniform(0.0, 1.0, size=(int(bad.sum()), 3)) * L
    x = np.where(x >= L, 0.0, x)
    s = math.sqrt(p["kT"] / p["mass"]) if velocity_scale is None else velocity_scale
    v = rng.normal(0.0, s, size=(n, 3))
    if n:
        v -= v.mean(axis=0)
    ids = rng.permutation(n).astype(np.uint32)
    st = np.zeros(n, dtype=np.uint8)
    if species_B_fraction > 0:
        st[rng.random(n) < species_B_fraction] |= 1
    if flag_fraction > 0:
        st[(rng.random(n) < flag_fraction) & ((st & 1) == 0)] |= 2
    if float32:
        x = x.astype(np.float32).astype(np.float64)
        x = np.where(x >= L, 0.0, x)
        v = v.astype(np.float32).astype(np.float64)
    nc = len(cols)
    X = np.array([c["x"] for c in cols], dtype=float).reshape(nc, 3)
    V = rng.normal(0.0, 1.0, size=(nc, 3)) * np.array(
        [math.sqrt(p["kT"] / c["mass"]) for c in cols]).reshape(nc, 1) if nc else np.zeros((0, 3))
    # keep bonded pairs' relative velocity free of a bond component
    for (a, b, d) in p["bonds"]:
        r = X[a] - X[b]
        dv = V[a] - V[b]
        k = np.dot(dv, r) / np.dot(r, r)
        ma, mb = cols[a]["mass"], cols[b]["mass"]
        V[a] -= k * r * mb / (ma + mb)
        V[b] += k * r * ma / (ma + mb)
    return dict(x=np.ascontiguousarray(x.T), v=np.ascontiguousarray(v.T), id=ids,
                state=st, X=X, V=V, md_step=0, coll_step=0)


def cluster_state(p: dict, seed: int, cell=(0, 0, 0), count=200):
    """A state with `count` particles crowded into one cell and the rest
    uniform: exercises cells far above the mean occupancy."""
    s = random_state(p, seed)
    rng = np.random.default_rng(seed + 1)
    k = min(count, s["x"].shape[1])
    for d in range(3):
        s["x"][d, :k] = cell[d] + rng.uniform(0.05, 0.95, size=k)
    return s


# ----------------------------------------------------------------------------
# key = value configuration files (the paper's appendix format)
# ----------------------------------------------------------------------------

def parse_parameters(text: str) -> dict:
    """Parse `key = value [value ...]` lines; '#' starts a comment.  Numbers
    become int/float, T/F become booleans, several values become a tuple."""
    out = {}
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line or "=" not in line:
            continue
        k, v = (t.strip() for t in line.split("=", 1))
        vals = []
        for tok in v.split():
            if tok in ("T", "F"):
                vals.append(tok == "T")
                continue
            try:
                vals.append(int(tok))
            except ValueError:
                vals.append(float(tok))
        out[k] = vals[0] if len(vals) == 1 else tuple(vals)
    return out


def params_from_config(cfg: dict, L_override=None, seed=None) -> dict:
    """Dimer-motor parameter set from a parsed configuration file."""
    L = tuple(L_override or cfg["L"])
    n_md = int(cfg["N_MD"])
    p = base_params(L=L, rho=cfg["rho"], dt=float(cfg["tau"]) / n_md, n_md=n_md,
                    kT=float(cfg.get("T", 1.0)))
    rng = np.random.default_rng(BASE_SEED if seed is None else seed)
    centre = tuple(l / 2.0 for l in L)
    eN, eC = cfg["epsilon_N"], cfg["epsilon_C"]
    add_dimer(p, centre, random_axis(rng), sigma_C=float(cfg["sigma_C"]),
              sigma_N=float(cfg["sigma_N"]), d=float(cfg["d"]),
              eps_C=(float(eC[0]), float(eC[1])), eps_N=(float(eN[0]), float(eN[1])))
    p["eps_cc"] = ((float(cfg.get("epsilon_C_C", 1.0)), float(cfg.get("epsilon_N_C", 1.0))),
                   (float(cfg.get("epsilon_N_C", 1.0)), float(cfg.get("epsilon_N_N", 1.0))))
    p["cat_prob"] = float(cfg.get("probability", 1.0))
    p["bulk_rate"] = float(cfg.get("bulk_rate", 0.0)) if cfg.get("bulk_rmpcd", False) else 0.0
    p["n_collide"] = int(cfg.get("N_loop", 1))
    return p
