"""Benchmark of the MPCD+MD solvent hot path on one MI355X.

Default workload (the one `value` is quoted on): chemically powered dimer
nanomotor, periodic 32^3 cells, 10 solvent particles per cell = 327,680
particles, catalytic C and non-catalytic N spheres (sigma 4, bond 6.7),
eps_B = 0.5 on N, catalytic conversion with probability 1, bulk B->A rate
0.01, dt = 0.01, tau = 0.5 (50 MD steps per collision), FP64 state.
Synthetic seeded input: the library's own initialisation (uniform positions
outside the colloids, Maxwellian velocities at kT = 1).

One benchmark step = one interval of the method: 50 velocity-Verlet MD steps
of all solvent particles and the dimer, then one MPCD collision with the
bulk reaction.  value = solvent particle-steps per second
= N * 50 * steps / wall time, inputs resident in HBM.

The roofline object reports the dominant kernel: its average launch
duration is measured with HIP events recorded by the library on the stream
that kernel runs on, over a second pass of the same workload; achieved =
algorithmic bytes per launch / that duration.  cpu_baseline times the FP64
CPU oracle on a bounded sample of the same workload on the host cores.

Extra objects on the same line: the same workload in FP32 state, and the
128^3-cell, 8-dimer system (20,971,520 particles, FP64 and FP32) where the
state exceeds the caches and the streaming and collision kernels are
HBM-bound.  Other modes (--workload batch / serve / large128 / sphere10)
print their own line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solvent particle-steps/s + % HBM peak; batched FP32 vs FP64; p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FLOPS_PER_LIST_STEP = 120.0


def algorithmic_bytes(kernel: str, n: int, ncell: int, tb: int, n_cand: int,
                      flow: bool = False) -> float:
    """Bytes the method must move per launch (not counting re-reads):
    stream_bin  per free particle: read x, v (6 tb) + list flag (1), write x
                (3 tb) + key/rank (8); cell counters 8 B per cell.
    collide     per particle: read perm (4), x, v (6 tb), id (4), state (1);
                write x, v (6 tb), id (4), state (1), list flag (1); per
                cell: read the start (4), zero the counter (4).
    scatter     per particle: read key/rank (8), write perm (4); starts 4/cell.
    scan_final  per cell: read count (4), write start (4).
    stream_bin  with a flow (acceleration, plates) every particle also writes
                its velocity: read x, v (6 tb) + flag (1), write x, v (6 tb)
                + key/rank (8).
    chain       per list entry: read and write x, v, state (12 tb + 2).
    analysis    per particle: read x (3 tb) and state (1); the histogram
                updates touch only particles inside a dimer's cylinder."""
    nf = max(n - n_cand, 0)
    if kernel == "stream_bin":
        return nf * ((12 if flow else 9) * tb + 9) + 8 * ncell
    if kernel == "collide":
        return n * (12 * tb + 15) + 8 * ncell
    if kernel == "scatter":
        return n * 12 + 4 * ncell
    if kernel == "scan_final":
        return 8 * ncell
    if kernel == "chain":
        return n_cand * (12 * tb + 2)
    if kernel == "analysis":
        return n * (3 * tb + 1)
    if kernel in ("chunk_scan", "cand_write"):
        return n * 1 + 8 * math.ceil(n / 1024)
    return 0.0


def kernel_source_hash() -> str:
    """Hash of the HIP sources: counter-derived traffic is only reported for
    the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1608_04904_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name: str, precision: int, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if the
    kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{workload_name}_fp{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else 1e6 * (k["fetch_MB"] + k["write_MB"])


def workload(name: str, precision: int):
    import workloads as W
    if name == "dimer32":
        p = W.dimer32(precision=precision)
        return p, 50, W.BASE_SEED + 2, ("dimer32: 32^3 cells, rho 10, N=327,680, 1 dimer (C+N, "
                                         "sigma 4, d 6.7), tau 0.5 (50 MD steps/collision)")
    if name == "sphere10":
        p = W.sphere10(precision=precision)
        return p, 10, W.BASE_SEED + 1, ("sphere10: 10^3 cells, rho 10, N=10,000, 1 WCA sphere "
                                         "sigma 2, tau 0.1 (10 MD steps/collision)")
    if name == "janus32":
        p = W.janus_system(L=32, rho=10, n_md=50, precision=precision)
        return p, 50, W.BASE_SEED + 6, ("janus32: 32^3 cells, rho 10, N=327,680, one composite Janus "
                                         "particle (13 beads, 42 rigid bonds, iterative RATTLE), "
                                         "tau 0.5 (50 MD steps/collision)")
    if name == "poiseuille":
        p = W.poiseuille(precision=precision)
        return p, 10, W.BASE_SEED + 5, ("poiseuille: 64 x 64 x 32 cells between plates at z = 0 "
                                         "and 32, rho 10, N=1,310,720, g = 0.001 along x, "
                                         "tau 0.1 (10 MD steps/collision), no colloid")
    if name == "large128":
        p = W.large128(precision=precision)
        return p, 50, W.BASE_SEED + 3, ("large128: 128^3 cells, rho 10, N=20,971,520, 8 dimers, "
                                         "tau 0.5 (50 MD steps/collision)")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(p, n_md, seed, budget_s: float):
    """Time the FP64 oracle on a bounded sample: whole intervals of the same
    workload until about budget_s seconds of work."""
    import oracle
    o = oracle.Oracle(p, seed)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o.run(n_md, 1)                                 # warm-up interval
    t0 = time.perf_counter()
    k = 0
    while True:
        o.run(n_md, 1)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=p["n_solvent"] * n_md * k / dt, unit="particle-steps/s", cores=threads,
                kind="oracle",
                sample=f"{k} intervals x {n_md} MD steps of the same workload "
                       f"({p['n_solvent']} particles), {dt:.1f} s")


def fp32_drift(intervals: int, oracle_intervals: int, with_oracle: bool, name: str = "dimer32"):
    """FP32 state against FP64 from the same initial state: total momentum
    P = sum m v (solvent and colloids, conserved exactly by the method), total
    energy E = KE + U - e_rxn (e_rxn: potential change booked at species
    flips), and the dimers' centre-of-mass displacements (MSD averaged over
    the dimers).  The FP64 run is checked bit for bit against the CPU oracle
    over the first `oracle_intervals` intervals, so it stands for the oracle
    trajectory."""
    import torch
    import paper_1608_04904_amd as rm
    import workloads as W
    make = W.dimer32 if name == "dimer32" else W.large128
    p64 = make(precision=64)
    p32 = make(precision=32)
    bonds = p64["bonds"]
    masses = np.array([c["mass"] for c in p64["colloids"]])
    n_md = int(p64["n_md"])
    seed = W.BASE_SEED + 77
    st0 = W.random_state(p64, seed)
    runs = {}
    for prec, p in ((64, p64), (32, p32)):
        s = rm.System(p, seed)
        s.set_state(st0)
        P, E, R = [], [], []
        for k in range(intervals + 1):
            if k:
                s.step(n_md, 1)
            o = s.observables(raise_on_flags=False)
            P.append(np.array(o["momentum"]))
            E.append(o["ke_solvent"] + o["ke_colloid"] + o["potential"] - o["e_rxn"])
            X = np.array(o["colloid_X"])
            R.append(np.array([(masses[a] * X[a] + masses[b] * X[b]) / (masses[a] + masses[b])
                               for a, b, _ in bonds]))
        torch.cuda.synchronize()
        runs[prec] = dict(P=np.array(P), E=np.array(E), R=np.array(R), flags=o["flags"])
        if prec == 64 and with_oracle:
            import oracle
            g = rm.System(p, seed)
            g.set_state(st0)
            g.step(n_md, oracle_intervals)
            oc = oracle.Oracle(p, seed, init=False)
            oc.set_state(st0)
            oc.run(n_md, oracle_intervals)
            gs, os_ = g.get_state(), oc.get_state()
            runs[64]["oracle_equal"] = all(np.array_equal(np.asarray(gs[k]), np.asarray(os_[k]))
                                          for k in ("id", "state", "x", "v", "X", "V"))
            g.close()
        s.close()
    r64, r32 = runs[64], runs[32]
    n = p64["n_solvent"]
    pscale = float(np.sqrt(n * p64["mass"] * p64["kT"]))     # thermal momentum of the system
    e0 = float(r64["E"][0])
    msd64 = float(np.mean(np.sum((r64["R"][-1] - r64["R"][0]) ** 2, axis=1)))
    msd32 = float(np.mean(np.sum((r32["R"][-1] - r32["R"][0]) ** 2, axis=1)))
    out = dict(
        workload=name, n_dimers=len(bonds), intervals=intervals, md_steps=intervals * n_md,
        momentum_drift_fp64=float(np.max(np.linalg.norm(r64["P"] - r64["P"][0], axis=1)) / pscale),
        momentum_drift_fp32=float(np.max(np.linalg.norm(r32["P"] - r32["P"][0], axis=1)) / pscale),
        energy_drift_fp64=float(np.max(np.abs(r64["E"] - e0)) / abs(e0)),
        energy_drift_fp32=float(np.max(np.abs(r32["E"] - r32["E"][0])) / abs(e0)),
        energy_fp32_vs_fp64=float(np.max(np.abs(r32["E"] - r64["E"])) / abs(e0)),
        dimer_msd_fp64=msd64, dimer_msd_fp32=msd32,
        # the two trajectories decorrelate (the dynamics is chaotic): rms
        # distance between the FP32 and FP64 dimer centres after k intervals
        dimer_com_diff={str(k): float(np.sqrt(np.mean(np.sum((r32["R"][k] - r64["R"][k]) ** 2, axis=1))))
                        for k in (1, 2, 5, 10, 20, 50, 100, 200) if k <= intervals},
        flags=[int(r64["flags"]), int(r32["flags"])],
        note="momentum drifts are max_t |P(t) - P(0)| / sqrt(N m kT); energy drifts max_t |E(t) - E(0)| / E(0)")
    if "oracle_equal" in r64:
        out["fp64_bitwise_equal_to_oracle"] = dict(intervals=oracle_intervals, equal=bool(r64["oracle_equal"]))
    return out


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def tuning_from_args(args) -> dict:
    tun = dict(use_graph=args.graph)
    for k in ("collide_cells", "chain_k", "chain_block", "chain_resident", "stream_block", "stream_ppt"):
        if getattr(args, k) > 0:
            tun[k] = getattr(args, k)
    return tun


def run_single(name, precision, steps, warmup, profile_steps, tun):
    """Time `steps` intervals of one system, then a profiled pass.  Returns a
    dict with value, wall, per-kernel averages and the roofline object."""
    import torch
    import paper_1608_04904_amd as rm
    p, n_md, seed, desc = workload(name, precision)
    n = p["n_solvent"]
    ncell = p["L"][0] * p["L"][1] * (p["L"][2] + p.get("walls", 0))
    tb = 8 if precision == 64 else 4
    flow = bool(p.get("walls", 0)) or any(p.get("accel", (0.0, 0.0, 0.0)))
    _log(f"workload {name} N={n} n_md={n_md} precision={precision}")
    s = rm.System(p, seed)
    s.set_tuning(**tun)
    s.step(n_md, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(n_md, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ob = s.observables(raise_on_flags=False)
    _log(f"{name} fp{precision}: {steps} steps in {wall:.4f} s, flags={ob['flags']}")
    s.profile(True)
    s.step(n_md, profile_steps)
    prof = s.profile_read()
    s.profile(False)
    n_cand = ob["n_candidates"]
    kern = {k: (ms / c, c) for k, (ms, c) in prof.items() if c > 0}
    dom = max(kern, key=lambda k: kern[k][0] * kern[k][1])
    avg_ms = kern[dom][0]
    if dom == "chain":
        # the MD chain is a dependent sequence of n_md small steps (latency
        # bound); its FP64 work is reported against the vector FP64 peak
        flops = FLOPS_PER_LIST_STEP * n_cand * n_md
        achieved = flops / (avg_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / FP64_PEAK_TFLOPS,
                    # what does bound it: one cross-workgroup exchange per MD step
                    us_per_md_step=1e3 * avg_ms / n_md,
                    note="latency-bound: n_md dependent MD steps, each ending in a "
                         "cross-workgroup exchange of the colloid forces")
    else:
        achieved = algorithmic_bytes(dom, n, ncell, tb, n_cand, flow) / (avg_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS)
    roof.update(traffic=measured_traffic(name, precision, dom), kernel=dom, avg_launch_ms=avg_ms)
    kernels = {k: dict(avg_ms=round(v[0], 5), launches=v[1],
                       algorithmic_GBps=round(algorithmic_bytes(k, n, ncell, tb, n_cand, flow)
                                              / (v[0] * 1e-3) / 1e9, 1))
               for k, v in kern.items()}
    _log(f"{name} fp{precision} kernels {json.dumps(kernels)}")
    out = dict(value=n * n_md * steps / wall, wall=wall, n=n, n_md=n_md, desc=desc,
               n_cand=n_cand, roofline=roof, kernels=kernels, tuning=s.get_tuning(),
               flags=ob["flags"])
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def poiseuille_profile(precision, warm_intervals=6000, snapshots=200, every=10):
    """Steady Poiseuille flow of the benchmark channel on the GPU (6000
    intervals = 600 time units, five relaxation times h^2 / (pi^2 nu)): the x
    velocity averaged in slabs of unit width across the channel, a quadratic
    fit, and its curvature against -g / (2 nu) with the MPCD kinematic
    viscosity of the closed form (Kikuchi et al. 2003); slip = fitted
    velocity at a plate over the centre velocity."""
    import torch
    import paper_1608_04904_amd as rm
    p, n_md, seed, _ = workload("poiseuille", precision)
    h, g = p["L"][2], p["accel"][0]
    tau = n_md * p["dt"]
    M, a = p["rho"], p["alpha"]
    gm = M - 1 + math.exp(-M)
    nu = tau / 2 * (5 * M / (gm * (2 - math.cos(a) - math.cos(2 * a))) - 1) + \
        (1 / (18 * tau)) * (gm / M) * (1 - math.cos(a))
    s = rm.System(p, seed)
    s.step(n_md, warm_intervals)
    prof = np.zeros(h)
    for _ in range(snapshots):
        s.step(n_md, every)
        st = s.get_state()
        k = np.minimum(st["x"][2].astype(int), h - 1)
        prof += np.bincount(k, weights=st["v"][0], minlength=h) / np.bincount(k, minlength=h)
    prof /= snapshots
    ob = s.observables(raise_on_flags=False)
    s.close()
    del s
    torch.cuda.empty_cache()
    zc = np.arange(h) + 0.5
    c = np.polyfit(zc, prof, 2)
    vmax = g * h * h / (8 * nu)
    return dict(curvature_over_closed_form=float(-c[0] / (g / (2 * nu))),
                slip_over_vmax=[float(np.polyval(c, 0.0) / vmax), float(np.polyval(c, float(h)) / vmax)],
                centre_velocity=float(prof[h // 2 - 1: h // 2 + 1].mean()), closed_form_vmax=vmax,
                temperature=ob["temperature"],
                sample=f"{warm_intervals} intervals to steady state, then {snapshots} snapshots "
                       f"{every} intervals apart")


ANALYSIS = dict(every=1, hist_nz=64, hist_nr=32, hist_zmax=12.0, hist_rmax=10.0)


def run_analysis(name, precision, steps, warmup, tun):
    """The workload with the dimer analysis sampled after every collision:
    cost of the analysis kernel per sample and of the whole interval."""
    import torch
    import paper_1608_04904_amd as rm
    p, n_md, seed, _ = workload(name, precision)
    n = p["n_solvent"]
    tb = 8 if precision == 64 else 4
    s = rm.System(p, seed)
    s.set_tuning(**tun)
    s.analysis_attach(series_cap=steps + warmup + 8, **ANALYSIS)
    s.step(n_md, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(n_md, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.profile(True)
    s.step(n_md, 4)
    prof = s.profile_read()
    s.profile(False)
    res = s.analysis_read()
    flags = s.observables(raise_on_flags=False)["flags"]
    ms, cnt = prof["analysis"]
    avg = ms / max(cnt, 1)
    gbs = algorithmic_bytes("analysis", n, 0, tb, 0) / (avg * 1e-3) / 1e9
    msd = s.analysis_msd(min(steps, 16))
    s.close()
    del s
    torch.cuda.empty_cache()
    return dict(value=n * n_md * steps / wall, analysis_avg_ms=round(avg, 5),
                analysis_GBps=round(gbs, 1), analysis_hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                samples=res["n_samples"], counted_per_sample=int(res["hist"].sum()) // max(
                    res["n_samples"] + res["n_dropped"], 1),
                dimers=len(p["bonds"]), bins=f"{ANALYSIS['hist_nz']}x{ANALYSIS['hist_nr']}",
                directed_velocity_mean=float(res["series"][:, :, 9].mean()),
                msd_lag1=float(msd[0][1]), flags=flags)


def run_batch(precision, ticks, warmup, tun, n_rep=64):
    """64 dimer replicas, box edges from {16,20,24,32}, per-replica seeds,
    one interval (50 MD steps + collision) per replica per tick."""
    import torch
    import paper_1608_04904_amd as rm
    import workloads as W
    reps = W.batch_replicas(n=n_rep, precision=precision)
    b = rm.Batch(len(reps), precision=precision)
    b.set_tuning(**tun)
    for i, p in enumerate(reps):
        b.set_slot(i, p, p["seed"], p["n_md"])
    n_tot = sum(p["n_solvent"] for p in reps)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(ticks)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flags = [b.observables(i, raise_on_flags=False)["flags"] for i in range(len(reps))]
    val = n_tot * 50 * ticks / wall
    _log(f"batch fp{precision}: {len(reps)} replicas, N_total={n_tot}, {ticks} ticks in "
         f"{wall:.3f} s -> {val:.3e} particle-steps/s, flags={sum(1 for f in flags if f)}")
    b.close()
    torch.cuda.empty_cache()
    return dict(value=val, wall=wall, n_total=n_tot, n_replicas=len(reps), ticks=ticks,
                flagged=sum(1 for f in flags if f))


def run_serve(n_jobs, rate, scale, budget_gb, slots, seed=None):
    """Poisson trace (box edge 12..48, density 5..20, sphere or dimer,
    tau 0.1..0.5, FP32 or FP64); collisions per job scaled by `scale`."""
    import workloads as W
    from paper_1608_04904_amd.serve import Server, summarize
    jobs = W.serve_trace(n_jobs=n_jobs, rate=rate, seed=seed)
    for j in jobs:
        j["n_collide"] = max(1, int(round(j["n_collide"] * scale)))
    srv = Server.on_gpu(hbm_budget=int(budget_gb * (1 << 30)), slots_per_pool=slots)
    t0 = time.perf_counter()
    res = srv.run(jobs, realtime=True)
    wall = time.perf_counter() - t0
    s = summarize(res)
    s.update(wall_s=wall, peak_hbm_bytes=srv.peak_used, n_jobs_offered=n_jobs,
             arrival_rate=rate, collision_scale=scale)
    _log(f"serve: {json.dumps(s)}")
    return s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="dimer32",
                    choices=["dimer32", "sphere10", "large128", "poiseuille", "janus32", "batch", "serve"])
    ap.add_argument("--precision", type=int, default=64)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--collide-cells", type=int, default=0)
    ap.add_argument("--chain-k", type=int, default=0)
    ap.add_argument("--chain-block", type=int, default=0)
    ap.add_argument("--chain-resident", type=int, default=0)
    ap.add_argument("--stream-block", type=int, default=0)
    ap.add_argument("--stream-ppt", type=int, default=0)
    ap.add_argument("--serve-jobs", type=int, default=60)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-scale", type=float, default=0.05)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB copied by one plain device copy before the run (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(each replica or job is independent; the design notes describe how a "
              "single large system would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        _log(f"calibration copy of {nbytes} bytes done")
        del src, dst

    tun = tuning_from_args(args)
    base = dict(metric=METRIC, unit="particle-steps/s", n_gpus=1, higher_is_better=True,
                scaling="weak", vs_baseline=None, data="synthetic")

    if args.workload == "batch":
        r64 = run_batch(64, args.steps, args.warmup, tun)
        r32 = run_batch(32, args.steps, args.warmup, tun)
        line = dict(base, value=r32["value"], steps=args.steps, warmup=args.warmup,
                    ms_per_step=1e3 * r32["wall"] / args.steps, dtype="f32",
                    config=dict(workload="batch: 64 dimer replicas, box edge from {16,20,24,32}, "
                                "rho 10, tau 0.5, per-replica seeds, one interval per replica "
                                "per step", tuning=tun),
                    fp32=r32, fp64=r64, fp32_over_fp64=r32["value"] / r64["value"])
        print(json.dumps(line), flush=True)
        return
    if args.workload == "serve":
        s = run_serve(args.serve_jobs, args.serve_rate, args.serve_scale,
                      args.serve_budget_gb, args.serve_slots)
        line = dict(base, value=s.get("particle_steps_per_s", 0.0), steps=s.get("n_jobs", 0),
                    warmup=0, ms_per_step=None, dtype="f32+f64",
                    config=dict(workload=f"serve: Poisson trace, {args.serve_jobs} jobs at "
                                f"{args.serve_rate}/s, collisions x{args.serve_scale}, budget "
                                f"{args.serve_budget_gb} GiB, {args.serve_slots} slots per pool"),
                    serve=s)
        print(json.dumps(line), flush=True)
        return

    main_r = run_single(args.workload, args.precision, args.steps, args.warmup,
                        args.profile_steps, tun)
    extras = {}
    if not args.no_extras and args.workload == "dimer32":
        other = 32 if args.precision == 64 else 64
        r = run_single("dimer32", other, args.steps, args.warmup, args.profile_steps, tun)
        extras[f"dimer32_fp{other}"] = dict(value=r["value"], roofline=r["roofline"])
        for prec in (64, 32):
            r = run_single("large128", prec, 6, 2, 3, tun)
            extras[f"large128_fp{prec}"] = dict(
                value=r["value"], roofline=r["roofline"],
                kernels={k: r["kernels"][k] for k in ("stream_bin", "collide", "chain")
                         if k in r["kernels"]})
        _log("janus32 fp64")
        r = run_single("janus32", 64, 10, 2, 3, tun)
        extras["janus32_fp64"] = dict(value=r["value"], roofline=r["roofline"],
                                      kernels={k: r["kernels"][k] for k in ("chain", "collide", "stream_bin")
                                               if k in r["kernels"]}, flags=r["flags"])
        for prec in (64, 32):
            _log(f"poiseuille fp{prec}")
            r = run_single("poiseuille", prec, args.steps, args.warmup, args.profile_steps, tun)
            extras[f"poiseuille_fp{prec}"] = dict(value=r["value"], roofline=r["roofline"],
                                                 kernels=r["kernels"])
        _log("poiseuille steady profile (fp32)")
        extras["poiseuille_profile_fp32"] = poiseuille_profile(32)
        for wl, st in (("dimer32", args.steps), ("large128", 6)):
            _log(f"dimer analysis, {wl}")
            extras[f"analysis_{wl}_fp64"] = run_analysis(wl, 64, st, 2, tun)
        _log("FP32 against FP64 drift, dimer32")
        extras["fp32_drift"] = fp32_drift(200, 3, not args.no_cpu)
        _log("FP32 against FP64 drift, large128")
        extras["fp32_drift_large128"] = fp32_drift(40, 1, not args.no_cpu, name="large128")
    cpu = None
    if not args.no_cpu:
        _log("timing the CPU oracle")
        p, n_md, seed, _ = workload(args.workload, 64)
        cpu = cpu_baseline(p, n_md, seed, args.cpu_seconds)
    line = dict(base, value=main_r["value"], steps=args.steps, warmup=args.warmup,
                ms_per_step=1e3 * main_r["wall"] / args.steps,
                dtype="f64" if args.precision == 64 else "f32",
                config=dict(workload=main_r["desc"], n_solvent=main_r["n"], n_md=main_r["n_md"],
                            precision=args.precision, n_candidates=main_r["n_cand"],
                            tuning=main_r["tuning"]),
                roofline=main_r["roofline"], cpu_baseline=cpu, kernels=main_r["kernels"],
                **extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
