"""Benchmark of the MPCD+MD solvent hot path on one MI355X.

Headline workload (the one `value` is quoted on): one large system of 128^3
cells with 10 solvent particles per cell = 20,971,520 particles and 8
chemically powered dimer motors at seeded random non-overlapping sites
(catalytic C and non-catalytic N spheres, sigma 4, bond 6.7, eps_B = 0.5 on
N, catalytic conversion with probability 1, bulk B->A rate 0.01), dt = 0.01,
tau = 0.5 (50 MD steps per collision), FP64 state.  Synthetic seeded input:
the library's own initialisation (uniform positions outside the colloids,
Maxwellian velocities at kT = 1).

One benchmark step = one interval of the method: 50 velocity-Verlet MD steps
of every solvent particle and the dimers, then one MPCD collision with the
bulk reaction.  value = solvent particle-steps per second = N * 50 * steps /
wall time, with the state resident in HBM.

The roofline object describes the dominant bandwidth-bound kernel (the
collision): its average launch duration is measured with HIP events that the
library records on the stream the kernel runs on, over a second pass of the
same workload; achieved = the kernel's algorithmic bytes per launch / that
duration.  `interval` relates the whole interval to HBM peak with the bytes
the method itself must move per particle and interval (streaming, binning,
scan, scatter, collision gather and write), and `chain` states the latency
of the MD chain (the Verlet-list particles and colloids, n_md dependent
steps).  cpu_baseline times the FP64 CPU oracle on a bounded sample of the
same workload on the host cores.

Objects on the same line: the same system in FP32 state; the batched
ensemble (64 dimer replicas, box edges from {16, 20, 24, 32}, FP32 and FP64,
launch shapes tuned per box class); the served Poisson trace (p50/p99 job
latency at the specified arrival rate and at 0.5x and 0.8x of the measured
capacity); the FP32-against-FP64 drift of the large system over 1000
collisions; the 32^3 single-dimer and 10^3 single-sphere systems; and the
flows, Janus and analysis extensions.
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
REC_BYTES = {8: 64, 4: 32}          # staging record of the scatter, per particle


def algorithmic_bytes(kernel: str, n: int, ncell: int, tb: int, n_cand: int,
                      flow: bool = False) -> float:
    """Bytes a kernel must move per launch given its inputs and outputs (not
    counting re-reads), tb = bytes of the storage type, R = staging record:
    stream_bin  per free particle: read x, v (6 tb) + list flag (1), write x
                (3 tb) + key/rank (8); cell counters 8 B per cell.  With a
                flow every particle also writes v (12 tb + 9).
    scatter     per particle: read key/rank (8), cell start (4), x, v (6 tb),
                id (4), state (1); write the record (R).
    collide     per particle: read the record (R); write x, v (6 tb), id (4),
                state (1), list flag (1); per cell: read the start (4), zero
                the counter (4).
    scan_final  per cell: read count (4), write start (4).
    chain       per list entry: read and write x, v, state (12 tb + 2).
    analysis    per particle: read x (3 tb) and state (1)."""
    nf = max(n - n_cand, 0)
    R = REC_BYTES[tb]
    if kernel == "stream_bin":
        return nf * ((12 if flow else 9) * tb + 9) + 8 * ncell
    if kernel == "scatter":
        return n * (6 * tb + 17 + R)
    if kernel == "collide":
        return n * (R + 6 * tb + 6) + 8 * ncell
    if kernel == "scan_final":
        return 8 * ncell
    if kernel == "chain":
        return n_cand * (12 * tb + 2)
    if kernel == "analysis":
        return n * (3 * tb + 1)
    if kernel in ("chunk_scan", "cand_write"):
        return n * 1 + 8 * math.ceil(n / 1024)
    return 0.0


def method_bytes_per_particle(tb: int, ncell_per_particle: float) -> float:
    """Bytes per particle and interval that the method itself must move with
    fused-interval streaming (the algorithmic floor, independent of this
    implementation's staging): streaming 9 tb + 9, cell key/rank 8, scatter
    of a 12-byte index, cell scan 12 per cell, and the collision's gather
    and write of the payload (4 + 2 P, P = 6 tb + 5: x, v, id, state)."""
    P = 6 * tb + 5
    return (9 * tb + 9) + 8 + 12 + 12 * ncell_per_particle + 4 + 2 * P


def traffic_table(workload_name: str, precision: int):
    """Per-phase HBM bytes per launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is
    none or the kernels changed since it was taken."""
    from paper_1608_04904_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"{workload_name}_fp{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return {k: 1048576.0 * (v["fetch_MB"] + v["write_MB"]) for k, v in d.get("kernels", {}).items()}


DESCS = {
    "large128": ("large128: 128^3 cells, rho 10, N=20,971,520, 8 dimers (C+N, sigma 4, d 6.7) at "
                 "random non-overlapping sites, tau 0.5 (50 MD steps/collision)"),
    "dimer32": ("dimer32: 32^3 cells, rho 10, N=327,680, 1 dimer (C+N, sigma 4, d 6.7), "
                "tau 0.5 (50 MD steps/collision)"),
    "sphere10": "sphere10: 10^3 cells, rho 10, N=10,000, 1 WCA sphere sigma 2, tau 0.1 (10 MD steps/collision)",
    "janus32": ("janus32: 32^3 cells, rho 10, N=327,680, one composite Janus particle (13 beads, 42 rigid "
                "bonds, iterative RATTLE), tau 0.5 (50 MD steps/collision)"),
    "poiseuille": ("poiseuille: 64 x 64 x 32 cells between plates at z = 0 and 32, rho 10, N=1,310,720, "
                   "g = 0.001 along x, tau 0.1 (10 MD steps/collision), no colloid"),
    "solvent128": ("solvent128: 128^3 cells, rho 10, N=20,971,520, no colloid (the streaming, sort and "
                   "collision kernels alone), tau 0.5 (50 MD steps/collision)"),
}


def workload(name: str, precision: int):
    import workloads as W
    mk = {"large128": (W.large128, 50, 3), "dimer32": (W.dimer32, 50, 2), "sphere10": (W.sphere10, 10, 1),
          "poiseuille": (W.poiseuille, 10, 5)}
    if name == "janus32":
        return W.janus_system(L=32, rho=10, n_md=50, precision=precision), 50, W.BASE_SEED + 6, DESCS[name]
    if name == "solvent128":
        p = W.base_params(L=(128, 128, 128), rho=10, dt=0.01, n_md=50, precision=precision)
        p["name"] = name
        return p, 50, W.BASE_SEED + 7, DESCS[name]
    if name not in mk:
        raise SystemExit(f"unknown workload {name}")
    f, n_md, k = mk[name]
    return f(precision=precision), n_md, W.BASE_SEED + k, DESCS[name]


def cpu_baseline(p, n_md, seed, budget_s: float):
    """Time the FP64 oracle on a bounded sample: one untimed warm-up
    interval, then whole intervals of the same workload until about
    budget_s seconds of work."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t_init = time.perf_counter()
    o = oracle.Oracle(p, seed)
    o.run(n_md, 1)
    t_init = time.perf_counter() - t_init
    t0 = time.perf_counter()
    k = 0
    while True:
        o.run(n_md, 1)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    del o
    return dict(value=p["n_solvent"] * n_md * k / dt, unit="particle-steps/s", cores=threads,
                kind="oracle",
                sample=f"{k} timed intervals x {n_md} MD steps of the same workload "
                       f"({p['n_solvent']} particles) after one untimed warm-up interval; "
                       f"{dt:.1f} s timed, {t_init:.1f} s init + warm-up")


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TUNING_KEYS = ("collide_cells", "collide_block", "collide_ppt", "chain_k", "chain_block", "chain_resident",
               "stream_block", "stream_ppt", "chain_serial")


def tuning_from_args(args) -> dict:
    tun = dict(use_graph=args.graph)
    for k in TUNING_KEYS:
        v = getattr(args, k)
        if v >= 0:
            tun[k] = v
    return tun


def copy_peak_gbps(mib=2048, reps=5):
    """Best of `reps` plain device-to-device copies of `mib` MiB, read plus
    write bytes over the copy's event time: what a pure streaming kernel
    reaches on this device, reported beside the nominal 8 TB/s."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def run_single(name, precision, steps, warmup, profile_steps, tun, keep=False):
    """Time `steps` intervals of one system, then a profiled pass.  Returns a
    dict with value, wall, per-kernel averages and the roofline objects."""
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
    kernels = {k: dict(avg_ms=round(v[0], 5), launches=v[1],
                       algorithmic_MB=round(algorithmic_bytes(k, n, ncell, tb, n_cand, flow) / 1048576.0, 3),
                       algorithmic_GBps=round(algorithmic_bytes(k, n, ncell, tb, n_cand, flow)
                                              / (v[0] * 1e-3) / 1e9, 1))
               for k, v in kern.items()}
    _log(f"{name} fp{precision} kernels {json.dumps(kernels)}")
    # the dominant bandwidth-bound kernel: the largest event time among the
    # particle kernels (the MD chain is latency-bound, reported apart)
    hbm_kernels = [k for k in ("collide", "stream_bin", "scatter") if k in kern]
    traffic = traffic_table(name, precision)
    dom = max(hbm_kernels, key=lambda k: kern[k][0] * kern[k][1])
    avg_ms = kern[dom][0]
    achieved = algorithmic_bytes(dom, n, ncell, tb, n_cand, flow) / (avg_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=(traffic or {}).get(dom), kernel=dom, avg_launch_ms=avg_ms,
                bytes_per_launch=algorithmic_bytes(dom, n, ncell, tb, n_cand, flow))
    value = n * n_md * steps / wall
    mb = method_bytes_per_particle(tb, ncell / max(n, 1))
    interval = dict(method_bytes_per_particle=round(mb, 2),
                    bytes_per_particle_step=round(mb / n_md, 4),
                    achieved_GBps=round(mb / n_md * value / 1e9, 1),
                    frac=mb / n_md * value / 1e9 / HBM_PEAK_GBS,
                    ms_per_interval=1e3 * wall / steps,
                    measured_traffic_GBps=None if traffic is None else round(
                        sum(traffic[k] * kern[k][1] / profile_steps for k in traffic if k in kern)
                        / (wall / steps) / 1e9, 1),
                    note="bytes the method must move per particle and interval (fused-interval "
                         "streaming, sort, collision gather and write) x particle rate, over 8 TB/s")
    chain = None
    if "chain" in kern and n_cand > 0:
        chain = dict(avg_launch_ms=kern["chain"][0], us_per_md_step=1e3 * kern["chain"][0] / n_md,
                     list_entries=n_cand,
                     note="latency-bound: n_md dependent MD steps, each ending in an exchange of the "
                          "colloid force sums between workgroups")
    out = dict(value=value, wall=wall, n=n, n_md=n_md, desc=desc, n_cand=n_cand, roofline=roof,
               interval=interval, chain=chain, kernels=kernels, tuning=s.get_tuning(), flags=ob["flags"])
    if keep:
        out["system"] = s
        return out
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


def fp32_drift(intervals: int, every: int, oracle_intervals: int, with_oracle: bool, name: str = "large128"):
    """FP32 state against FP64 from the same initial state over `intervals`
    collisions, sampled every `every`: total momentum P = sum m v (solvent and
    colloids, conserved exactly by the method), total energy E = KE + U - e_rxn
    (e_rxn: potential change booked at species flips), and the dimers'
    centre-of-mass MSD in each precision.  The FP64 run is checked bit for bit
    against the CPU oracle over the first `oracle_intervals` intervals (a
    separate run from the same state), so it stands for the oracle."""
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
        t0 = time.perf_counter()
        for k in range(0, intervals + 1, every):
            if k:
                s.step(n_md, every)
            o = s.observables(raise_on_flags=False)
            P.append(np.array(o["momentum"]))
            E.append(o["ke_solvent"] + o["ke_colloid"] + o["potential"] - o["e_rxn"])
            X = np.array(o["colloid_X"])
            R.append(np.array([(masses[a] * X[a] + masses[b] * X[b]) / (masses[a] + masses[b])
                               for a, b, _ in bonds]))
        torch.cuda.synchronize()
        runs[prec] = dict(P=np.array(P), E=np.array(E), R=np.array(R), flags=o["flags"],
                          wall=time.perf_counter() - t0)
        s.close()
        del s
        torch.cuda.empty_cache()
    out_eq = None
    if with_oracle:
        import oracle
        g = rm.System(p64, seed)
        g.set_state(st0)
        g.step(n_md, oracle_intervals)
        oc = oracle.Oracle(p64, seed, init=False)
        oc.set_state(st0)
        oc.run(n_md, oracle_intervals)
        gs, os_ = g.get_state(), oc.get_state()
        out_eq = all(np.array_equal(np.asarray(gs[k]), np.asarray(os_[k]))
                     for k in ("id", "state", "x", "v", "X", "V"))
        g.close()
        del g, oc
        torch.cuda.empty_cache()
    r64, r32 = runs[64], runs[32]
    n = p64["n_solvent"]
    pscale = float(np.sqrt(n * p64["mass"] * p64["kT"]))     # thermal momentum of the system
    e0 = float(r64["E"][0])
    lags = np.arange(len(r64["R"])) * every

    def msd(R):
        return [float(np.mean(np.sum((R[i] - R[0]) ** 2, axis=1))) for i in range(len(R))]
    m64, m32 = msd(r64["R"]), msd(r32["R"])
    pick = [i for i in range(len(lags)) if lags[i] in (0, 10, 50, 100, 200, 500, 1000) or i == len(lags) - 1]
    out = dict(
        workload=name, n_dimers=len(bonds), intervals=intervals, md_steps=intervals * n_md,
        sample_every=every,
        momentum_drift_fp64=float(np.max(np.linalg.norm(r64["P"] - r64["P"][0], axis=1)) / pscale),
        momentum_drift_fp32=float(np.max(np.linalg.norm(r32["P"] - r32["P"][0], axis=1)) / pscale),
        energy_drift_fp64=float(np.max(np.abs(r64["E"] - e0)) / abs(e0)),
        energy_drift_fp32=float(np.max(np.abs(r32["E"] - r32["E"][0])) / abs(e0)),
        energy_fp32_vs_fp64=float(np.max(np.abs(r32["E"] - r64["E"])) / abs(e0)),
        dimer_msd_fp64={str(int(lags[i])): m64[i] for i in pick},
        dimer_msd_fp32={str(int(lags[i])): m32[i] for i in pick},
        # the two trajectories decorrelate (the dynamics is chaotic): rms
        # distance between the FP32 and FP64 dimer centres
        dimer_com_diff={str(int(lags[i])): float(np.sqrt(np.mean(np.sum((r32["R"][i] - r64["R"][i]) ** 2,
                                                                           axis=1)))) for i in pick},
        flags=[int(r64["flags"]), int(r32["flags"])],
        wall_s=[round(r64["wall"], 2), round(r32["wall"], 2)],
        note="momentum drifts are max_t |P(t) - P(0)| / sqrt(N m kT); energy drifts max_t |E(t) - E(0)| / E(0); "
             "MSD averaged over the dimers; single trajectories decorrelate, so the MSDs are two samples")
    if out_eq is not None:
        out["fp64_bitwise_equal_to_oracle"] = dict(intervals=oracle_intervals, equal=bool(out_eq))
    return out


def tune_batch_classes(precision, intervals=4):
    """Autotuned launch shapes per box class of the ensemble (one seeded
    system per class over the autotuner's grid, measured afresh each run)."""
    from paper_1608_04904_amd import autotune
    import workloads as W
    reps = W.batch_replicas(n=64, precision=precision)
    best = {}
    for p in reps:
        key = autotune.box_class(p)
        if key not in best:
            best[key] = autotune.tune(p, seed=1, intervals=intervals, cache_path=None, force=True)
    return best


def run_batch(precision, ticks, warmup, tun, n_rep=64, tuned=None):
    """64 dimer replicas, box edges from {16,20,24,32}, per-replica seeds,
    one interval (50 MD steps + collision) per replica per tick; with
    `tuned`, each slot's collision tile size comes from its box class and
    the batch-wide shapes from the class holding most particles."""
    import torch
    import paper_1608_04904_amd as rm
    import workloads as W
    from paper_1608_04904_amd import autotune
    reps = W.batch_replicas(n=n_rep, precision=precision)
    b = rm.Batch(len(reps), precision=precision)
    bt = dict(tun)
    if tuned:
        weight = {}
        for p in reps:
            k = autotune.box_class(p)
            weight[k] = weight.get(k, 0) + p["n_solvent"]
        top = max(weight, key=weight.get)
        for k in ("chain_k", "stream_ppt"):
            if k in tuned[top]:
                bt[k] = tuned[top][k]
    b.set_tuning(**bt)
    for i, p in enumerate(reps):
        b.set_slot(i, p, p["seed"], p["n_md"])
        if tuned:
            cc = int(tuned[autotune.box_class(p)].get("collide_cells", 0))
            if cc > 0:
                b.set_slot_tuning(i, cc)
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
                ms_per_tick=1e3 * wall / ticks, flagged=sum(1 for f in flags if f), tuning=bt)


def run_serve(n_jobs, rate, budget_gb, slots, realtime=True, seed=None):
    """Poisson trace at `rate` jobs/s (box edge 12..48, density 5..20, sphere
    or dimer, tau 0.1..0.5, 500..5000 collisions, FP32 or FP64); with
    realtime False every job is queued at the start (a saturated server)."""
    import workloads as W
    from paper_1608_04904_amd.serve import Server, summarize
    jobs = W.serve_trace(n_jobs=n_jobs, rate=rate, seed=seed)
    work = sum(j["params"]["n_solvent"] * j["params"]["n_md"] * j["n_collide"] for j in jobs)
    srv = Server.on_gpu(hbm_budget=int(budget_gb * (1 << 30)), slots_per_pool=slots)
    t0 = time.perf_counter()
    res = srv.run(jobs, realtime=realtime)
    wall = time.perf_counter() - t0
    s = summarize(res)
    s.update(wall_s=wall, peak_hbm_bytes=srv.peak_used, n_jobs_offered=n_jobs,
             arrival_rate=rate if realtime else None,
             offered_particle_steps_per_s=(work / max(jobs[-1]["arrival"], 1e-9)) if realtime else None,
             restarted=sum(1 for r in res if r.restarts))
    for pool in srv.pools.values():
        pool.batch.close()
    import torch
    torch.cuda.empty_cache()
    _log(f"serve: {json.dumps(s)}")
    return s, work / n_jobs


def serve_block(n_jobs, budget_gb, slots):
    """The served trace at its specified arrival rate (20 jobs/s); the
    capacity of the server (aggregate particle-steps/s with every job of the
    trace queued at the start); then the trace with arrival rates that offer
    0.5x and 0.8x of that capacity."""
    spec, mean_job = run_serve(n_jobs, 20.0, budget_gb, slots)
    sat, _ = run_serve(n_jobs, 20.0, budget_gb, slots, realtime=False)
    cap = sat.get("particle_steps_per_s", 0.0)
    out = dict(at_spec=spec, saturated=sat, capacity_particle_steps_per_s=cap,
               mean_job_particle_steps=mean_job)
    if cap > 0:
        for f in (0.5, 0.8):
            rate = f * cap / mean_job
            r, _ = run_serve(n_jobs, rate, budget_gb, slots)
            out[f"at_{f}x_capacity"] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large128",
                    choices=["large128", "dimer32", "sphere10", "poiseuille", "janus32", "solvent128", "batch",
                             "serve"])
    ap.add_argument("--precision", type=int, default=64)
    ap.add_argument("--profile-steps", type=int, default=6)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--graph", type=int, default=1)
    for k in TUNING_KEYS:
        ap.add_argument("--" + k.replace("_", "-"), dest=k, type=int, default=-1)
    ap.add_argument("--serve-jobs", type=int, default=40)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--batch-ticks", type=int, default=30)
    ap.add_argument("--drift-intervals", type=int, default=1000)
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
        tuned = {prec: tune_batch_classes(prec) for prec in (64, 32)}
        r64 = run_batch(64, args.steps, args.warmup, tun, tuned=tuned[64])
        r32 = run_batch(32, args.steps, args.warmup, tun, tuned=tuned[32])
        line = dict(base, value=r32["value"], steps=args.steps, warmup=args.warmup,
                    ms_per_step=1e3 * r32["wall"] / args.steps, dtype="f32",
                    config=dict(workload="batch: 64 dimer replicas, box edge from {16,20,24,32}, rho 10, "
                                "tau 0.5, per-replica seeds, one interval per replica per step"),
                    fp32=r32, fp64=r64, fp32_over_fp64=r32["value"] / r64["value"], tuned=tuned)
        print(json.dumps(line), flush=True)
        return
    if args.workload == "serve":
        s = serve_block(args.serve_jobs, args.serve_budget_gb, args.serve_slots)
        line = dict(base, value=s["at_spec"].get("particle_steps_per_s", 0.0),
                    steps=s["at_spec"].get("n_jobs", 0), warmup=0, ms_per_step=None, dtype="f32+f64",
                    config=dict(workload=f"serve: Poisson trace of {args.serve_jobs} jobs at 20/s, "
                                f"500-5000 collisions each, budget {args.serve_budget_gb} GiB"),
                    serve=s)
        print(json.dumps(line), flush=True)
        return

    main_r = run_single(args.workload, args.precision, args.steps, args.warmup, args.profile_steps, tun)
    # with a calibration copy asked for, the same size, so that a counter
    # run's largest copy dispatch is the calibration copy
    copy = copy_peak_gbps(args.calibrate_copy if args.calibrate_copy > 0 else 2048)
    _log(f"plain device copy: {copy:.1f} GB/s")
    main_r["roofline"].update(measured_copy_GBps=round(copy, 1), frac_of_copy=main_r["roofline"]["achieved"] / copy)
    main_r["interval"].update(frac_of_copy=main_r["interval"]["achieved_GBps"] / copy)
    extras = {}
    if not args.no_extras and args.workload == "large128":
        other = 32 if args.precision == 64 else 64
        r = run_single("large128", other, args.steps, args.warmup, args.profile_steps, tun)
        extras[f"large128_fp{other}"] = dict(value=r["value"], roofline=r["roofline"], interval=r["interval"],
                                            chain=r["chain"], kernels=r["kernels"])
        v64 = main_r["value"] if args.precision == 64 else r["value"]
        v32 = r["value"] if args.precision == 64 else main_r["value"]
        extras["large128_fp32_over_fp64"] = v32 / v64
        for prec in (64, 32):
            r = run_single("dimer32", prec, 40, 5, 10, tun)
            extras[f"dimer32_fp{prec}"] = dict(value=r["value"], interval=r["interval"], chain=r["chain"],
                                              kernels=r["kernels"])
        r = run_single("sphere10", 64, 100, 10, 10, tun)
        extras["sphere10_fp64"] = dict(value=r["value"], chain=r["chain"], kernels=r["kernels"])
        _log("batched ensemble (config 4): autotuning per box class")
        tuned = {prec: tune_batch_classes(prec) for prec in (64, 32)}
        b64 = run_batch(64, args.batch_ticks, 3, tun, tuned=tuned[64])
        b32 = run_batch(32, args.batch_ticks, 3, tun, tuned=tuned[32])
        extras["batch"] = dict(fp64=b64, fp32=b32, fp32_over_fp64=b32["value"] / b64["value"], tuned=tuned,
                               workload="64 dimer replicas, box edge from {16,20,24,32}, rho 10, tau 0.5, "
                                        "per-replica seeds; one interval per replica per tick")
        _log("served trace (config 5)")
        extras["serve"] = serve_block(args.serve_jobs, args.serve_budget_gb, args.serve_slots)
        _log(f"FP32 against FP64 drift, large128, {args.drift_intervals} collisions")
        extras["fp32_drift_large128"] = fp32_drift(args.drift_intervals, 10, 1, not args.no_cpu, "large128")
        _log("janus32 fp64")
        r = run_single("janus32", 64, 10, 2, 3, tun)
        extras["janus32_fp64"] = dict(value=r["value"], chain=r["chain"],
                                      kernels={k: r["kernels"][k] for k in ("chain", "collide", "stream_bin")
                                               if k in r["kernels"]}, flags=r["flags"])
        for prec in (64, 32):
            _log(f"poiseuille fp{prec}")
            r = run_single("poiseuille", prec, 40, 5, 10, tun)
            extras[f"poiseuille_fp{prec}"] = dict(value=r["value"], interval=r["interval"],
                                                 kernels=r["kernels"])
        _log("poiseuille steady profile (fp32)")
        extras["poiseuille_profile_fp32"] = poiseuille_profile(32)
        for wl, st in (("dimer32", 40), ("large128", 6)):
            _log(f"dimer analysis, {wl}")
            extras[f"analysis_{wl}_fp64"] = run_analysis(wl, 64, st, 2, tun)
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
                roofline=main_r["roofline"], interval=main_r["interval"], chain=main_r["chain"],
                cpu_baseline=cpu, kernels=main_r["kernels"], **extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
