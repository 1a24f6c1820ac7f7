"""Benchmark of the MI355X Wilson-HMC hot path (one JSON line on stdout).

Workloads (--workload):
  hmc     (default) HMC seconds per trajectory on 16^3x32, beta 5.6,
          kappa 0.156, tau 1 with 20 leapfrog steps, CG to 1e-10 (FP64),
          trajectories 0..K-1 of the chain from the weak-field eps=0.3 start.
          A step is one trajectory.
  dslash  field-kernel bandwidth at 48^3x96 (FP64 and FP32 Dslash, staple
          force, exp+reunit, norm2 / innerProduct), GB/s against HBM peak.
  cg      24^3x48 kappa 0.157 Wilson solves of Gaussian sources to
          |b - M x| <= 1e-10 |b|: FP64 CGLS against mixed precision
          (FP32, FP16 and BF16 inner storage).
  mts     the same 16^3x32 chain with the mass-preconditioned (Hasenbusch)
          action on nested time scales: kappa_h 0.10, 5 ratio steps x 2
          heavy steps x 2 gauge steps (the innermost step equals the plain
          run's 0.05), FP64 solves to 1e-10.
  copy    a plain 2 GiB device-to-device copy (torch), the calibration
          kernel for the HBM byte counters (known bytes read and written).
  serve   Poisson stream of Wilson solves over {8^4, 16^3x32, 24^3x48}
          through the continuous-batching service (mixed precision),
          throughput and p50/p99 latency against a one-at-a-time FP64 FIFO
          baseline on the same requests.

Inputs are synthetic (weak-field gauge fields and sources drawn on the device
from seeds) and resident in HBM when the timed region starts.  The roofline
object reports the dominant kernel's algorithmic bytes per launch over its
average duration, measured with HIP events on the launch stream inside the
timed region.  Algorithmic bytes count each datum of the operation read once
and each output written once, an SU(3) link as its nine complex entries (the
half Dslash: 1536 / 1728 / 1920 B per output site in FP64 for the plain, axpy
and CG-update forms); the `implemented` entry gives the same launches with
the bytes the kernel as implemented must move (compact links).  The CPU
baseline times the FP64 oracle on a bounded sample of the same workload on
the host cores (and, smaller, on one core).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
METRIC = "HMC s/traj @16^3x32; Dslash HBM GB/s; mixed vs FP64 CG; solve p50/p99"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dslash_kernels.h", "device.h"):
        h.update(open(os.path.join(ROOT, "paper_1212_0785_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# F64 Dslash launch decisions a committed counter figure depends on
TRAFFIC_LAUNCH_KEYS = ("dslash_f64", "dslash_links_f64", "dslash_stream_f64", "dslash_order_f64",
                       "dslash_occupancy_f64")


def load_traffic(workload: str, launch=None):
    """HBM bytes per Dslash launch from the committed rocprofv3 counter runs,
    or None when the kernel source or (given `launch`, the choices of
    TRAFFIC_LAUNCH_KEYS in force) the launch changed since they were taken."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = d.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    if launch is not None and e.get("launch") != launch:
        return None
    return e.get("bytes_per_launch")


def launch_shapes(H, L, db):
    """The launch decisions in force for lattice L and where each came from:
    Dslash shape (1 = one site per work-item, 2/4 = direction split) and
    link form (reals read per SU(3) link: 12 = two rows, 10 = row 0 and
    column 2), streaming (non-temporal link loads and output stores), site
    order (0 linear, 1 tiled by z-planes, n tiled by y-blocks of n 64-site
    chunks) and workgroups per CU of the tiled order (2, or 0 = as registers
    allow) per storage, staple-force shape (0 = one link per work-item,
    1 = plane split, 2 = four directions of 64 sites per block) and link
    form."""
    table = db or (os.environ.get("HMC_TUNE_DB") or H.TUNE_TABLE)
    if os.path.isabs(table) and table.startswith(ROOT + os.sep):
        table = os.path.relpath(table, ROOT)
    out = {"table": table}
    for p, name in ((H.F64, "f64"), (H.F32, "f32"), (H.F16, "f16"), (H.BF16, "bf16")):
        c, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH, p)
        out[f"dslash_{name}"] = [c, "table" if tuned else "rule"]
        c, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH_LINKS, p)
        out[f"dslash_links_{name}"] = [c, "table" if tuned else "rule"]
        c, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH_STREAM, p)
        out[f"dslash_stream_{name}"] = [c, "table" if tuned else "rule"]
        c, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH_ORDER, p)
        out[f"dslash_order_{name}"] = [c, "table" if tuned else "rule"]
        c, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH_OCC, p)
        out[f"dslash_occupancy_{name}"] = [c, "table" if tuned else "rule"]
    c, tuned = H.hmc_tune_query(L, H.TUNE_GAUGE_FORCE)
    out["gauge_force_shape"] = [c, "table" if tuned else "rule"]
    c, tuned = H.hmc_tune_query(L, H.TUNE_GAUGE_FORCE_LINKS)
    out["gauge_force_links"] = [c, "table" if tuned else "rule"]
    return out


def event_floor(H, torch, n=200):
    """Average duration an empty one-wavefront kernel shows through the
    kernel-stamped event pair that times the sampled launches: the part of
    a timed launch that is the events' own."""
    H.hmc_timing_reset()
    H.hmc_timing_enable(1)
    H.hmc_timing_probe(n, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    t = H.hmc_timing_read().get("other")
    H.hmc_timing_enable(0)
    H.hmc_timing_reset()
    return t["total_ms"] / t["launches"] if t and t["launches"] else None


def triad_ceiling(H, torch, mib=512, reps=10):
    """Live STREAM-triad rate (GB/s, best of plain and non-temporal) over
    three arrays of `mib` MiB: the attainable streaming rate the roofline
    fraction is also read against."""
    n = mib * (1 << 20) // 8
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.ones(n, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    st = torch.cuda.current_stream()
    best = 0.0
    for nt in (False, True):
        H.hmc_stream_triad(a, b, c, 2.0, nt, stream=st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            H.hmc_stream_triad(a, b, c, 2.0, nt, stream=st)
        e1.record(st)
        torch.cuda.synchronize()
        best = max(best, 3 * 8 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b, c
    return best


def timed_kernel_roofline(H, name="dslash", timing=None):
    """Average launch time and rates of a timed kernel family: `achieved`
    on the algorithmic bytes, `achieved_moved` on the bytes as implemented."""
    t = (timing if timing is not None else H.hmc_timing_read()).get(name)
    if not t or not t["launches"]:
        return None
    avg_ms = t["total_ms"] / t["launches"]
    bytes_per_launch = t["bytes"] / t["launches"]
    moved_per_launch = t["bytes_moved"] / t["launches"]
    return {"avg_ms": avg_ms, "bytes_per_launch": bytes_per_launch,
            "achieved": bytes_per_launch / (avg_ms * 1e-3) / 1e9, "moved_per_launch": moved_per_launch,
            "achieved_moved": moved_per_launch / (avg_ms * 1e-3) / 1e9, "launches_timed": t["launches"]}


def implemented(rf):
    """The same launches' rate on the bytes the kernel as implemented moves."""
    return {"bytes_per_launch": rf["moved_per_launch"], "achieved": rf["achieved_moved"],
            "frac": rf["achieved_moved"] / HBM_PEAK_GBS}


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count()}


# ------------------------------------------------------------------- HMC


def oracle_hmc_sample(L, seed, beta, kappa, nsteps, cg_iters_per_solve, n_cg_sample=400, n_rep=3, threads=0):
    """Time the oracle's pieces of one trajectory (forces and link update
    n_rep times each, the CG over a fixed n_cg_sample iterations; about 15 s
    on 16 host cores) and project seconds per trajectory with the measured
    GPU iteration count per solve (same algorithm, same count).  threads > 0
    runs the oracle's site loops on that many threads."""
    import numpy as np  # noqa: F401

    import oracle as O
    prev = O.set_threads(threads)
    try:
        return _oracle_hmc_sample(O, L, seed, beta, kappa, nsteps, cg_iters_per_solve, n_cg_sample, n_rep)
    finally:
        O.set_threads(prev)


def _oracle_hmc_sample(O, L, seed, beta, kappa, nsteps, cg_iters_per_solve, n_cg_sample, n_rep):
    t0 = time.perf_counter()
    U = O.weak_field(L, seed, 0.3)
    ta = time.perf_counter()
    P = O.refresh_momenta(L, seed, 0)
    eta = O.eta(L, seed, 0, 0)
    phi = O.mhat(L, U, kappa, eta, dagger=True)
    O.kinetic(L, P), O.gauge_action(L, U, beta)
    t_refresh = time.perf_counter() - ta
    ta = time.perf_counter()
    for _ in range(n_rep):
        O.gauge_force(L, U, beta)
    t_gf = (time.perf_counter() - ta) / n_rep
    ta = time.perf_counter()
    Xe, _ = O.cg_mhat(L, U, kappa, phi, fixed_iters=n_cg_sample)
    t_cg = (time.perf_counter() - ta) / n_cg_sample
    ta = time.perf_counter()
    for _ in range(n_rep):
        odd = O.parity_mask(L)
        X = Xe.copy()
        X[odd] = O.dslash(L, U, Xe, 1)[odd]
        Y = O.mhat(L, U, kappa, Xe)
        Y[odd] = O.dslash(L, U, Y, 1, dagger=True)[odd]
        O.fermion_force(L, U, kappa * kappa, X, Y)
    t_ff = (time.perf_counter() - ta) / n_rep
    ta = time.perf_counter()
    for _ in range(n_rep):
        O.update_links(L, U, P, 1.0 / nsteps)
    t_up = (time.perf_counter() - ta) / n_rep
    sample = time.perf_counter() - t0
    n_force = nsteps + 1
    proj = 2 * t_refresh + n_force * (t_gf + t_ff + cg_iters_per_solve * t_cg) + nsteps * t_up
    cores = O.set_threads(0)
    return {"value": proj, "unit": "s/traj", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle on 16^3x32, trajectory 0 pieces: refresh + actions once, gauge force, "
                       f"fermion force and link update {n_rep} times each, {n_cg_sample} CG iterations; "
                       f"projected to {n_force} force evaluations x {cg_iters_per_solve:.0f} CG iterations "
                       f"(the GPU's mean per solve) + {nsteps} link updates; sample wall {sample:.1f} s"),
            "per_kernel_s": {"cg_iteration": t_cg, "gauge_force": t_gf, "fermion_force": t_ff,
                             "exp_update_reunit": t_up, "refresh_and_actions": t_refresh}}


def oracle_hmc_trajectory(L, seed, beta, kappa, nsteps):
    """One whole oracle trajectory (trajectory 0 of the chain), timed: the
    measured counterpart of the projected baseline (about a minute on 16
    host cores, so only on request)."""
    import oracle as O
    U = O.weak_field(L, seed, 0.3)
    t0 = time.perf_counter()
    _, r = O.hmc_trajectory(L, U, beta, kappa, seed, 0, 1.0, nsteps, tol=1e-10)
    return {"seconds": time.perf_counter() - t0, "cores": O.set_threads(0), "dH": r["dH"],
            "cg_iters_total": r["cg_iters_total"]}


def effective_delta(args):
    """The reliable-update delta the solves use (the library picks it when
    --reliable-delta is not given)."""
    if args.reliable_delta > 0:
        return args.reliable_delta
    return 0.01 if args.cg_prec == "f32" else 0.1


def run_hmc(args, H, torch):
    L = (16, 16, 16, 32)
    seed, beta, kappa, tau, nsteps = 12120785, 5.6, 0.156, 1.0, 20
    cg_prec = H.PREC_NAMES[args.cg_prec]
    F = H.Fields(L, beta, kappa, flags=H.FIELDS_LOWPREC if cg_prec != H.F64 else 0)
    stream = torch.cuda.current_stream()
    prm = H.cg_params(tol=1e-10, maxiter=10000, prec=cg_prec, reliable_delta=args.reliable_delta)
    H.hmc_weak_field_start(F, seed, 0.3)
    for w in range(args.warmup):
        H.hmc_trajectory(F, seed, w, tau, nsteps, prm, n_chrono=args.chrono)
    H.hmc_weak_field_start(F, seed, 0.3)  # timed chain starts at trajectory 0
    torch.cuda.synchronize()
    H.hmc_timing_reset()
    H.hmc_timing_enable(args.sample_every)
    t0 = time.perf_counter()
    results = [H.hmc_trajectory(F, seed, k, tau, nsteps, prm, stream=stream, n_chrono=args.chrono)
               for k in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    H.hmc_timing_enable(0)
    timing = H.hmc_timing_read()
    rf = timed_kernel_roofline(H, "dslash", timing)
    iters = sum(r["cg_iters_total"] for r in results)
    solves = args.steps * (nsteps + 1)
    out = {
        "metric": METRIC, "value": dt / args.steps, "unit": "s/traj", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if cg_prec == H.F64 else f"f64 ({args.cg_prec} inner solver storage)", "data": "synthetic",
        "config": {"workload": "hmc_16c32", "lattice": list(L), "beta": beta, "kappa": kappa, "tau": tau,
                   "nsteps": nsteps, "cg_tol": 1e-10, "start": "weak-field eps=0.3 seed 12120785",
                   "trajectories": f"0..{args.steps - 1}", "initial_guess": (
                       f"chronological, last {args.chrono} solutions" if args.chrono else "zero"),
                   "force_solves": ("FP64 CG" if cg_prec == H.F64 else
                                    f"mixed-precision CG, {args.cg_prec} inner storage, FP64 reliable updates "
                                    f"(delta {effective_delta(args)})"),
                   "parallelism": "1 GPU"},
        "trajectories": [{"traj": k, "seconds": r["seconds"], "dH": r["dH"], "accepted": r["accepted"],
                          "plaquette": r["plaquette"], "cg_iters": r["cg_iters_total"]}
                         for k, r in enumerate(results)],
        "s_per_traj_median": statistics.median(r["seconds"] for r in results),
        "cg_iters_per_solve": iters / solves,
        "kernels_sampled": {k: {"launches_timed": v["launches"], "launches_all": v["calls"],
                                "avg_ms": v["total_ms"] / v["launches"],
                                "GBps": v["bytes"] / (v["total_ms"] * 1e-3) / 1e9 if v["bytes"] else None,
                                "GBps_implemented": (v["bytes_moved"] / (v["total_ms"] * 1e-3) / 1e9
                                                     if v["bytes_moved"] else None)}
                            for k, v in timing.items() if v["launches"]},
        # per kernel family: sampled average x all launches, per trajectory
        "time_split_ms_per_traj": {k: v["total_ms"] / v["launches"] * v["calls"] / args.steps
                                   for k, v in timing.items() if v["launches"]},
    }
    if rf:
        out["roofline"] = {"bound": "hbm", "achieved": rf["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": rf["achieved"] / HBM_PEAK_GBS, "traffic": load_traffic("hmc_16c32"),
                           "kernel": ("F64 half-lattice hop, k_dslash or k_dslash_split (shape in "
                                      "config.launch_shapes.dslash_f64; plain, axpy/norm and CG-update "
                                      "epilogues; link form in config.launch_shapes.dslash_links_f64)"),
                           "bytes": ("algorithmic: 1536 / 1728 / 1920 B per output site (8 links of 144 B, "
                                     "spinors of 192 B) for the plain, axpy and CG-update hops"),
                           "avg_launch_ms": rf["avg_ms"], "bytes_per_launch": rf["bytes_per_launch"],
                           "launches_timed": rf["launches_timed"], "implemented": implemented(rf)}
    return out, iters / solves, L, seed, beta, kappa, nsteps


def run_mts(args, H, torch):
    L = (16, 16, 16, 32)
    seed, beta, kappa, kappa_h, tau = 12120785, 5.6, 0.156, args.kappa_h, 1.0
    steps = tuple(int(v) for v in args.mts_steps.split(","))
    F = H.Fields(L, beta, kappa)
    p = H.mts_params(tau, kappa_h, *steps, H.cg_params(tol=1e-10, maxiter=10000))
    H.hmc_weak_field_start(F, seed, 0.3)
    for w in range(args.warmup):
        H.hmc_trajectory_mts(F, seed, w, p)
    H.hmc_weak_field_start(F, seed, 0.3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [H.hmc_trajectory_mts(F, seed, k, p) for k in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    keys = ("seconds", "dH", "accepted", "plaquette", "S1_old", "S2_old", "S1_new", "S2_new", "solves_ratio",
            "solves_heavy", "iters_ratio", "iters_heavy", "gauge_forces", "link_updates")
    return {
        "metric": METRIC, "value": dt / args.steps, "unit": "s/traj", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "hmc_mts_16c32", "lattice": list(L), "beta": beta, "kappa": kappa,
                   "kappa_h": kappa_h, "tau": tau, "steps_ratio_heavy_gauge": list(steps), "cg_tol": 1e-10,
                   "start": "weak-field eps=0.3 seed 12120785", "trajectories": f"0..{args.steps - 1}",
                   "parallelism": "1 GPU"},
        "trajectories": [{"traj": k, **{x: r[x] for x in keys}} for k, r in enumerate(results)],
        "acceptance": sum(r["accepted"] for r in results) / len(results),
    }


# ----------------------------------------------------------------- Dslash


def synth_vh(L):
    return L[0] * L[1] * L[2] * L[3] // 2


def run_dslash(args, H, torch):
    L = (48, 48, 48, 96)
    F = H.Fields(L, 5.6, 0.15, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, 2, 0.3)
    H.hmc_sync_lowprec(F)
    hb = {p: H.hmc_field_bytes(L, p, H.KIND_HALF_SPINOR) for p in (H.F64, H.F32)}
    src = F.spinor(full=True)
    H.hmc_make_source(F, src, 0, 2, 0)
    inp = {H.F64: src[hb[H.F64]:]}
    inp[H.F32] = F.spinor(prec=H.F32)
    H.hmc_convert_spinor(F, inp[H.F32], H.F32, inp[H.F64], H.F64)
    outb = {p: F.spinor(prec=p) for p in (H.F64, H.F32)}
    res = {}
    for p, name in ((H.F64, "f64"), (H.F32, "f32")):
        for _ in range(args.warmup):
            H.hmc_wilson_dslash(F, outb[p], inp[p], 0, 0, p)
        torch.cuda.synchronize()
        H.hmc_timing_reset()
        H.hmc_timing_enable(1)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            H.hmc_wilson_dslash(F, outb[p], inp[p], 0, 0, p)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        H.hmc_timing_enable(0)
        rf = timed_kernel_roofline(H, "dslash")
        res[name] = {"avg_ms": rf["avg_ms"], "GBps": rf["achieved"], "frac": rf["achieved"] / HBM_PEAK_GBS,
                     "wall_ms": 1e3 * wall, "bytes_per_launch": rf["bytes_per_launch"],
                     "implemented": implemented(rf)}
    # other field kernels (FP64); flops per site (all four links) are the
    # approximate counts of the kernels' arithmetic, for the FP64 fraction
    # of the kernels near the ridge
    V = 2 * synth_vh(L)
    xe = inp[H.F64]  # a Gaussian half spinor as X_e of the fermion force
    for name, fn, kern, flops_site in (
            ("gauge_force", lambda: H.hmc_gauge_force(F, 1e-3), "gauge_force", 11500),
            ("fermion_force", lambda: H.hmc_fermion_force(F, xe, 1e-3), "fermion_force", 2800),
            ("exp_update", lambda: H.hmc_exp_update_reunit(F, 1e-3), "exp_update", 2800),
            ("plaquette", lambda: H.hmc_plaquette(F), "plaquette", 3600),
            ("norm2", lambda: H.hmc_norm2(F, inp[H.F64], 1), "reduce", None),
            ("inner", lambda: H.hmc_inner(F, inp[H.F64], outb[H.F64], 1), "reduce", None)):
        H.hmc_refresh(F, 5, 0, H.REFRESH_MOM)
        fn()
        torch.cuda.synchronize()
        H.hmc_timing_reset()
        H.hmc_timing_enable(1)
        for _ in range(max(3, args.steps // 4)):
            fn()
        torch.cuda.synchronize()
        H.hmc_timing_enable(0)
        rf = timed_kernel_roofline(H, kern)
        res[name] = {"avg_ms": rf["avg_ms"], "GBps": rf["achieved"], "frac": rf["achieved"] / HBM_PEAK_GBS,
                     "bytes_per_launch": rf["bytes_per_launch"], "implemented": implemented(rf)}
        if flops_site:
            tf = flops_site * V / (rf["avg_ms"] * 1e-3) / 1e12
            res[name].update({"TFLOPs_approx": tf, "fp64_frac_approx": tf / FP64_PEAK_TFLOPS})
    best = res["f64"]
    out = {
        "metric": METRIC, "value": best["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": best["avg_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "dslash_48c96", "lattice": list(L), "gauge": "weak-field eps=0.3 seed 2",
                   "spinor": "Gaussian seed 2", "parallelism": "1 GPU"},
        "kernels": res,
        "roofline": {"bound": "hbm", "achieved": best["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": best["frac"], "traffic": load_traffic("dslash_48c96"),
                     "kernel": f"k_dslash F64 plain, {best['bytes_per_launch'] / (synth_vh(L)):.0f} B/site",
                     "bytes": "algorithmic: 8 links of 144 B + in and out spinors of 192 B per output site",
                     "avg_launch_ms": best["avg_ms"], "bytes_per_launch": best["bytes_per_launch"],
                     "implemented": best["implemented"]},
    }
    return out, L, {k: v["avg_ms"] for k, v in res.items()}


def _slab_sample(L, t_lo, t_hi):
    """Lexicographic sites of the t-slices t_lo..t_hi (inclusive)."""
    import numpy as np
    slab = L[0] * L[1] * L[2]
    return np.arange(t_lo * slab, (t_hi + 1) * slab, dtype=np.int64)


def oracle_field_kernel_sample(L, gpu_ms, threads=0, reps=64):
    """The oracle's Dslash and staple force on a slab of the 48^3x96 field
    (the even sites, resp. all sites, of t-slices 10 and 11, with the links
    and spinors they read drawn from the same seeds as the GPU's), timed and
    projected to one whole-lattice launch."""
    import numpy as np

    import oracle as O
    prev = O.set_threads(threads)
    try:
        V = L[0] * L[1] * L[2] * L[3]
        t0 = time.perf_counter()
        need = _slab_sample(L, 9, 12)
        U = np.zeros((V, 4, 3, 3), np.complex128)  # lazily zero pages: only the slab is touched
        psi = np.zeros((V, 4, 3), np.complex128)
        O.weak_field_sites(L, 2, 0.3, need, U)
        O.gauss_source_sites(2, 0, need, psi)
        sites = _slab_sample(L, 10, 11)
        c = np.stack([sites % L[0], (sites // L[0]) % L[1], (sites // (L[0] * L[1])) % L[2],
                      sites // (L[0] * L[1] * L[2])], 1)
        even = sites[c.sum(1) % 2 == 0]
        ta = time.perf_counter()
        for _ in range(reps):
            O.dslash_sites(L, U, psi, even)
        t_ds = (time.perf_counter() - ta) / reps * (V // 2) / len(even)
        ta = time.perf_counter()
        for _ in range(reps):
            O.gauge_force_sites(L, U, 5.6, sites)
        t_gf = (time.perf_counter() - ta) / reps * V / len(sites)
        wall = time.perf_counter() - t0
        cores = O.set_threads(0)
    finally:
        O.set_threads(prev)
    alg = 1536.0 * (V // 2)
    return {"value": alg / t_ds / 1e9, "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle Dslash on the {len(even)} even sites and staple force on the {len(sites)} "
                       f"sites of t-slices 10-11 of 48^3x96 ({reps} passes each), projected to one launch over "
                       f"the lattice; algorithmic bytes 1536 B per output site; sample wall {wall:.1f} s"),
            "per_kernel_ms": {"dslash": 1e3 * t_ds, "gauge_force": 1e3 * t_gf},
            "gpu_speedup": {"dslash": 1e3 * t_ds / gpu_ms["f64"], "gauge_force": 1e3 * t_gf / gpu_ms["gauge_force"]}}


# ------------------------------------------------------------------- triad


def run_triad(args, H, torch):
    """STREAM triad a = b + s c over three 2 GiB FP64 arrays with the
    library's kernel, with and without non-temporal hints: the attainable
    streaming rate for 16-byte lanes."""
    n = (2 << 30) // 8
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    st = torch.cuda.current_stream()
    res = {}
    for nt in (False, True):
        for _ in range(args.warmup):
            H.hmc_stream_triad(a, b, c, 3.0, nt, stream=st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(args.steps):
            H.hmc_stream_triad(a, b, c, 3.0, nt, stream=st)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res["nontemporal" if nt else "plain"] = {"avg_ms": ms, "GBps": 3 * 8 * n / (ms * 1e-3) / 1e9}
    assert float(a[12345]) == 2.5 and float(a[-1]) == 2.5
    best = max(res.values(), key=lambda r: r["GBps"])
    return {"metric": METRIC, "value": best["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": best["avg_ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "stream_triad_3x2GiB", "bytes_per_launch": 3 * 8 * n, "parallelism": "1 GPU"},
            "kernels": res,
            "roofline": {"bound": "hbm", "achieved": best["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": best["GBps"] / HBM_PEAK_GBS, "traffic": None, "kernel": "k_triad",
                         "avg_launch_ms": best["avg_ms"]}}


# ------------------------------------------------------------------- copy


def run_copy(args, H, torch):
    nbytes = 2 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(st)
    for _ in range(args.steps):
        dst.copy_(src)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    gbps = 2 * nbytes / (ms * 1e-3) / 1e9
    return {"metric": METRIC, "value": gbps, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "copy_2GiB", "bytes_read": nbytes, "bytes_written": nbytes,
                       "parallelism": "1 GPU"},
            "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbps / HBM_PEAK_GBS, "traffic": None, "kernel": "torch copy_",
                         "avg_launch_ms": ms}}


# --------------------------------------------------------------------- CG


def run_cg(args, H, torch):
    L = (24, 24, 24, 48)
    kappa = 0.157
    F = H.Fields(L, 5.6, kappa, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, 1, 0.5)
    nsrc = args.steps
    rows = {}
    ref = {}
    first = {}  # solution of source 0 per precision (for the oracle comparison)
    b = F.spinor(full=True)
    x = F.spinor(full=True)
    for prec, name in ((H.F64, "f64"), (H.F32, "f32"), (H.F16, "f16"), (H.BF16, "bf16")):
        prm = H.cg_params(tol=1e-10, maxiter=50000, mode=H.CG_WILSON_SOLVE, prec=prec)
        H.hmc_make_source(F, b, 0, 1, 0)
        H.hmc_cg_solve(F, x, b, prm)  # warm-up
        recs = []
        for k in range(nsrc):
            H.hmc_make_source(F, b, 0, 1, k)
            torch.cuda.synchronize()
            st = H.hmc_cg_solve(F, x, b, prm)
            torch.cuda.synchronize()
            if k == 0:
                first[name] = x.clone()
            if prec == H.F64:
                ref[k] = x.clone()
                err = 0.0
            else:
                d = (x.view(torch.float64) - ref[k].view(torch.float64)).norm() / ref[k].view(torch.float64).norm()
                err = float(d)
            recs.append({"src": k, "seconds": st["seconds"], "iters": st["iters"],
                         "reliable_updates": st["reliable_updates"], "true_rel_res": st["true_rel_res"],
                         "rel_diff_vs_f64": err})
        t = sum(r["seconds"] for r in recs) / len(recs)
        rows[name] = {"mean_seconds": t, "solves": recs}
    best = min(("f32", "f16", "bf16"), key=lambda n: rows[n]["mean_seconds"])
    out = {
        "metric": METRIC, "value": rows["f64"]["mean_seconds"] / rows[best]["mean_seconds"],
        "unit": "x speedup (FP64 CG time / mixed time to 1e-10)", "n_gpus": 1, "steps": nsrc,
        "warmup": 1, "ms_per_step": 1e3 * rows[best]["mean_seconds"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": best, "data": "synthetic",
        "config": {"workload": "wilson_solve_24c48", "lattice": list(L), "kappa": kappa,
                   "gauge": "weak-field eps=0.5 seed 1", "sources": f"Gaussian seed 1 epochs 0..{nsrc - 1}",
                   "tol": 1e-10, "parallelism": "1 GPU"},
        "solvers": {k: {"mean_seconds": v["mean_seconds"],
                        "mean_iters": sum(r["iters"] for r in v["solves"]) / len(v["solves"]),
                        "max_true_rel_res": max(r["true_rel_res"] for r in v["solves"]),
                        "max_rel_diff_vs_f64": max(r["rel_diff_vs_f64"] for r in v["solves"])}
                    for k, v in rows.items()},
        "fastest_mixed": best,
        "_fields": F,
    }
    return out, first


def oracle_solve_sample(L, kappa, first, H, F, torch):
    """The FP64 oracle's CGLS Wilson solve of source 0 (the CPU baseline,
    one solve, ~10-20 s on 16 host cores) and the difference of every GPU
    precision's solution of the same source from it."""
    import numpy as np

    import oracle as O
    U = O.weak_field(L, 1, 0.5)
    b = O.source(L, 0, 1, 0)
    t0 = time.perf_counter()
    xo, st = O.wilson_solve(L, U, kappa, b, tol=1e-10, maxiter=50000)
    dt = time.perf_counter() - t0
    err = {}
    for name, xg in first.items():
        c = H.canon_spinor_zeros(L)
        H.hmc_export_spinor(F, c, xg, -1)
        torch.cuda.synchronize()
        xgn = c.cpu().numpy()
        err[name] = float(np.linalg.norm(xgn - xo) / np.linalg.norm(xo))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": dt, "unit": "s/solve", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle CGLS Wilson solve of source 0 (24^3x48, kappa {kappa}) to 1e-10: "
                       f"{st['iters']} iterations, true residual {st['true_rel_res']:.2e}"),
            "rel_err_vs_oracle": err}


# ------------------------------------------------------------------ serve


def serve_requests(n, seed=3):
    """Request mix: volume uniform over {8^4, 16^3x32, 24^3x48}, kappa
    U[0.150, 0.157], gauge eps U[0.2, 0.5], Z2 or point source (p = 1/2),
    per-request seeds drawn from the master seed."""
    import numpy as np
    g = np.random.default_rng(seed)
    vols = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48)]
    out = []
    for i in range(n):
        out.append({"L": vols[int(g.integers(0, 3))], "kappa": float(g.uniform(0.150, 0.157)),
                    "gauge_seed": int(g.integers(1, 2**62)), "eps": float(g.uniform(0.2, 0.5)),
                    "kind": 1 if g.random() < 0.5 else 2, "source_seed": int(g.integers(1, 2**62))})
    return out


def run_serve(args, H, torch):
    import threading

    import numpy as np
    reqs = serve_requests(args.steps)
    # one-at-a-time FP64 baseline: measured service time of every request
    fields = {}
    svc_time = []
    b, x = {}, {}
    for r in reqs:
        L = r["L"]
        if L not in fields:
            fields[L] = H.Fields(L, 5.6, r["kappa"])
            b[L] = fields[L].spinor(full=True)
            x[L] = fields[L].spinor(full=True)
        F = fields[L]
        H.hmc_set_action(F, 5.6, r["kappa"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.hmc_weak_field_start(F, r["gauge_seed"], r["eps"])
        H.hmc_make_source(F, b[L], r["kind"], r["source_seed"], 0)
        st = H.hmc_cg_solve(F, x[L], b[L], H.cg_params(tol=1e-10, maxiter=50000, mode=H.CG_WILSON_SOLVE),
                            allow_noconv=True)
        torch.cuda.synchronize()
        svc_time.append(time.perf_counter() - t0)
        r["f64_iters"] = st["iters"]
    del fields, b, x
    torch.cuda.empty_cache()
    mu1 = 1.0 / (sum(svc_time) / len(svc_time))
    lam = args.rho * mu1
    arr = np.cumsum(np.random.default_rng(4).exponential(1.0 / lam, len(reqs)))
    # FIFO single server on the measured service times
    done, lat_base = 0.0, []
    for a, s_ in zip(arr, svc_time):
        start = max(a, done)
        done = start + s_
        lat_base.append(done - a)
    base = {"throughput": len(reqs) / (done - arr[0]), "p50": float(np.percentile(lat_base, 50)),
            "p99": float(np.percentile(lat_base, 99)), "mean_service_s": 1.0 / mu1}
    # continuous-batching service, real-time Poisson submissions
    svc = H.Service(args.arena_gb * (1 << 30), inner_prec=H.PREC_NAMES[args.inner], max_batch=64,
                    chunk=args.serve_chunk, reliable_delta=args.reliable_delta)
    tickets = [None] * len(reqs)

    def submitter():
        t0 = time.perf_counter()
        for i, (a, r) in enumerate(zip(arr - arr[0], reqs)):
            dt = a - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets[i] = svc.submit(H.solve_request(r["L"], r["kappa"], r["gauge_seed"], r["eps"], r["kind"],
                                                    r["source_seed"], 0))

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    res = [svc.wait(t) for t in tickets]
    svc.close()
    lat = [r["t_done"] - r["t_submit"] for r in res]
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    ok = sum(r["status"] == 0 for r in res)
    serv = {"throughput": len(res) / span, "p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "converged": ok, "max_true_rel_res": max(r["true_rel_res"] for r in res),
            "max_group": max(r["max_group"] for r in res)}
    out = {
        "metric": METRIC, "value": serv["throughput"], "unit": "solves/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 0, "ms_per_step": 1e3 / serv["throughput"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.inner, "data": "synthetic",
        "config": {"workload": "serve_mix", "volumes": ["8^4", "16^3x32", "24^3x48"], "kappa": [0.150, 0.157],
                   "gauge_eps": [0.2, 0.5], "sources": "Z2 or point, p=1/2", "master_seed": 3,
                   "rho": args.rho, "arrival_rate_per_s": lam, "tol": 1e-10, "arena_gb": args.arena_gb,
                   "inner": args.inner, "chunk": args.serve_chunk,
                   "reliable_delta": args.reliable_delta if args.reliable_delta > 0 else (
                       0.01 if args.inner == "f32" else 0.1),
                   "parallelism": "1 GPU"},
        "service": serv,
        "fifo_fp64_baseline": base,
        "p50_ratio_vs_baseline": base["p50"] / serv["p50"],
        "p99_ratio_vs_baseline": base["p99"] / serv["p99"],
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="hmc", choices=["hmc", "mts", "dslash", "cg", "serve", "copy", "triad"])
    ap.add_argument("--rho", type=float, default=0.9, help="serve: offered load relative to FP64 FIFO capacity")
    ap.add_argument("--inner", default="f32", choices=["f64", "f32", "f16", "bf16"], help="serve: inner precision")
    ap.add_argument("--arena-gb", type=int, default=16, help="serve: arena for request state")
    ap.add_argument("--serve-chunk", type=int, default=16, help="serve: solver iterations per service round")
    ap.add_argument("--sample-every", type=int, default=31,
                    help=("time every n-th launch of each kernel kind with HIP events (the four Dslash "
                          "launches of a CG iteration count as one, bracketed by one event pair; each sampled "
                          "launch costs the GPU a few us)"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="hmc: also time one whole oracle trajectory (about a minute on 16 host cores)")
    ap.add_argument("--kappa-h", type=float, default=0.10, help="mts: heavy hopping parameter")
    ap.add_argument("--chrono", type=int, default=0,
                    help="hmc: start each force solve from the chronological guess over the last N solutions")
    ap.add_argument("--mts-steps", default="5,2,2", help="mts: ratio,heavy,gauge steps per enclosing step")
    ap.add_argument("--cg-prec", default="f64", choices=["f64", "f32", "f16", "bf16"],
                    help="hmc: storage of the force solves' inner iteration (default f64: the plain FP64 HMC)")
    ap.add_argument("--reliable-delta", type=float, default=0.0,
                    help=("hmc with --cg-prec other than f64, and serve: reliable-update threshold delta "
                          "(default: the library's, 0.01 for f32 and 0.1 for f16 / bf16)"))
    ap.add_argument("--tune-db", default=None,
                    help=("extra launch-shape table to load (hmc_tune_load) before the run; the binding "
                          "already loads paper_1212_0785_amd/tune/mi355x.txt unless HMC_TUNE_DB is set "
                          "(HMC_TUNE_DB=none: built-in rules only)"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    defaults = {"hmc": (5, 1), "dslash": (50, 5), "cg": (16, 1), "serve": (64, 0), "copy": (20, 2), "mts": (5, 1),
                "triad": (20, 2)}[args.workload]
    args.steps = args.steps if args.steps is not None else defaults[0]
    args.warmup = args.warmup if args.warmup is not None else defaults[1]

    import torch

    import paper_1212_0785_amd.hmc as H
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    H.lib()
    torch.cuda.set_device(0)
    if args.tune_db:
        H.hmc_tune_load(args.tune_db)
    if args.workload == "hmc":
        out, iters_per_solve, L, seed, beta, kappa, nsteps = run_hmc(args, H, torch)
        if not args.no_cpu_baseline:
            cb = oracle_hmc_sample(L, seed, beta, kappa, nsteps, iters_per_solve)
            out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "per_kernel_s")}
            out["cpu_baseline"].update(cpu_info())
            out["cpu_baseline"]["gpu_speedup"] = cb["value"] / out["value"]
            c1 = oracle_hmc_sample(L, seed, beta, kappa, nsteps, iters_per_solve, n_cg_sample=16, n_rep=1,
                                   threads=1)
            out["cpu_baseline"]["single_thread"] = {k: c1[k] for k in ("value", "unit", "cores", "sample",
                                                                       "per_kernel_s")}
            if args.cpu_full:
                out["cpu_baseline"]["measured_trajectory"] = oracle_hmc_trajectory(L, seed, beta, kappa, nsteps)
    elif args.workload == "dslash":
        out, L, gpu_ms = run_dslash(args, H, torch)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = oracle_field_kernel_sample(L, gpu_ms)
            out["cpu_baseline"].update(cpu_info())
            c1 = oracle_field_kernel_sample(L, gpu_ms, threads=1, reps=2)
            out["cpu_baseline"]["single_thread"] = {k: c1[k] for k in ("value", "unit", "cores", "sample",
                                                                       "per_kernel_ms")}
    elif args.workload == "serve":
        out = run_serve(args, H, torch)
    elif args.workload == "copy":
        out = run_copy(args, H, torch)
    elif args.workload == "triad":
        out = run_triad(args, H, torch)
    elif args.workload == "mts":
        out = run_mts(args, H, torch)
    else:
        out, first = run_cg(args, H, torch)
        if not args.no_cpu_baseline:
            ob = oracle_solve_sample((24, 24, 24, 48), 0.157, first, H, out.pop("_fields"), torch)
            out["cpu_baseline"] = {k: ob[k] for k in ("value", "unit", "cores", "kind", "sample")}
            out["rel_err_vs_oracle"] = ob["rel_err_vs_oracle"]
        out.pop("_fields", None)
    if "config" in out and "lattice" in out["config"]:
        out["config"]["launch_shapes"] = launch_shapes(H, out["config"]["lattice"], args.tune_db)
        if args.workload in ("hmc", "dslash") and "roofline" in out:
            out["roofline"]["event_floor_ms"] = event_floor(H, torch)
            tri = triad_ceiling(H, torch)
            out["roofline"]["attainable"] = {"triad_GBps": tri, "frac": out["roofline"]["achieved"] / tri}
            out["roofline"]["dslash_shape"] = out["config"]["launch_shapes"]["dslash_f64"][0]
            out["roofline"]["link_reals"] = out["config"]["launch_shapes"]["dslash_links_f64"][0]
            out["roofline"]["stream"] = out["config"]["launch_shapes"]["dslash_stream_f64"][0]
            out["roofline"]["tiled_order"] = out["config"]["launch_shapes"]["dslash_order_f64"][0]
            out["roofline"]["tiled_occupancy"] = out["config"]["launch_shapes"]["dslash_occupancy_f64"][0]
            launch = {k: out["config"]["launch_shapes"][k][0] for k in TRAFFIC_LAUNCH_KEYS}
            out["roofline"]["traffic"] = load_traffic(out["config"]["workload"], launch)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
