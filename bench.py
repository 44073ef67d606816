"""Benchmark: wall time and matvecs per outer IRN step, recycled vs plain CG.

Headline workload: the 256 x 256 deblurring problem (Gaussian PSF sigma = 3 at
15 x 15, 20 shifts log-spaced in 1e-5..1e1, principal recycle dimension 40,
local dimension 5, one shift solved at a time, relative residual 1e-8), whose
configured outer loop has 5 steps.  A "step" is one outer step of the
edge-preserving iteration: new weights, principal recycle space (Algorithm 1,
A U, E U, blocks), and all 20 shifted solves (Algorithm 5, per-k phase).

Timing: W untimed warm-up steps, then exactly K timed outer steps, taken as
consecutive runs of the configured 5-step loop (each run starts afresh at
k = 0, so the first-step spike is inside every run; a last partial run covers
k = 0..K mod 5 - 1).  `value` is the configured loop's mean step time: the
median over runs of each k, averaged over k = 0..4.  `ms_per_step` is the raw
mean over all K timed steps.

Variants, each timed the same way on the same kernels:
  plain per-shift CG (x0 = 0, one shift per launch): the target's denominator;
  plain batched CG (x0 = 0, all shifts in one launch);
  plain warm-started CG (x0 = the previous outer step's solution of the shift);
  recycled, one shift at a time (the headline) and recycled batched.

The default line also carries the 1024 x 1024 / 32-shift workload and the
64-instance workload (each over its configured outer steps, one run per
variant) with their own rooflines, and the oracle timed on the host
(single-threaded and on the host's allotted cores) on a bounded sample.

Prints one JSON line.  Inputs are seeded synthetic data resident in HBM before
the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "wall time & matvecs per outer IRN step, recycled vs plain CG @1e-8 relres"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
HOST_CORE_SHARE = 16      # CPU threads a one-GPU machine allots to its job


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, HOST_CORE_SHARE))


def host_cpu() -> dict:
    """Model name and thread count of the timing host (from lscpu)."""
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Socket(s)", "CPU max MHz"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cg_alg_bytes_per_px_iter(q: int, m_share: int) -> float:
    """Algorithmic HBM bytes per pixel per CG iteration of one system.

    One iteration reads r_{j-1}, w_{j-1}, ph_{j-1}, x, p_{j-1} and the q
    columns of W and of Z, and writes r_j, ph_j, x, p_j and w_j (each pixel
    once; the halo re-reads are not algorithmic); the two weight planes
    (16 B/px) are shared by the m_share systems of a launch.
    """
    return 80.0 + 16.0 * q + 16.0 / max(1, m_share)


def cg_alg_flops_per_px_iter(s: int, q: int) -> float:
    """K^T K as two banded passes of 2s - 1 taps (2 flops each), E (13), the
    vector updates and the p.w, r.r, r.w, w.w, Z^T r, Z^T w partial sums."""
    return 8.0 * s - 4.0 + 13.0 + 14.0 + 8.0 * q


# HBM bytes per CG launch measured with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE on
# the recycled loop of each workload (FETCH_SIZE scaled by 2.0, WRITE_SIZE by 1.0:
# the factors a 256 MiB device copy gives), keyed by the workload, the solve mode and
# the hash of the sources of the kernels that mode launches; any other build reports null.
MEASURED_TRAFFIC = {
    ("C2", "sequential", "66bfc4247badd383"): 0.7960e9,   # profiles/k_cg1_256x256_sequential_recycled.md
    ("C3", "batched", "af3dceadc2bcabfa"): 2.0434e12,        # profiles/k_cg_1024x1024_batched_recycled.md
    ("C4", "batched", "af3dceadc2bcabfa"): 3.4616e12,        # profiles/k_cg_64_instances_batched_recycled.md
}
# the measured traffic holds for these sources: the CG kernels a mode launches
# (batched launches hold several systems and never run the single-system
# kernel), and the outer loop whose defaults decide how the iterations are
# split into launches
_COMMON_SOURCES = ["paper_2306_15049_amd/csrc/cg.hip", "paper_2306_15049_amd/csrc/cgcore.hpp",
                   "paper_2306_15049_amd/csrc/stencil.hpp", "paper_2306_15049_amd/csrc/internal.hpp",
                   "paper_2306_15049_amd/irn.py"]
KERNEL_SOURCES = {"batched": _COMMON_SOURCES,
                  "sequential": _COMMON_SOURCES + ["paper_2306_15049_amd/csrc/cg1.hip"]}
KERNEL_NAMES = {"batched": "k_cg (persistent deflated CG, one stencil + update phase per iteration)",
                "sequential": "k_cg1 / k_cg (persistent deflated CG of one system / of many; "
                              "one stencil + update phase per iteration)"}


def kernel_source_hash(label: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[label]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def desc_problems(cfg) -> str:
    pr = cfg.problems
    if pr[0].ct is not None:
        return f"{pr[0].ny}x{pr[0].nx} parallel-beam CT, {len(pr[0].ct[0])} angles, {pr[0].ct[1]} bins"
    if len(pr) == 1:
        s = pr[0].psf.shape[0]
        return f"{pr[0].ny}x{pr[0].nx} deblur, PSF {s}x{s} sigma={pr[0].sigma}"
    sides = sorted({p.ny for p in pr})
    return (f"{len(pr)} deblurring instances, sides {sides[0]}..{sides[-1]}, "
            f"PSF sigma {min(p.sigma for p in pr):.2f}..{max(p.sigma for p in pr):.2f}")


def roofline(cfg, recs, mode_batched: bool, label: str):
    """Algorithmic bytes of every timed CG iteration over the CG kernel time
    (HIP events on the solve stream).  Each system counts with its own size,
    PSF and reported local-space width q; the weight planes are shared by the
    systems of one launch."""
    from paper_2306_15049_amd import rsr  # noqa: F401
    M = len(cfg.gammas)
    tot_bytes = tot_flops = tot_ms = 0.0
    tot_iters = launches = 0
    for r in recs:
        m_share = M if mode_batched else 1
        for j, its in enumerate(r.iters):
            pr = cfg.problems[j // M]
            npx = pr.ny * pr.nx
            q = r.local_dim[j]
            tot_bytes += its * npx * cg_alg_bytes_per_px_iter(q, m_share)
            tot_flops += its * npx * cg_alg_flops_per_px_iter(pr.psf.shape[0], q)
            tot_iters += its
        tot_ms += r.cg_kernel_ms
        launches += r.cg_launches
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    key = (cfg.name, label, kernel_source_hash(label))
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": MEASURED_TRAFFIC.get(key),
            "kernel": KERNEL_NAMES[label],
            "alg_bytes_per_launch": tot_bytes / max(1, launches),
            "avg_launch_ms": tot_ms / max(1, launches),
            "launches": launches,
            "fp64_tflops": tot_flops / (tot_ms * 1e-3) / 1e12 if tot_ms > 0 else 0.0,
            "fp64_frac": (tot_flops / (tot_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS) if tot_ms > 0 else 0.0,
            "cg_kernel_ms_per_step": tot_ms / max(1, len(recs)),
            "us_per_cg_iteration": tot_ms * 1e3 / max(1, tot_iters)}


def summarize(recs, steps_per_loop: int):
    """Per-k medians over the runs of the loop, and their mean over the loop."""
    by_k = {}
    for r in recs:
        by_k.setdefault(r.k, []).append(r)
    med_ms = {k: statistics.median(x.wall_ms for x in v) for k, v in by_k.items()}
    med_mv = {k: statistics.median(x.matvec_A for x in v) for k, v in by_k.items()}
    ks = sorted(med_ms)
    loop_ms = sum(med_ms[k] for k in ks) / len(ks)
    loop_mv = sum(med_mv[k] for k in ks) / len(ks)
    ge1 = [k for k in ks if k >= 1]
    return {"ms_per_step": loop_ms,
            "ms_per_step_k_ge_1": (sum(med_ms[k] for k in ge1) / len(ge1)) if ge1 else None,
            "matvecs_A_per_step": loop_mv,
            "matvecs_E_per_step": sum(statistics.median(x.matvec_E for x in by_k[k]) for k in ks) / len(ks),
            "per_k_ms": [round(med_ms[k], 3) for k in ks],
            "per_k_matvecs_A": [med_mv[k] for k in ks],
            "per_k_p": [by_k[k][0].p for k in ks],
            "runs": max(len(v) for v in by_k.values()),
            "covers_k": ks,
            "complete_loop": len(ks) == steps_per_loop,
            "max_relres": max(max(r.relres) for r in recs)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed outer steps (runs of the configured loop)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C2", help="headline workload")
    ap.add_argument("--no-variants", action="store_true", help="only the recycled method and plain per-shift CG")
    ap.add_argument("--no-plain", action="store_true", help="only the recycled method (profiling runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-minres", action="store_true", help="skip the recycled-vs-plain MINRES block")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^2 and 64-instance blocks")
    ap.add_argument("--large-only", default=None, help="comma list of large workloads to run (C3, C4)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-cache", default=None, help="autotune cache file (read if it holds the case, else appended)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device three times (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is a design note, "
              "not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_15049_amd import irn, rsr, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8, "copies": 3}))
        return
    log = sys.stderr if args.verbose else None
    ctx = rsr.Context(0)

    def run_variant(cfg, method, mode, steps, warmup, label, tiles_cache, solver="cg"):
        """warmup untimed steps, then `steps` timed steps as runs of the configured loop."""
        loop = irn.OuterLoop(ctx, cfg, method, mode=mode, solver=solver)
        n_inst = len(cfg.problems)
        key = (cfg.name, mode)
        if not args.no_autotune and cfg.problems[0].ct is None:
            if key not in tiles_cache:
                M = len(cfg.gammas)
                tiles_cache[key] = {i: ctx.autotune(i, 1 if mode == rsr.SEQUENTIAL else M, args.tune_cache)
                                    for i in range(n_inst)}
                if log:
                    print(f"[{cfg.name} {label}] autotuned tiles {tiles_cache[key]}", file=log, flush=True)
            for i, t in tiles_cache[key].items():
                ctx.set_tile(i, *t)
        if warmup > 0:
            loop.reset()
            loop.run(warmup, log=log)
        recs = []
        t_all = 0.0
        left = steps
        while left > 0:
            loop.reset()
            torch.cuda.synchronize()
            n = min(left, cfg.outer_steps)
            t0 = time.perf_counter()
            recs += loop.run(n, log=log)
            torch.cuda.synchronize()
            t_all += time.perf_counter() - t0
            left -= n
        out = summarize(recs, cfg.outer_steps)
        out["ms_per_timed_step"] = t_all * 1e3 / steps
        return out, recs

    tiles_cache = {}
    cfg = synth.config(args.config)
    seq = rsr.SEQUENTIAL if cfg.mode == "sequential" else rsr.BATCHED
    head, head_recs = run_variant(cfg, "recycled", seq, args.steps, args.warmup, "recycled", tiles_cache)
    variants = {}
    if args.no_plain:
        pl = head
    else:
        pl = run_variant(cfg, "plain", rsr.SEQUENTIAL, args.steps, args.warmup, "plain per-shift", tiles_cache)[0]
        variants["plain_per_shift"] = pl
    if not args.no_variants and not args.no_plain:
        other = rsr.BATCHED if seq == rsr.SEQUENTIAL else rsr.SEQUENTIAL
        variants["recycled_" + ("batched" if other == rsr.BATCHED else "sequential")] = run_variant(
            cfg, "recycled", other, args.steps, args.warmup, "recycled other", tiles_cache)[0]
        variants["plain_batched"] = run_variant(cfg, "plain", rsr.BATCHED, args.steps, args.warmup, "plain batched",
                                                tiles_cache)[0]
        variants["plain_warm_start"] = run_variant(cfg, "warm", rsr.SEQUENTIAL, args.steps, args.warmup,
                                                   "warm start", tiles_cache)[0]
    for v in variants.values():
        v["speedup_of_recycled_headline"] = v["ms_per_step"] / head["ms_per_step"]
    t_plain = pl["ms_per_step"]
    for name, v in list(variants.items()) + [("recycled_headline", head)]:
        v["speedup_vs_plain_per_shift"] = t_plain / v["ms_per_step"]

    if cfg.problems[0].ct is None:
        roof = roofline(cfg, head_recs, seq == rsr.BATCHED, "sequential" if seq == rsr.SEQUENTIAL else "batched")
    else:   # no persistent CG kernel: the projector launches of the host-driven solvers dominate
        roof = None

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cfg, pl["matvecs_A_per_step"])

    # the paper's own inner solver: recycled MINRES against MINRES from zero, in
    # the unit the paper counts (matrix-vector products per outer step)
    minres = None
    if not args.no_minres:
        mr = run_variant(cfg, "recycled", rsr.BATCHED, args.steps, args.warmup, "recycled MINRES", tiles_cache,
                         solver="minres")[0]
        mp = run_variant(cfg, "plain", rsr.BATCHED, args.steps, args.warmup, "plain MINRES", tiles_cache,
                         solver="minres")[0]
        minres = {"recycled_batched": mr, "plain_batched": mp,
                  "matvec_ratio_plain_over_recycled": mp["matvecs_A_per_step"] / mr["matvecs_A_per_step"],
                  "speedup_vs_plain_minres": mp["ms_per_step"] / mr["ms_per_step"]}

    large = {}
    if not args.no_large:
        names = args.large_only.split(",") if args.large_only else ["C3", "C4"]
        for nm in names:
            large[nm] = large_block(nm, run_variant, tiles_cache, args, synth, rsr, log)

    out = {
        "metric": METRIC,
        "value": round(head["ms_per_step"], 4),
        "unit": "ms/outer-step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_timed_step"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded rectangle phantom, Gaussian PSF, 1% noise)",
        "config": {"workload": f"{cfg.name}: {desc_problems(cfg)}, {len(cfg.gammas)} shifts 1e-5..1e1, "
                               f"p={cfg.p}, q={cfg.q}, {cfg.outer_steps} outer steps, "
                               f"{'one shift at a time' if seq == rsr.SEQUENTIAL else 'all shifts batched'}, "
                               f"tol={cfg.tol}",
                   "outer_steps_per_loop": cfg.outer_steps, "parallelism": "single GPU"},
        "recycled": head,
        "variants": variants,
        "speedup_vs_plain_per_shift": t_plain / head["ms_per_step"],
        "matvec_ratio_plain_over_recycled": pl["matvecs_A_per_step"] / head["matvecs_A_per_step"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "minres": minres,
        "large": large,
        "paper_context": "paper reports matvec savings 'on the order of 10,000' (MINRES, tol 1e-6, MATLAB); no timings",
    }
    print(json.dumps(out))
    ctx.close()


def large_block(name, run_variant, tiles_cache, args, synth, rsr, log):
    """One run of the configured loop per variant on a large workload, with its roofline."""
    cfg = synth.config(name)
    steps = cfg.outer_steps
    rec, recs = run_variant(cfg, "recycled", rsr.BATCHED, steps, 0, "recycled batched", tiles_cache)
    vs = {"plain_per_shift": run_variant(cfg, "plain", rsr.SEQUENTIAL, steps, 0, "plain per-shift", tiles_cache)[0]}
    if not args.no_variants:
        vs["plain_batched"] = run_variant(cfg, "plain", rsr.BATCHED, steps, 0, "plain batched", tiles_cache)[0]
        vs["plain_warm_start"] = run_variant(cfg, "warm", rsr.SEQUENTIAL, steps, 0, "warm start", tiles_cache)[0]
    for v in vs.values():
        v["speedup_of_recycled"] = v["ms_per_step"] / rec["ms_per_step"]
    out = {"workload": f"{cfg.name}: {desc_problems(cfg)}, {len(cfg.gammas)} shifts, p={cfg.p}, "
                       f"{cfg.outer_steps} outer steps, all shifts{' and instances' if len(cfg.problems) > 1 else ''}"
                       f" batched, tol={cfg.tol}",
           "recycled_batched": rec, "variants": vs,
           "speedup_vs_plain_per_shift": vs["plain_per_shift"]["ms_per_step"] / rec["ms_per_step"],
           "roofline": roofline(cfg, recs, True, "batched")}
    if not args.no_cpu:
        out["cpu_oracle_sample"] = oracle_rate_sample(cfg)
    if log:
        print(f"[{name}] {json.dumps(out)[:400]}", file=log, flush=True)
    return out


def oracle_rate_sample(cfg, iters: int = 4):
    """Oracle seconds per matvec on outer step 0, shifts 1, ceil(M/2) and M of the
    first instance, `iters` CG iterations each (one thread per shift)."""
    import oracle
    L = oracle.native_lib()
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    wh, wv = oracle.unit_weights(pr.ny, pr.nx)
    M = len(cfg.gammas)
    g = [cfg.gammas[0], cfg.gammas[(M + 1) // 2 - 1], cfg.gammas[M - 1]]
    t0 = time.perf_counter()
    _, st = oracle.cg_shifts(pr.psf, wh, wv, g, b, tol=cfg.tol, maxit=iters, nthreads=len(g), L=L)
    dt = time.perf_counter() - t0
    mv = sum(s["matvecs"] for s in st)
    return {"s_per_matvec_per_thread": dt * len(g) / mv, "matvecs": mv, "threads": len(g), "seconds": dt,
            "instance": f"{pr.ny}x{pr.nx}, PSF {pr.psf.shape[0]}x{pr.psf.shape[1]}"}


def cpu_baseline(cfg, plain_matvecs_per_step: float, budget_s: float = 8.0):
    """The oracle (plain C CG, direct-loop operators, built -O3 -march=native on
    this host) timed on outer step 0 of the workload: all shifts, each capped
    at the same iteration count, once single-threaded and once with OpenMP over
    shifts on the host's allotted cores.  The per-step time is extrapolated as
    the plain-CG matvecs per step measured on the GPU / the oracle's matvec rate."""
    import oracle
    L = oracle.native_lib()
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    wh, wv = oracle.unit_weights(pr.ny, pr.nx)
    M = len(cfg.gammas)
    cores = host_cores()
    # size the cap so that the single-threaded leg takes about budget_s
    t0 = time.perf_counter()
    _, st = oracle.cg_shifts(pr.psf, wh, wv, cfg.gammas[:1], b, tol=cfg.tol, maxit=2, nthreads=1, L=L)
    per_mv = (time.perf_counter() - t0) / max(1, st[0]["matvecs"])
    cap = max(2, int(budget_s / per_mv / M))
    legs = {}
    for threads in (1, cores):
        t0 = time.perf_counter()
        _, st = oracle.cg_shifts(pr.psf, wh, wv, cfg.gammas, b, tol=cfg.tol, maxit=cap, nthreads=threads, L=L)
        dt = time.perf_counter() - t0
        mv = sum(s["matvecs"] for s in st)
        legs[threads] = (mv / dt, mv, dt)
    rate, mv, dt = legs[cores]
    rate1, mv1, dt1 = legs[1]
    return {"value": plain_matvecs_per_step / rate * 1e3, "unit": "ms/outer-step (extrapolated)", "cores": cores,
            "kind": "oracle",
            "sample": (f"outer step 0, all {M} shifts, plain CG capped at {cap} iterations each, oracle built "
                       f"-O3 -march=native on this host: {mv} matvecs in {dt:.2f} s on {cores} threads "
                       f"(OpenMP over shifts), {mv1} in {dt1:.2f} s on 1 thread; per-step time = plain-CG "
                       f"matvecs per step measured on the GPU / the oracle's matvec rate"),
            "single_thread_value": plain_matvecs_per_step / rate1 * 1e3,
            "matvecs_per_s": rate, "matvecs_per_s_single_thread": rate1,
            "host": host_cpu()}


if __name__ == "__main__":
    main()
