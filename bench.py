#!/usr/bin/env python3
"""Throughput of the EPR iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch64]

A step is one complete solve (all iterations) of the workload's synthetic projections, with the
inputs resident in device memory.  Workloads:

  batch64              64 non-local polychromatic problems (8 lines, 30 iterations): 24 x 1024^2,
                       32 x 2048^2, 8 x 2160x2560, per-problem distance 5-20 m.  The timed solver
                       is the batched one (one launch per stage for all problems, the whole
                       iteration loop replayed from a HIP graph); the plain solver (one
                       projection per launch sequence, no graph) is timed beside it.
  nonlocal-poly8-2048  one 2048^2 projection, 8 lines, 30 iterations (plain solver)
  nonlocal-mono-2048   one 2048^2 projection, 1 line, 30 iterations (plain solver)
  local-mono-256       one 256^2 projection, local second-order closure, 20 iterations

value = 2048^2-equivalent projections per second (total pixels / 2048^2 / seconds per step),
timed over exactly K steps of the solver as a user runs it: the batched solver replays its
cached HIP graph, the plain solver replays one cached graph per projection, with stage timing
off.  A separate pass of E steps (--eager-steps) enqueues the identical launch sequence
directly, with HIP events recorded on the launch stream around every stage launch: it gives
the stage shares and the roofline of the dominant kernel (algorithmic bytes per launch over
its average duration).  The FP64 CPU oracle is timed on a bounded sample of the same work,
on one core and on several worker processes, before the GPU is touched.
"""

import argparse
import hashlib
import json
import os
import platform
import sys
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2048² projections/s to 1e-4 rel. phase err, batched vs plain; % HBM peak"
UNIT = "2048^2 projections/s"
HBM_PEAK_GBS = 8000.0
STAGES = ("maxgrad", "splat", "local", "rowfft", "colfft", "rowinv", "vjp", "binsplit")
KERNEL_SOURCE = {"maxgrad": "k_transport.hip", "splat": "k_transport.hip",
                 "local": "k_local.hip", "rowfft": "k_spectral.hip",
                 "colfft": "k_spectral.hip", "rowinv": "k_spectral.hip", "vjp": "k_vjp.hip",
                 "binsplit": "k_transport.hip"}


def stage_bytes(stage, ny, nx, L, f=1):
    """Algorithmic HBM bytes of one problem's share of a stage launch (float32 / complex64):
    every array the stage must read or write, once; halo re-reads are not counted.  ny x nx is
    the detector; with oversampling f the stages work on the (f ny) x (f nx) internal grid, the
    splat / closure write every line's prediction and the bin-split stage forms the residual."""
    P = ny * nx * f * f
    H = f * ny * (f * nx // 2 + 1)  # half-spectrum bins per line
    pred = 4 * P + 4 * L * P if f > 1 else 8 * P + 4 * L * P
    return {
        "maxgrad": 4 * P,                       # read tau
        "splat": pred,                          # read tau (and d); write e_s or P_s
        "local": pred,
        "rowfft": 4 * P + 4 * L * P + 8 * L * H,  # read tau, e_s; write spectra
        "colfft": 16 * L * H,                   # read + write spectra
        "rowinv": 8 * L * H + 8 * P,            # read spectra, tau; write tau
        "vjp": 0,
        "binsplit": 8 * L * P + 4 * ny * nx,    # read P_s, write e_s, read d
    }[stage]


def _phantom(w):
    """Seeded true object of one workload (phase and absorption at the reference)."""
    obj = w.true_object()
    return obj["phase"], obj["absorb"]


def build_problems(wls, ctx, torch, threads, f=1):
    """Synthetic data on the device: phantoms on the CPU (threads of this one process, so a
    profiler sees a single process), forward model + Poisson noise on the GPU."""
    from paper_2601_22793_amd import Geometry, Material, Spectrum
    if len(wls) > 1 and threads > 1:
        with ThreadPoolExecutor(threads) as ex:
            objs = list(ex.map(_phantom, wls))
    else:
        objs = [_phantom(w) for w in wls]
    probs = []
    gen = torch.Generator(device="cuda")
    for w, (ph, ab) in zip(wls, objs):
        geom = Geometry(w.ny, w.nx, w.pixel_m, w.distance_m)
        spec = Spectrum(list(map(float, w.energies_kev)), list(map(float, w.weights)),
                        w.energy_ref_kev, w.delta_exponent, w.beta_exponent)
        mat = Material(w.delta_ref, w.beta_ref)
        phase = torch.from_numpy(ph).cuda()
        absorb = torch.from_numpy(ab).cuda()
        model = "nonlocal" if w.model == "nonlocal" else w.model
        clean = ctx.forward(phase, absorb, geom, spec, model)
        if w.photons:
            gen.manual_seed(w.seed + 500)
            d = torch.poisson(clean.clamp_min(0) * w.photons, generator=gen) / w.photons
        else:
            d = clean
        tau = torch.zeros((w.ny * f, w.nx * f), dtype=torch.float32, device=d.device)
        probs.append((d.contiguous(), tau, geom, spec, mat))
        del phase, absorb, clean
    torch.cuda.synchronize()
    return probs


def size_class(ny, nx):
    """Size class of a problem: 0 up to 2048 x 2048 pixels (512-thread spectral kernels),
    1 beyond (1024 threads).  A batched solve launches each stage once per class."""
    return 0 if (ny <= 2048 and nx <= 2048) else 1


def kernel_instance(stage, cls, batched, n_lines, row_lines):
    """Name of the kernel template instance a (stage, size class) launch runs, as rocprofv3
    lists it (without the namespace).  row_lines: lines per row-pass workgroup."""
    b = "true" if batched else "false"
    if stage == "rowfft":
        return f"k_rowfft<{b}, {512 if cls == 0 else 1024}, {row_lines}>"
    if stage in ("rowfft", "colfft", "rowinv"):
        return f"k_{stage}<{b}, {512 if cls == 0 else 1024}>"
    if stage == "splat":
        nl = next(v for v in (1, 2, 4, 8, 16) if v >= n_lines)
        return f"k_splat<{b}, {nl}>"
    return f"k_{stage}<{b}>"


def source_digest(stage):
    """SHA-256 of the kernel's translation unit and the device headers it includes."""
    csrc = os.path.join(ROOT, "paper_2601_22793_amd", "csrc")
    h = hashlib.sha256()
    for f in (KERNEL_SOURCE[stage], "dev_common.h", "epr_internal.h", "fft_lds.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def counters_for(kernel, stage, workload):
    """Committed rocprofv3 counter record of a kernel instance (profiles/traffic_<workload>.json:
    HBM bytes and VALU wave instructions per launch), if it was taken with the current kernel
    sources; else an empty dict."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return {}
    rec = json.load(open(path)).get("kernels", {}).get(kernel)
    if not rec or rec.get("source_sha256") != source_digest(stage):
        return {}
    return rec


# Vector issue capacity: 256 CUs x 4 SIMDs, one wave64 FP32 instruction per SIMD every 4
# cycles (16 lanes), at 2.4 GHz.
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4


def _oracle_case(w, f=1):
    """Oracle inputs of one workload: line constants (internal grid) and the noisy data."""
    from oracle import epr_oracle as O
    obj = w.true_object()
    L = O.line_constants(w.energies_kev, w.weights, w.pixel_m, w.distance_m, w.delta_ref,
                         w.beta_ref, w.energy_ref_kev, w.delta_exponent, w.beta_exponent)
    d = w.add_noise(O.forward(obj["phase"], obj["absorb"], L, w.model))
    Li = O.line_constants(w.energies_kev, w.weights, w.pixel_m / f, w.distance_m, w.delta_ref,
                          w.beta_ref, w.energy_ref_kev, w.delta_exponent, w.beta_exponent)
    return d, Li


def _oracle_iteration_seconds(w, f=1, warm=True):
    """Seconds of one oracle iteration (from tau = 0) of workload w, after a warm-up call."""
    import numpy as np
    from oracle import epr_oracle as O
    d, Li = _oracle_case(w, f)
    tau = np.zeros((w.ny * f, w.nx * f), dtype=np.float64)
    if warm:
        O.iterate(tau, d, Li, w.model, w.relaxation, oversample=f)  # first-touch costs
    t0 = time.perf_counter()
    O.iterate(tau, d, Li, w.model, w.relaxation, oversample=f)
    return time.perf_counter() - t0


def _worker_iteration(w, barrier, results, idx):
    """Worker process (numpy only, never the GPU): set up one oracle case, wait for every
    worker, then time one oracle iteration; puts (idx, start, end) wall-clock times."""
    import numpy as np
    from oracle import epr_oracle as O
    d, Li = _oracle_case(w)
    tau = np.zeros((w.ny, w.nx), dtype=np.float64)
    barrier.wait()
    t0 = time.time()
    O.iterate(tau, d, Li, w.model, w.relaxation)
    results.put((idx, t0, time.time()))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wls, n_iter, f=1, workers=16):
    """FP64 oracle on a bounded sample of the workload, scaled to 2048^2-equivalent projections
    per second at the full iteration count.

    Per core: one oracle iteration of one projection (a 2048 x 2048 one when the workload has
    it) in this process.  All cores: `workers` processes (numpy only; started before the GPU
    is touched) each time one oracle iteration of a different projection of the workload's
    smallest size, all at once; the throughput is their pixels over the wall time.  The
    oracle's FFT is single-threaded, so one process uses one core."""
    sample_w = next((w for w in wls if w.ny == 2048), wls[0])
    dt1 = _oracle_iteration_seconds(sample_w, f)
    per_core = sample_w.ny * sample_w.nx / 2048.0 ** 2 / (dt1 * n_iter)
    out = {"value": per_core, "unit": UNIT, "cores": 1, "kind": "oracle",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
           "per_core_value": per_core,
           "sample": f"1 iteration of one {sample_w.ny}x{sample_w.nx} projection with "
                     f"{sample_w.n_lines} line(s), model {sample_w.model}, oversampling {f}, FP64 "
                     f"numpy on 1 core ({dt1:.2f} s per iteration), scaled to {n_iter} iterations"}
    avail = out["affinity"] or out["nproc"] or 1
    k = min(workers, avail, len(wls))
    if k > 1 and f == 1:
        import multiprocessing as mp
        smallest = min(w.ny * w.nx for w in wls)
        picks = [w for w in wls if w.ny * w.nx == smallest][:k]
        k = len(picks)
        env = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                               "MKL_NUM_THREADS")}
        for v in env:
            os.environ[v] = "1"
        try:
            ctx = mp.get_context("spawn")
            barrier, results = ctx.Barrier(k), ctx.Queue()
            procs = [ctx.Process(target=_worker_iteration, args=(w, barrier, results, i))
                     for i, w in enumerate(picks)]
            for pr in procs:
                pr.start()
            spans = [results.get(timeout=600) for _ in procs]
            for pr in procs:
                pr.join()
        finally:
            for v, val in env.items():
                if val is None:
                    os.environ.pop(v, None)
                else:
                    os.environ[v] = val
        wall = max(sp[2] for sp in spans) - min(sp[1] for sp in spans)
        secs = [sp[2] - sp[1] for sp in spans]
        eq = sum(w.ny * w.nx for w in picks) / 2048.0 ** 2
        all_core = eq / (wall * n_iter)
        out.update(value=all_core, cores=k, all_core_value=all_core,
                   sample=out["sample"] + f"; all cores: {k} worker processes, each one "
                   f"iteration of a different {picks[0].ny}x{picks[0].nx} projection "
                   f"(setup excluded; {min(secs):.2f}-{max(secs):.2f} s each, {wall:.2f} s wall), "
                   f"scaled to {n_iter} iterations")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eager-steps", type=int, default=2,
                    help="steps of the event-timed pass (stage shares, roofline)")
    ap.add_argument("--plain-steps", type=int, default=3, help="batch64: plain solver samples")
    ap.add_argument("--workload", default="batch64",
                    choices=["batch64", "nonlocal-poly8-2048", "nonlocal-mono-2048",
                             "local-mono-256"])
    ap.add_argument("--no-plain", action="store_true", help="batch64: skip the plain solver")
    ap.add_argument("--oversample", type=int, default=1, choices=[1, 2, 4],
                    help="single-projection workloads: internal grid factor (detector-level "
                         "residual, thickness on the internal grid)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (use under a profiler: it starts processes)")
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch choices (no autotuner before timing)")
    ap.add_argument("--tune-cache", default=None, metavar="PATH",
                    help="autotuner cache (JSON): used if valid, else written")
    ap.add_argument("--splat-tile", default=None, metavar="TXxTY",
                    help="use this splat tile shape (e.g. 64x32) and skip the autotuner")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (calibrates HBM "
                         "counters under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the projections "
              "are independent and would shard across GPUs without communication.",
              file=sys.stderr)
        sys.exit(2)

    from synthetic import batch_workloads, workload
    if args.workload == "batch64":
        wls = batch_workloads()
    else:
        wls = [workload(args.workload)]
    w0 = wls[0]
    model, n_iter, relax = w0.model, w0.n_iter, w0.relaxation
    f = args.oversample
    if f > 1 and args.workload == "batch64":
        print("--oversample applies to the single-projection workloads", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the worker processes only ever load numpy
        t_cpu = time.perf_counter()
        cpu = cpu_baseline(wls, n_iter, f=f, workers=args.cpu_workers)
        print(f"# cpu baseline {time.perf_counter() - t_cpu:.1f} s", file=sys.stderr, flush=True)

    import torch
    from paper_2601_22793_amd import Context

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    ctx = Context.get(0)
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_setup = time.perf_counter()
    probs = build_problems(wls, ctx, torch, min(16, os.cpu_count() or 1), f)
    print(f"# setup {time.perf_counter() - t_setup:.1f} s, {len(probs)} problem(s)",
          file=sys.stderr, flush=True)
    tuned = None
    if args.splat_tile:
        tx, ty = (int(v) for v in args.splat_tile.lower().split("x"))
        # a cached tuning result pins the shape without timing anything
        with tempfile.TemporaryDirectory() as tmp:
            path = os.path.join(tmp, "splat_tile.json")
            with open(path, "w") as fh:
                json.dump({"splat_tx": tx, "splat_ty": ty}, fh)
            tuned = ctx.autotune(probs[:1], model, cache_json=path)
    elif not args.no_autotune:
        # the autotuner (splat tile on a warm state, radix order per transform length), timed
        # on the workload's own problems before the timed region
        t_tune = time.perf_counter()
        if args.tune_cache:
            tuned = ctx.autotune(probs, model, relaxation=relax, cache_json=args.tune_cache,
                                 oversample=f)
        else:
            with tempfile.TemporaryDirectory() as tmp:
                tuned = ctx.autotune(probs, model, relaxation=relax,
                                     cache_json=os.path.join(tmp, "tune.json"), oversample=f)
        print(f"# autotune {time.perf_counter() - t_tune:.1f} s: {tuned}", file=sys.stderr,
              flush=True)
    total_px = sum(p[2].ny * p[2].nx for p in probs)
    eq = total_px / 2048.0 ** 2
    L = w0.n_lines
    batched = args.workload == "batch64"

    def step_plain():
        for d, tau, geom, spec, mat in probs:
            tau.zero_()
            ctx.solve(d, geom, spec, mat, model, n_iter, relax, thickness=tau, oversample=f)

    def step_batched():
        for p in probs:
            p[1].zero_()
        ctx.solve_batched(probs, model, n_iter, relax)

    step = step_batched if batched else step_plain

    def timed(fn, k, w):
        """k steps after w warm-up steps, timing off (graphs replayed): (mean seconds per
        step over the whole bracket, per-step seconds from events on the current stream)."""
        ctx.set_timing(False)
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        t0 = time.perf_counter()
        ev[0].record()
        for i in range(k):
            fn()
            ev[i + 1].record()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        per = [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(k)]
        return dt, per

    def eager(fn, k):
        """k steps with stage timing on: the same launches enqueued directly, with events."""
        fn()
        torch.cuda.synchronize()
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        tim, tim_cls = ctx.timing(), ctx.timing(by_class=True)
        ctx.set_timing(False)
        return dt, tim, tim_cls

    plain = None
    if batched and not args.no_plain:
        plain = timed(step_plain, args.plain_steps, 1)
    dt, per_step = timed(step, args.steps, args.warmup)
    value = eq / dt
    eager_dt, tim, tim_cls = eager(step, max(args.eager_steps, 1))

    # roofline of the dominant kernel: the (stage, size class) launch with the most time in the
    # event-timed pass.  One such launch covers every problem of that class (batched) or the
    # one problem (plain).
    stage_ms = {s: tim[s][0] for s in STAGES}
    dom, cls = max(tim_cls, key=lambda k: tim_cls[k][0])
    ms_total, launches = tim_cls[(dom, cls)]
    members = [p for p in probs if size_class(p[2].ny * f, p[2].nx * f) == cls]
    per_launch_bytes = sum(stage_bytes(dom, p[2].ny, p[2].nx, L, f) for p in members)
    if not batched:
        per_launch_bytes = stage_bytes(dom, members[0][2].ny, members[0][2].nx, L, f)
    avg_s = ms_total / 1e3 / max(launches, 1)
    achieved = per_launch_bytes / avg_s / 1e9
    # (the library's default is two lines per row-pass workgroup when nothing was tuned)
    kname = kernel_instance(dom, cls, batched, L, (tuned or {}).get("row_lines", 2))
    ctr = counters_for(kname, dom, args.workload if f == 1 else f"{args.workload}-os{f}")
    valu = ctr.get("valu_insts_per_launch")
    roof = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": ctr.get("bytes_per_launch"),
            # what limits it instead: the share of the vector-issue capacity its counted
            # VALU instructions take over the measured duration
            "valu_insts_per_launch": valu,
            "valu_issue_frac": round(valu / avg_s / VALU_ISSUE_PEAK, 4) if valu else None,
            "avg_launch_ms": round(avg_s * 1e3, 4), "launches": int(launches),
            "problems_per_launch": len(members) if batched else 1,
            "algorithmic_bytes_per_launch": int(per_launch_bytes),
            "timed_in": "event-timed pass of the same launch sequence (eager)"}
    stage_share = {s: round(v / max(sum(stage_ms.values()), 1e-12), 4)
                   for s, v in stage_ms.items() if v > 0}
    stages = (("maxgrad", "splat") if model == "nonlocal" else ("local",))
    stages += (("binsplit",) if f > 1 else ()) + ("rowfft", "colfft", "rowinv")
    alg_iter = sum(stage_bytes(s, p[2].ny, p[2].nx, L, f) for p in probs for s in stages)
    whole = alg_iter * n_iter / dt / 1e9
    per_sorted = sorted(per_step)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "problems": len(probs), "lines": L,
                   "iterations": n_iter, "model": model, "relaxation": relax,
                   "pixels": total_px,
                   "solver": "batched, HIP graph replay" if batched
                             else "plain, HIP graph replay per projection",
                   "tuned": tuned, "oversample": f},
        "roofline": roof,
        "median_ms_per_step": round(per_sorted[len(per_sorted) // 2] * 1e3, 3),
        "eager_ms_per_step": round(eager_dt * 1e3, 3),
        "stage_time_share": stage_share,
        "whole_iteration_GBps": round(whole, 1),
        "whole_iteration_hbm_frac": round(whole / HBM_PEAK_GBS, 4),
    }
    if plain is not None:
        out["plain_value"] = round(eq / plain[0], 3)
        out["plain_steps"] = args.plain_steps
        out["batched_over_plain"] = round(plain[0] / dt, 3)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
