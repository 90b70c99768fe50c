"""Throughput of the staggered-grid pressure Poisson solve on one MI355X.

Workload: 512 x 384 x 512 cells, x and z periodic (Lx = Lz = 2 pi), y on
[-1, 1] with tanh stretching beta = 2 and Neumann walls; right-hand side =
discrete divergence (computed by the library's divergence kernel) of a seeded
staggered velocity field whose components have a k^-5/3 spectrum up to k = 64
(inputs resident in HBM before timing).  One step = one complete solve.

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed|mixed_f64sweep]

Prints one JSON line.  `value` is FP64 solves/s (the direct solve); the mixed
forms (FP32 transforms and line solves wrapped in FP64 iterative refinement
to a 1e-10 relative residual) are timed beside it on the same input and
reported under "mixed".  The roofline entry is the dominant kernel of the
FP64 solve, its duration taken from HIP events recorded around every launch
over a second timed region of the same number of steps (the first, which
gives `value`, records no per-launch events).
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Poisson solves/s + HBM GB/s at 512x384x512, mixed vs FP64 at 1e-10 resid"
HBM_PEAK_GBS = 8000.0
SOURCES = ["ibp_api.cpp", "ibp_host.cpp", "ibp_host.hpp", "ibp_xz.hip", "ibp_xz_narrow.hip", "ibp_xz_kernels.hpp", "ibp_fastxz.hip", "ibp_ytri.hip",
           "ibp_ytri_body.hpp", "ibp_misc.hip", "ibp_lines.hip", "ibp_persist.hip", "ibp_bluereg.hip", "ibp_device.hpp",
           "ibp_internal.hpp", "ibp_regfft.hpp"]


def source_hash():
    h = hashlib.sha256()
    for name in SOURCES:
        with open(os.path.join(ROOT, "paper_2609_19130_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_solves(plan, f, phi, steps, warmup, profile=True):
    import torch
    for _ in range(warmup):
        plan.solve(f, phi)
    torch.cuda.synchronize()
    plan.set_profiling(profile)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        plan.solve(f, phi)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile() if profile else {}
    plan.set_profiling(False)
    return start.elapsed_time(stop) / steps, wall, prof


def traffic_for(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, when they
    were taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def copy_gbs(n_doubles):
    """Device copy bandwidth (read + write) of an FP64 array half the dominant
    kernel's bytes, measured live with torch's copy: the practical HBM ceiling
    next to the 8 TB/s peak."""
    import torch
    a = torch.ones(n_doubles, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    del a, b
    return 2.0 * n_doubles * 8 / (ms * 1e-3) / 1e9


def cpu_threads():
    """Host threads this process may use: the CPU affinity set, capped at the
    share of one GPU's host (16 threads)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if env > 0:
        n = min(n, env)
    return max(1, min(n, 16))


def cpu_baseline(args, keep=None, uvw=None):
    """The oracle as it stands, on the host cores, on full solves of the same
    workload: numpy FFTs (one thread) and scipy.fft with `workers` threads
    (the FFT steps only; the Thomas sweep is single-threaded numpy in both).
    `keep`, if a dict, receives the oracle's solution of the full workload
    (`phi`) for the GPU forms' error against it."""
    import numpy as np

    import oracle
    from oracle.grid import geometry
    from oracle.operators import divergence
    from paper_2609_19130_amd import synth

    nx, ny, nz = args.nx, args.ny, args.nz
    if args.cpu_sample == "quarter":
        nx, nz = nx // 2, nz // 2
    yf = synth.tanh_faces(ny, args.beta)
    g = geometry(nx, ny, nz, 2 * np.pi, 2 * np.pi, yf)
    if uvw is not None and args.cpu_sample == "full":
        u, v, w = uvw
    else:
        u, v, w = synth.kolmogorov_velocity(nx, ny, nz, seed=3, kmax=64)
    f = divergence(u, v, w, g)
    del u, v, w
    threads = cpu_threads()

    def timed(workers):
        times = []
        phi = None
        while len(times) < 3 and sum(times) < 30.0:
            t0 = time.perf_counter()
            phi, _ = oracle.solve(f, 2 * np.pi, 2 * np.pi, yf, workers=workers)
            times.append(time.perf_counter() - t0)
        return float(np.median(times)), len(times), phi

    dt, n1, phi = timed(None)
    dtm, nm, _ = timed(threads)
    if keep is not None and args.cpu_sample == "full":
        keep["phi"] = phi
        keep["f"] = f
    scale = (nx * ny * nz) / float(args.nx * args.ny * args.nz)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    import scipy
    return {"value": scale / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host": {"cpu": cpu, "logical_cpus": os.cpu_count(), "numpy": np.__version__,
                     "scipy": scipy.__version__},
            "sample": f"median of {n1} full oracle solves at {nx}x{ny}x{nz}: {dt:.2f} s each (numpy FFTs, 1 thread)"
                      + ("" if scale == 1.0 else f"; rate scaled by the cell ratio {scale:.3f}"),
            "threaded": {"value": scale / dtm, "unit": "solves/s", "cores": threads,
                         "sample": f"median of {nm} full oracle solves: {dtm:.2f} s each (scipy.fft with "
                                   f"workers={threads}; the Thomas sweep stays one thread)"}}


def run_c4(args):
    """64 uneven grids (each dimension in {32, 48, ..., 192}, beta in [1.5, 3],
    divergence of a uniform random velocity as right-hand side): one batched
    solve of all grids (one launch per stage) against the loop of per-grid
    solves, FP64 and mixed.  A step solves all 64 grids."""
    import numpy as np
    import torch

    from paper_2609_19130_amd import ibpoisson as ibp
    from paper_2609_19130_amd import synth

    grids = synth.batch_grids(seed=4, count=64)
    rhs, yfs = [], []
    for gd in grids:
        nx, ny, nz = gd["nx"], gd["ny"], gd["nz"]
        yf = synth.tanh_faces(ny, gd["beta"])
        u, v, w = synth.uniform_velocity(nx, ny, nz, seed=gd["seed"])
        yfs.append(yf)
        rhs.append((u, v, w))
    cells = sum(gd["nx"] * gd["ny"] * gd["nz"] for gd in grids)
    out = {"metric": METRIC, "unit": "grid solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic: divergence of i.i.d. U[-1,1] staggered velocity per grid",
           "config": {"workload": "poisson_batch64_dims32to192_seed4", "grids": len(grids), "cells": cells}}
    for form in [s for s in args.forms.split(",") if s in ("fp64", "mixed")]:
        plans = [ibp.Plan(gd["nx"], gd["ny"], gd["nz"], gd["Lx"], gd["Lz"], yf, precision=form,
                          max_iters=args.mixed_iters) for gd, yf in zip(grids, yfs)]
        fs = [p.divergence(*(torch.from_numpy(a).cuda() for a in uvw)) for p, uvw in zip(plans, rhs)]
        phis = [torch.empty_like(f) for f in fs]

        def loop():
            for p, f, q in zip(plans, fs, phis):
                p.solve(f, q)

        def batched():
            ibp.solve_batched(plans, fs, phis)

        staged_b = ibp.Batch(plans)
        staged_b.set_persistent(False)
        persist_b = ibp.Batch(plans)
        try:
            persist_b.set_persistent(True)
            has_persist = True
        except ibp.IbpError:
            has_persist = False

        def staged():
            staged_b.solve(fs, phis)

        def persistent():
            persist_b.solve(fs, phis)

        batch = ibp.Batch(plans)
        tune = batch.autotune(fs, phis)
        log(f"[bench c4] {form} autotuned batch: {tune}")

        def tuned():
            batch.solve(fs, phis)

        res = {"autotune": tune}
        variants = [("per_grid_loop", loop), ("batched", batched), ("batched_staged", staged)]
        if has_persist:
            variants.append(("batched_persistent", persistent))
        variants.append(("batched_autotuned", tuned))
        for name, fn in variants:
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.steps
            res[name] = {"ms_per_step": ms, "grid_solves_per_s": 64 * 1000.0 / ms, "cells_per_s": cells * 1000.0 / ms}
            log(f"[bench c4] {form} {name}: {ms:.3f} ms for 64 grids")
        if form == "mixed":
            res["converged"] = int(sum(p.info()["converged"] for p in plans))
        res["batched_vs_loop"] = res["per_grid_loop"]["ms_per_step"] / res["batched"]["ms_per_step"]
        res["autotuned_vs_loop"] = res["per_grid_loop"]["ms_per_step"] / res["batched_autotuned"]["ms_per_step"]
        out[form] = res
        batch.close()
        staged_b.close()
        persist_b.close()
        for p in plans:
            p.close()
    if "fp64" in out:
        out["value"] = out["fp64"]["batched_autotuned"]["grid_solves_per_s"]
        out["ms_per_step"] = out["fp64"]["batched_autotuned"]["ms_per_step"]
    out["source_hash"] = source_hash()
    return out


def run_c5(args, steps=None):
    """One GPU's share at paper scale: 1024 x 768 x 1024 cells, beta = 3.  A
    bank of 4 right-hand sides (divergences of seeded k^-5/3 velocity fields,
    drawn on the GPU) feeds an AR(1) sequence f_{t+1} = 0.95 f_t +
    sqrt(1 - 0.95^2) s_t roll(bank[t mod 4]).  `--seq` steps of (solve,
    advance) are captured as one graph per form and replayed; the advance
    steps alone are captured and timed too, and their time is subtracted."""
    import numpy as np
    import torch

    from paper_2609_19130_amd import ibpoisson as ibp
    from paper_2609_19130_amd import synth

    nx, ny, nz, beta, seed, nbank = 1024, 768, 1024, 3.0, 5, 4
    steps = args.seq if steps is None else steps
    workload = f"poisson_{nx}x{ny}x{nz}_beta{beta:g}_ar1_kolmogorov_graph{steps}"
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(ny, beta)
    log(f"[bench c5] drawing a bank of {nbank} k^-5/3 velocity fields on the GPU")
    plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf)
    bank = []
    for b in range(nbank):
        u, v, w = synth.kolmogorov_velocity_device(nx, ny, nz, seed=1000 * seed + b)
        bank.append(plan.divergence(u, v, w))
        del u, v, w
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    sched = synth.ar1_schedule(seed, steps + 1, nx, nz, nbank)
    f0 = bank[0] * sched[0][3]
    f = torch.empty_like(f0)
    gbuf = torch.empty_like(f0)
    phi = torch.empty_like(f0)

    def capture(with_solve):
        g = torch.cuda.CUDAGraph()
        f.copy_(f0)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            for t in range(steps):
                if with_solve:
                    plan.solve(f, phi)
                synth.ar1_advance(f, gbuf, bank, sched[t + 1])
        return g

    def replay_ms(g, reps):
        times = []
        for _ in range(reps):
            f.copy_(f0)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            g.replay()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        return float(np.median(times))

    log("[bench c5] timing the AR(1) advance alone")
    g_adv = capture(False)
    g_adv.replay()
    adv_ms = replay_ms(g_adv, 3)
    del g_adv
    forms = [s for s in args.forms.split(",") if s in ("fp64", "mixed", "mixed_f64sweep", "mixed_f64inv")]
    res = {}
    finals = {}
    for form in forms:
        plan.set_precision(form, 1e-10, args.mixed_iters)
        plan.solve(f0, phi)
        torch.cuda.synchronize()
        log(f"[bench c5] {form}: capturing {steps} x (solve, advance)")
        g = capture(True)
        g.replay()                       # warm-up replay
        torch.cuda.synchronize()
        ms = replay_ms(g, 3)
        info = plan.info()
        finals[form] = phi.clone()
        res[form] = dict(seq_ms=ms, solve_ms=(ms - adv_ms) / steps, info=info)
        log(f"[bench c5] {form}: {ms:.1f} ms per sequence, {(ms - adv_ms) / steps:.3f} ms per solve, {info}")
        del g
    N = nx * ny * nz
    Nh = (nx // 2 + 1) * ny * nz
    stage_bytes = 16.0 * N + 8 * 16.0 * Nh
    r64 = res.get("fp64")
    out = {"metric": METRIC, "unit": "solves/s", "n_gpus": 1, "steps": steps, "warmup": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic: AR(1) blend (rho 0.95) of rolled, sign-flipped divergences of 4 seeded "
                   "k^-5/3 velocity fields drawn on the GPU",
           "config": {"workload": workload, "nx": nx, "ny": ny, "nz": nz, "beta": beta,
                      "form": "captured graph of (solve, AR(1) advance) steps; advance time subtracted"},
           "ar1_advance_ms_per_step": adv_ms / steps}
    if r64 is not None:
        out["value"] = 1000.0 / r64["solve_ms"]
        out["ms_per_step"] = r64["solve_ms"]
        out["hbm_gbs_stage_model"] = stage_bytes / (r64["solve_ms"] * 1e-3) / 1e9
        out["roofline_frac_stage_model"] = out["hbm_gbs_stage_model"] / HBM_PEAK_GBS
    mixed = {}
    for form in forms:
        if form == "fp64":
            continue
        r = res[form]
        d = None
        if "fp64" in finals:
            d = float(torch.linalg.vector_norm(finals[form] - finals["fp64"]) / torch.linalg.vector_norm(finals["fp64"]))
        mixed[form] = {"solves_per_s": 1000.0 / r["solve_ms"], "ms_per_step": r["solve_ms"],
                       "iterations_last": r["info"]["iterations"], "converged_last": r["info"]["converged"],
                       "rel_residual_last": r["info"]["rel_residual"], "rel_diff_vs_fp64_last": d,
                       "backward_error_last": r["info"]["backward_error"],
                       "residual_history_last": r["info"]["residual_history"],
                       "vs_fp64": (r64["solve_ms"] / r["solve_ms"]) if r64 else None}
    out["mixed"] = mixed
    out["source_hash"] = source_hash()
    return out


def run_paper_grids(args, steps=10, warmup=2):
    """FP64 solves on the paper's two scaling grids (501 x 501 x 1001 and
    632 x 632 x 1263 cells, stretched direction second): time per solve, the
    stage model's rate and the per-pass times.  Right-hand sides are seeded
    normal values (the direct solve's time does not depend on them)."""
    import numpy as np
    import torch

    from paper_2609_19130_amd import ibpoisson as ibp
    from paper_2609_19130_amd import synth

    out = {}
    for nx, ny, nz in ((501, 1001, 501), (632, 1263, 632)):
        yf = synth.tanh_faces(ny, args.beta)
        plan = ibp.Plan(nx, ny, nz, 2 * np.pi, 2 * np.pi, yf)
        g = torch.Generator(device="cuda")
        g.manual_seed(nx)
        f = torch.randn((ny, nz, nx), generator=g, device="cuda", dtype=torch.float64)
        phi = torch.empty_like(f)
        ms, _, _ = timed_solves(plan, f, phi, steps, warmup, False)
        _, _, prof = timed_solves(plan, f, phi, steps, 0, True)
        N = nx * ny * nz
        Nh = (nx // 2 + 1) * ny * nz
        model = 16.0 * N + 8 * 16.0 * Nh
        out[f"{nx}x{ny}x{nz}"] = {
            "ms_per_solve": ms, "solves_per_s": 1000.0 / ms,
            "hbm_gbs_stage_model": model / (ms * 1e-3) / 1e9,
            "roofline_frac_stage_model": model / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "passes_ms": {k: v["total_ms"] / v["launches"] for k, v in prof.items()}}
        log(f"[bench] paper grid {nx}x{ny}x{nz}: {ms:.2f} ms")
        del f, phi
        plan.close()
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=384)
    ap.add_argument("--nz", type=int, default=512)
    ap.add_argument("--beta", type=float, default=2.0)
    ap.add_argument("--mixed-iters", type=int, default=2,
                    help="refinement corrections allowed after the initial FP32 solve (each form reports how "
                         "many it took)")
    ap.add_argument("--forms", default="fp64,mixed,mixed_f64sweep,mixed_f64inv")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-substep", action="store_true", help="skip the fractional-step substep timing")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without the per-launch events (no per-pass breakdown or roofline)")
    ap.add_argument("--cpu-sample", choices=["full", "quarter"], default="full")
    ap.add_argument("--config", choices=["c3", "c4", "c5", "paper"], default="c3",
                    help="c3: the 512x384x512 solve (default, the headline line); "
                         "c5: a captured graph of --seq solves at 1024x768x1024, beta 3, AR(1) right-hand sides; "
                         "paper: FP64 solves on the 501x1001x501 and 632x1263x632 grids")
    ap.add_argument("--seq", type=int, default=100, help="solves per captured sequence (c5)")
    ap.add_argument("--no-extra", action="store_true",
                    help="c3 only: skip the batched, paper-scale and paper-grid summaries appended to the line")
    ap.add_argument("--extra-seq", type=int, default=20, help="solves per captured sequence of the c5 summary")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.config == "c5":
        print(json.dumps(run_c5(args)), flush=True)
        return
    if args.config == "c4":
        print(json.dumps(run_c4(args)), flush=True)
        return
    if args.config == "paper":
        print(json.dumps({"config": "paper_grids", "beta": args.beta, "unit": "ms per FP64 solve",
                          "grids": run_paper_grids(args, steps=args.steps, warmup=args.warmup)}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2609_19130_amd import ibpoisson as ibp
    from paper_2609_19130_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nx, ny, nz = args.nx, args.ny, args.nz
    workload = f"poisson_{nx}x{ny}x{nz}_beta{args.beta:g}_kolmogorov"
    Lx = Lz = 2 * np.pi
    yf = synth.tanh_faces(ny, args.beta)
    log(f"[bench] generating k^-5/3 velocity {nx}x{ny}x{nz}")
    t0 = time.perf_counter()
    u, v, w = synth.kolmogorov_velocity(nx, ny, nz, seed=3, kmax=64)
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s; uploading")
    plan = ibp.Plan(nx, ny, nz, Lx, Lz, yf)
    ud, vd, wd = (torch.from_numpy(a).cuda() for a in (u, v, w))
    host_uvw = (u, v, w) if not args.no_cpu_baseline else None   # the oracle leg's input
    del u, v, w
    f = plan.divergence(ud, vd, wd)
    phi = torch.empty_like(f)
    torch.cuda.synchronize()

    forms = [s for s in args.forms.split(",") if s]
    results = {}
    for form in forms:
        plan.set_precision(form, 1e-10, args.mixed_iters)
        log(f"[bench] timing {form}: {args.warmup} warmup + {args.steps} steps")
        ms, wall, _ = timed_solves(plan, f, phi, args.steps, args.warmup, False)
        info = plan.info()
        prof, ms_prof = {}, None
        if not args.no_profile:
            # the same steps again with HIP events around every launch (on the
            # stream the kernels run on) for the per-kernel durations
            log(f"[bench] {form}: per-launch events over {args.steps} more steps")
            ms_prof, _, prof = timed_solves(plan, f, phi, args.steps, 0, True)
        results[form] = dict(ms=ms, wall=wall, prof=prof, info=info, ms_prof=ms_prof)
        log(f"[bench] {form}: {ms:.3f} ms/solve, info {info}")

    substep = None
    if "fp64" in forms and not args.no_substep:
        # one fractional-step substep around the FP64 solve: right-hand side
        # from the velocity, solve, projection + pressure update
        plan.set_precision("fp64")
        adt = 0.01
        pr = torch.zeros_like(f)
        fbuf = torch.empty_like(f)

        def fused():
            plan.solve_divergence(ud, vd, wd, adt, phi=phi)
            plan.project(phi, adt, ud, vd, wd, p=pr)

        def unfused():
            plan.divergence(ud, vd, wd, fbuf)
            fbuf.mul_(1.0 / adt)
            plan.solve(fbuf, phi)
            plan.project(phi, adt, ud, vd, wd, p=pr)

        substep = {}
        for name, fn in (("fused_rhs", fused), ("separate_divergence", unfused)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            a0 = torch.cuda.Event(enable_timing=True)
            b0 = torch.cuda.Event(enable_timing=True)
            a0.record()
            for _ in range(args.steps):
                fn()
            b0.record()
            torch.cuda.synchronize()
            substep[name + "_ms"] = a0.elapsed_time(b0) / args.steps
        log(f"[bench] substep (rhs + solve + projection): {substep}")
        # implicit viscous step: factored line solves of the three velocity
        # components (eq. nstime_discr with Crank-Nicolson terms), beta =
        # alpha dt / (2 Re) = 1e-4; the cost does not depend on beta
        plan.helmholtz_set(1e-4)

        def viscous():
            plan.helmholtz(ud, "cells")
            plan.helmholtz(vd, "yfaces")
            plan.helmholtz(wd, "cells")

        for _ in range(2):
            viscous()
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        b0 = torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(args.steps):
            viscous()
        b0.record()
        torch.cuda.synchronize()
        substep["viscous_uvw_ms"] = a0.elapsed_time(b0) / args.steps
        plan.set_profiling(True)
        for _ in range(args.steps):
            viscous()
        vprof = plan.profile()
        plan.set_profiling(False)
        substep["viscous_passes"] = {
            k: {"avg_ms": v["total_ms"] / v["launches"], "launches": v["launches"],
                "gbs": v["bytes_per_launch"] / (v["total_ms"] / v["launches"] * 1e-3) / 1e9}
            for k, v in vprof.items()}
        log(f"[bench] viscous u, v, w: {substep['viscous_uvw_ms']:.3f} ms, passes {substep['viscous_passes']}")
    del ud, vd, wd

    N = nx * ny * nz
    Nh = (nx // 2 + 1) * ny * nz
    stage_bytes = 16.0 * N + 8 * 16.0 * Nh      # five passes, each a full read + write (FP64)
    r64 = results.get("fp64")
    out = {"metric": METRIC, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic: seeded k^-5/3 staggered velocity, rhs = its discrete divergence",
           "config": {"workload": workload, "nx": nx, "ny": ny, "nz": nz, "beta": args.beta,
                      "Lx": "2pi", "Lz": "2pi", "form": "fp64 direct solve"}}
    if r64 is not None:
        out["value"] = 1000.0 / r64["ms"]
        out["ms_per_step"] = r64["ms"]
        out["hbm_gbs_stage_model"] = stage_bytes / (r64["ms"] * 1e-3) / 1e9
        out["stage_model_bytes"] = stage_bytes
        out["roofline_frac_stage_model"] = out["hbm_gbs_stage_model"] / HBM_PEAK_GBS
        passes = {}
        for name, p in r64["prof"].items():
            avg = p["total_ms"] / p["launches"]
            passes[name] = {"avg_ms": avg, "launches": p["launches"],
                            "gbs": p["bytes_per_launch"] / (avg * 1e-3) / 1e9}
        out["passes_fp64"] = passes
        out["ms_per_step_with_launch_events"] = r64["ms_prof"]
    if r64 is not None and r64["prof"]:
        dom = max(r64["prof"].items(), key=lambda kv: kv[1]["total_ms"])
        name, p = dom
        avg = p["total_ms"] / p["launches"]
        ach = p["bytes_per_launch"] / (avg * 1e-3) / 1e9
        copy = copy_gbs(int(p["bytes_per_launch"] // 16))
        out["roofline"] = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                           "copy_gbs": copy, "frac_of_copy": ach / copy,
                           "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                           "bytes_per_launch": p["bytes_per_launch"], "avg_launch_ms": avg,
                           "traffic": traffic_for(name, workload)}
    mixed = {}
    for form in forms:
        if form == "fp64":
            continue
        r = results[form]
        mixed[form] = {"solves_per_s": 1000.0 / r["ms"], "ms_per_step": r["ms"],
                       "iterations": r["info"]["iterations"], "converged": r["info"]["converged"],
                       "rel_residual": r["info"]["rel_residual"],
                       "rel_residual_vw": r["info"]["rel_residual_vw"],
                       "backward_error": r["info"]["backward_error"],
                       "residual_history": r["info"]["residual_history"],
                       "vs_fp64": (r64["ms"] / r["ms"]) if r64 else None}
        if r["prof"]:
            mixed[form]["passes"] = {
                name: {"avg_ms": p["total_ms"] / p["launches"], "launches": p["launches"],
                       "gbs": p["bytes_per_launch"] / (p["total_ms"] / p["launches"] * 1e-3) / 1e9}
                for name, p in r["prof"].items()}
    out["mixed"] = mixed
    if substep is not None:
        out["substep_fp64"] = substep
    out["source_hash"] = source_hash()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: oracle on the host")
        keep = {}
        out["cpu_baseline"] = cpu_baseline(args, keep, host_uvw)
        del host_uvw
        if "phi" in keep:
            # each form's error against the oracle: the oracle's right-hand
            # side solved by every form, ||phi - phi_oracle|| / ||phi_oracle||
            ref = keep["phi"]
            fo = torch.from_numpy(keep["f"]).cuda()
            errs = {}
            for form in forms:
                plan.set_precision(form, 1e-10, args.mixed_iters)
                po = plan.solve(fo).cpu().numpy()
                errs[form] = float(np.linalg.norm(po - ref) / np.linalg.norm(ref))
            del fo, keep
            log(f"[bench] error against the oracle: {errs}")
            out["err_vs_oracle"] = errs
            if "fp64" in errs:
                out["err_vs_oracle_fp64"] = errs["fp64"]
            for form in mixed:
                mixed[form]["err_vs_oracle"] = errs.get(form)
    del plan, f, phi
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_extra:
        # the batched (64 uneven grids) and paper-scale (1024x768x1024 graph
        # sequence) workloads, summarised; `--config c4` / `--config c5` give
        # their full records
        log("[bench] c4: 64-grid batch")
        c4 = run_c4(args)
        out["c4"] = {k: c4[k] for k in ("config", "value", "unit", "ms_per_step") if k in c4}
        for form in ("fp64", "mixed"):
            if form in c4:
                out["c4"][form] = {k: c4[form][k] for k in c4[form] if k != "autotune"}
        torch.cuda.empty_cache()
        log(f"[bench] c5: {args.extra_seq}-solve graph sequence at 1024x768x1024")
        c5 = run_c5(args, steps=args.extra_seq)
        out["c5"] = {k: c5[k] for k in ("config", "value", "unit", "ms_per_step", "hbm_gbs_stage_model",
                                         "roofline_frac_stage_model", "mixed") if k in c5}
        torch.cuda.empty_cache()
        log("[bench] paper grids 501x1001x501 and 632x1263x632 (FP64)")
        out["paper_grids"] = run_paper_grids(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
