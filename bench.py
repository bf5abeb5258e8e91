"""Throughput of the local-potential application V_loc|psi> on one MI355X.

One step = one vloc_apply over the whole batch: 256 bands on a 96^3 grid with
the |G| <= 24 sphere (57,777 plane waves, 1,793 z-sticks), K1 -> K2 -> K3 per
band chunk.  Inputs are synthetic (seeded), resident in HBM before timing.
Prints one JSON line on stdout; details go to stderr.

Timing: every throughput figure comes from a timed region with no per-launch
events (HIP events only at its two ends), after an untimed warm-up of at least
--warmup steps and at least 0.3 s (the clock settles in that time).  The per-kernel split and the
roofline of the dominant kernel come from a second timed region of the same
steps in which the library records HIP events around each of its launches on
the plan's stream.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
VECTOR_PEAK = 78.6e12      # FLOP/s, MI355X FP64 vector (and non-packed FP32)
VECTOR_PEAK = 78.6e12      # FLOP/s: FP64 vector; FP32 without packed instructions runs the same


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "dft_codelets.h", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1601_07378_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(precision: str, nbands_per_launch: float):
    """HBM bytes per plane-kernel launch from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"k2_plane_96cubed_{precision}_hbm_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_band"]) * nbands_per_launch
    except (KeyError, ValueError):
        return None


def workload_sizes(plan, grid, nbands, precision):
    st = plan.sticks()
    nst = st.shape[0]
    npw = plan.npw
    nxo = plan.layout()["nxo"]
    N1, N2, N3 = grid
    N = N1 * N2 * N3
    s = 16 if precision == "f64" else 8
    sv = s // 2
    # algorithmic bytes per band (c in, out out, one stick-buffer exchange per
    # direction, V once per apply)
    b_alg = 2 * npw * s + 4 * nst * N3 * s + N * sv / nbands
    lg = np.log2
    f_alg = 2 * (nst * 5 * N3 * lg(N3) + nxo * N3 * 5 * N2 * lg(N2) + N2 * N3 * 5 * N1 * lg(N1)) + 2 * N
    return dict(nst=nst, npw=npw, nxo=nxo, N=N, s=s, sv=sv, b_alg=b_alg, f_alg=f_alg)


def timed_region(run, steps, stream):
    """ms over `steps` calls of run(), HIP events at the two ends only."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


# Untimed warm-up lasts at least `--warmup` steps and at least this long: the
# device's clock takes some tens of milliseconds of back-to-back work to settle
# (K2 launches run about 15% slower in the first ~25 ms of a cold start).
WARM_MIN_S = 0.3


def warm(run, warmup):
    """`warmup` untimed calls of run(), then more until WARM_MIN_S has passed."""
    import torch
    t0 = time.perf_counter()
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < WARM_MIN_S:
        run()
        torch.cuda.synchronize()


SCHEDULES = os.path.join(ROOT, "paper_1601_07378_amd", "schedules.json")


def schedule(grid, cell, ecut, kpts, nbands, precision):
    """(knobs, source) of the tuned schedule stored for this workload on this
    device, or ({}, 'planner default')."""
    from paper_1601_07378_amd import autotune
    key = autotune._cache_key(grid, cell, ecut, kpts, nbands, precision)
    if os.path.exists(SCHEDULES):
        with open(SCHEDULES) as f:
            entry = json.load(f).get(key)
        if entry:
            return entry["best"], "autotuned (paper_1601_07378_amd/schedules.json)"
    return {}, "planner default"


def measure(workload, precision, steps, warmup, gamma=False, kernel_pass=True, keep=False,
            tuned=True, per_apply=False):
    """Throughput of one plan on a named workload (with its tuned schedule when
    one is stored); optionally a second pass with per-launch events for the
    kernel split."""
    import torch

    import synth
    from paper_1601_07378_amd import autotune, vloc

    w = synth.WORKLOADS[workload]
    grid, cell, ecut, nb = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"]), w["nbands"]
    knobs, source = ({}, "planner default")
    if tuned:
        # the real mode takes the schedule stored for the same grid, sphere and
        # bands: it runs the same plane kernels on half as many transforms
        knobs, source = schedule(grid, cell, ecut, [(0.0, 0.0, 0.0)], [nb], precision)
    opts = autotune.to_options(knobs) if knobs else {}
    plan = vloc.Plan(grid, cell, ecut, precision=precision, gamma=gamma, **opts)
    hkl = plan.gvectors()
    ct, rt = (torch.complex128, torch.float64) if precision == "f64" else (torch.complex64, torch.float32)
    c = torch.from_numpy(synth.coefficients(hkl, nb)).to("cuda", ct)
    V = torch.from_numpy(synth.potential(grid, w["ngauss"])).to("cuda", rt)
    out = torch.empty_like(c)
    stream = torch.cuda.current_stream()
    plan.set_stream(stream)

    def run():
        plan.apply(c, V, out=out, stream=stream)

    warm(run, warmup)
    ms = timed_region(run, steps, stream)
    res = dict(plan=plan, grid=grid, nb=nb, ms_step=ms / steps, bands_per_s=nb * steps / (ms / 1e3),
               sizes=workload_sizes(plan, grid, nb, precision), layout=plan.layout(),
               schedule=knobs or "planner default", schedule_source=source)
    if kernel_pass:
        plan.enable_timing(True)
        plan.read_timing()
        ms_k = timed_region(run, steps, stream)
        kms, kn = plan.read_timing()
        plan.enable_timing(False)
        res.update(ms_step_kernel_pass=ms_k / steps, kms=kms, kn=kn)
    if per_apply:
        # one HIP event pair around each apply (a pass of its own)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record(stream)
            run()
            e1.record(stream)
        torch.cuda.synchronize()
        t = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
        res["per_apply_ms"] = {"median": round(float(np.median(t)), 4),
                               "min": round(float(t.min()), 4),
                               "max": round(float(t.max()), 4),
                               "timing": "HIP events around each apply, a pass after the timed region and the per-launch event pass"}
    if keep:
        res.update(out=out, c=c, V=V)
    return res


def balance_report(workload):
    """Plane waves per stick group (the analogue of the paper's Tab. 2 statistic,
    per workgroup instead of per process) for the greedy deal (the paper's rule,
    Sec. 3.2), the snake variant and the unsorted cyclic deal it improves on, at
    the plan's group count; and the grid-sufficiency flag N_i >= 4 R_i (Sec.
    3.1: the product V psi is band-limited to twice the sphere's radius)."""
    import synth
    from paper_1601_07378_amd import vloc

    w = synth.WORKLOADS[workload]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    out = {}
    for deal in ("greedy", "snake", "unsorted"):
        b = vloc.Plan(grid, cell, ecut, deal=deal).balance()
        out[deal] = {"max": int(b.max()), "min": int(b.min()), "mean": round(float(b.mean()), 2),
                     "max_over_mean": round(float(b.max() / b.mean()), 4)}
    p = vloc.Plan(grid, cell, ecut)
    out["groups"] = int(p.balance().size)
    out["sticks"] = int(p.sticks().shape[0])
    hkl = p.gvectors()
    # 2 R_i = the sphere's extent along axis i minus one
    two_r = [int(x) for x in hkl.max(0) - hkl.min(0)]
    out["grid_check"] = {"N": list(grid), "four_R": [2 * t for t in two_r],
                         "N_ge_4R": [bool(n >= 2 * t) for n, t in zip(grid, two_r)]}
    return out


def measure_batch(steps, warmup, workload="c4_kpts"):
    """Several k-points with uneven spheres and band counts (72x96x128, R = 18,
    4 k-points, 64/128/256/512 bands): the batch (one launch per kernel per
    chunk) against plain per-k plans applied one after another, in FP32 (graph
    replay, tuned schedule) and FP64."""
    import torch

    import synth
    from paper_1601_07378_amd import autotune, vloc

    w = synth.BATCH_WORKLOADS[workload]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    kpts, nbs = w["kpts"], w["nbands"]
    total = sum(nbs)
    sched = {p: schedule(grid, cell, ecut, kpts, nbs, p) for p in ("f32", "f64")}
    res = {}
    stream = torch.cuda.current_stream()
    # every leg uses the tuned schedule of its precision (the plain plans take
    # the same knobs but the batch's band chunk); batches replay HIP graphs
    legs = (("f32", True, "f32_batch_graph"), ("f32", False, "f32_plain"),
            ("f64", True, "f64_batch_graph"), ("f64", False, "f64_plain"))
    for prec, is_batch, name in legs:
        knobs = sched[prec][0]
        opts = autotune.to_options(knobs) if knobs else {}
        plain_opts = {k: v for k, v in opts.items() if k != "band_chunk"}
        ct, rt = (torch.complex128, torch.float64) if prec == "f64" else \
            (torch.complex64, torch.float32)
        b = vloc.Batch(grid, cell, ecut, kpts, precision=prec, **opts)
        cs = [torch.from_numpy(synth.coefficients(p.gvectors(), nb, k, ik=i)).to("cuda", ct)
              for i, (p, nb, k) in enumerate(zip(b.plans, nbs, kpts))]
        outs = [torch.empty_like(c) for c in cs]
        V = torch.from_numpy(synth.potential(grid, w["ngauss"])).to("cuda", rt)
        if not is_batch:
            plans = [vloc.Plan(grid, cell, ecut, k, precision=prec, **plain_opts) for k in kpts]
            for p in plans:
                p.set_stream(stream)

            def run():
                for p, c, o in zip(plans, cs, outs):
                    p.apply(c, V, out=o, stream=stream)
        else:
            b.set_stream(stream)
            b.use_graph(True)

            def run():
                b.apply(cs, V, outs=outs, stream=stream)
        warm(run, warmup)
        ms = timed_region(run, steps, stream) / steps
        res[name] = {"value": round(total / (ms / 1e3), 1), "ms_per_apply": round(ms, 4)}
        del b, cs, outs, V
        torch.cuda.empty_cache()
    res["speedup_f32_batch_vs_f32_plain"] = round(res["f32_batch_graph"]["value"] /
                                                  res["f32_plain"]["value"], 3)
    res["speedup_f64_batch_vs_f64_plain"] = round(res["f64_batch_graph"]["value"] /
                                                  res["f64_plain"]["value"], 3)
    res["speedup_f32_batch_vs_f64_plain"] = round(res["f32_batch_graph"]["value"] /
                                                  res["f64_plain"]["value"], 3)
    res["unit"] = "bands/s"
    res["workload"] = (f"{grid[0]}x{grid[1]}x{grid[2]} grid, |g+k| <= {w['R']:g}, k = "
                       + ", ".join("(" + ",".join(f"{x:g}" for x in k) + ")" for k in kpts)
                       + f" with {'/'.join(map(str, nbs))} bands ({total} per apply)")
    res["schedule"] = {p: sched[p][0] or "planner default" for p in sched}
    res["schedule_source"] = {p: sched[p][1] for p in sched}
    return res


def measure_grad(steps, warmup):
    """The differentiable energy at 128^3, |G| <= 32 (137,065 PW), 512 bands:
    one step = forward (apply, band energies, weighted sum) and backward
    (dE/dc, dE/dV by the density pass, dE/dw), FP32 with FP64 reductions, and
    the same in FP64."""
    import torch

    import synth
    from paper_1601_07378_amd import autograd, autotune, vloc

    w_ = synth.WORKLOADS["c5_128"]
    grid, cell, ecut, nb = w_["grid"], synth.cubic_cell(), synth.ecut_for_radius(w_["R"]), w_["nbands"]
    res = {}
    splits = ("L1x", "L2x", "L1y", "L2y", "L1z", "L2z")
    for prec in ("f32", "f64"):
        ct, rt = (torch.complex128, torch.float64) if prec == "f64" else \
            (torch.complex64, torch.float32)
        # the stored schedule (tuned on the application) when it keeps the
        # planner's line splits: the density kernels are compiled for those, and
        # another split would send the density passes of a step to the
        # runtime-sized kernels; else the planner's schedule
        plan = vloc.Plan(grid, cell, ecut, precision=prec)
        knobs, source = schedule(grid, cell, ecut, [(0.0, 0.0, 0.0)], [nb], prec)
        if knobs:
            tuned_plan = vloc.Plan(grid, cell, ecut, precision=prec, **autotune.to_options(knobs))
            if all(tuned_plan.layout()[k] == plan.layout()[k] for k in splits):
                plan.close()
                plan = tuned_plan
            else:
                tuned_plan.close()
                knobs, source = {}, "planner default (the stored schedule changes the line splits)"
        c = torch.from_numpy(synth.coefficients(plan.gvectors(), nb)).to("cuda", ct)
        V = torch.from_numpy(synth.potential(grid, w_["ngauss"])).to("cuda", rt)
        w = torch.from_numpy(synth.band_weights(nb)).to("cuda", torch.float64)
        c.requires_grad_(True)
        V.requires_grad_(True)
        w.requires_grad_(True)
        stream = torch.cuda.current_stream()

        def step():
            c.grad = V.grad = w.grad = None
            E = autograd.local_energy(plan, c, V, w)
            E.backward()
            return E

        warm(step, warmup)
        ms = timed_region(step, steps, stream) / steps
        res[prec] = {"value": round(nb / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                     "plane_xmode": plan.layout()["plane_xmode"],
                     "schedule": knobs or "planner default", "schedule_source": source}
        del c, V, w, plan
        torch.cuda.empty_cache()
    res["unit"] = "bands/s (energy + all gradients)"
    res["workload"] = "128^3 grid, |G|<=32 sphere (137065 PW), 512 bands, Gamma, cubic cell"
    res["speedup_f32_vs_f64"] = round(res["f32"]["value"] / res["f64"]["value"], 3)
    return res


def cpu_baseline(nbands_sample: int, threads: int):
    import oracle
    import synth

    w = synth.WORKLOADS["c2_96"]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    hkl = oracle.sphere_py(cell, ecut)
    c = synth.coefficients(hkl, w["nbands"])[:nbands_sample]
    V = synth.potential(grid, w["ngauss"])
    t0 = time.perf_counter()
    oracle.apply(grid, cell, ecut, (0, 0, 0), c, V, nthreads=threads)
    dt = time.perf_counter() - t0
    return dict(value=nbands_sample / dt, unit="bands/s", cores=threads, kind="oracle",
                sample=f"{nbands_sample} of the 256 bands of the 96^3/R=24 workload, "
                       f"FP64, full-cube unpruned FFTs, OpenMP over bands; {dt:.1f} s")


def r_default_needed(result) -> bool:
    return result.get("schedule") != "planner default"


def path_figures(r, precision):
    sz = r["sizes"]
    v = r["bands_per_s"]
    return {"value": round(v, 1), "ms_per_step": round(r["ms_step"], 4),
            "hbm_frac_path": round(sz["b_alg"] * v / HBM_PEAK, 4),
            "flop_rate_tflops": round(sz["f_alg"] * v / 1e12, 2),
            # FP32 issues at the FP64 rate here (packed FP32 instructions are
            # not used), so both precisions take the 78.6 TFLOP/s vector peak
            "flop_frac_vector_peak": round(sz["f_alg"] * v / VECTOR_PEAK, 4),
            "algorithmic_bytes_per_band": round(sz["b_alg"])}


def kernel_figures(r, steps):
    """Per-kernel split and the roofline of the plane kernel K2 from the
    per-launch event pass."""
    sz = r["sizes"]
    kms, kn = r["kms"], r["kn"]
    N3 = r["grid"][2]
    # plane kernel: S read and written for its bands, plus the arranged
    # potential once per launch
    b_k2_band = 2 * sz["nst"] * N3 * sz["s"]
    launch_bands = r["nb"] * steps / kn[1]
    k2_launch_bytes = b_k2_band * launch_bands + sz["N"] * sz["sv"]
    k2_avg_s = kms[1] / kn[1] / 1e3
    achieved = k2_launch_bytes / k2_avg_s
    split = {"k1_stick_fwd": round(kms[0] / steps, 4), "k2_plane": round(kms[1] / steps, 4),
             "k3_stick_bwd": round(kms[2] / steps, 4),
             "launches_per_step": [n // steps for n in kn],
             "ms_per_step_with_events": round(r["ms_step_kernel_pass"], 4)}
    return split, achieved, k2_launch_bytes, launch_bands, k2_avg_s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--cpu-sample-1thread", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="the 96^3 FP64 and FP32 legs only (profiling runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the M0, real-mode, batch and gradient legs")
    ap.add_argument("--only-grad", action="store_true",
                    help="the 128^3 energy + gradient leg only, its figures as the one "
                         "JSON line (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain device copy of 256 MiB so that "
                         "profiler byte counters can be scaled by a kernel of known traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the path shards over bands with no exchange, "
              f"so --gpus {args.gpus} is not run (see the sharding notes in the design "
              f"document).", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1601_07378_amd import autotune
    log(f"# device: {torch.cuda.get_device_name(0)} ({autotune.device_tag()})")
    steps, warmup = args.steps, args.warmup
    if args.only_grad:
        rg = measure_grad(steps, warmup)
        log(f"# energy + gradients 128^3 x 512: f32 {rg['f32']['value']:,.0f} bands/s, "
            f"f64 {rg['f64']['value']:,.0f} bands/s")
        print(json.dumps({"differentiable_energy": rg, "steps": steps, "warmup": warmup}),
              flush=True)
        return

    # ---- headline: 96^3, 256 bands, FP64
    r = measure("c2_96", "f64", steps, warmup, keep=True, per_apply=True)
    head = path_figures(r, "f64")
    split, achieved, k2_bytes, launch_bands, k2_avg_s = kernel_figures(r, steps)
    log(f"# f64: {r['ms_step']:.4f} ms/step ({r['ms_step_kernel_pass']:.4f} with per-launch "
        f"events), {r['bands_per_s']:,.0f} bands/s, {head['hbm_frac_path'] * 100:.1f}% of HBM "
        f"peak; K1 {split['k1_stick_fwd']:.4f} K2 {split['k2_plane']:.4f} K3 "
        f"{split['k3_stick_bwd']:.4f} ms/step; K2 {k2_avg_s * 1e3:.4f} ms/launch; "
        f"layout {r['layout']}")
    sz = r["sizes"]
    result = {
        "metric": "band V_loc|psi> applications/sec at 96^3 (FP64 vs FP32) + % HBM peak",
        "value": head["value"],
        "unit": "bands/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian coefficients scaled by 1/(1+|G|^2); V = 0.5 + 32 Gaussians)",
        "config": {"workload": "96^3 grid, |G|<=24 sphere (57777 PW, 1793 sticks), 256 bands, Gamma, "
                               "cubic cell", "grid": list(r["grid"]), "nbands": r["nb"],
                   "npw": sz["npw"], "band_chunk_max": r["layout"]["band_chunk"],
                   "bands_per_launch": round(launch_bands, 2), "precision": "f64"},
        "hbm_frac_path": head["hbm_frac_path"],
        "flop_rate_tflops": head["flop_rate_tflops"],
        "flop_frac_vector_peak": head["flop_frac_vector_peak"],
        "per_apply_ms": r["per_apply_ms"],
        "roofline": {"bound": "hbm", "kernel": "k_plane (K2)",
                     "achieved": round(achieved / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK, 4),
                     "traffic": read_traffic("f64", launch_bands),
                     "algorithmic_bytes_per_launch": round(k2_bytes),
                     "avg_launch_ms": round(k2_avg_s * 1e3, 4),
                     "timing": "per-launch HIP events on the plan stream, second timed region of "
                               "the same steps",
                     "measured_limiter": "LDS traffic and VALU issue (SQ counters in profiles/)"},
        "kernel_ms_per_step": split,
        "schedule": r["schedule"],
        "schedule_source": r["schedule_source"],
    }
    e64 = r["plan"].band_dot(r["c"], r["out"])
    out64 = r["out"]
    del r
    torch.cuda.empty_cache()
    if args.copy_calibration:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("# copy calibration: 268435456 B read + 268435456 B written")
        del src, dst

    # the planner's default schedule on the same workload, for comparison
    if r_default_needed(result):
        rd = measure("c2_96", "f64", steps, warmup, kernel_pass=False, tuned=False)
        result["default_schedule"] = {"value": round(rd["bands_per_s"], 1),
                                      "ms_per_step": round(rd["ms_step"], 4)}
        del rd
    # ---- the metric's FP32 column, timed the same way
    r32 = measure("c2_96", "f32", steps, warmup, keep=True, per_apply=True)
    f32 = path_figures(r32, "f32")
    s32, a32, b32, lb32, k2s32 = kernel_figures(r32, steps)
    f32["speedup_vs_f64"] = round(r32["bands_per_s"] / head["value"], 3)
    f32["schedule"] = r32["schedule"]
    f32["kernel_ms_per_step"] = s32
    f32["per_apply_ms"] = r32["per_apply_ms"]
    f32["k2_roofline"] = {"achieved_GBps": round(a32 / 1e9, 1), "frac": round(a32 / HBM_PEAK, 4),
                          "avg_launch_ms": round(k2s32 * 1e3, 4),
                          "algorithmic_bytes_per_launch": round(b32),
                          "traffic": read_traffic("f32", lb32)}
    # accuracy of the FP32 path against the FP64 path (itself within 1e-12 of the
    # oracle in the parity tests), every band; the band energies use the FP64
    # reductions
    o32 = r32["out"].to(torch.complex128)
    rel = (torch.linalg.vector_norm(o32 - out64, dim=1) / torch.linalg.vector_norm(out64, dim=1))
    e32 = r32["plan"].band_dot(r32["c"], r32["out"])
    erel = ((e32 - e64).abs() / e64.abs()).max().item()
    f32["max_rel_err_per_band_vs_f64"] = float(f"{rel.max().item():.3e}")
    f32["max_rel_err_band_energy_vs_f64"] = float(f"{erel:.3e}")
    result["f32"] = f32
    log(f"# f32: {r32['bands_per_s']:,.0f} bands/s ({f32['speedup_vs_f64']:.2f}x f64), "
        f"{f32['hbm_frac_path'] * 100:.1f}% of HBM peak; K2 {k2s32 * 1e3:.4f} ms/launch; max "
        f"per-band rel err {rel.max().item():.2e}, band-energy rel err {erel:.2e}")
    del r32, o32, out64
    torch.cuda.empty_cache()
    result["balance"] = balance_report("c2_96")
    log(f"# balance: {result['balance']}")

    if not args.only_headline and not args.no_extra:
        # the paper's workload shape (80^3 grid, ~35k plane waves, 1001 bands)
        m0 = {}
        for prec in ("f64", "f32"):
            rm = measure("m0_80", prec, max(3, steps // 4), warmup, kernel_pass=False)
            m0[prec] = path_figures(rm, prec)
            del rm
        m0["workload"] = ("80^3 grid, |G|^2 <= 413 sphere (35273 PW), 1001 bands, Gamma, cubic "
                          "cell: the shape of the paper's 80^3 / 35160-PW / 1001-state workload")
        m0["unit"] = "bands/s"
        result["m0_paper_shape"] = m0
        log(f"# m0 80^3 x 1001: f64 {m0['f64']['value']:,.0f} bands/s "
            f"({m0['f64']['hbm_frac_path'] * 100:.1f}%), f32 {m0['f32']['value']:,.0f}")
        # the paper's real mode (Gamma point, half sphere, two bands per transform)
        # on the same grid and sphere: a different input class (real psi), so it
        # is reported beside the complex-path value, not as it
        gm = {}
        for prec in ("f64", "f32"):
            rg = measure("c2_96", prec, steps, warmup, gamma=True, kernel_pass=False)
            gm[prec] = {"value": round(rg["bands_per_s"], 1), "ms_per_step": round(rg["ms_step"], 4),
                        "schedule": rg["schedule"], "schedule_source": rg["schedule_source"]}
            del rg
        gm["unit"] = "bands/s"
        gm["speedup_f64_vs_complex_f64"] = round(gm["f64"]["value"] / head["value"], 3)
        gm["workload"] = ("96^3, |G|<=24, 256 real bands (half sphere 28889 coefficients per "
                          "band), two bands per complex transform")
        result["gamma_real_mode"] = gm
        log(f"# gamma real mode: f64 {gm['f64']['value']:,.0f} bands/s, "
            f"f32 {gm['f32']['value']:,.0f} bands/s")
        rb = measure_batch(steps, warmup)
        result["batched_kpoints"] = rb
        log(f"# batch: f32 graph {rb['f32_batch_graph']['value']:,.0f} vs f32 plain "
            f"{rb['f32_plain']['value']:,.0f}; f64 graph {rb['f64_batch_graph']['value']:,.0f} vs "
            f"f64 plain {rb['f64_plain']['value']:,.0f} bands/s ({rb['schedule_source']})")
        rs = measure_batch(steps, warmup, "small_kpts")
        result["batched_small_kpoints"] = rs
        log(f"# small k-points batch: f32 graph {rs['f32_batch_graph']['value']:,.0f} vs plain "
            f"{rs['f32_plain']['value']:,.0f}; f64 graph {rs['f64_batch_graph']['value']:,.0f} vs "
            f"plain {rs['f64_plain']['value']:,.0f} bands/s")
        rg = measure_grad(max(2, steps // 4), 1)
        result["differentiable_energy"] = rg
        log(f"# energy + gradients 128^3 x 512: f32 {rg['f32']['value']:,.0f} bands/s, "
            f"f64 {rg['f64']['value']:,.0f} bands/s")
    if not args.no_cpu_baseline:
        import oracle
        cb = cpu_baseline(args.cpu_sample, oracle.max_threads())
        result["cpu_baseline"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in cb.items()}
        log(f"# cpu oracle: {cb['value']:.2f} bands/s on {cb['cores']} threads")
        c1 = cpu_baseline(args.cpu_sample_1thread, 1)
        result["cpu_baseline_1thread"] = {k: (round(v, 3) if isinstance(v, float) else v)
                                          for k, v in c1.items()}
        log(f"# cpu oracle, 1 thread: {c1['value']:.3f} bands/s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
