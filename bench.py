"""Throughput of the local-potential application V_loc|psi> on one MI355X.

One step = one vloc_apply over the whole batch: 256 bands on a 96^3 grid with
the |G| <= 24 sphere (57,777 plane waves, 1,793 z-sticks), K1 -> K2 -> K3 per
band chunk.  Inputs are synthetic (seeded), resident in HBM before timing.
Prints one JSON line on stdout; details go to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--precision f64]
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
FP64_PEAK = 78.6e12        # FLOP/s vector FP64
FP32_PEAK_NONPACKED = 78.6e12  # FLOP/s FP32 without packed instructions


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "dft_codelets.h", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1601_07378_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(precision: str, nbands: int):
    """HBM bytes per plane-kernel launch from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"vloc_apply_96cubed_256bands_{precision}.txt")
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
        return float(kv["hbm_bytes_per_band"]) * nbands
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


def measure(precision, steps, warmup, chunk=0, timing=True, gamma=False):
    import torch

    import synth
    from paper_1601_07378_amd import vloc

    w = synth.WORKLOADS["c2_96"]
    grid, cell, ecut, nb = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"]), w["nbands"]
    plan = vloc.Plan(grid, cell, ecut, precision=precision, band_chunk=chunk, gamma=gamma)
    hkl = plan.gvectors()
    ct, rt = (torch.complex128, torch.float64) if precision == "f64" else (torch.complex64, torch.float32)
    c = torch.from_numpy(synth.coefficients(hkl, nb)).to("cuda", ct)
    V = torch.from_numpy(synth.potential(grid, w["ngauss"])).to("cuda", rt)
    out = torch.empty_like(c)
    stream = torch.cuda.current_stream()
    plan.set_stream(stream)
    for _ in range(warmup):
        plan.apply(c, V, out=out, stream=stream)
    torch.cuda.synchronize()
    if timing:
        plan.enable_timing(True)
        plan.read_timing()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.apply(c, V, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    kms, kn = plan.read_timing() if timing else ([0, 0, 0], [0, 0, 0])
    sizes = workload_sizes(plan, grid, nb, precision)
    lay = plan.layout()
    bal = plan.balance()
    return dict(plan=plan, grid=grid, nb=nb, ms_total=ms_total, wall=wall, kms=kms, kn=kn,
                sizes=sizes, layout=lay, balance=bal, out=out, c=c, V=V)


SCHEDULES = os.path.join(ROOT, "paper_1601_07378_amd", "schedules.json")


def measure_batch(steps, warmup):
    """Several k-points with uneven spheres and band counts (72x96x128, R = 18,
    4 k-points, 64/128/256/512 bands): FP32 batch replayed from a HIP graph with
    the tuned schedule, against the plain FP64 path (one plan per k-point, one
    apply after another) and the FP64 batch."""
    import torch

    import synth
    from paper_1601_07378_amd import autotune, vloc

    w = synth.BATCH_WORKLOADS["c4_kpts"]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    kpts, nbs = w["kpts"], w["nbands"]
    total = sum(nbs)
    tuned, source = {}, "planner default"
    key = autotune._cache_key(grid, cell, ecut, kpts, nbs, "f32")
    if os.path.exists(SCHEDULES):
        with open(SCHEDULES) as f:
            entry = json.load(f).get(key)
        if entry:
            tuned, source = entry["best"], "autotuned (paper_1601_07378_amd/schedules.json)"
    res = {}
    stream = torch.cuda.current_stream()

    def timed(run):
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    for prec, opts, graph, name in (("f32", autotune.to_options(tuned) if tuned else {}, True,
                                     "f32_batch_graph"),
                                    ("f64", {}, False, "f64_batch"),
                                    ("f64", {}, False, "f64_plain")):
        ct, rt = (torch.complex128, torch.float64) if prec == "f64" else \
            (torch.complex64, torch.float32)
        b = vloc.Batch(grid, cell, ecut, kpts, precision=prec, **opts)
        cs = [torch.from_numpy(synth.coefficients(p.gvectors(), nb, k, ik=i)).to("cuda", ct)
              for i, (p, nb, k) in enumerate(zip(b.plans, nbs, kpts))]
        outs = [torch.empty_like(c) for c in cs]
        V = torch.from_numpy(synth.potential(grid, w["ngauss"])).to("cuda", rt)
        if name == "f64_plain":
            plans = [vloc.Plan(grid, cell, ecut, k, precision=prec) for k in kpts]
            for p in plans:
                p.set_stream(stream)

            def run():
                for p, c, o in zip(plans, cs, outs):
                    p.apply(c, V, out=o, stream=stream)
        else:
            b.set_stream(stream)
            if graph:
                b.use_graph(True)

            def run():
                b.apply(cs, V, outs=outs, stream=stream)
        ms = timed(run)
        res[name] = {"value": round(total / (ms / 1e3), 1), "ms_per_apply": round(ms, 4)}
        del b, cs, outs, V
        torch.cuda.empty_cache()
    res["speedup_f32_graph_vs_f64_plain"] = round(res["f32_batch_graph"]["value"] /
                                                  res["f64_plain"]["value"], 3)
    res["unit"] = "bands/s"
    res["workload"] = ("72x96x128 grid, |g+k| <= 18, k = (0,0,0), (1/4,0,0), (1/4,1/4,0), "
                       "(1/4,1/4,1/4) with 64/128/256/512 bands (960 per apply)")
    res["schedule"] = tuned or "planner default"
    res["schedule_source"] = source
    return res


def measure_grad(steps, warmup):
    """The differentiable energy at 128^3, |G| <= 32 (137,065 PW), 512 bands:
    one step = forward (apply, band energies, weighted sum) and backward
    (dE/dc, dE/dV by the density pass, dE/dw), FP32 with FP64 reductions, and
    the same in FP64."""
    import torch

    import synth
    from paper_1601_07378_amd import autograd, vloc

    w_ = synth.WORKLOADS["c5_128"]
    grid, cell, ecut, nb = w_["grid"], synth.cubic_cell(), synth.ecut_for_radius(w_["R"]), w_["nbands"]
    res = {}
    for prec in ("f32", "f64"):
        ct, rt = (torch.complex128, torch.float64) if prec == "f64" else \
            (torch.complex64, torch.float32)
        plan = vloc.Plan(grid, cell, ecut, precision=prec)
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

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[prec] = {"value": round(nb / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                     "plane_xmode": plan.layout()["plane_xmode"]}
        del c, V, w, plan
        torch.cuda.empty_cache()
    res["unit"] = "bands/s (energy + all gradients)"
    res["workload"] = "128^3 grid, |G|<=32 sphere (137065 PW), 512 bands, Gamma, cubic cell"
    res["speedup_f32_vs_f64"] = round(res["f32"]["value"] / res["f64"]["value"], 3)
    return res


def cpu_baseline(nbands_sample: int):
    import oracle
    import synth

    w = synth.WORKLOADS["c2_96"]
    grid, cell, ecut = w["grid"], synth.cubic_cell(), synth.ecut_for_radius(w["R"])
    hkl = oracle.sphere_py(cell, ecut)
    c = synth.coefficients(hkl, w["nbands"])[:nbands_sample]
    V = synth.potential(grid, w["ngauss"])
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.apply(grid, cell, ecut, (0, 0, 0), c, V, nthreads=threads)
    dt = time.perf_counter() - t0
    return dict(value=nbands_sample / dt, unit="bands/s", cores=threads, kind="oracle",
                sample=f"{nbands_sample} of the 256 bands of the 96^3/R=24 workload, "
                       f"FP64, full-cube unpruned FFTs, OpenMP over bands; {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-gamma", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
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
    log(f"# device: {torch.cuda.get_device_name(0)}")
    r = measure(args.precision, args.steps, args.warmup, args.chunk)
    sz = r["sizes"]
    nb = r["nb"]
    ms_step = r["ms_total"] / args.steps
    bands_per_s = nb * args.steps / (r["ms_total"] / 1e3)
    kms, kn = r["kms"], r["kn"]
    chunk = r["layout"]["band_chunk"]
    # plane kernel (dominant): bytes per launch = S read + S written for its
    # bands + V once
    N3 = r["grid"][2]
    b_k2_band = 2 * sz["nst"] * N3 * sz["s"]
    k2_bytes = b_k2_band * nb * args.steps + sz["N"] * sz["sv"] * kn[1]
    k2_time = kms[1] / 1e3
    achieved = k2_bytes / k2_time if k2_time > 0 else None
    log(f"# {args.precision}: {ms_step:.3f} ms/step, {bands_per_s:,.0f} bands/s; kernels ms/step "
        f"K1 {kms[0] / args.steps:.3f} K2 {kms[1] / args.steps:.3f} K3 {kms[2] / args.steps:.3f}; "
        f"launches {kn}; layout {r['layout']}")
    path_frac = sz["b_alg"] * bands_per_s / HBM_PEAK
    flop_rate = sz["f_alg"] * bands_per_s
    bal = r["balance"]
    log(f"# path: B_alg/band {sz['b_alg']:.0f} B -> {path_frac * 100:.1f}% of HBM peak; "
        f"F_alg/band {sz['f_alg']:.3e} -> {flop_rate / 1e12:.1f} TFLOP/s; group PW max/min/mean "
        f"{bal.max()}/{bal.min()}/{bal.mean():.1f}")
    k2_launch_bytes = k2_bytes / kn[1] if kn[1] else None
    # bands per launch: a call is cut into equal chunks of at most band_chunk
    launch_bands = nb * args.steps / kn[1] if kn[1] else chunk
    traffic = read_traffic(args.precision, launch_bands)
    result = {
        "metric": "band V_loc|psi> applications/sec at 96^3 (FP64 vs FP32) + % HBM peak",
        "value": round(bands_per_s, 1),
        "unit": "bands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded Gaussian coefficients scaled by 1/(1+|G|^2); V = 0.5 + 32 Gaussians)",
        "config": {"workload": "96^3 grid, |G|<=24 sphere (57777 PW, 1793 sticks), 256 bands, Gamma, "
                               "cubic cell", "grid": list(r["grid"]), "nbands": nb,
                   "npw": sz["npw"], "band_chunk_max": chunk,
                   "bands_per_launch": round(launch_bands, 2), "precision": args.precision},
        "hbm_frac_path": round(path_frac, 4),
        "roofline": {"bound": "hbm", "kernel": "k_plane (K2)",
                     "achieved": round(achieved / 1e9, 1) if achieved else None,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK, 4) if achieved else None,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": round(k2_launch_bytes) if k2_launch_bytes else None,
                     "avg_launch_ms": round(kms[1] / kn[1], 4) if kn[1] else None},
        "kernel_ms_per_step": {"k1_stick_fwd": round(kms[0] / args.steps, 4),
                               "k2_plane": round(kms[1] / args.steps, 4),
                               "k3_stick_bwd": round(kms[2] / args.steps, 4)},
    }
    # FP64 band energies e_n = Re<c_n|V c_n> (FP64 reductions), kept to check FP32
    e64 = r["plan"].band_dot(r["c"], r["out"]) if args.precision == "f64" else None
    out64 = r["out"] if args.precision == "f64" else None
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
    if not args.no_f32 and args.precision == "f64":
        r32 = measure("f32", args.steps, args.warmup, args.chunk, timing=False)
        v32 = r32["nb"] * args.steps / (r32["ms_total"] / 1e3)
        result["f32"] = {"value": round(v32, 1), "ms_per_step": round(r32["ms_total"] / args.steps, 4),
                         "speedup_vs_f64": round(v32 / bands_per_s, 3),
                         "hbm_frac_path": round(r32["sizes"]["b_alg"] * v32 / HBM_PEAK, 4)}
        # accuracy of the FP32 path against the FP64 path (itself within 1e-12 of
        # the oracle in the parity tests), every band of the workload; the FP32
        # band energies use the FP64 reductions
        o32 = r32["out"].to(torch.complex128)
        rel = (torch.linalg.vector_norm(o32 - out64, dim=1) /
               torch.linalg.vector_norm(out64, dim=1))
        e32 = r32["plan"].band_dot(r32["c"], r32["out"])
        erel = ((e32 - e64).abs() / e64.abs()).max().item()
        result["f32"]["max_rel_err_per_band_vs_f64"] = float(f"{rel.max().item():.3e}")
        result["f32"]["max_rel_err_band_energy_vs_f64"] = float(f"{erel:.3e}")
        log(f"# f32: {v32:,.0f} bands/s ({v32 / bands_per_s:.2f}x f64); max per-band rel err "
            f"{rel.max().item():.2e}, band-energy rel err {erel:.2e}")
        del r32, o32
    if not args.no_gamma and args.precision == "f64":
        # the paper's real mode (Gamma point, half sphere, two bands per transform)
        # on the same grid and sphere: a different input class (real psi), so it
        # is reported beside the complex-path value, not as it
        gm = {}
        for prec in ("f64", "f32"):
            rg = measure(prec, args.steps, args.warmup, args.chunk, timing=False, gamma=True)
            vg = rg["nb"] * args.steps / (rg["ms_total"] / 1e3)
            gm[prec] = {"value": round(vg, 1), "ms_per_step": round(rg["ms_total"] / args.steps, 4)}
            del rg
        gm["unit"] = "bands/s"
        gm["speedup_f64_vs_complex_f64"] = round(gm["f64"]["value"] / bands_per_s, 3)
        gm["workload"] = ("96^3, |G|<=24, 256 real bands (half sphere 28889 coefficients per "
                          "band), two bands per complex transform")
        result["gamma_real_mode"] = gm
        log(f"# gamma real mode: f64 {gm['f64']['value']:,.0f} bands/s, "
            f"f32 {gm['f32']['value']:,.0f} bands/s")
    if not args.no_batch and args.precision == "f64":
        rb = measure_batch(args.steps, args.warmup)
        result["batched_kpoints"] = rb
        log(f"# batch: f32 graph {rb['f32_batch_graph']['value']:,.0f} bands/s, f64 batch "
            f"{rb['f64_batch']['value']:,.0f}, f64 plain {rb['f64_plain']['value']:,.0f} "
            f"({rb['schedule_source']})")
    if not args.no_grad and args.precision == "f64":
        rg = measure_grad(max(2, args.steps // 4), 1)
        result["differentiable_energy"] = rg
        log(f"# energy + gradients 128^3 x 512: f32 {rg['f32']['value']:,.0f} bands/s, "
            f"f64 {rg['f64']['value']:,.0f} bands/s")
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.cpu_sample)
        result["cpu_baseline"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in cb.items()}
        log(f"# cpu oracle: {cb['value']:.2f} bands/s on {cb['cores']} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
