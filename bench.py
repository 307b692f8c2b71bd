#!/usr/bin/env python3
"""Benchmark of the shadow-map shading path on one MI355X.

A step is one whole year of the rooftop BIPV workload (2,000 flat modules,
120,000 cells, on a roof among 200 buildings and 1,000 trees, 522,010
triangles, 8192 x 8192 depth picture, 8 x 8 samples per cell, the 4,379 suns
above the horizon at 40.4 N), evaluated through the C ABI (pv3d_evaluate,
suns in groups of up to 32 per launch sequence) with device-resident inputs
and outputs: view set-up, triangle set-up and binning, raster, sample depth
check, bypass-diode losses and the energy sums all run on the GPU.

Prints one JSON line with the throughput (sample x sun shadow tests per
second; triangles rasterized per second beside it), the roofline of the
dominant kernel (priced on its exclusive time: the union of its launches'
intervals), the CPU oracle timed on a bounded sample of the same workload,
and legs: the row plant year, the batched and serving forms, trackers, many
generators, the single-diode model and sky view factors.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


LEGS = ("row_plant", "batched", "c4", "trackers", "stadium", "electrical", "sky", "serving")
WORKLOAD_KEY = {"c1": "c1_tiny", "c2": "c2_row_plant", "c3": "c3_rooftop"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--suns", type=int, default=0,
                    help="profiling runs only: use every n-th sun of the year (0 = all)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--cpu-every", type=int, default=100, help="oracle leg: every n-th sun of the year")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--route", default="sparse", choices=["sparse", "materialised"],
                    help="sparse: picture evaluated at sample texels only (default); materialised: every "
                         "sun's full picture written to HBM and read back by a separate depth-check kernel")
    ap.add_argument("--no-materialised", action="store_true",
                    help="skip the extra one-step run of the materialised route")
    ap.add_argument("--no-extra", action="store_true", help="skip every leg")
    ap.add_argument("--extra-legs", default="all",
                    help="comma-separated legs to run (" + ", ".join(LEGS) + "); default all")
    ap.add_argument("--c4-every", type=int, default=1, help="C4 leg: every n-th sun of the year (1 = full year)")
    ap.add_argument("--stadium-every", type=int, default=4, help="stadium leg: every n-th sun of the year")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="serving leg: arrivals per second")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="serving leg: seconds of arrivals")
    ap.add_argument("--light-rate", type=float, default=4.0, help="serving leg: light-load arrivals per second")
    ap.add_argument("--light-seconds", type=float, default=3.0, help="serving leg: light-load seconds of arrivals")
    ap.add_argument("--sweep-requests", type=int, default=40,
                    help="serving leg: requests per rate of the rate sweep (0 = no sweep)")
    return ap.parse_args()


def workload(name, every):
    from paper_1410_5780_amd import workloads as W
    yr = W.year_sweep()
    if every > 1:
        yr = yr.subset(np.arange(0, yr.n, every))
    if name == "c1":
        return W.c1_tiny(d_poa=100.0)
    if name == "c2":
        return W.c2_row_plant(sweep=yr)
    return W.c3_rooftop(sweep=yr)


# Peaks of one MI355X: HBM3E 8 TB/s; VALU lane operations (int32 / fp32 / fp64
# non-packed: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Lane operations the depth check of one sample needs at least: the FP64 affine
# map to light space (3 x 4), three floors and clamps (12), and at its texel
# the edge functions and depth plane of the two surfaces every sample sees
# (its own module and what lies behind it): 2 x (3 edges + 1 plane) x 2 int64
# multiply-adds x 4 int32 operations = 64; 88 in all.
SAMPLE_LANE_OPS = 88


def stage_roofline(stage, w, route):
    """(bound, algorithmic units per sun, unit, peak) of a stage."""
    V = w.scene.n_vert + 4 * w.gen.n_mod
    if stage == "raster" and route == "materialised":
        return "hbm", 4 * w.map_n * w.map_n, "GB/s", HBM_PEAK_GBS        # the picture, written once
    if stage == "raster":
        return "alu", SAMPLE_LANE_OPS * w.n_samples, "TOP/s", VALU_PEAK_TOPS
    if stage == "sample_test":
        return "hbm", 4 * w.n_samples + 4 * w.gen.n_cells, "GB/s", HBM_PEAK_GBS
    if stage == "tri_setup":
        return "hbm", 24 * V + 12 * w.n_tri_submitted, "GB/s", HBM_PEAK_GBS
    return "hbm", 0, "GB/s", HBM_PEAK_GBS


def profile_path(wname):
    return os.path.join(ROOT, "profiles", f"tile_{wname}.md")


def measured_traffic(kernel, route, wname="c2_row_plant"):
    """HBM bytes per sun of the tile kernel from the committed rocprofv3 counter summary of
    that workload, or None when the kernel source changed since the counters were taken."""
    import hashlib
    if kernel != "raster" or route != "sparse":
        return None
    prof = profile_path(wname)
    src = os.path.join(ROOT, "paper_1410_5780_amd", "csrc", "pv3d_kernels.hip")
    try:
        kv = dict(line.split(" = ", 1) for line in open(prof).read().splitlines() if " = " in line)
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if kv.get("kernel_source_sha256_16", "").strip() != sha or "tile_traffic_bytes_per_sun" not in kv:
        return None
    return int(kv["tile_traffic_bytes_per_sun"])


def timed_year(ctx, w, sh, gh, steps, warmup, route="sparse", tile=0, log=None):
    """Warm-up passes (the first times every stage), then `steps` timed passes of the sweep
    with every launch of the dominant stage bracketed by events: seconds per pass, the
    stage table, and the dominant stage's event time and exclusive (union) time per sun."""
    import torch
    from paper_1410_5780_amd import pv3d
    counts = torch.empty((w.sweep.n, w.gen.n_cells), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(r=route):
        return ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k, stream=stream, counts=counts, tile=tile,
                                   separate_test=(r == "materialised"))

    stage_ms = {}
    res = None
    for i in range(max(warmup, 1)):
        if i == 0:
            ctx.profile_enable((1 << pv3d.N_STAGES) - 1)
        res = step()
        torch.cuda.synchronize()
        if i == 0:
            for nm, sid in pv3d.STAGE.items():
                ms, n = ctx.profile_read(sid)
                busy, suns = ctx.profile_busy(sid)
                stage_ms[nm] = {"total_ms": ms, "launches": n, "busy_ms": busy, "suns": suns,
                                "busy_us_per_sun": 1e3 * busy / max(suns, 1)}
            ctx.profile_enable(0)
        if log:
            log(f"[bench] {w.name}: warmup {i} done")
    dominant = max(stage_ms, key=lambda k: stage_ms[k]["busy_ms"])
    sid = pv3d.STAGE[dominant]
    ctx.profile_sample(1)
    ctx.profile_enable(1 << sid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n = ctx.profile_read(sid)
    busy_ms, suns = ctx.profile_busy(sid)
    ctx.profile_enable(0)
    if log:
        log(f"[bench] {w.name}: timed {steps} passes in {t1 - t0:.3f} s")
    work = ctx.path_stats()                # the last timed pass: set-up records and binned pairs
    return {"sec_per_step": (t1 - t0) / steps, "stage_ms": stage_ms, "dominant": dominant, "work": work,
            "event_ms": k_ms, "launches": k_n, "busy_ms": busy_ms, "suns": suns, "result": res, "step": step}


def roofline_of(t, w, route):
    bound, units, unit, peak = stage_roofline(t["dominant"], w, route)
    scale = 1e9 if unit == "GB/s" else 1e12
    busy_s = t["busy_ms"] * 1e-3
    achieved = units * t["suns"] / busy_s / scale if units and busy_s > 0 else None
    return {"kernel": t["dominant"], "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": (achieved / peak) if achieved else None,
            "traffic": measured_traffic(t["dominant"], route, w.name.split(":")[0]),
            "exclusive_us_per_sun": 1e3 * t["busy_ms"] / max(t["suns"], 1),
            "event_us_per_launch": 1e3 * t["event_ms"] / max(t["launches"], 1),
            "launches": t["launches"], "suns": t["suns"], "units_per_sun": units,
            "model": ("88 lane-ops per sample (FP64 light-space map, floors, two covering surfaces' edge and "
                      "depth evaluations), over the union of the kernel's launch intervals" if bound == "alu"
                      else "algorithmic bytes over the union of the kernel's launch intervals")}


def row_plant_leg(ctx, log, steps):
    """The row plant year (C2) through the same per-sun path, with its own roofline."""
    from paper_1410_5780_amd import workloads as W
    w = W.c2_row_plant()
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    t = timed_year(ctx, w, sh, gh, steps, 1, log=log)
    res = t["result"]
    out = {"workload": f"{w.name}: {w.note}; {w.sweep.n} suns", "year_seconds": t["sec_per_step"],
           "value": w.n_samples * w.sweep.n / t["sec_per_step"], "unit": "sample-sun tests/s",
           "triangles_per_s": w.n_tri_submitted * w.sweep.n / t["sec_per_step"],
           "roofline": roofline_of(t, w, "sparse"), "energy_loss": res.loss,
           "stage_busy_us_per_sun": {k: round(v["busy_us_per_sun"], 3) for k, v in t["stage_ms"].items()}}
    log(f"[bench] row plant year {t['sec_per_step']:.3f} s")
    return out, (w, sh, gh, res)


def batched_leg(ctx, w, sh, gh, plain_energy, plain_power, plain_year_s, log):
    """The same year in one persistent launch (pv3d_evaluate_batched), results checked against the loop."""
    import torch
    spec = dict(scene=sh, gen=gh, generator=w.gen, sweep=w.sweep, map_n=w.map_n, k=w.k, counts=False)
    best = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.evaluate_batched([spec], device=True)[0]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    st = ctx.batch_stats()
    same = bool(np.array_equal(r.energy.cpu().numpy(), plain_energy) and np.array_equal(r.power.cpu().numpy(), plain_power))
    log(f"[bench] batched year: {best:.3f} s, identical {same}")
    return {"value": w.n_samples * w.sweep.n / best, "unit": "sample-sun tests/s", "year_seconds": best,
            "speedup_vs_plain_loop": plain_year_s / best, "identical_to_plain_loop": same,
            "launch_us": st["launch_us"], "units": st["units"], "slots": st["slots"],
            "workgroups": st["workgroups"], "xcd_groups": st["xcd_groups"]}


def c4_leg(ctx, every, log):
    """64 uneven sites: the plain per-sun loop against one persistent launch (autotuned per size class)."""
    import torch
    from paper_1410_5780_amd import workloads as W
    yr = W.year_sweep()
    sub = yr.subset(np.arange(0, yr.n, every))
    ws = W.c4_batched(sweep=sub)
    specs = [dict(scene=ctx.load_scene(x.scene), gen=ctx.define_generator(x.gen), generator=x.gen, sweep=x.sweep,
                  map_n=x.map_n, k=x.k, counts=False) for x in ws]
    # every site goes through the autotuner; the library times one site per class (map size, k,
    # triangle and cell decades) and hands the others its cached choice
    import json as _json
    import tempfile
    from paper_1410_5780_amd import pv3d
    ctx.tuning_cache(pv3d.TUNE_CLEAR)
    t0 = time.perf_counter()
    for sp in specs:
        sp["tile"], sp["bin_limit"] = ctx.autotune(sp, n_probe=4)[:2]
    tune_s = time.perf_counter() - t0
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "tuning.json")
        ctx.tuning_cache(pv3d.TUNE_SAVE, path)
        tuned = _json.load(open(path))
    log(f"[bench] c4: {len(ws)} sites x {sub.n} suns, autotuned {len(tuned)} classes in {tune_s:.2f} s")
    best_p = best_b = None
    for _ in range(1 if every == 1 else 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = [ctx.evaluate_device(sp["scene"], sp["gen"], sp["generator"], sp["sweep"], sp["map_n"], sp["k"])
                 for sp in specs]
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        t0 = time.perf_counter()
        bat = ctx.evaluate_batched(specs, device=True)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        best_p = tp if best_p is None else min(best_p, tp)
        best_b = tb if best_b is None else min(best_b, tb)
    st = ctx.batch_stats()
    same = all(np.array_equal(a.energy.cpu().numpy(), b.energy.cpu().numpy()) and
               np.array_equal(a.power.cpu().numpy(), b.power.cpu().numpy()) for a, b in zip(plain, bat))
    samples = sum(x.n_samples * x.sweep.n for x in ws)
    tris = sum(x.n_tri_submitted * x.sweep.n for x in ws)
    for sp in specs:
        ctx.release_scene(sp["scene"])
        ctx.release_generator(sp["gen"])
    log(f"[bench] c4: plain {best_p:.3f} s, batched {best_b:.3f} s, identical {same}")
    return {"workload": f"64 sites (1k-2M triangles, 60-24,000 cells, N 2048-8192), every {every}th sun of the "
                        f"year ({sub.n} suns each, {st['items']} items)",
            "plain_loop_s": best_p, "batched_s": best_b, "speedup": best_p / best_b, "identical": same,
            "batched_tests_per_s": samples / best_b, "batched_triangles_per_s": tris / best_b,
            "autotune_s": tune_s,
            "autotuned": {f"N{e['map_n']}_1e{e['tri_decade']}tri_1e{e['cell_decade']}cells": [e["tile"], e["bin_limit"]]
                          for e in tuned},
            "units": st["units"], "slots": st["slots"], "redone_per_sun": st["redone"]}


def tracker_leg(ctx, log):
    """The two-axis tracker plant on terrain (Sec. 3.4's case): a year on the per-sun loop,
    modules posed for every sun on the device."""
    import torch
    from paper_1410_5780_amd import workloads as W
    w = W.c6_tracker_plant()
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    best = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    loss = r.loss
    spec = dict(scene=sh, gen=gh, generator=w.gen, sweep=w.sweep, map_n=w.map_n, k=w.k, counts=False)
    bbest = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = ctx.evaluate_batched([spec], device=True)[0]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bbest = dt if bbest is None else min(bbest, dt)
    same = bool(np.array_equal(b.energy.cpu().numpy(), r.energy.cpu().numpy())
                and np.array_equal(b.power.cpu().numpy(), r.power.cpu().numpy()))
    ctx.release_scene(sh)
    ctx.release_generator(gh)
    log(f"[bench] trackers: {w.gen.trackers.shape[0]} two-axis trackers, {w.gen.n_cells} cells, year {best:.3f} s, "
        f"batched {bbest:.3f} s, identical {same}")
    return {"workload": f"{w.name}: {w.note}", "suns": w.sweep.n, "year_seconds": best,
            "value": w.n_samples * w.sweep.n / best, "unit": "sample-sun tests/s",
            "triangles_per_s": w.n_tri_submitted * w.sweep.n / best, "energy_loss": loss,
            "batched_year_seconds": bbest, "batched_identical": same}


def stadium_leg(ctx, log, every):
    """Sec. 3.3's case: 88 generators of 14 x 4 modules in one stadium scene, each with its own
    window and picture. The scene is loaded once; the per-generator loop (one per-sun-path call
    per generator) against one persistent launch over all 88 generators' suns."""
    import torch
    from paper_1410_5780_amd import workloads as W
    yr = W.year_sweep()
    ws = W.c7_stadium(sweep=yr.subset(np.arange(0, yr.n, every)))
    sh = ctx.load_scene(ws[0].scene)
    ghs = [ctx.define_generator(w.gen) for w in ws]
    best = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = [ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k) for gh, w in zip(ghs, ws)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    specs = [dict(scene=sh, gen=gh, generator=w.gen, sweep=w.sweep, map_n=w.map_n, k=w.k, counts=False)
             for gh, w in zip(ghs, ws)]
    bbest = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs = ctx.evaluate_batched(specs, device=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bbest = dt if bbest is None else min(bbest, dt)
    same = all(np.array_equal(a.power.cpu().numpy(), b.power.cpu().numpy())
               and np.array_equal(a.energy.cpu().numpy(), b.energy.cpu().numpy()) for a, b in zip(rs, bs))
    loss = np.array([r.loss for r in rs])
    for gh in ghs:
        ctx.release_generator(gh)
    ctx.release_scene(sh)
    n_sun = ws[0].sweep.n
    tests = sum(w.n_samples for w in ws) * n_sun
    log(f"[bench] stadium: {len(ws)} generators x {n_sun} suns, loop {best:.3f} s, batched {bbest:.3f} s, "
        f"identical {same}, loss {loss.min():.4f}..{loss.max():.4f}")
    return {"workload": f"c7_stadium: {len(ws)} generators of 14x4 modules, {ws[0].scene.n_tri} scene triangles, "
                        f"N={ws[0].map_n}, k={ws[0].k}, every {every}th sun of the year",
            "generators": len(ws), "suns": n_sun, "loop_seconds": best, "batched_seconds": bbest,
            "value": tests / bbest, "unit": "sample-sun tests/s", "loop_value": tests / best,
            "batched_identical": same, "energy_loss_min": float(loss.min()), "energy_loss_mean": float(loss.mean()),
            "energy_loss_max": float(loss.max())}


def electrical_leg(ctx, log):
    """The C2 year with the single-diode cell model (bypass diodes, a maximum power point per string)
    against the ideal string model: whole year and the loss stage alone (HIP events)."""
    import torch
    from paper_1410_5780_amd import pv3d, workloads as W
    w = W.c2_row_plant()
    sh = ctx.load_scene(w.scene)
    out = {}
    for name, d in (("ideal", None), ("single_diode", W.DIODE_CELL)):
        g = dataclasses.replace(w.gen, diode=d)
        gh = ctx.define_generator(g)
        best = None
        for i in range(2):
            if i == 1:
                ctx.profile_enable(1 << pv3d.STAGE["loss"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.evaluate_device(sh, gh, g, w.sweep, w.map_n, w.k)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        ms, n = ctx.profile_read(pv3d.STAGE["loss"])
        ctx.profile_enable(0)
        out[name] = {"year_seconds": best, "loss_stage_ms": ms / max(n, 1), "energy_loss": r.loss,
                     "energy_wh": float(r.energy.cpu().numpy()[0])}
        ctx.release_generator(gh)
    ctx.release_scene(sh)
    log(f"[bench] electrical: ideal year {out['ideal']['year_seconds']:.3f} s (loss stage "
        f"{out['ideal']['loss_stage_ms']:.2f} ms), single-diode {out['single_diode']['year_seconds']:.3f} s "
        f"(loss stage {out['single_diode']['loss_stage_ms']:.2f} ms), losses {out['ideal']['energy_loss']:.4f} / "
        f"{out['single_diode']['energy_loss']:.4f}")
    return {"workload": f"{w.name}: {w.note}; 20 strings of 1,200 cells, 4,379 suns", **out}


def sky_leg(ctx, log, n_dir=145):
    """Diffuse shading: per-cell sky view factors of C2 from n_dir sky directions (each evaluated as a
    sun), then the year with the factors attached."""
    import torch
    from paper_1410_5780_amd import workloads as W
    w = W.c2_row_plant()
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    dirs = W.sky_directions(n_dir)
    best = None
    for _ in range(2):
        t0 = time.perf_counter()
        svf = ctx.sky_view(sh, gh, w.gen, dirs, w.map_n, w.k)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    base = ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k)
    ctx.set_sky(gh, svf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k)
    torch.cuda.synchronize()
    year = time.perf_counter() - t0
    ctx.release_scene(sh)
    ctx.release_generator(gh)
    log(f"[bench] sky view: {n_dir} directions in {best:.3f} s, svf {svf.min():.3f}..{svf.max():.3f} "
        f"(mean {svf.mean():.3f}); year with it {year:.3f} s, loss {base.loss:.4f} -> {r.loss:.4f}")
    return {"workload": f"{w.name}: {w.note}", "directions": n_dir, "sky_view_seconds": best,
            "svf_min": float(svf.min()), "svf_mean": float(svf.mean()), "year_seconds_with_svf": year,
            "energy_loss_beam_only": base.loss, "energy_loss_with_diffuse": r.loss}


def highest_flat_rate(sweep):
    """The highest swept arrival rate whose p99 stays within twice the lowest p99 of the sweep
    (a straggler at one rate does not move the reference of the others)."""
    if not sweep:
        return None
    ref = min(x["p99_ms"] for x in sweep)
    return max(x["rate_hz"] for x in sweep if x["p99_ms"] <= 2.0 * ref)


def serving_leg(ctx, log, rate_hz, duration_s, light_rate, light_s, sweep_n):
    """Poisson request streams through the serving loop: latency from arrival to completion.
    The configured stream (200 req/s) offers more than one GPU evaluates, so it reports the
    offered and the sustained rates; a sweep below the sustained rate finds the highest
    arrival rate at which p99 stays within twice the lowest p99 of the sweep."""
    from paper_1410_5780_amd import serve, workloads as W
    out = {}
    reqs = W.serving_stream(seed=5, rate_hz=rate_hz, duration_s=duration_s)
    log(f"[bench] serving configured: {len(reqs)} requests at {rate_hz} /s")
    r = serve.run_stream(ctx, reqs, seed=5, log=log)
    r.update({"rate_hz": rate_hz, "duration_s": duration_s,
              "offered_req_per_s": len(reqs) / duration_s, "sustained_req_per_s": len(reqs) / r["wall_s"],
              "offered_tests_per_s": r["tests"] / duration_s, "sustained_tests_per_s": r["tests"] / r["wall_s"]})
    log(f"[bench] serving configured: {r['requests']} requests, p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms, "
        f"sustained {r['sustained_req_per_s']:.1f} of {r['offered_req_per_s']:.1f} req/s offered")
    out["configured_rate"] = r
    lr = W.serving_stream(seed=6, rate_hz=light_rate, duration_s=light_s)
    if lr:
        r2 = serve.run_stream(ctx, lr, seed=6, log=log)
        r2.update({"rate_hz": light_rate, "duration_s": light_s})
        out["light_load"] = r2
        log(f"[bench] serving light load: {r2['requests']} requests, p50 {r2['p50_ms']:.1f} ms, p99 {r2['p99_ms']:.1f} ms")
    if sweep_n > 0:
        cap = out["configured_rate"]["sustained_req_per_s"]
        sweep = []
        for i, f in enumerate((0.25, 0.5, 0.75)):
            rate = f * cap
            rq = W.serving_stream(seed=20 + i, rate_hz=rate, duration_s=sweep_n / rate)
            if not rq:
                continue
            rs = serve.run_stream(ctx, rq, seed=20 + i, log=log)
            sweep.append({"rate_hz": rate, "requests": rs["requests"], "p50_ms": rs["p50_ms"], "p99_ms": rs["p99_ms"],
                          "sustained_req_per_s": rs["requests"] / rs["wall_s"]})
            log(f"[bench] serving sweep {rate:.1f} req/s: p50 {rs['p50_ms']:.1f} ms, p99 {rs['p99_ms']:.1f} ms")
        out["rate_sweep"] = sweep
        out["highest_flat_p99_rate_hz"] = highest_flat_rate(sweep)
    return out


def cpu_baseline(w_full, every, threads=0):
    from oracle import oracle as O
    sw = w_full.sweep.subset(np.arange(0, w_full.sweep.n, every))
    cores = threads or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    r = O.evaluate(w_full.scene, w_full.gen, sw, w_full.map_n, w_full.k, threads=cores)
    dt = time.perf_counter() - t0
    tests = w_full.n_samples * sw.n
    return {"value": tests / dt, "unit": "sample-sun tests/s", "cores": cores, "kind": "oracle",
            "sample": f"{w_full.name}: every {every}th sun of the year ({sw.n} suns) of the same workload, "
                      f"{dt:.1f} s wall on {cores} threads; per-sun time extrapolates to "
                      f"{dt / sw.n * 4379:.0f} s for the year",
            "seconds": dt, "suns": sw.n, "triangles_per_s": w_full.n_tri_submitted * sw.n / dt,
            "loss_sample": r.loss}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not part of this "
                                   "build (sun positions would shard across GPUs, see the design notes)"}))
        sys.exit(2)
    import torch
    from paper_1410_5780_amd import pv3d

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    w = workload(a.workload, a.suns)
    n_sun = w.sweep.n
    log(f"[bench] workload {w.name}: {w.n_tri_submitted} triangles, {w.gen.n_cells} cells, "
        f"{n_sun} suns, N={w.map_n}, k={w.k}")
    ctx = pv3d.Context(0)
    sh = ctx.load_scene(w.scene)
    gh = ctx.define_generator(w.gen)
    t = timed_year(ctx, w, sh, gh, a.steps, a.warmup, a.route, a.tile, log)
    res = t["result"]

    if a.calib_copy_mb:
        nb = a.calib_copy_mb << 20
        src = torch.empty(nb // 4, dtype=torch.int32, device="cuda").fill_(7)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {nb} bytes done")

    sec_per_step = t["sec_per_step"]
    tests = w.n_samples * n_sun
    tris = w.n_tri_submitted * n_sun

    mat = None
    if not a.no_materialised and a.route != "materialised":
        # every 10th sun with the picture materialised in HBM: raster writes it, a second kernel reads it
        sub = w.sweep.subset(np.arange(0, n_sun, 10))
        ctx.profile_sample(1)
        ctx.profile_enable((1 << pv3d.STAGE["raster"]) | (1 << pv3d.STAGE["sample_test"]))
        torch.cuda.synchronize()
        m0 = time.perf_counter()
        mres = ctx.evaluate_device(sh, gh, w.gen, sub, w.map_n, w.k, separate_test=True)
        torch.cuda.synchronize()
        m1 = time.perf_counter()
        r_busy, r_suns = ctx.profile_busy(pv3d.STAGE["raster"])
        t_busy, _ = ctx.profile_busy(pv3d.STAGE["sample_test"])
        ctx.profile_enable(0)
        lean = ctx.evaluate_device(sh, gh, w.gen, sub, w.map_n, w.k)
        mb = 4 * w.map_n * w.map_n
        r_per = r_busy * 1e-3 / max(r_suns, 1)
        mat = {"suns": sub.n, "year_seconds": (m1 - m0) * (n_sun / sub.n), "identical_energy": bool(
                   np.array_equal(mres.energy.cpu().numpy(), lean.energy.cpu().numpy())),
               "raster_exclusive_us_per_sun": r_per * 1e6, "sample_test_exclusive_us_per_sun": t_busy * 1e3 / max(r_suns, 1),
               "raster_roofline": {"bound": "hbm", "achieved": mb / r_per / 1e9, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": mb / r_per / 1e9 / HBM_PEAK_GBS,
                                   "bytes_per_sun": mb}}
        log(f"[bench] materialised route: {sub.n} suns in {m1 - m0:.3f} s")
    line = {
        "metric": "sample\u00d7sun shadow tests/s + triangles rasterized/s; p50/p99 request latency",
        "value": tests / sec_per_step,
        "unit": "sample-sun tests/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * sec_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.note}; {n_sun} suns per step, per-sun path (groups of up to 32 suns "
                               f"per launch sequence)",
                   "route": a.route,
                   "triangles": w.n_tri_submitted, "cells": w.gen.n_cells, "samples_per_sun": w.n_samples,
                   "suns": n_sun, "map_n": w.map_n, "k": w.k},
        "triangles_per_s": tris / sec_per_step,
        "in_window_records_per_s": t["work"]["records"] / sec_per_step,
        "work_per_step": dict(t["work"], note="set-up records: triangles inside the window after culling, a "
                                              "triangle cut at the guard band once per piece"),
        "year_seconds": sec_per_step * (4379.0 / n_sun),
        "roofline": roofline_of(t, w, a.route),
        "route": a.route,
        "materialised_route": mat,
        "stage_busy_us_per_sun": {k: round(v["busy_us_per_sun"], 3) for k, v in t["stage_ms"].items()},
        "energy_loss": res.loss,
    }
    if not a.no_extra and a.route == "sparse" and a.suns <= 1:
        legs = set(LEGS) if a.extra_legs == "all" else set(a.extra_legs.split(","))
        if legs - set(LEGS):
            raise SystemExit(f"unknown legs {sorted(legs - set(LEGS))}; known: {', '.join(LEGS)}")
        rp = None
        if "row_plant" in legs or "batched" in legs:
            line["row_plant"], rp = row_plant_leg(ctx, log, max(1, min(a.steps, 10)))
        if "batched" in legs:
            w2, sh2, gh2, r2 = rp
            line["batched"] = batched_leg(ctx, w2, sh2, gh2, r2.energy.cpu().numpy(), r2.power.cpu().numpy(),
                                          line["row_plant"]["year_seconds"], log)
        if "c4" in legs:
            line["c4_batched"] = c4_leg(ctx, a.c4_every, log)
        if "trackers" in legs:
            line["trackers"] = tracker_leg(ctx, log)
        if "stadium" in legs:
            line["stadium"] = stadium_leg(ctx, log, a.stadium_every)
        if "electrical" in legs:
            line["electrical"] = electrical_leg(ctx, log)
        if "sky" in legs:
            line["sky"] = sky_leg(ctx, log)
        if "serving" in legs:
            # the serving loop in a context of its own, with the GPU to itself
            ctx.close()
            sctx = pv3d.Context(0)
            try:
                line["serving"] = serving_leg(sctx, log, a.serve_rate, a.serve_seconds, a.light_rate,
                                              a.light_seconds, a.sweep_requests)
            finally:
                sctx.close()
            cr = line["serving"]["configured_rate"]
            line["request_latency_ms"] = {"p50": cr["p50_ms"], "p99": cr["p99_ms"], "requests": cr["requests"],
                                          "offered_req_per_s": cr["offered_req_per_s"],
                                          "sustained_req_per_s": cr["sustained_req_per_s"],
                                          "stream": "the configured Poisson stream through the serving loop"}
    if not a.no_cpu:
        log("[bench] cpu oracle legs ...")
        full = w if a.suns <= 1 else workload(a.workload, 1)
        line["cpu_baseline"] = cpu_baseline(full, a.cpu_every)
        from paper_1410_5780_amd import workloads as W
        line["cpu_single_thread"] = {"c1_tiny": cpu_baseline(W.c1_tiny(d_poa=100.0), 1, threads=1),
                                     "c2_row_plant": cpu_baseline(W.c2_row_plant(), 100, threads=1)}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
