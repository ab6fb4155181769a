#!/usr/bin/env python3
"""Throughput of the hybrid force-free / PIC step on one MI355X.

Workload (the 4096^2 magnetosphere): 4096 x 4096 (r, theta) grid, r log-spaced
on [1, 100], light cylinder at r = 10, 4e8 e+- macro-particles (99% in a sech^2
current sheet of width 0.02 rad beyond the light cylinder drifting at
+-0.5c in phi, 1% at rest in the closed zone), open-dipole field with the
force-free domain on open lines below 0.85 Psi_pc, radiation reaction on,
sort every 8 steps.  Inputs are seeded and synthetic and resident in HBM
before the timed region.

A "step" is one full hybrid step: flux function + mask, (every 8th step)
stable sort, push + deposit of both species, fused field update with the
force-free current and E correction.  The headline is the FP32-mixed path;
the plain FP64 GPU path is timed on the same workload beside it.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec + cell-updates/sec at 4096² grid; FP32-mixed vs FP64 GPU"
HBM_PEAK_GBS = 8000.0
BYTES_PER_PARTICLE = {1: 48.0, 0: 80.0}   # algorithmic push+deposit bytes (read + write state)


# HBM counters of the dominant kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
# this script, scaled by the same counters for a plain copy); valid only for the
# kernel source they were taken from
COUNTER_FILE = {1: "profiles/k_push32_sheet4096_hbm_counters.txt",
                0: "profiles/k_push64_sheet4096_hbm_counters.txt"}
KERNEL_SOURCES = {1: ["paper_2406_14512_amd/csrc/k_push32.hip"],
                  0: ["paper_2406_14512_amd/csrc/k_push64.hip",
                      "paper_2406_14512_amd/csrc/gather.h"]}
# headers whose device code the push kernels compile in (the context struct
# of ffpic_internal.h is host-side bookkeeping, left out)
COMMON_SOURCES = ["paper_2406_14512_amd/csrc/device_common.h",
                  "paper_2406_14512_amd/csrc/sort_view.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(precision):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[precision] + COMMON_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision):
    """HBM bytes per launch from the committed counter summary, or None when
    the summary is absent or the kernel source has changed since."""
    path = os.path.join(ROOT, COUNTER_FILE[precision])
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash(precision):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Plain device-to-device copy of nbytes, timed with events: GB/s of
    read + written bytes (the measured ceiling beside the 8 TB/s spec)."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / s / 1e9


def make_sim(ffpic, w, precision):
    d = w.desc()
    d["precision"] = precision
    return ffpic.Sim(d, capacity=[w.n_per_species] * w.nspec)


def run_timed(ffpic, sim, steps, warmup, nspec, sort_interval, phase_steps=16):
    """Wall time of `steps` steps as the library runs them (whole sort cycles
    as replayed graphs), then the per-phase device times of `phase_steps`
    more steps launched one by one with events between the phases, then the
    push phase alone over the steps of one sort cycle that do not sort
    (their pushes are the plain kernel instance; a step that sorts also
    places the new order in its push)."""
    sim.step(warmup)
    sim.sync()
    alive0 = sum(sim.diagnostics(ffpic.DIAG_MOMENTS)["alive"])
    g0 = sim.graph_stats()
    sim.sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    t1 = time.perf_counter()
    g1 = sim.graph_stats()
    alive1 = sum(sim.diagnostics(ffpic.DIAG_MOMENTS)["alive"])
    sim.set_timing(True)
    sim.step(phase_steps)
    sim.sync()
    sim.set_timing(False)
    ph = sim.phase_times()
    wall = t1 - t0
    out = dict(wall=wall, phases=ph, phase_steps=phase_steps, alive0=alive0, alive1=alive1,
               graphs={"captured": g1[0] - g0[0], "launched": g1[1] - g0[1]})
    if sort_interval > 1:
        # to the step after the next sort, then the cycle's steps without one
        step = sim.diagnostics(ffpic.DIAG_MOMENTS)["step"]
        sim.step(1 + (-step) % sort_interval)
        sim.sync()
        n0 = sum(sim.diagnostics(ffpic.DIAG_MOMENTS)["alive"])
        sim.set_timing(True)
        sim.step(sort_interval - 1)
        sim.sync()
        sim.set_timing(False)
        n1 = sum(sim.diagnostics(ffpic.DIAG_MOMENTS)["alive"])
        out["plain"] = dict(push_ms=sim.phase_times()[2], steps=sort_interval - 1,
                            alive=0.5 * (n0 + n1))
    return out


def roofline(precision, res, steps, nspec, copy_gbs):
    # dominant kernel: the push + deposit kernel, one launch per species and
    # step; algorithmic bytes = state read + written per live particle.  The
    # launch time is that of the plain instance (steps without a sort) where
    # measured; the average over whole sort cycles, which includes the
    # pushes that also place the new order, is reported beside it
    n_avg = 0.5 * (res["alive0"] + res["alive1"])
    cycle_launch_s = res["phases"][2] / 1e3 / (res["phase_steps"] * nspec)
    avg_launch_s = cycle_launch_s
    timing = "push phase of whole sort cycles, placing pushes included"
    if "plain" in res:
        pl = res["plain"]
        n_avg = pl["alive"]
        avg_launch_s = pl["push_ms"] / 1e3 / (pl["steps"] * nspec)
        timing = (f"push phase of the {pl['steps']} steps of a sort cycle without a sort "
                  "(plain kernel instance), launched one by one")
    bytes_per_launch = BYTES_PER_PARTICLE[precision] * n_avg / nspec
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = measured_traffic(precision)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": traffic,
           "kernel": "k_push32" if precision == 1 else "k_push64",
           "achieved_basis": f"algorithmic bytes: {BYTES_PER_PARTICLE[precision]} B per live "
                             "particle (state read + written once)",
           "avg_launch_ms": round(avg_launch_s * 1e3, 4),
           "launch_timing": "HIP events on the push's stream: " + timing,
           "avg_launch_ms_cycle": round(cycle_launch_s * 1e3, 4),
           "bytes_per_launch": bytes_per_launch,
           "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
           "target_frac": 0.6}
    if traffic:
        # the counter-measured bytes over the same launch time
        out["traffic_gbs"] = round(traffic / avg_launch_s / 1e9, 1)
        out["traffic_frac"] = round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    valu = valu_per_particle(precision)
    if valu:
        # VALU issue against the SIMDs' capacity: one wave64 instruction per
        # SIMD every 4 clocks, 256 CUs x 4 SIMDs at 2.4 GHz
        issue = valu * (n_avg / nspec) / 64.0 * 4.0 / (256 * 4 * 2.4e9 * avg_launch_s)
        out["alu"] = {"valu_per_particle": valu, "issue_frac": round(issue, 3),
                      "source": SQ_FILE}
    return out


SQ_FILE = "profiles/push_sheet4096_sq_counters.txt"


def valu_per_particle(precision):
    """VALU wave instructions x 64 per particle of the push (steps without a
    sort), from the committed instruction-counter summary; None if absent."""
    path = os.path.join(ROOT, SQ_FILE)
    if not os.path.exists(path):
        return None
    want = "k_push32<false, 16, false>" if precision == 1 else "k_push64 :"
    block = False
    with open(path) as fh:
        for line in fh:
            if line.startswith("ffpic::"):
                block = want in line
            elif block and line.strip().startswith("SQ_INSTS_VALU") and "per particle" in line:
                try:
                    return float(line.split()[-3])
                except ValueError:
                    return None
    return None


def batch_run(ffpic, W, steps, warmup, scale, tune_ms=0.0):
    """The batched workload: 64 independent magnetospheres (grids 256^2 to
    1024^2, 1e6-1e7 particles each, FP32-mixed) stepped together through
    ffpic_batch_step; wall time around the batch step and a full sync."""
    ws = W.batched_systems(64, scale=scale)
    descs, caps = [], []
    for w in ws:
        d = w.desc()
        d["precision"] = w.precision
        descs.append(d)
        caps.append([w.n_per_species] * w.nspec)
    b = ffpic.Batch(descs, caps)
    for w, v in zip(ws, b.views):
        for s in range(w.nspec):
            for c in range(w.n_chunks()):
                v.load_particles(s, w.chunk(s, c))
    tuned = None
    cycle = 8
    if tune_ms > 0:
        # sort interval, push chunk and slab rows of every system, timed
        # from its state after loading (and restored)
        t = b.autotune(tune_ms)
        tuned = {}
        for key in ("sort_interval", "push_ppt", "field_rows"):
            vals = [x[key] for x in t]
            tuned[key] = {str(v): vals.count(v) for v in sorted(set(vals))}
        tuned["ms"] = round(sum(x["total_ms"] for x in t), 1)
        # the batch's graph mode, chosen by timing both from one checkpoint
        mode, gppt, mode_ms = b.graph_settings()
        tuned["graph_mode"] = mode
        tuned["grouped_push_ppt"] = gppt or "own"
        tuned["graph_mode_ms_per_step"] = {str(k): round(v, 3) for k, v in mode_ms.items()}
        cycle = 1
        for x in t:
            cycle = cycle * x["sort_interval"] // math.gcd(cycle, x["sort_interval"])
    # whole batch cycles (the least common multiple of the sort intervals):
    # the first (launched step by step after the tuner's restore, whose
    # sorts are full ones), two to capture the graphs of both buffer
    # parities, then the timed ones
    warmup = max(warmup, 3 * cycle)
    warmup = -(-warmup // cycle) * cycle
    steps = -(-steps // cycle) * cycle
    b.step(warmup)
    b.sync()
    alive = lambda: sum(sum(v.diagnostics(ffpic.DIAG_MOMENTS)["alive"]) for v in b.views)
    n0 = alive()
    g0 = b.graph_stats()
    grouped0 = b.grouped_launches()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t1 = time.perf_counter()
    g1 = b.graph_stats()
    n1 = alive()
    grouped = b.grouped_launches() - grouped0
    mode = b.get_graph()[0]
    # for comparison: the same steps in the other graph mode (two cycles to
    # capture its graphs first), then launched one by one
    other = b.GRAPH_PER_SYSTEM if mode == b.GRAPH_GROUPED else b.GRAPH_GROUPED
    b.set_graph(other)
    b.step(2 * cycle)
    b.sync()
    n2 = alive()
    t4 = time.perf_counter()
    b.step(steps)
    b.sync()
    t5 = time.perf_counter()
    n3 = alive()
    b.set_graph(False)
    t2 = time.perf_counter()
    b.step(steps)
    b.sync()
    t3 = time.perf_counter()
    cells = sum(w.nr * w.nth for w in ws)
    b.close()
    wall = t1 - t0
    return {"systems": len(ws), "particles": int(0.5 * (n0 + n1)), "cells": cells,
            "steps": steps, "ms_per_step": wall / steps * 1e3,
            "particle_steps_per_s": 0.5 * (n0 + n1) * steps / wall,
            "cell_updates_per_s": cells * steps / wall,
            "graphs": {"captured": g1[0] - g0[0], "launched": g1[1] - g0[1],
                       "grouped": grouped},
            "graph_mode": {1: "per-system", 2: "grouped"}.get(mode, "off"),
            "other_graph_mode_ms_per_step": (t5 - t4) / steps * 1e3,
            # later in the run, with fewer live particles: compare per particle
            "other_graph_mode_particle_steps_per_s": 0.5 * (n2 + n3) * steps / (t5 - t4),
            "eager_ms_per_step": (t3 - t2) / steps * 1e3, "tuned": tuned}


def host_cpu():
    """CPU model (/proc/cpuinfo), logical CPUs (nproc) and the threads a
    process is meant to use here (OMP_NUM_THREADS if set, else nproc)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        threads = int(os.environ.get("OMP_NUM_THREADS", "")) or nproc
    except ValueError:
        threads = nproc
    return model, nproc, min(threads, nproc)


def oracle_rate(w, n_sample, threads, steps=2):
    """Particle-steps/s and cell-updates/s of the oracle on a sample of the
    workload: the full grid and n_sample particles for `steps` steps; the
    push time per particle and the grid time per step are scaled to the
    workload's particle count."""
    import oracle
    o = oracle.Oracle(w.desc(), threads=threads)
    per = n_sample // w.nspec
    for s in range(w.nspec):
        o.load(s, w.particles(s, limit=per))
    n = sum(o.n(s) for s in range(w.nspec))
    t_push = t_grid = 0.0
    for k in range(steps):
        t0 = time.perf_counter()
        o.phases(oracle.PHASE_MASK | oracle.PHASE_KILL | (oracle.PHASE_SORT if k == 0 else 0))
        t1 = time.perf_counter()
        o.phases(oracle.PHASE_PUSH)
        t2 = time.perf_counter()
        o.phases(oracle.PHASE_FIELDS)
        t3 = time.perf_counter()
        t_push += t2 - t1
        t_grid += (t1 - t0) + (t3 - t2)
    o.close()
    per_particle = t_push / (steps * n)
    grid_step = t_grid / steps
    n_full = w.n_per_species * w.nspec
    step_full = grid_step + per_particle * n_full
    return {"value": n_full / step_full, "per_particle_ns": per_particle * 1e9,
            "grid_s": grid_step, "cell_updates_per_s": w.nr * w.nth / grid_step, "n": n}


def cpu_baseline(w, n_sample, steps=2):
    """The oracle (its OpenMP build: grid loops over rows, pushes over slot
    ranges) on the host's threads and on one thread."""
    import oracle
    oracle.build(force=False)
    model, nproc, threads = host_cpu()
    allc = oracle_rate(w, n_sample, threads, steps)
    one = oracle_rate(w, n_sample, 1, steps)
    return {"value": allc["value"], "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"{allc['n']} particles of the same workload on the full {w.nr}x{w.nth} grid, "
                       f"{steps} steps on {threads} threads; push time per particle "
                       f"({allc['per_particle_ns']:.1f} ns) and grid time per step "
                       f"({allc['grid_s']:.3f} s) scaled to {w.n_per_species * w.nspec:.3g} particles"),
            "cell_updates_per_s": allc["cell_updates_per_s"],
            "one_core": {"value": one["value"], "cell_updates_per_s": one["cell_updates_per_s"],
                         "per_particle_ns": round(one["per_particle_ns"], 1),
                         "grid_s": round(one["grid_s"], 3)},
            "cpu_model": model, "nproc": nproc}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--n-total", type=int, default=400_000_000)
    ap.add_argument("--grid", type=int, default=4096)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched workload (64 systems), reported under 'batch'")
    ap.add_argument("--batch-tune-ms", type=float, default=30000.0,
                    help="autotuning budget of the batch (all systems together), 0 = none")
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="particle-count scale of the batched workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain 1 GiB device copies (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, device="cuda", dtype=torch.float32)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 1 << 30, "copies": 3}), flush=True)
        return

    from paper_2406_14512_amd import ffpic
    from paper_2406_14512_amd import workloads as W

    w = W.sheet_4096(n_total=args.n_total)
    w.nr = w.nth = args.grid
    copy_gbs = copy_bandwidth()
    log(f"plain device copy: {copy_gbs:.0f} GB/s")
    precisions = [1] if args.no_fp64 else [1, 0]
    sims = {p: make_sim(ffpic, w, p) for p in precisions}
    t0 = time.perf_counter()
    for s in range(w.nspec):
        for c in range(w.n_chunks()):
            chunk = w.chunk(s, c)
            for p in precisions:
                sims[p].load_particles(s, chunk)
        log(f"loaded species {s}: {sims[1].n(s)} live particles "
            f"({time.perf_counter() - t0:.1f} s)")

    results = {}
    for p in precisions:
        log(f"timing {'FP32-mixed' if p == 1 else 'FP64'}: {args.warmup} warmup + {args.steps} steps")
        results[p] = run_timed(ffpic, sims[p], args.steps, args.warmup, w.nspec,
                               w.sort_interval)
        r = results[p]
        log(f"  {r['wall'] / args.steps * 1e3:.3f} ms/step ({r['graphs']['launched']} graph "
            f"launches), phases (ms/step) mask/sort/push/fields "
            + " ".join(f"{x / r['phase_steps']:.3f}" for x in r["phases"]))
        if "plain" in r:
            pl = r["plain"]
            log(f"  push launch without a sort: {pl['push_ms'] / (pl['steps'] * w.nspec):.4f} ms "
                f"(over {pl['steps']} steps)")
        if p == 0:
            sims[p].close()

    r = results[1]
    n_avg = 0.5 * (r["alive0"] + r["alive1"])
    ms = r["wall"] / args.steps * 1e3
    value = n_avg * args.steps / r["wall"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"sheet_{w.nr}: {w.nr}x{w.nth} (r, theta) grid, r in [1, 100], "
                                f"R_LC = 10, {w.n_per_species * w.nspec:.3g} e+- (99% sech^2 sheet "
                                "of width 0.02, 1% closed-zone background), open dipole with "
                                "force-free open lines, radiation reaction on, sort every 8 steps"),
                   "grid": f"{w.nr}x{w.nth}", "particles": int(n_avg),
                   "precision": "fp32-mixed", "sort_interval": w.sort_interval},
        "cell_updates_per_s": w.nr * w.nth * args.steps / r["wall"],
        "phase_ms_per_step": {k: round(v / r["phase_steps"], 4)
                              for k, v in zip(("mask", "sort", "push_deposit", "fields"), r["phases"])},
        "graphs": r["graphs"],
        "roofline": roofline(1, r, args.steps, w.nspec, copy_gbs),
    }
    if 0 in results:
        r64 = results[0]
        n64 = 0.5 * (r64["alive0"] + r64["alive1"])
        out["fp64"] = {"value": n64 * args.steps / r64["wall"], "unit": "particle-steps/s",
                       "ms_per_step": r64["wall"] / args.steps * 1e3,
                       "cell_updates_per_s": w.nr * w.nth * args.steps / r64["wall"],
                       "phase_ms_per_step": {k: round(v / r64["phase_steps"], 4) for k, v in
                                             zip(("mask", "sort", "push_deposit", "fields"),
                                                 r64["phases"])},
                       "roofline": roofline(0, r64, args.steps, w.nspec, copy_gbs)}
        out["fp32_over_fp64"] = out["value"] / out["fp64"]["value"]
    sims[1].close()
    if not args.no_batch:
        log("timing the batched workload (64 systems)")
        out["batch"] = batch_run(ffpic, W, args.steps, args.warmup, args.batch_scale,
                                 args.batch_tune_ms)
        bo = out["batch"]
        log(f"  batch: {bo['ms_per_step']:.3f} ms/step, "
            f"{bo['particle_steps_per_s']:.3e} particle-steps/s, graphs {bo['graphs']}; "
            f"mode {bo['graph_mode']}, other mode {bo['other_graph_mode_ms_per_step']:.3f} ms/step "
            f"({bo['other_graph_mode_particle_steps_per_s']:.3e} particle-steps/s), "
            f"one by one {bo['eager_ms_per_step']:.3f} ms/step")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
