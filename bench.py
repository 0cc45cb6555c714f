#!/usr/bin/env python
"""Throughput of the particle hot path on one MI355X.

Workload (one "step" = one pass of advect + locate + re-sort over the store):
64^3 uniform hex mesh on the unit cube, Q2 velocity = curl of a random
8-mode Fourier vector potential (normalised to max nodal speed 1), 20
particles per cell (5,242,880), FP64 locations, FP32 field evaluation,
3 FP32 properties, classical RK4, dt = 0.5/64 (CFL 0.5).

Prints ONE JSON line: particle-steps/s over exactly --steps timed steps
(live particles summed over the steps), the HBM roofline of the dominant
kernel (HIP events on the library's stream), the FP64 CPU oracle timed on a
bounded sample, and extra measurements (adjoint/forward time ratio on the
32^3 adjoint workload, batched vs per-problem, per-kernel times).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
REPO = os.path.dirname(os.path.abspath(__file__))
# byte counters of the dominant kernel, taken by --summarize-traffic from two rocprofv3 --pmc runs
TRAFFIC_FILE = os.path.join(REPO, "profiles", "traffic_gather_advect_uniform64_rk4_f32.json")
DOMINANT_KERNEL = "k_advect_blk<3, 4, float, 4, 4, 4, true, false, false>"
ADJOINT_TRAFFIC_FILE = os.path.join(REPO, "profiles", "traffic_adjoint_blk_adjoint32_rk4.json")
ADJOINT_KERNEL = "k_adjoint_blk<3, 4, 4, 2, 2>"
COPY_BYTES = 64 * 1024 * 1024 * 4          # the calibration copy below: 256 MiB read, 256 MiB written


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# algorithmic bytes per particle and launch (see the design notes): d = 3,
# 3 float properties, int32 cell/key/src, uint32 id
def source_digest():
    """sha256 over the library sources: byte counters are valid only for the code they were taken on."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(REPO, "paper_1612_03369_amd", "csrc")
    for name in sorted(os.listdir(src)):
        with open(os.path.join(src, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(REPO, "include", "pic.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def _pmc_per_dispatch(run_dir, counter):
    """{kernel name: [(counter value of one dispatch in KiB, duration ns), ...]} of a rocpd database."""
    import glob
    import sqlite3
    out = {}
    for db in glob.glob(os.path.join(run_dir, "**", "*results.db"), recursive=True):
        con = sqlite3.connect(db)
        q = ("select kernel_name, dispatch_id, sum(value), avg(duration) from counters_collection "
             "where counter_name = ? group by dispatch_id")
        for name, _, total, dur in con.execute(q, (counter,)):
            out.setdefault(name, []).append((total, dur))
        con.close()
    return out


def _copy_kib(per_kernel):
    """Counter value of the 256 MiB copies: median over the copy dispatches within half of the largest."""
    import statistics
    vals = [v for k, lst in per_kernel.items() if "copyBuffer" in k for v, _ in lst]
    top = max(vals)
    return statistics.median(v for v in vals if v >= 0.5 * top)


def summarize_traffic(fetch_dir, write_dir, command, kernel=DOMINANT_KERNEL):
    """HBM bytes per launch of one kernel (the dominant one by default) from FETCH_SIZE and WRITE_SIZE runs, each
    scaled by what the same counter reads for the 256 MiB device copy of the same run."""
    fetch = _pmc_per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _pmc_per_dispatch(write_dir, "WRITE_SIZE")
    dom = [k for k in fetch if kernel in k]
    if len(dom) != 1:
        raise SystemExit(f"dominant kernel not found once in {fetch_dir}: {dom}")
    dom = dom[0]
    f_n = len(fetch[dom])
    f_kib = sum(v for v, _ in fetch[dom]) / f_n
    f_dur = sum(d for _, d in fetch[dom]) / f_n
    w_kib = sum(v for v, _ in write[dom]) / len(write[dom])
    cp = "__amd_rocclr_copyBuffer"
    cf_kib = _copy_kib(fetch)
    cw_kib = _copy_kib(write)
    f_scale = COPY_BYTES / (cf_kib * 1024.0)
    w_scale = COPY_BYTES / (cw_kib * 1024.0)
    rec = {"kernel": dom, "dispatches": f_n, "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
           "copy_kernel": cp, "copy_bytes_each_way": COPY_BYTES, "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "traffic_bytes_per_launch": f_kib * 1024.0 * f_scale + w_kib * 1024.0 * w_scale,
           "mean_duration_ns_under_counters": f_dur, "source_sha256": source_digest(), "command": command}
    print(json.dumps(rec, indent=1))


def summarize_trace(trace_dir, title, command):
    """Per-kernel call count, total and mean duration of a rocprofv3 --kernel-trace --stats run."""
    import glob
    import sqlite3
    print(f"# rocprofv3 kernel-trace summary: {title}")
    print(f"# command: {command}")
    print("# columns: kernel, calls, total_us, average_us, percent")
    for db in glob.glob(os.path.join(trace_dir, "**", "*results.db"), recursive=True):
        con = sqlite3.connect(db)
        for name, n, tot, avg, pct in con.execute(
                "select name, total_calls, total_duration, average, percentage from top_kernels"):
            print(f"{name}\t{n}\t{tot:.1f}\t{avg:.3f}\t{pct:.2f}")
        con.close()


def summarize_counters(run_dir, title, command):
    """Per-kernel averages per dispatch of the SQ counters of a rocprofv3 --pmc run (the re-sort and advect
    kernels), with the wait fraction SQ_WAIT_ANY / SQ_WAVE_CYCLES and the VALU issue fraction
    SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES."""
    import glob
    import sqlite3
    acc = {}
    for db in glob.glob(os.path.join(run_dir, "**", "*results.db"), recursive=True):
        con = sqlite3.connect(db)
        q = ("select kernel_name, counter_name, dispatch_id, sum(value), avg(duration) from counters_collection "
             "group by kernel_name, counter_name, dispatch_id")
        for name, counter, _, total, dur in con.execute(q):
            k = acc.setdefault(name, {})
            k.setdefault(counter, []).append(total)
            k.setdefault("duration_ns", []).append(dur)
        con.close()
    print(f"# rocprofv3 counter summary: {title}")
    print(f"# command: {command}")
    print("# per kernel: dispatches, mean duration, mean of each counter per dispatch, wait and VALU-issue fractions")
    keep = ("k_advect_blk", "k_place", "k_fix", "k_scan", "k_gather", "k_adjoint_blk")
    for name in sorted(acc, key=lambda n: -sum(acc[n]["duration_ns"])):
        if not any(k in name for k in keep):
            continue
        c = {k: sum(v) / len(v) for k, v in acc[name].items()}
        n = max(len(v) for k, v in acc[name].items() if k != "duration_ns")
        print(f"{name.split('(')[0]}\tdispatches {n}\tduration_us {c.pop('duration_ns') / 1e3:.1f}")
        for k in sorted(c):
            print(f"    {k} {c[k]:.0f}")
        if c.get("SQ_WAVE_CYCLES"):
            if "SQ_WAIT_ANY" in c:
                print(f"    wait_fraction {c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:.3f}")
            if "SQ_ACTIVE_INST_VALU" in c:
                print(f"    valu_issue_fraction {c['SQ_ACTIVE_INST_VALU'] / c['SQ_WAVE_CYCLES']:.3f}")
        for prec in ("F32", "F64"):
            names = [f"SQ_INSTS_VALU_{op}_{prec}" for op in ("FMA", "MUL", "ADD")]
            if all(n in c for n in names):
                # wave instructions x 64 lanes: an upper bound (partly masked waves count in full)
                flop = 64.0 * (2 * c[names[0]] + c[names[1]] + c[names[2]])
                dur = sum(acc[name]["duration_ns"]) / len(acc[name]["duration_ns"])
                print(f"    {prec.lower()}_flop_upper {flop:.4g}  ({flop / dur / 1e3:.2f} TFLOP/s over the mean duration)")


def measured_traffic(path=TRAFFIC_FILE):
    """Bytes per launch of a kernel (the dominant one by default) from its committed counter summary, or None when
    the summary is missing or was taken on other sources."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, "no counter summary"
    if rec.get("source_sha256") != source_digest():
        return None, "counter summary taken on other sources"
    return rec["traffic_bytes_per_launch"], os.path.relpath(path, REPO)


def bytes_per_particle(kernel, dim=3, prop_bytes=12):
    """Bytes a kernel must move per particle as built for uniform meshes: the reference coordinates and the cell
    are derived from the position and the block row (not read), and only the final gather stores them."""
    x = 8 * dim
    return {
        "advect": x + (x + 4),                                          # r: x; w: x, key
        "place": 4 + 4,                                                 # r: key; w: src
        "fix": 0,
        "gather": (4 + 4 + x + 4 + prop_bytes) + (x + x + 4 + 4 + prop_bytes),  # r: src, key, x, id, props
        "gather_advect": (4 + x + 4 + prop_bytes) + (x + 4 + prop_bytes + 4),   # r: src, x, id, props; w: + key
    }[kernel]


# The same per particle-step in the paper-faithful layout (x and x-hat stored and read every step, one scatter
# pass over the whole state): 48 + 48 + 4 written by the advect, 4 + 64 + 64 by the scatter, the key read, about
# 5 B of field and 0.4 B of counts per particle at 64^3 -- about 237 B, the model the 64^3 gate is priced on.
PAPER_STEP_BYTES = 237.0


KERNELS = ("advect", "gather_advect", "scan_reduce", "scan_down", "place", "fix", "gather", "flip")


def run_main(args):
    import numpy as np
    import torch

    from paper_1612_03369_amd import _lib as L
    from paper_1612_03369_amd import inputs as I
    from paper_1612_03369_amd.api import Problem

    torch.cuda.init()
    dev = torch.device("cuda", 0)
    cfg = I.config2(eval_f32=True)
    mesh = cfg["mesh"]
    n0 = cfg["xr"].shape[1]
    log(f"[bench] workload {cfg['name']}: {mesh.n_cells} cells, {n0} particles")
    p = Problem(0)
    p.mesh_uniform(3, mesh.n)
    p.set_velocity(cfg["U"])
    p.allocate(n0, n_prop=3, prop_dtype="float32")
    dt = cfg["dt"]

    def reseed():
        p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"])
        p.stats_reset()
        torch.cuda.synchronize()

    # warmup
    reseed()
    if args.warmup:
        p.advance(dt, args.warmup, L.PIC_RK4, L.PIC_F32)
    torch.cuda.synchronize()
    # timed region: exactly K steps from the seeded state
    reseed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.advance(dt, args.steps, L.PIC_RK4, L.PIC_F32)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = p.stats()
    elapsed = t1 - t0
    psteps = st["particle_steps"]
    value = psteps / elapsed
    log(f"[bench] {args.steps} steps in {elapsed * 1e3:.2f} ms, {psteps} particle-steps, live {st['live']}, "
        f"lost {st['lost']}, moved/step {st['moved'] / max(1, args.steps):.0f}")

    # per-kernel durations with HIP events on the library's stream (same K steps)
    reseed()
    p.profile(True)
    p.advance(dt, args.steps, L.PIC_RK4, L.PIC_F32)
    kernels = {}
    for k in KERNELS:
        ms, n = p.profile_read(k)
        kernels[k] = {"total_ms": ms, "launches": n, "avg_us": 1e3 * ms / max(n, 1)}
    p.profile(False)
    st2 = p.stats()
    dom = max(("advect", "gather_advect", "gather", "place"), key=lambda k: kernels[k]["total_ms"])
    avg_particles = st2["particle_steps"] / max(1, st2["steps"])
    n_nodes = int(np.prod(mesh.node_shape))
    field_bytes = n_nodes * 3 * 4                     # Q2 nodal field (3 f32 components), read once per step
    bytes_launch = avg_particles * bytes_per_particle(dom) + (field_bytes if "advect" in dom else 0)
    achieved = bytes_launch / (kernels[dom]["avg_us"] * 1e-6) / 1e9
    step_bytes = avg_particles * (bytes_per_particle("gather_advect") + bytes_per_particle("place")) + field_bytes
    step_ms = 1e3 * elapsed / args.steps
    traffic, traffic_src = measured_traffic()
    line = {
        "metric": "particle-steps/s (advect+locate+sort)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 locations / f32 field evaluation",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "cells": mesh.n_cells, "particles": n0, "scheme": "rk4",
                   "dt": dt, "eval": "f32", "n_prop": 3, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic if dom == "gather_advect" else None,
                     "traffic_source": traffic_src, "bytes_per_launch": bytes_launch,
                     "bytes_per_particle": bytes_per_particle(dom),
                     "bytes_model": "as built: x-hat and cell derived from x and the block row, stored only by the "
                                    "final gather; plus 12 B per Q2 node of field",
                     "avg_launch_us": kernels[dom]["avg_us"]},
        "step_hbm_frac": step_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_bytes_per_particle": step_bytes / avg_particles,
        "step_hbm_frac_paper_model": avg_particles * PAPER_STEP_BYTES / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernels": kernels,
        "stats": st,
    }

    # plain copy kernel of known size (calibrates the byte counters of a profiled run)
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    line["copy_gbs"] = 2 * a.numel() * 4 * 10 / (time.perf_counter() - t) / 1e9
    # the dominant kernel's algorithmic rate against what a plain device copy reaches on this GPU
    line["roofline"]["frac_of_copy"] = line["roofline"]["achieved"] / line["copy_gbs"]
    del a, b
    p.close()

    if args.extras:
        extras = {}
        if "adjoint" in args.extras:
            extras["adjoint"] = bench_adjoint(args)
        if "batch" in args.extras:
            extras["batch"] = bench_batch(args)
        if "octree" in args.extras:
            extras["octree"] = bench_octree(args)
        if "odes" in args.extras:
            extras["odes"] = bench_odes(args)
        if "time_field" in args.extras:
            extras["time_field"] = bench_time_field(args)
        if "interp" in args.extras:
            extras["interp"] = bench_interp(args)
        line["extras"] = extras

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args)
    return line


def bench_adjoint(args):
    """Adjoint/forward time ratio on 32^3, 32 per cell (1,048,576 particles), RK4 x 50, checkpoints every 10."""
    import torch

    from paper_1612_03369_amd import _lib as L
    from paper_1612_03369_amd import inputs as I
    from paper_1612_03369_amd.api import Problem

    cfg = I.config5()
    mesh = cfg["mesh"]
    n0 = cfg["xr"].shape[1]
    p = Problem(0)
    p.mesh_uniform(3, mesh.n)
    p.set_velocity(cfg["U"])
    p.allocate(n0, n_prop=0)
    ws = p.adjoint_workspace(cfg["steps"], cfg["ckpt_every"])
    dt, ns = cfg["dt"], cfg["steps"]

    def timed(fn, reps=3):
        best = []
        for _ in range(reps):
            p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"])
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best.append(time.perf_counter() - t)
        return sorted(best)[len(best) // 2]

    fwd = timed(lambda: p.advance(dt, ns, L.PIC_RK4, L.PIC_F64))
    dl = torch.ones((3, n0), dtype=torch.float64, device=p.device) * 1e-3
    dU = torch.zeros((3, mesh.n_nodes), dtype=torch.float64, device=p.device)

    def fwd_bwd():
        p.advance_checkpointed(dt, ns, L.PIC_RK4, cfg["ckpt_every"], ws)
        p.adjoint(dl, ws, dU)

    both = timed(fwd_bwd)
    # the reverse-step kernel alone: its mean launch time from the library's HIP events, priced at the bytes it
    # must move (per particle-step: x, cell, dst and lambda' read, lambda written -- the first stage point's
    # reference coordinates come from x and the cell; per launch: the field's nodes and dU read and written once)
    p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"])
    p.profile(True)
    fwd_bwd()
    torch.cuda.synchronize()
    ms, cnt = p.profile_read("adjoint_step")
    p.profile(False)
    per_particle = 8 * 3 + 4 + 4 + 8 * 3 + 8 * 3
    per_node = 32 + 2 * 8 * 3
    bytes_launch = n0 * per_particle + mesh.n_nodes * per_node
    avg_us = 1e3 * ms / max(cnt, 1)
    traffic, traffic_src = measured_traffic(ADJOINT_TRAFFIC_FILE)
    r = {"workload": cfg["name"], "particles": n0, "forward_ms": fwd * 1e3, "forward_plus_adjoint_ms": both * 1e3,
         "ratio": both / fwd,
         "reverse_kernel": {"name": "k_adjoint_blk", "launches": cnt, "avg_launch_us": avg_us,
                            "bytes_per_launch": bytes_launch, "achieved_gbs": bytes_launch / (avg_us * 1e3),
                            "hbm_frac": bytes_launch / (avg_us * 1e-6) / 8e12,
                            "bytes_model": f"{per_particle} B per particle-step + {per_node} B per node",
                            "traffic": traffic, "traffic_source": traffic_src}}
    log(f"[bench] adjoint: forward {fwd * 1e3:.1f} ms, checkpointed forward + adjoint {both * 1e3:.1f} ms; "
        f"reverse step {avg_us:.0f} us x {cnt} ({bytes_launch / (avg_us * 1e3):.0f} GB/s of algorithmic bytes)")
    p.close()
    return r


def bench_batch(args):
    """64 problems stepped from one graph vs the same problems one by one (20 steps each)."""
    import torch

    from paper_1612_03369_amd import _lib as L
    from paper_1612_03369_amd import inputs as I
    from paper_1612_03369_amd.api import Batch, Problem

    cfgs = I.config4()
    probs = []
    for c in cfgs:
        m = c["mesh"]
        q = Problem(0)
        q.mesh_uniform(m.dim, m.n[: m.dim])
        q.set_velocity(c["U"])
        q.allocate(c["xr"].shape[1], n_prop=1)
        probs.append(q)

    def reseed():
        for q, c in zip(probs, cfgs):
            q.seed_reference(c["counts"], c["xr"], c["ids"])
            q.stats_reset()
        torch.cuda.synchronize()

    total = sum(c["xr"].shape[1] for c in cfgs)
    reseed()
    t = time.perf_counter()
    for q, c in zip(probs, cfgs):
        q.advance(c["dt"], c["steps"], c["scheme"], L.PIC_F64)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t
    ps_single = sum(q.stats()["particle_steps"] for q in probs)
    bt = Batch(probs)
    dts, schemes = [c["dt"] for c in cfgs], [c["scheme"] for c in cfgs]

    def run_batch():
        reseed()
        bt.advance(dts, schemes, 20)                 # graph build + warm
        torch.cuda.synchronize()
        reseed()
        t = time.perf_counter()
        bt.advance(dts, schemes, 20)
        torch.cuda.synchronize()
        return time.perf_counter() - t, sum(q.stats()["particle_steps"] for q in probs)

    t_default, _ = run_batch()                       # default cell-block shapes
    reseed()
    t = time.perf_counter()
    tuned = bt.tune(dts, schemes, trials=3)          # the library's autotuner
    t_tune = time.perf_counter() - t
    t_batch, ps_batch = run_batch()
    bt.close()
    for q in probs:
        q.close()
    log(f"[bench] batch: {len(cfgs)} problems, {total} particles: per-problem {t_single * 1e3:.1f} ms, "
        f"batched graph {t_default * 1e3:.1f} ms (default shapes), {t_batch * 1e3:.1f} ms (tuned {tuned['variants']}, "
        f"tuning {t_tune * 1e3:.0f} ms)")
    return {"problems": len(cfgs), "particles": total, "per_problem_ms": t_single * 1e3, "batched_ms": t_batch * 1e3,
            "batched_default_shapes_ms": t_default * 1e3, "tuning_ms": t_tune * 1e3,
            "tuned_variants": tuned["variants"], "tuned_times_ms": tuned["times_ms"],
            "speedup": t_single / t_batch, "particle_steps_per_s": ps_batch / t_batch,
            "per_problem_particle_steps_per_s": ps_single / t_single}


def bench_octree(args):
    """Shell-refined octree (1,005,152 leaves), 5..80 per cell, RK2 x 50 with population [8, 64] each step,
    linear least squares at the end; FP32 evaluation, FP64 locations."""
    import numpy as np
    import torch

    from paper_1612_03369_amd import _lib as L
    from paper_1612_03369_amd import inputs as I
    from paper_1612_03369_amd.api import Problem

    cfg = I.config3()
    t0 = time.perf_counter()
    p = Problem(0)
    p.mesh_octree(cfg["level"], cfg["anchor"], cfg["max_level"])
    xyz, _ = p.q2_nodes()
    U = I.normalise_nodal(I.sample_nodes(cfg["field"].velocity, xyz))
    p.set_velocity(U)
    n0 = cfg["xr"].shape[1]
    cap = int(n0 * 1.1) + 1_000_000
    p.allocate(cap, n_prop=cfg["n_prop"], prop_dtype="float64")
    log(f"[bench] octree: {p.n_cells} leaves, {p.n_nodes} nodes, {n0} particles, set-up {time.perf_counter() - t0:.1f} s")
    dt = cfg["dt"]
    steps = min(cfg["steps"], max(args.steps, 1))

    def run(timed):
        p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"])
        p.stats_reset()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * steps + 1)]
        ps = []
        torch.cuda.synchronize()
        for s in range(steps):
            ev[3 * s].record()
            p.advance(dt, 1, L.PIC_RK2, L.PIC_F32)
            ev[3 * s + 1].record()
            p.population(cfg["pop_min"], cfg["pop_max"], cfg["pop_seed"], s)
            ev[3 * s + 2].record()
        coef, xbar, cnt = p.interpolate(L.PIC_INTERP_LINEAR_LS)
        ev[3 * steps].record()
        torch.cuda.synchronize()
        adv = sum(ev[3 * s].elapsed_time(ev[3 * s + 1]) for s in range(steps))
        pop = sum(ev[3 * s + 1].elapsed_time(ev[3 * s + 2]) for s in range(steps))
        lls = ev[3 * steps - 1].elapsed_time(ev[3 * steps])
        return adv, pop, lls, cnt

    run(False)                                       # warm-up (first touch of every buffer)
    adv, pop, lls, cnt = run(True)
    st = p.stats()
    c = cnt.cpu().numpy()
    r = {"workload": cfg["name"], "leaves": p.n_cells, "particles_initial": n0, "steps": steps, "dt": dt,
         "eval": "f32", "advect_sort_ms": adv, "population_ms": pop, "lls_ms": lls,
         "particle_steps_per_s": st["particle_steps"] / (adv * 1e-3),
         "live_final": st["live"], "added": st["added"], "deleted": st["deleted"], "lost": st["lost"],
         "moved": st["moved"], "first_try": st["first_try"], "fallback": st["fallback"],
         "cells_min_max": [int(c.min()), int(c.max())]}
    log(f"[bench] octree: {steps} steps: advect+sort {adv:.1f} ms ({r['particle_steps_per_s']:.3e} p-s/s), "
        f"population {pop:.1f} ms, LLS {lls:.2f} ms, live {st['live']}")
    # mesh coarsening and refinement (Sec. 2.5): every finest sibling group merged, then split again
    cl, ca = I.coarsen_finest(cfg["level"], cfg["anchor"], cfg["max_level"])
    q = Problem(0)
    q.mesh_octree(cl, ca, cfg["max_level"])
    q.set_velocity(np.zeros((3, q.n_nodes)))
    q.allocate(cap, n_prop=cfg["n_prop"], prop_dtype="float64")

    def timed_transfer(dst, src):
        torch.cuda.synchronize()
        t = time.perf_counter()
        dst.transfer_from(src)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t)

    timed_transfer(q, p)                             # warm-up
    r["coarse_leaves"] = int(cl.size)
    r["transfer_coarsen_ms"] = timed_transfer(q, p)
    r["transfer_refine_ms"] = timed_transfer(p, q)
    r["transferred"] = p.stats()["live"]
    log(f"[bench] octree: transfer of {r['transferred']} particles to the coarsened mesh ({cl.size} leaves) "
        f"{r['transfer_coarsen_ms']:.1f} ms, back to the fine mesh {r['transfer_refine_ms']:.1f} ms")
    q.close()
    p.close()
    return r


def bench_odes(args):
    """The 64^3 RK4 workload with the damage and deformation-gradient equations (Sec. 2.6) integrated
    with the positions: 1 + 9 double-precision properties per particle, same K fused steps."""
    import numpy as np
    import torch

    from paper_1612_03369_amd import _lib as L
    from paper_1612_03369_amd import inputs as I
    from paper_1612_03369_amd.api import Problem

    cfg = I.config2(eval_f32=True)
    mesh = cfg["mesh"]
    n0 = cfg["xr"].shape[1]
    p = Problem(0)
    p.mesh_uniform(3, mesh.n)
    p.set_velocity(cfg["U"])
    p.allocate(n0, n_prop=10, prop_dtype="float64")
    P0 = np.zeros((10, n0))
    P0[[1, 5, 9]] = 1.0                              # d = 0, F = I
    P0 = torch.as_tensor(P0).to(p.device)
    dt = cfg["dt"]

    def run():
        p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"], prop=P0)
        p.set_property_odes(0, 1, 1.0, 0.5)
        p.stats_reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        p.advance(dt, args.steps, L.PIC_RK4, L.PIC_F32)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    run()
    el = run()
    st = p.stats()
    p.profile(True)
    run()
    ms, n = p.profile_read("gather_advect")
    p.profile(False)
    g = p.current()
    F = g["prop"][1:10]
    detF = torch.linalg.det(F.T.reshape(-1, 3, 3)).double()
    r = {"workload": cfg["name"] + "+damage+F", "particles": n0, "n_prop": 10, "steps": args.steps,
         "ms_per_step": 1e3 * el / args.steps, "particle_steps_per_s": st["particle_steps"] / el,
         "gather_advect_avg_us": 1e3 * ms / max(n, 1),
         "detF_min_max": [float(detF.min()), float(detF.max())],
         "damage_max": float(g["prop"][0].max())}
    log(f"[bench] odes: {r['ms_per_step']:.3f} ms/step, {r['particle_steps_per_s']:.3e} p-s/s, "
        f"gather_advect {r['gather_advect_avg_us']:.0f} us, det F in {r['detF_min_max']}")
    p.close()
    return r


def bench_time_field(args):
    """The 64^3 RK4 workload in a field that changes in time: u^n and u^{n+1} evaluated at every stage,
    four particle steps per field step, the next field loaded (shift) after each field step."""
    import torch

    from paper_1612_03369_amd import _lib as L
    from paper_1612_03369_amd import inputs as I
    from paper_1612_03369_amd.api import Problem

    cfg = I.config2(eval_f32=True)
    mesh = cfg["mesh"]
    n0 = cfg["xr"].shape[1]
    nodes = I.uniform_q2_nodes(mesh)
    fields = [torch.as_tensor(I.normalise_nodal(I.sample_nodes(I.FourierField(3, seed=2 + k).velocity, nodes))).cuda()
              for k in range(3)]
    p = Problem(0)
    p.mesh_uniform(3, mesh.n)
    p.set_velocity(fields[0])
    p.allocate(n0, n_prop=3, prop_dtype="float32")
    dt, sub = cfg["dt"], 4
    n_field = max(1, args.steps // sub)

    def run(timed_shift):
        p.set_velocity(fields[0])
        p.set_velocity_end(fields[1], sub * dt)
        p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"])
        p.stats_reset()
        torch.cuda.synchronize()
        t_adv = t_shift = 0.0
        for k in range(n_field):
            t = time.perf_counter()
            p.advance(dt, sub, L.PIC_RK4, L.PIC_F32)
            torch.cuda.synchronize()
            t_adv += time.perf_counter() - t
            t = time.perf_counter()
            p.shift_velocity(fields[(k + 2) % 3], sub * dt)
            torch.cuda.synchronize()
            t_shift += time.perf_counter() - t
        return t_adv, t_shift

    run(False)
    t_adv, t_shift = run(True)
    st = p.stats()
    steps = n_field * sub
    r = {"workload": cfg["name"] + "+time-interpolated", "particles": n0, "steps": steps, "substeps": sub,
         "ms_per_step": 1e3 * t_adv / steps, "shift_ms": 1e3 * t_shift / n_field,
         "particle_steps_per_s": st["particle_steps"] / t_adv}
    log(f"[bench] time field: {r['ms_per_step']:.3f} ms/step, {r['particle_steps_per_s']:.3e} p-s/s, "
        f"shift {r['shift_ms']:.2f} ms per field step")
    p.close()
    return r


def bench_interp(args):
    """On the 64^3 store (5,242,880 particles, three f64 properties): every interpolator, with the
    eight Gauss points of Q1 plus the centre as evaluation points; and Metropolis-Hastings generation
    of the same 20 particles per cell (J = 10) from a varying density."""
    import math

    import numpy as np
    import torch

    from paper_1612_03369_amd import _lib as L
    from paper_1612_03369_amd import inputs as I
    from paper_1612_03369_amd.api import Problem

    cfg = I.config2()
    mesh = cfg["mesh"]
    n0 = cfg["xr"].shape[1]
    p = Problem(0)
    p.mesh_uniform(3, mesh.n)
    p.set_velocity(cfg["U"])
    p.allocate(n0, n_prop=3, prop_dtype="float64")
    P = torch.rand((3, n0), dtype=torch.float64, device=p.device) + 0.5
    p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"], prop=P)
    g = 1 / math.sqrt(3)
    pts = np.array(list(np.ndindex(2, 2, 2)), float).T
    q = np.concatenate([0.5 + (pts - 0.5) * g, np.full((3, 1), 0.5)], axis=1)
    r = {"workload": cfg["name"] + " store", "particles": n0, "eval_points": q.shape[1]}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / reps

    for name, kind in (("arithmetic", L.PIC_INTERP_CELL_AVERAGE), ("geometric", L.PIC_INTERP_GEOMETRIC_AVERAGE),
                       ("harmonic", L.PIC_INTERP_HARMONIC_AVERAGE), ("linear_ls", L.PIC_INTERP_LINEAR_LS)):
        r[name + "_ms"] = timed(lambda: p.interpolate(kind))
    for name, kind in (("nearest", L.PIC_INTERP_NEAREST), ("inv_distance", L.PIC_INTERP_INV_DISTANCE),
                       ("shape_weighted", L.PIC_INTERP_SHAPE_WEIGHTED)):
        r[name + "_ms"] = timed(lambda: p.interpolate_points(kind, q))
    nodes = I.uniform_q2_nodes(mesh)
    rho = 1.0 + 0.5 * np.sin(6.0 * nodes[0]) * np.cos(4.0 * nodes[1]) + 0.3 * nodes[2]
    lr = []
    r["mh_seed_ms"] = timed(lambda: lr.append(p.seed_mh(cfg["counts"], rho, 10, 7)), reps=3)
    r["mh_longest_run"] = lr[-1]
    log(f"[bench] interpolators: " + ", ".join(f"{k[:-3]} {v:.2f} ms" for k, v in r.items() if k.endswith("_ms")))
    p.close()
    return r


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """FP64 oracle on the host cores: a bounded sample of the same workload (the whole 64^3 store, its
    first steps: one single-threaded, --cpu-steps on all the cores the process may use), median of 3
    runs each (the paper averages 3 runs)."""
    import statistics

    from oracle import oracle as O
    from paper_1612_03369_amd import inputs as I

    cfg = I.config2(eval_f32=True)
    om = O.OracleMesh.uniform(cfg["mesh"])
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp_env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    all_threads = min(avail, omp_env) if omp_env else avail

    def one_run(threads, steps):
        used = O.set_threads(threads)
        st = O.seed(om, cfg["counts"], cfg["xr"], cfg["ids"], 3)
        s = O.Stats()
        psteps = 0
        t = time.perf_counter()
        for _ in range(steps):
            psteps += st.n
            O.step(om, cfg["U"], cfg["dt"], 4, st, s)
        return psteps / (time.perf_counter() - t), used

    out = {}
    for label, threads, steps in (("single", 1, 1), ("all", all_threads, args.cpu_steps)):
        runs = [one_run(threads, steps) for _ in range(3)]
        out[label] = (statistics.median(r[0] for r in runs), runs[0][1], steps)
    O.set_threads(all_threads)
    log(f"[bench] cpu oracle: single thread {out['single'][0]:.3e} p-s/s, {out['all'][1]} threads "
        f"{out['all'][0]:.3e} p-s/s ({_cpu_model()}, {avail} cores available)")
    return {"value": out["all"][0], "unit": "particle-steps/s", "cores": out["all"][1], "kind": "oracle",
            "sample": f"the 64^3 RK4 store ({cfg['xr'].shape[1]} particles): first {out['all'][2]} steps on all "
                      f"cores, first {out['single'][2]} single-threaded, FP64 evaluation, median of 3 runs each",
            "single_thread_value": out["single"][0], "cpu_model": _cpu_model(), "nproc": avail,
            "os_cpu_count": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--extras", default="adjoint,batch,octree,odes,time_field,interp",
                    help="comma list: adjoint,batch,octree,odes,time_field,interp ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "COMMAND"),
                    help="print the counter summary of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--traffic-kernel", default=DOMINANT_KERNEL,
                    help="kernel whose bytes --summarize-traffic reports (default: the fused advect)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("RUN_DIR", "TITLE", "COMMAND"),
                    help="print a per-kernel SQ counter summary of a rocprofv3 --pmc run (for profiles/)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_DIR", "TITLE", "COMMAND"),
                    help="print the per-kernel summary of a rocprofv3 --kernel-trace --stats run and exit")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, kernel=args.traffic_kernel)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the particle path has no "
              "multi-GPU form (one MI355X holds the whole mesh and particle set).", file=sys.stderr)
        sys.exit(2)
    args.extras = [e for e in args.extras.split(",") if e]
    line = run_main(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
