#!/usr/bin/env python
"""Benchmark of the FDTD hot path on one MI355X.

Headline (value): FP32 forward throughput in Mcell-updates/s on the largest
workload: 536^3 = 512^3 + 12-cell CPML, diagonal eps with each component in
[1,5], a central 128^3 one-pole Lorentz box, an Ex sheet source and an Ex
64x64 patch monitor over 8 frequencies, 4000 time steps per solve.  One
"step" of this benchmark is 100 time steps of that solve with the monitor
recording (two captured 50-step chunks); the solve restarts from rest after
its 4000 steps.  Inputs are resident in HBM before the timed region.

Alongside, on the same JSON line:
  * roofline: the stepping kernels of one time step against the HBM peak,
    timed live with HIP events on the library stream, and the HBM traffic of
    the same launch shape from the committed counter summary in profiles/;
  * cpu_baseline: the FP64 C oracle on the host, on all cores and on one
    core, forward and adjoint steps of the same workload (a bounded sample);
  * adjoint_536: the same workload's reverse sweep over 4000 steps with
    binomial replay in 32 FP32 slots and in 32 BF16 slots, gradient against
    an FP64 reference (20 slots) on a 64^3 subsample of the gradient box;
  * cache_resident_148: the 148^3 one-pole Lorentz workload (its working set
    fits the 256 MB Infinity Cache), its FP32 fields and flux after 1000
    steps against the oracle's stored record, the FP64 GPU path, and the
    full-solve time from construction to the final transfer (median of 3);
  * adjoint_212: the 212^3 design workload's reverse sweep (24 slots) and its
    gradient against the oracle's stored record; the 48-domain ragged batch;
    the 148^3 workload with 3 and 16 poles;
  * tensor_536: the 536^3 domain with a rotated symmetric tensor at every
    interior node (the two-pass tensor E update), FP32 forward;
  * tensor_adjoint_536: its reverse sweep with the gradient over every node
    tensor (160 steps, 8 slots, FP32 and FP64) and the adjoint step's
    kernel time against the forward step's;
  * periodic_536: a 512 x 512 x 536 Bloch-periodic cell, forward rate and
    roofline, and the adjoint step's kernel time against the forward step's;
  * streamed_536: the headline workload through host-streamed causal slabs
    (state in host memory, 64-plane slabs, 32 steps per visit);
  * streamed_adjoint_256: resident against streamed time to gradient and
    device memory on a matched 256^3 adjoint of 128 steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra] [--no-adjoint] [--shape K,R,Z]
"""
import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

BENCH_CHUNK = 50           # captured time steps per graph
BENCH_STEP = 100           # time steps per benchmark step


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fdtd_kernels.hip", "fdtd_dev.h"):
        with open(os.path.join(ROOT, "paper_2609_30039_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_hash, tile, name):
    """HBM bytes per time step of the stepping kernels from a committed counter
    summary, only if it was taken on the current kernel source and the launch
    shape that was timed."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    key = f"{tile.get('kernel')},{tile.get('tile_rows', 0)},{tile.get('tile_kz', 0)}"
    e = d.get("per_launch_shape", {}).get(key)
    return None if e is None else e.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run_forward(spec, dtype, stream, K, Wm, tile=None, graph_chunk=32):
    """K timed solves from rest (after Wm warm-up solves) with captured step
    chunks, then one solve with per-step kernel timing (eager launches, HIP
    events on the library stream) for the roofline."""
    from paper_2609_30039_amd.sim import Simulation
    import torch
    kw = dict(tile or {})
    if kw.get("kernel") not in ("split", "onepass"):
        graph_chunk = 0
    sim = Simulation(spec, dtype=dtype, stream=stream, graph_chunk=graph_chunk, **kw)

    def solve():
        sim.reset()
        sim.step(spec.n_steps, record=True)

    for _ in range(Wm):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.timing(1)
    solve()
    kms, nl = sim.timing(2)
    sim.timing(0)
    return sim, el, kms, nl


SPLIT_SHAPES = [{"kernel": "split", "tile_rows": r, "tile_kz": z} for (r, z) in ((8, 2), (8, 3), (8, 4), (8, 8), (0, 8))]


# ------------------------------------------------------------------ headline
def headline(args, stream, khash):
    """The 536^3 workload: K benchmark steps of 100 time steps each after W
    warm-up steps, then 100 eagerly launched time steps with HIP events
    around each step's stepping launches."""
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import roofline as RL
    from paper_2609_30039_amd import autotune as AT
    from paper_2609_30039_amd.sim import Simulation
    spec = W.anisotropic_lorentz()
    if args.shape:
        kk, rr, zz = args.shape.split(",")
        tile = {"kernel": kk, "tile_rows": int(rr), "tile_kz": int(zz)}
    else:
        tile = AT.tune(spec, "f32", stream=stream, log=log, steps=3, candidates=SPLIT_SHAPES[2:4])
    K, Wm = args.steps, args.warmup
    log(f"headline: anisotropic_lorentz {spec.shape} FP32, {BENCH_STEP} time steps per step, warmup {Wm}, "
        f"timed {K}, launch shape {tile}")
    sim = Simulation(spec, dtype="f32", stream=stream, graph_chunk=BENCH_CHUNK if tile["kernel"] in ("split", "onepass") else 0,
                     **tile)
    N = spec.n_steps
    done = [0]

    def bench_step():
        if done[0] + BENCH_STEP > N:
            sim.reset()
            done[0] = 0
        sim.step(BENCH_STEP, record=True)
        done[0] += BENCH_STEP

    for _ in range(Wm):
        bench_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        bench_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.timing(1)
    bench_step()
    kms, nl = sim.timing(2)
    sim.timing(0)
    sim.close()
    ncell = spec.ncells
    mcups = ncell * BENCH_STEP * K / el / 1e6
    avg_ms = kms / nl
    bytes_step = RL.forward_bytes(spec, 4)
    achieved = bytes_step / (avg_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(khash, tile, "fwd_anisotropic_lorentz_f32_pmc.json")
    log(f"headline: {el / K * 1e3:.1f} ms per step, {mcups:.0f} Mcell-upd/s, stepping kernels {avg_ms * 1e3:.1f} us "
        f"per time step, {achieved:.0f} GB/s algorithmic")
    out = {
        "metric": "Mcell-updates/s fwd & adjoint (FP32 vs FP64), % HBM roofline, grad rel. err",
        "value": round(mcups, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(el / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "536^3 cells (512^3 + 12-cell CPML, m=3, kappa_max=5), diagonal eps in [1,5] "
                               "(seed 1005), 128^3 one-pole Lorentz box, Ex sheet source, Ex 64x64 patch monitor "
                               "(8 frequencies); one step = 100 of the solve's 4000 time steps",
                   "cells": ncell, "time_steps_per_step": BENCH_STEP, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": RL.HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / RL.HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1),
                     "kernel": {"split": "split E and H kernels (k_fwd_e with the Lorentz-box blocks leading, "
                                         "then k_fwd_h)",
                                "onepass": "single-pass interior kernel k_fwd_one beside the split E and H kernels "
                                           "on the absorbing, wall and dispersive blocks",
                                "fused": "fused single-pass tile kernels"}[tile["kernel"]]
                               + ": all stepping launches of one time step",
                     "launch_shape": tile,
                     "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": bytes_step,
                     "kernel_source_hash": khash},
    }
    return spec, tile, out


# ------------------------------------------------------------------ CPU oracle
def cpu_baseline(spec, budget_s=30.0):
    """The FP64 oracle as it stands on the host's cores: forward steps with
    every core and with one, and adjoint steps with every core, of the same
    536^3 workload (a bounded sample of its 4000 steps)."""
    import ctypes
    from oracle import oracle as O
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    gomp = None
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        pass
    t0 = time.perf_counter()
    osim = O.OracleSim(spec)
    osim.step(2)                       # first steps: page faults and thread start-up
    log(f"oracle: set-up and 2 steps {time.perf_counter() - t0:.1f} s")
    n_all = 6
    t0 = time.perf_counter()
    osim.step(n_all)
    el_all = time.perf_counter() - t0
    one = None
    if gomp is not None:
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        osim.step(1)
        one = time.perf_counter() - t0
        gomp.omp_set_num_threads(cores)
    # adjoint steps against the current forward state
    a = np.zeros_like(osim.u)
    g = np.zeros((3, osim.N))
    osim.adjoint_step_state(a, osim.u, g)      # page faults
    n_adj = 3
    t0 = time.perf_counter()
    for _ in range(n_adj):
        osim.adjoint_step_state(a, osim.u, g)
    el_adj = time.perf_counter() - t0
    del osim, a, g
    ncell = spec.ncells
    out = {"value": round(ncell * n_all / el_all / 1e6, 2), "unit": "Mcell-updates/s", "cores": cores,
           "kind": "oracle",
           "sample": f"FP64 C oracle on the same 536^3 workload: forward time steps 3..{2 + n_all} of 4000 with the "
                     f"monitor recorded ({el_all:.1f} s on {cores} threads); one thread: 1 step; adjoint: {n_adj} "
                     f"steps on {cores} threads",
           "cpu_model": cpu_model(),
           "adjoint_value": round(ncell * n_adj / el_adj / 1e6, 2)}
    if one is not None:
        out["one_core_value"] = round(ncell / one / 1e6, 2)
    log(f"oracle: {out['value']} Mcell-upd/s forward on {cores} threads, {out.get('one_core_value')} on one, "
        f"adjoint {out['adjoint_value']}")
    return out


# ------------------------------------------------------------------ 536^3 adjoint
def adjoint_536(stream):
    """4000 steps, |DFT Ex|^2 on the 64x64 patch: binomial replay with 32 FP32
    slots and with 32 BF16 slots (per-array max-abs scale), and an FP64
    reference (20 slots, to fit in memory); gradients compared on a 64^3
    subsample of the gradient box (every 8th cell per axis)."""
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import adjoint as A
    from paper_2609_30039_amd import autotune as AT
    from paper_2609_30039_amd.sim import Simulation
    spec = W.anisotropic_lorentz()
    N = spec.n_steps
    out = {"workload": "536^3 (512^3 + 12-cell CPML), diagonal eps in [1,5], 128^3 Lorentz box, Ex sheet, |DFT Ex|^2 "
                       "on a 64x64 patch (8 frequencies), 4000 steps", "cells": spec.ncells}
    grads = {}
    for tag, dtype, slots, storage in (("fp32_slots", "f32", 32, None), ("bf16_slots", "f32", 32, "bf16"),
                                       ("fp64", "f64", 20, None)):
        tile = AT.tune(spec, dtype, adjoint=True, stream=stream, log=log, steps=3, candidates=SPLIT_SHAPES[2:4])
        kw = dict(tile)
        if storage:
            kw["ckpt_storage"] = storage
        sim = Simulation(spec, dtype=dtype, n_ckpt=slots, stream=stream, graph_chunk=32 if tile["kernel"] in ("split", "onepass")
                         else 0, **kw)
        plan = A.RevolvePlan(N, slots)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = A.forward_record(sim, plan)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.set_cotangent(0, 2.0 * sim.spectra(0))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        A.reverse_sweep(sim, plan, *last, progress=lambda m: log(f"  536^3 {tag}: adjoint at step {m}"))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g = sim.grad(0)
        grads[tag] = g[:, ::8, ::8, ::8].astype(np.float64)   # 64^3 subsample per component
        out[tag] = {"slots": slots, "launch_shape": tile, "forward_s": round(t1 - t0, 3),
                    "reverse_s": round(t3 - t2, 3), "reverse_over_forward": round((t3 - t2) / (t1 - t0), 3),
                    "forward_evaluations": plan.forward_evals + 1, "device_bytes": sim.memory_bytes(),
                    "adjoint_mcups": round(spec.ncells * N / (t3 - t2) / 1e6, 1)}
        log(f"536^3 adjoint {tag}: forward {t1 - t0:.2f} s, reverse {t3 - t2:.2f} s")
        sim.close()
        del sim
    ref = grads["fp64"]
    for tag in ("fp32_slots", "bf16_slots"):
        out[tag]["grad_rel_l2_vs_fp64_64cube"] = float(f"{np.linalg.norm(grads[tag] - ref) / np.linalg.norm(ref):.3e}")
    out["reversible"] = "not admissible: the 128^3 Lorentz box is lossy (gamma > 0) and lies in the gradient box"
    out["bf16_vs_fp32_slots_grad_rel_l2"] = float(
        f"{np.linalg.norm(grads['bf16_slots'] - grads['fp32_slots']) / np.linalg.norm(grads['fp32_slots']):.3e}")
    return out


# ------------------------------------------------------------------ 148^3
def cache_resident_148(stream, khash):
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import roofline as RL
    from paper_2609_30039_amd import autotune as AT
    from paper_2609_30039_amd.sim import Simulation
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_golden_full as G
    spec = W.lorentz_flux()
    ncell = spec.ncells
    tile = AT.tune(spec, "f32", stream=stream, log=log)
    sim32, el, kms, nl = run_forward(spec, "f32", stream, 3, 1, tile)
    bytes_step = RL.forward_bytes(spec, 4)
    avg_ms = kms / nl
    traffic = traffic_from_profiles(khash, tile, "fwd_lorentz_flux_f32_pmc.json")
    out = {"workload": "148^3 (128^3 + 10-cell CPML), 48^3 one-pole Lorentz block, Ex sheet, 16-frequency flux "
                       "plane, 1000 steps FP32; working set inside the 256 MB Infinity Cache",
           "mcups": round(ncell * spec.n_steps * 3 / el / 1e6, 1), "launch_shape": tile,
           "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": bytes_step,
           "achieved_GBs": round(bytes_step / (avg_ms * 1e-3) / 1e9, 1),
           "frac_hbm": round(bytes_step / (avg_ms * 1e-3) / 1e9 / RL.HBM_PEAK_GBS, 4),
           "traffic_GBs": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1)}
    # FP32 after 1000 steps against the oracle's record (strided node sample, flux)
    rec = G.read("lorentz_flux_1000")
    a, s_ = (int(v) for v in rec["field_sample_spec"])
    errs = {}
    for q in range(6):
        f = sim32.field(q)[a::s_, a::s_, a::s_].astype(np.float64)
        r = rec["fields_sample"][q]
        errs[W.COMP_NAMES[q]] = float(f"{np.linalg.norm(f - r) / np.linalg.norm(r):.3e}")
    fl = sim32.flux(0)
    out["fp32_vs_oracle_at_1000"] = {
        **errs, "flux_max_rel": float(f"{np.max(np.abs(fl - rec['flux']) / np.abs(rec['flux'])):.3e}"),
        "float32_storage_floor": {W.COMP_NAMES[q]: float(f"{rec['f32store_rel_sample'][q]:.3e}") for q in range(6)},
        "note": "rel. L2 on every 6th node per axis; the floor is the oracle with its state rounded to float32 each step"}
    sim32.close()
    # FP64 GPU path
    tile64 = AT.tune(spec, "f64", stream=stream, log=log)
    sim64, el64, kms64, nl64 = run_forward(spec, "f64", stream, 1, 1, tile64)
    errs64 = max(np.linalg.norm(sim64.field(q)[a::s_, a::s_, a::s_] - rec["fields_sample"][q]) /
                 np.linalg.norm(rec["fields_sample"][q]) for q in range(6))
    out["fp64"] = {"mcups": round(ncell * spec.n_steps / el64 / 1e6, 1), "launch_shape": tile64,
                   "achieved_GBs": round(RL.forward_bytes(spec, 8) / (kms64 / nl64 * 1e-3) / 1e9, 1),
                   "max_field_rel_l2_vs_oracle_at_1000": float(f"{errs64:.3e}")}
    sim64.close()
    # full solve: construction, 1000 steps with the monitor, final transfer of
    # the six fields and the flux; median of 3 after one warm repetition
    reps = []
    for r in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim = Simulation(spec, dtype="f32", stream=stream, graph_chunk=32 if tile["kernel"] in ("split", "onepass") else 0, **tile)
        sim.step(spec.n_steps, record=True)
        _ = [sim.field(q) for q in range(6)]
        _ = sim.flux(0)
        torch.cuda.synchronize()
        sim.close()
        if r:
            reps.append(time.perf_counter() - t0)
    out["full_solve_s_median_of_3"] = round(statistics.median(reps), 4)
    out["full_solve_mcups"] = round(ncell * spec.n_steps / statistics.median(reps) / 1e6, 1)
    log(f"148^3: {out['mcups']} Mcell/s stepping, full solve {out['full_solve_s_median_of_3']} s")
    return out


# ------------------------------------------------------------------ 212^3 adjoint
def adjoint_212(stream):
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import adjoint as A
    from paper_2609_30039_amd import autotune as AT
    from paper_2609_30039_amd.sim import Simulation
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_golden_full as G
    spec3, _ = W.design_patch()
    log(f"design_patch adjoint: {spec3.shape} x {spec3.n_steps}, 24 checkpoint slots")
    rec = G.read("design_patch_full") if os.path.exists(G.path("design_patch_full")) else None
    out = {"workload": "212^3 (192^3 + 10-cell CPML), 64^3 design box eps in [1,6], |DFT Ez|^2 on a 32x32 patch, "
                       "8 frequencies, 2000 steps, 24 checkpoints (binomial)"}
    grads = {}
    for dt in ("f32", "f64"):
        tile3 = AT.tune(spec3, dt, adjoint=True, stream=stream, log=log)
        sim3 = Simulation(spec3, dtype=dt, n_ckpt=24, stream=stream,
                          graph_chunk=32 if tile3["kernel"] in ("split", "onepass") else 0, **tile3)
        plan = A.RevolvePlan(spec3.n_steps, 24)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = A.forward_record(sim3, plan)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim3.set_cotangent(0, 2.0 * sim3.spectra(0))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        A.reverse_sweep(sim3, plan, *last)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        grads[dt] = sim3.grad(0)[0]
        tf, tr = t1 - t0, t3 - t2
        n3 = spec3.ncells
        out[dt] = {"forward_s": round(tf, 4), "reverse_s": round(tr, 4), "reverse_over_forward": round(tr / tf, 3),
                   "adjoint_mcups": round(n3 * spec3.n_steps / tr / 1e6, 1),
                   "forward_mcups": round(n3 * spec3.n_steps / tf / 1e6, 1),
                   "forward_evaluations": plan.forward_evals + 1, "launch_shape": tile3}
        if rec is not None:
            out[dt]["grad_rel_l2_vs_oracle"] = float(
                f"{np.linalg.norm(grads[dt] - rec['grad']) / np.linalg.norm(rec['grad']):.3e}")
        log(f"design_patch {dt}: forward {tf:.3f} s, reverse {tr:.3f} s")
        sim3.close()
        del sim3
    out["grad_rel_l2_fp32_vs_fp64"] = float(
        f"{np.linalg.norm(grads['f32'] - grads['f64']) / np.linalg.norm(grads['f64']):.3e}")
    # reversible mode: the design box lies in the lossless interior, so the
    # reverse sweep steps it backward with the recorded interface (no replay)
    for dt in ("f32", "f64"):
        tile3 = out[dt]["launch_shape"]
        sim3 = Simulation(spec3, dtype=dt, stream=stream, reversible=True, max_steps=spec3.n_steps, **tile3)
        sim3.step(4, record=False)
        sim3.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim3.step(spec3.n_steps, record=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim3.set_cotangent(0, 2.0 * sim3.spectra(0))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        A.reversible_sweep(sim3, spec3.n_steps)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g = sim3.grad(0)[0]
        tf, tr = t1 - t0, t3 - t2
        r = {"forward_s": round(tf, 4), "reverse_s": round(tr, 4),
             "reverse_over_forward": round(tr / out[dt]["forward_s"], 3),
             "reverse_over_own_forward": round(tr / tf, 3),
             "note": "reverse_over_forward divides by the plain forward solve above (captured chunks); the "
                     "reversible forward launches steps one by one and records the interface",
             "grad_rel_l2_vs_checkpointed": float(f"{np.linalg.norm(g - grads[dt]) / np.linalg.norm(grads[dt]):.3e}")}
        if rec is not None:
            r["grad_rel_l2_vs_oracle"] = float(f"{np.linalg.norm(g - rec['grad']) / np.linalg.norm(rec['grad']):.3e}")
        out[dt]["reversible"] = r
        log(f"design_patch {dt} reversible: forward {tf:.3f} s, reverse {tr:.3f} s")
        sim3.close()
        del sim3
    return out


# ------------------------------------------------------------------ ragged batch
def batch_48(stream):
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import adjoint as A
    from paper_2609_30039_amd import autotune as AT
    from paper_2609_30039_amd.sim import Simulation
    specs4 = W.batch_domains()
    cells4 = sum(s_.ncells for s_ in specs4)
    n4 = specs4[0].n_steps
    tile4 = AT.tune(specs4, "f32", stream=stream, log=log, steps=3)
    log(f"batch_domains: {len(specs4)} domains, {cells4} cells, {n4} steps, launch shape {tile4}")
    sim4 = Simulation(specs4, dtype="f32", n_ckpt=16, stream=stream,
                      graph_chunk=32 if tile4["kernel"] in ("split", "onepass") else 0, **tile4)
    sim4.step(4, record=False)
    sim4.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim4.step(n4, record=True)
    torch.cuda.synchronize()
    el4 = time.perf_counter() - t0
    plan4 = A.RevolvePlan(n4, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last4 = A.forward_record(sim4, plan4)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for d_, s_ in enumerate(specs4):
        if s_.grad_box is None:
            continue
        sp = sim4.spectra(0, domain=d_)
        g = np.zeros_like(sp)     # J = sum_f Re sum (Ex Hy* - Ey Hx*)
        g[:, 0], g[:, 3], g[:, 1], g[:, 2] = sp[:, 3], sp[:, 0], -sp[:, 2], -sp[:, 1]
        sim4.set_cotangent(0, g, domain=d_)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    A.reverse_sweep(sim4, plan4, *last4)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    sim4.close()
    return {"workload": f"{len(specs4)} ragged domains (per-axis interior from {{48,64,96,128,160}} + 10-cell CPML), "
                        f"eps in [1,4], Ez dipole, {n4} steps FP32; even domains forward+adjoint of a flux objective, "
                        f"16 checkpoints",
            "cells": cells4, "forward_mcups": round(cells4 * n4 / el4 / 1e6, 1),
            "record_s": round(t1 - t0, 4), "reverse_s": round(t3 - t2, 4),
            "reverse_over_forward": round((t3 - t2) / (t1 - t0), 3),
            "forward_evaluations": plan4.forward_evals + 1, "launch_shape": tile4}


def several_poles(stream, tile):
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import roofline as RL
    out = {"workload": "148^3 headline-sized domain, flux plane recorded, its 48^3 box with 3 poles (2 Lorentz, "
                       "1 Drude) or 16 poles (10 Lorentz, 6 Drude), 1000 steps FP32", "launch_shape": tile}
    for key in (3, 16):
        specp = W.with_poles(W.lorentz_flux(), W.pole_set(key))
        simp, elp, kmsp, nlp = run_forward(specp, "f32", stream, 1, 1, tile)
        bp = RL.forward_bytes(specp, 4)
        out[f"poles_{key}"] = {"mcups": round(specp.ncells * specp.n_steps / elp / 1e6, 1),
                               "avg_launch_us": round(kmsp / nlp * 1e3, 2),
                               "algorithmic_bytes_per_launch": bp,
                               "achieved_GBs": round(bp / (kmsp / nlp * 1e-3) / 1e9, 1)}
        simp.close()
    return out


def tensor_536(stream):
    """Symmetric tensor media at the headline size: 536^3 with a rotated
    tensor at every interior node, FP32 forward, captured 50-step chunks;
    per-time-step kernel time from HIP events over eager launches."""
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import roofline as RL
    from paper_2609_30039_amd.sim import Simulation
    t0 = time.perf_counter()
    spec = W.anisotropic_tensor()
    t1 = time.perf_counter()
    tile = {"kernel": "split", "tile_rows": 8, "tile_kz": 8}
    sim = Simulation(spec, dtype="f32", stream=stream, graph_chunk=BENCH_CHUNK, **tile)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"tensor_536: inputs {t1 - t0:.1f} s, create {t2 - t1:.1f} s")
    sim.step(BENCH_STEP)
    torch.cuda.synchronize()
    K = 3
    t3 = time.perf_counter()
    sim.step(K * BENCH_STEP)
    torch.cuda.synchronize()
    el = time.perf_counter() - t3
    sim.timing(1)
    sim.step(BENCH_STEP)
    kms, nl = sim.timing(2)
    sim.timing(0)
    sim.close()
    per_step_ms = kms / BENCH_STEP
    bstep = RL.forward_bytes(spec, 4)
    achieved = bstep / (per_step_ms * 1e-3) / 1e9
    mc = spec.ncells * K * BENCH_STEP / el / 1e6
    log(f"tensor_536: {mc:.0f} Mcell-upd/s, stepping kernels {per_step_ms * 1e3:.1f} us per time step, "
        f"{achieved:.0f} GB/s algorithmic")
    return {"workload": "536^3 (512^3 + 12-cell CPML), a rotated symmetric tensor with eigenvalues in [1,5] at "
                        "every interior node (a 64^3 block of independent tensors repeated, seed 1006), Ex sheet, "
                        "Ex patch, FP32 forward",
            "mcups": round(mc, 1), "stepping_us_per_time_step": round(per_step_ms * 1e3, 2),
            "algorithmic_bytes_per_time_step": bstep, "achieved_GBs": round(achieved, 1),
            "frac": round(achieved / RL.HBM_PEAK_GBS, 4), "launch_shape": tile,
            "inputs_s": round(t1 - t0, 1), "create_s": round(t2 - t1, 1)}


def tensor_adjoint_536(stream):
    """The reverse sweep of tensor media at 536^3: dJ/deps of all six entries
    of every interior node tensor (512^3 nodes), |DFT Ex|^2 on the 64x64
    patch moved 60 planes past the source so that 160 steps reach it;
    binomial replay in 8 slots, FP32 and FP64, the FP32 gradient against
    FP64 on the 64^3 block of nodes between the source and the patch; and
    the adjoint step's kernel time (HIP events on the library's stream,
    one adjoint step at a time from a stored state) against the forward
    step's."""
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import adjoint as A
    from paper_2609_30039_amd.sim import Simulation
    N, slots, R = 160, 8, 10
    spec = W.anisotropic_tensor(n_steps=N)
    pml = spec.pml[4]
    spec.monitors[0].pos = (0, 0, pml + 65)
    spec.grad_box = spec.eps_box
    (gx0, gy0, gz0), _ = spec.grad_box
    p0 = spec.monitors[0].rect
    blk = (slice(0, 64), slice(p0[2] - gy0, p0[2] - gy0 + 64), slice(p0[0] - gx0, p0[0] - gx0 + 64))
    out = {"workload": f"536^3 tensor workload with the gradient over every interior node tensor (6 entries), "
                       f"|DFT Ex|^2 on the 64x64 patch 60 planes past the source, {N} steps, {slots} binomial slots",
           "cells": spec.ncells}
    grads = {}
    for dtype, tile in (("f32", {"kernel": "split", "tile_rows": 8, "tile_kz": 8}),
                        ("f64", {"kernel": "split", "tile_rows": 8, "tile_kz": 4})):
        t0 = time.perf_counter()
        sim = Simulation(spec, dtype=dtype, n_ckpt=slots, max_steps=N, stream=stream, graph_chunk=32, **tile)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # kernel time of single steps: forward, then the adjoint step from the stored u^0
        sim.save(0)
        sim.timing(1)
        sim.step(R, record=False)
        fms, _ = sim.timing(2)
        sim.timing(0)
        sim.restore(0)
        sim.timing(1)
        for _ in range(R):
            sim.restore(0)
            sim.adjoint_begin(1)
            sim.step_adjoint(1)
        ams, na = sim.timing(2)
        sim.timing(0)
        sim.reset()
        plan = A.RevolvePlan(N, slots)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        last = A.forward_record(sim, plan)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        sim.set_cotangent(0, 2.0 * sim.spectra(0))
        A.reverse_sweep(sim, plan, *last)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        g = sim.grad(0)
        grads[dtype] = g[(slice(None),) + blk].astype(np.float64)
        del g
        out[dtype] = {"launch_shape": tile, "create_s": round(t1 - t0, 1), "forward_s": round(t3 - t2, 3),
                      "reverse_s": round(t4 - t3, 3), "reverse_over_forward": round((t4 - t3) / (t3 - t2), 3),
                      "forward_evaluations": plan.forward_evals + 1, "device_bytes": sim.memory_bytes(),
                      "forward_step_ms_events": round(fms / R, 3), "adjoint_step_ms_events": round(ams / na, 3),
                      "adjoint_over_forward_step": round((ams / na) / (fms / R), 3)}
        log(f"tensor adjoint 536^3 {dtype}: {out[dtype]}")
        sim.close()
        del sim
    ref = grads["f64"]
    out["grad_rel_l2_fp32_vs_fp64_64cube"] = float(f"{np.linalg.norm(grads['f32'] - ref) / np.linalg.norm(ref):.3e}")
    out["grad_offdiag_share"] = float(f"{np.linalg.norm(ref[3:]) / np.linalg.norm(ref):.3e}")
    return out


def periodic_536(stream):
    """The Bloch-periodic cell at the headline's size (512 x 512 x 536, x and
    y periodic with factors -1 and +1, absorbing z ends, a 64-plane
    patterned layer): FP32 forward in captured 50-step chunks with the flux
    plane recording, its stepping kernels' time per step (HIP events) and
    roofline, and the adjoint step's kernel time with the gradient over the
    layer (one adjoint step at a time from a stored state)."""
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import roofline as RL
    from paper_2609_30039_amd.sim import Simulation
    spec = W.bloch_cell()
    tile = {"kernel": "split", "tile_rows": 8, "tile_kz": 8}
    sim = Simulation(spec, dtype="f32", n_ckpt=1, stream=stream, graph_chunk=BENCH_CHUNK, **tile)
    sim.step(BENCH_STEP)
    torch.cuda.synchronize()
    K, R = 3, 10
    t0 = time.perf_counter()
    sim.step(K * BENCH_STEP)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.timing(1)
    sim.step(BENCH_STEP, record=False)
    fms, _ = sim.timing(2)
    sim.timing(0)
    sim.save(0)
    sim.timing(1)
    for _ in range(R):
        sim.restore(0)
        sim.adjoint_begin(sim.steps[0] + 1)
        sim.step_adjoint(1)
    ams, na = sim.timing(2)
    sim.timing(0)
    sim.close()
    fstep = fms / BENCH_STEP
    astep = ams / na
    bstep = RL.forward_bytes(spec, 4)
    achieved = bstep / (fstep * 1e-3) / 1e9
    mc = spec.ncells * K * BENCH_STEP / el / 1e6
    log(f"periodic_536: {mc:.0f} Mcell-upd/s, forward step {fstep * 1e3:.0f} us, adjoint step {astep * 1e3:.0f} us")
    return {"workload": "512 x 512 x 536 Bloch cell (x, y periodic, factors -1 and +1; 12-cell CPML at the z ends), "
                        "64-plane diagonal-eps layer in [1,5] (seed 1007) as the gradient box, Ex sheet, flux plane, "
                        "FP32", "cells": spec.ncells, "mcups": round(mc, 1), "launch_shape": tile,
            "stepping_us_per_time_step": round(fstep * 1e3, 2), "algorithmic_bytes_per_time_step": bstep,
            "achieved_GBs": round(achieved, 1), "frac": round(achieved / RL.HBM_PEAK_GBS, 4),
            "adjoint_step_us_events": round(astep * 1e3, 2), "adjoint_over_forward_step": round(astep / fstep, 3)}


def streamed_536(stream):
    """Host-streamed causal slabs on the 536^3 workload: slabs of 64 core
    planes, K = 32 steps per visit (33 halo planes per cut), FP32 forward
    over two passes (64 steps), against the resident stepping rate."""
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd.sim import StreamedSimulation
    spec = W.anisotropic_lorentz()
    spec.grad_box = None          # forward only
    Wp, Kp, passes = 64, 32, 2
    t0 = time.perf_counter()
    s = StreamedSimulation(spec, Wp, Kp, dtype="f32", stream=stream, tile_rows=8, tile_kz=8)
    t1 = time.perf_counter()
    s.step(Kp)                    # warm-up pass
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.step(passes * Kp)
    torch.cuda.synchronize()
    el = time.perf_counter() - t2
    info = s.info()
    s.close()
    mc = spec.ncells * passes * Kp / el / 1e6
    log(f"streamed_536: {mc:.0f} Mcell-upd/s, {info}")
    return {"workload": "536^3 anisotropic workload streamed: z slabs of <= 64 core planes, K = 32 steps per visit, "
                        "33 halo planes per cut, FP32 forward, state in two pinned host banks",
            "mcups": round(mc, 1), "s_per_pass": round(el / passes, 3), "create_s": round(t1 - t0, 2),
            "n_slabs": info["n_slabs"], "max_extent_planes": info["max_extent"],
            "device_bytes": info["device_bytes"], "host_bytes": info["host_bytes"],
            "resident_bytes": info["resident_bytes"]}


def streamed_adjoint_256(stream):
    """The memory-time trade-off of host streaming on a matched 256^3 adjoint
    (the paper's protocol: 128 steps, two checkpoints for the resident run):
    |DFT Ez|^2 of a patch, dJ/deps over a 128^3 design box.  Resident: two
    binomial checkpoint slots; streamed: 64-plane slabs, K = 16 (a forward
    bank per 16 steps in host memory), one workspace, 4 local slots per
    block.  Both FP32, from construction to the gradient on the host.  The
    streamed run is repeated with 4 forward banks on the host (a binomial
    schedule over the 8 passes)."""
    import torch
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import adjoint as A
    from paper_2609_30039_amd.sim import Simulation, StreamedSimulation
    spec, _ = W.design_patch(interior=236, pml=10, design=128, patch=32, n_steps=128, n_f=8)
    # the patch where the 128-step pulse has arrived: 60 planes past the sheet source
    spec.monitors[0].pos = (0, 0, spec.sources[0].pos[2] + 60)
    N = spec.n_steps
    tile = {"kernel": "split", "tile_rows": 8, "tile_kz": 8}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = Simulation(spec, dtype="f32", n_ckpt=2, stream=stream, **tile)
    plan = A.RevolvePlan(N, 2)
    last = A.forward_record(sim, plan)
    sim.set_cotangent(0, 2.0 * sim.spectra(0))
    A.reverse_sweep(sim, plan, *last)
    g_res = sim.grad(0)[0]
    t1 = time.perf_counter()
    dev_res = sim.memory_bytes()
    sim.close()
    t2 = time.perf_counter()
    st_ = StreamedSimulation(spec, 64, 16, dtype="f32", stream=stream, overlap=False, local_slots=4,
                             **{k: v for k, v in tile.items() if k != "kernel"})
    st_.step(N)
    st_.set_cotangent(0, 2.0 * st_.spectra(0))
    st_.reverse()
    g_str = st_.grad()[0]
    t3 = time.perf_counter()
    info = st_.info()
    st_.close()
    r = float(np.linalg.norm(g_str - g_res) / np.linalg.norm(g_res))
    log(f"streamed_adjoint_256: resident {t1 - t0:.2f} s ({dev_res / 1e9:.2f} GB), streamed {t3 - t2:.2f} s "
        f"({info['device_bytes'] / 1e9:.2f} GB device, {info['host_bytes'] / 1e9:.2f} GB host), grad rel {r:.2e}")
    # the same with 4 forward banks on the host (binomial over the 8 passes)
    t4 = time.perf_counter()
    sb = StreamedSimulation(spec, 64, 16, dtype="f32", stream=stream, overlap=False, local_slots=4, host_banks=4,
                            **{k: v for k, v in tile.items() if k != "kernel"})
    sb.step(N)
    sb.set_cotangent(0, 2.0 * sb.spectra(0))
    sb.reverse()
    g_b = sb.grad()[0]
    t5 = time.perf_counter()
    info_b = sb.info()
    sb.close()
    rb = float(np.linalg.norm(g_b - g_res) / np.linalg.norm(g_res))
    return {"workload": "256^3 (236^3 + 10-cell CPML), 128^3 design box eps in [1,6], |DFT Ez|^2 on a 32x32 "
                        "patch, 8 frequencies, 128 steps, FP32; resident with 2 binomial slots (forward "
                        f"evaluations {plan.forward_evals + 1}), streamed with 64-plane slabs, K = 16, one "
                        "workspace and 4 local slots",
            "resident_s": round(t1 - t0, 3), "streamed_s": round(t3 - t2, 3),
            "streamed_over_resident": round((t3 - t2) / (t1 - t0), 2),
            "resident_device_bytes": dev_res, "streamed_device_bytes": info["device_bytes"],
            "streamed_host_bytes": info["host_bytes"], "n_slabs": info["n_slabs"],
            "grad_rel_l2_streamed_vs_resident": float(f"{r:.3e}"),
            "four_host_banks": {"streamed_s": round(t5 - t4, 3), "host_bytes": info_b["host_bytes"],
                                "replay_passes": info_b["replay_passes"],
                                "grad_rel_l2_vs_resident": float(f"{rb:.3e}")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline only (with the CPU baseline)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 536^3 adjoint study")
    ap.add_argument("--shape", default=None,
                    help="launch shape KERNEL,ROWS,KZ for the headline (skips the autotuner), e.g. split,8,8")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the path is single-GPU (no collectives); --gpus {args.gpus} is not "
              f"supported", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs the GPU", file=sys.stderr)
        sys.exit(1)
    stream = torch.cuda.current_stream().cuda_stream
    khash = kernel_source_hash()
    t_start = time.perf_counter()

    spec5, tile5, out = headline(args, stream, khash)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec5)
    if not args.no_extra:
        if not args.no_adjoint:
            out["adjoint_536"] = adjoint_536(stream)
        out["cache_resident_148"] = cache_resident_148(stream, khash)
        out["adjoint_212"] = adjoint_212(stream)
        out["batch_48"] = batch_48(stream)
        out["several_poles"] = several_poles(stream, out["cache_resident_148"]["launch_shape"])
        out["tensor_536"] = tensor_536(stream)
        out["tensor_adjoint_536"] = tensor_adjoint_536(stream)
        out["periodic_536"] = periodic_536(stream)
        out["streamed_536"] = streamed_536(stream)
        out["streamed_adjoint_256"] = streamed_adjoint_256(stream)
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
