#!/usr/bin/env python
"""Benchmark of the FDTD hot path on one MI355X.

Headline (value): FP32 forward throughput in Mcell-updates/s on the 128^3 +
10-cell CPML workload with a 48^3 Lorentz block, a z-sheet source and a
16-frequency flux plane, 1000 time steps (one "step" of this benchmark = one
complete 1000-time-step solve from rest, monitors included).  Alongside: the
dominant kernel against the HBM roofline (HIP events on the library stream),
the FP64 oracle on the host cores, the FP64 GPU path, the adjoint sweep with
binomial replay on the 192^3 + CPML design-patch workload, and a 512^3 + CPML
forward whose working set is far beyond the on-die cache.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra] [--shape K,R,Z]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fdtd_kernels.hip", "fdtd_dev.h"):
        with open(os.path.join(ROOT, "paper_2609_30039_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_hash, tile, name="fwd_lorentz_flux_f32_pmc.json"):
    """HBM bytes per step of the stepping kernels from a committed PMC summary,
    only if it was taken on the current kernel source and the launch shape
    that was timed."""
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


def run_forward(spec, dtype, stream, K, Wm, tile=None, graph_chunk=32):
    """K timed solves from rest (after Wm warm-up solves) with captured step
    chunks, then one solve with per-step kernel timing (eager launches, HIP
    events on the library stream) for the roofline."""
    from paper_2609_30039_amd.sim import Simulation
    import torch
    kw = dict(tile or {})
    if kw.get("kernel") != "split":
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


def large_adjoint(stream, log):
    """512^3 + 12-cell CPML, diagonal eps, 128^3 Lorentz box, |DFT Ex|^2 on a
    64x64 patch, 4000 steps: binomial replay with 32 FP32 slots and with 32 BF16
    slots (per-array max-abs scale), and an FP64 reference (20 slots, to fit in
    memory); gradients compared on a 64^3 subsample of the gradient box."""
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
        tile = AT.tune(spec, dtype, adjoint=True, stream=stream, log=log, steps=3)
        kw = dict(tile)
        if storage:
            kw["ckpt_storage"] = storage
        sim = Simulation(spec, dtype=dtype, n_ckpt=slots, stream=stream, graph_chunk=32 if tile["kernel"] == "split"
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
        A.reverse_sweep(sim, plan, *last, progress=lambda m: log(f"  {tag}: adjoint at step {m}"))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g = sim.grad(0)
        grads[tag] = g[:, ::8, ::8, ::8].astype(np.float64)   # 64^3 subsample per component
        out[tag] = {"slots": slots, "launch_shape": tile, "forward_s": round(t1 - t0, 3),
                    "reverse_s": round(t3 - t2, 3), "reverse_over_forward": round((t3 - t2) / (t1 - t0), 3),
                    "forward_evaluations": plan.forward_evals + 1, "device_bytes": sim.memory_bytes()}
        log(f"large adjoint {tag}: forward {t1 - t0:.2f} s, reverse {t3 - t2:.2f} s")
        sim.close()
        del sim
    ref = grads["fp64"]
    for tag in ("fp32_slots", "bf16_slots"):
        out[tag]["grad_rel_l2_vs_fp64_64cube"] = float(f"{np.linalg.norm(grads[tag] - ref) / np.linalg.norm(ref):.3e}")
    out["bf16_vs_fp32_slots_grad_rel_l2"] = float(
        f"{np.linalg.norm(grads['bf16_slots'] - grads['fp32_slots']) / np.linalg.norm(grads['fp32_slots']):.3e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--large-adjoint", action="store_true",
                    help="run only the 512^3 + CPML adjoint study (FP32 vs BF16 checkpoints vs FP64) and print its JSON")
    ap.add_argument("--shape", default=None,
                    help="launch shape KERNEL,ROWS,KZ for the headline (skips the autotuner), e.g. split,0,8")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the path is single-GPU (no collectives); --gpus {args.gpus} is not "
              f"supported", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs the GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2609_30039_amd import workloads as W
    from paper_2609_30039_amd import roofline as RL
    from paper_2609_30039_amd.sim import Simulation
    from paper_2609_30039_amd import adjoint as A

    stream = torch.cuda.current_stream().cuda_stream
    K, Wm = args.steps, args.warmup
    khash = kernel_source_hash()

    from paper_2609_30039_amd import autotune as AT

    if args.large_adjoint:
        print(json.dumps(large_adjoint(stream, log)), flush=True)
        return

    # ---------------------------------------------------------------- headline
    spec = W.lorentz_flux()
    ncell = spec.ncells
    if args.shape:
        kk, rr, zz = args.shape.split(",")
        tile = {"kernel": kk, "tile_rows": int(rr), "tile_kz": int(zz)}
    else:
        tile = AT.tune(spec, "f32", stream=stream, log=log)
    log(f"lorentz_flux FP32 forward: {spec.shape} x {spec.n_steps} steps, warmup {Wm}, timed {K}, launch shape {tile}")
    sim32, el, kms, nl = run_forward(spec, "f32", stream, K, Wm, tile)
    mcups = ncell * spec.n_steps * K / el / 1e6
    avg_ms = kms / nl
    bytes_launch = RL.forward_bytes(spec, 4)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    log(f"lorentz_flux FP32: {el / K * 1e3:.2f} ms/solve, {mcups:.0f} Mcell-upd/s, kernel {avg_ms * 1e3:.1f} us/launch, "
        f"{achieved:.0f} GB/s algorithmic")
    traffic = traffic_from_profiles(khash, tile)
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
        "config": {"workload": "148^3 cells (128^3 + 10-cell CPML, m=3, kappa_max=5), 48^3 one-pole Lorentz "
                               "block, Ex sheet source, 16-frequency flux plane, 1000 time steps per step",
                   "cells": ncell, "time_steps_per_step": spec.n_steps, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": RL.HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / RL.HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1),
                     "kernel": ("split E and H kernels (k_fwd_e with the Lorentz-box blocks leading, then k_fwd_h)"
                                if tile["kernel"] == "split" else "fused single-pass tile kernels")
                               + ": all stepping launches of one time step",
                     "launch_shape": tile,
                     "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": bytes_launch,
                     "kernel_source_hash": khash},
    }

    # ---------------------------------------------------------------- CPU oracle
    if not args.no_cpu:
        from oracle import oracle as O
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        osim = O.OracleSim(spec)
        osim.step(2)                       # first steps: page faults and thread start-up
        t0 = time.perf_counter()
        osim.step(3)
        per = (time.perf_counter() - t0) / 3
        nsteps = int(max(2, min(spec.n_steps - 5, args.cpu_seconds / max(per, 1e-6))))
        log(f"oracle: {per * 1e3:.0f} ms/step on {cores} threads, running {nsteps} more steps")
        t0 = time.perf_counter()
        osim.step(nsteps)
        cel = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(ncell * nsteps / cel / 1e6, 2), "unit": "Mcell-updates/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"FP64 C oracle, same workload, time steps 6..{nsteps + 5} of 1000 "
                                         f"({cel:.1f} s), monitors recorded"}
        # FP32 GPU fields against the oracle at the same step
        n_cmp = nsteps + 5
        cmp_sim = Simulation(spec, dtype="f32", stream=stream)
        cmp_sim.step(n_cmp)
        errs = {W.COMP_NAMES[q]: float(np.linalg.norm(cmp_sim.field(q) - osim.field(q)) /
                                       max(np.linalg.norm(osim.field(q)), 1e-300)) for q in range(6)}
        out["accuracy_vs_oracle"] = {"fp32_field_rel_l2_at_step": n_cmp, **{k: float(f"{v:.3e}") for k, v in
                                                                           errs.items()}}
        del cmp_sim, osim

    if not args.no_extra:
        # ------------------------------------------------------------ FP64 path and FP32 accuracy at 1000 steps
        tile64 = AT.tune(spec, "f64", stream=stream, log=log)
        log(f"lorentz_flux FP64 forward, launch shape {tile64}")
        sim64, el64, kms64, nl64 = run_forward(spec, "f64", stream, 1, 1, tile64)
        out["fp64"] = {"value": round(ncell * spec.n_steps / el64 / 1e6, 1), "unit": "Mcell-updates/s",
                       "ms_per_solve": round(el64 * 1e3, 2),
                       "achieved_GBs": round(RL.forward_bytes(spec, 8) / (kms64 / nl64 * 1e-3) / 1e9, 1)}
        f32e = {}
        for q in range(6):
            a, b = sim32.field(q).astype(np.float64), sim64.field(q)
            f32e[W.COMP_NAMES[q]] = float(f"{np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300):.3e}")
        fl32, fl64 = sim32.flux(0), sim64.flux(0)
        f32e["flux_max_rel"] = float(f"{np.max(np.abs(fl32 - fl64) / np.abs(fl64)):.3e}")
        # By step 1000 most of the pulse has left through the absorbers, so the
        # figures above are relative to late-time residual fields.  Diagnostic:
        # the same differences over each field's largest norm in time (FP64 run
        # sampled every 50 steps).
        tsim = Simulation(spec, dtype="f64", stream=stream, **tile64)
        peak = np.zeros(6)
        for _ in range(spec.n_steps // 50):
            tsim.step(50, record=False)
            for q in range(6):
                peak[q] = max(peak[q], float(np.linalg.norm(tsim.field(q))))
        tsim.close()
        f32e["rel_to_time_max_norm"] = {
            W.COMP_NAMES[q]: float(f"{np.linalg.norm(sim32.field(q).astype(np.float64) - sim64.field(q)) / max(peak[q], 1e-300):.3e}")
            for q in range(6)}
        out["fp32_vs_fp64_gpu_at_1000"] = f32e
        del sim64

        # ------------------------------------------------------------ adjoint (192^3 + CPML, 2000 steps, 24 slots)
        spec3, fd_cells = W.design_patch()
        log(f"design_patch adjoint: {spec3.shape} x {spec3.n_steps}, 24 checkpoint slots")

        def cot(s):
            sp = s.spectra(0)
            return {(0, 0): 2.0 * sp}

        grads = {}
        for dt in ("f32", "f64"):
            tile3 = AT.tune(spec3, dt, adjoint=True, stream=stream, log=log)
            sim3 = Simulation(spec3, dtype=dt, n_ckpt=24, stream=stream,
                              graph_chunk=32 if tile3["kernel"] == "split" else 0, **tile3)
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
            if dt == "f32":
                # kernel time of the reverse sweep, from a second, untimed pass with
                # per-launch events (which also keep the replays out of captured chunks)
                last = A.forward_record(sim3, plan)
                sim3.set_cotangent(0, 2.0 * sim3.spectra(0))
                sim3.timing(1)
                A.reverse_sweep(sim3, plan, *last)
                akms, anl = sim3.timing(2)
                sim3.timing(0)
            tf, tr = t1 - t0, t3 - t2
            n3 = spec3.ncells
            if dt == "f32":
                out["adjoint"] = {
                    "workload": "212^3 (192^3 + 10-cell CPML), 64^3 design box eps in [1,6], |DFT Ez|^2 on a "
                                "32x32 patch, 8 frequencies, 2000 steps, 24 checkpoints (binomial)",
                    "forward_s": round(tf, 4), "reverse_s": round(tr, 4),
                    "reverse_over_forward": round(tr / tf, 3),
                    "adjoint_mcups": round(n3 * spec3.n_steps / tr / 1e6, 1),
                    "forward_mcups": round(n3 * spec3.n_steps / tf / 1e6, 1),
                    "forward_evaluations": plan.forward_evals + 1, "launch_shape": tile3,
                    "reverse_stepping_kernel_ms": round(akms, 2), "reverse_stepping_launches": anl}
            else:
                out["adjoint"]["fp64_reverse_s"] = round(tr, 4)
                out["adjoint"]["fp64_forward_s"] = round(tf, 4)
            log(f"design_patch {dt}: forward {tf:.3f} s, reverse {tr:.3f} s")
            del sim3
        g32, g64 = grads["f32"], grads["f64"]
        out["adjoint"]["grad_rel_l2_fp32_vs_fp64"] = float(f"{np.linalg.norm(g32 - g64) / np.linalg.norm(g64):.3e}")

        # ------------------------------------------------------------ ragged batch: 48 domains in every launch
        specs4 = W.batch_domains()
        cells4 = sum(s_.ncells for s_ in specs4)
        n4 = specs4[0].n_steps
        tile4 = AT.tune(specs4, "f32", stream=stream, log=log, steps=3)
        log(f"batch_domains: {len(specs4)} domains, {cells4} cells, {n4} steps, launch shape {tile4}")
        sim4 = Simulation(specs4, dtype="f32", n_ckpt=16, stream=stream,
                          graph_chunk=32 if tile4["kernel"] == "split" else 0, **tile4)
        sim4.step(4, record=False)
        sim4.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim4.step(n4, record=True)
        torch.cuda.synchronize()
        el4 = time.perf_counter() - t0
        # forward + adjoint of the flux objective on the even domains (binomial, 16 slots)
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
        out["batch"] = {
            "workload": f"{len(specs4)} ragged domains (per-axis interior from {{48,64,96,128,160}} + 10-cell CPML), "
                        f"eps in [1,4], Ez dipole, {n4} steps FP32; even domains forward+adjoint of a flux objective, "
                        f"16 checkpoints",
            "cells": cells4, "forward_mcups": round(cells4 * n4 / el4 / 1e6, 1),
            "record_s": round(t1 - t0, 4), "reverse_s": round(t3 - t2, 4),
            "reverse_over_forward": round((t3 - t2) / (t1 - t0), 3),
            "forward_evaluations": plan4.forward_evals + 1, "launch_shape": tile4}
        log(f"batch: forward {cells4 * n4 / el4 / 1e6:.0f} Mcell/s, reverse/forward {(t3 - t2) / (t1 - t0):.2f}")
        del sim4

        # ------------------------------------------------------------ large forward (cache-free roofline)
        spec5 = W.anisotropic_lorentz()
        spec5.n_steps = 200
        for s_ in spec5.sources:
            s_.waveform = s_.waveform[:200]
        tile5 = AT.tune(spec5, "f32", stream=stream, log=log, steps=3)
        log(f"anisotropic_lorentz forward: {spec5.shape} x 200 steps, launch shape {tile5}")
        sim5, el5, kms5, nl5 = run_forward(spec5, "f32", stream, 1, 1, tile5)
        b5 = RL.forward_bytes(spec5, 4)
        t5 = traffic_from_profiles(khash, tile5, "fwd_anisotropic_lorentz_f32_pmc.json")
        out["large_forward"] = {
            "workload": "536^3 (512^3 + 12-cell CPML), diagonal eps, 128^3 Lorentz box, Ex sheet, Ex patch "
                        "monitor, 200 steps FP32",
            "mcups": round(spec5.ncells * 200 / el5 / 1e6, 1),
            "avg_launch_us": round(kms5 / nl5 * 1e3, 1),
            "achieved_GBs": round(b5 / (kms5 / nl5 * 1e-3) / 1e9, 1),
            "frac_hbm": round(b5 / (kms5 / nl5 * 1e-3) / 1e9 / RL.HBM_PEAK_GBS, 4),
            "traffic_GBs": None if t5 is None else round(t5 / (kms5 / nl5 * 1e-3) / 1e9, 1),
            "launch_shape": tile5}
        del sim5

        # ------------------------------------------------------------ dispersive box with several poles
        # the headline domain and launch shape, its 48^3 box holding two Lorentz
        # poles and a Drude pole, then the maximum of 16 poles
        poles_out = {"workload": "148^3 headline domain, flux plane recorded, its 48^3 box with 3 poles (2 Lorentz, "
                                 "1 Drude) or 16 poles (10 Lorentz, 6 Drude), 1000 steps FP32",
                     "launch_shape": tile}
        for key in (3, 16):
            specp = W.with_poles(W.lorentz_flux(), W.pole_set(key))
            simp, elp, kmsp, nlp = run_forward(specp, "f32", stream, 1, 1, tile)
            bp = RL.forward_bytes(specp, 4)
            poles_out[f"poles_{key}"] = {
                "mcups": round(specp.ncells * specp.n_steps / elp / 1e6, 1),
                "avg_launch_us": round(kmsp / nlp * 1e3, 2),
                "algorithmic_bytes_per_launch": bp,
                "achieved_GBs": round(bp / (kmsp / nlp * 1e-3) / 1e9, 1)}
            log(f"lorentz_flux with {key} poles: {specp.ncells * specp.n_steps / elp / 1e6:.0f} Mcell/s, "
                f"{kmsp / nlp * 1e3:.1f} us/launch")
            simp.close()
            del simp
        out["several_poles"] = poles_out

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
