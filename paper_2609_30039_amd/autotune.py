"""Launch-shape autotuner for the stepping kernels.

Candidates are the kernel family (split E/H launches or fused single pass)
and the tile shape (register-blocked rows per wave, z planes per block).  Each
candidate is timed through the C-ABI on a handle of the real workload (HIP
events around the stepping launches only, monitors off), forward steps and
optionally adjoint steps, and the fastest is kept.  Results are cached in a
JSON file keyed by the dtype, the device name and a signature of the domain
geometry (shapes, absorber depths, dispersive boxes with their pole kinds, eps
boxes, sources), because the best shape depends on how the tiles fall onto
absorbers and dispersive regions as much as on the size.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Sequence

from . import binding as B
from .sim import Simulation

CANDIDATES = [
    {"kernel": "split", "tile_rows": 0, "tile_kz": 4},
    {"kernel": "split", "tile_rows": 0, "tile_kz": 8},
    {"kernel": "split", "tile_rows": 0, "tile_kz": 16},
    {"kernel": "split", "tile_rows": 8, "tile_kz": 2},
    {"kernel": "split", "tile_rows": 8, "tile_kz": 3},
    {"kernel": "split", "tile_rows": 8, "tile_kz": 4},
    {"kernel": "split", "tile_rows": 8, "tile_kz": 8},
    {"kernel": "onepass", "tile_rows": 8, "tile_kz": 8},
    {"kernel": "onepass", "tile_rows": 8, "tile_kz": 16},
    {"kernel": "onepass", "tile_rows": 0, "tile_kz": 16},
    {"kernel": "fused", "tile_rows": 2, "tile_kz": 8},
    {"kernel": "fused", "tile_rows": 2, "tile_kz": 16},
    {"kernel": "fused", "tile_rows": 4, "tile_kz": 8},
    {"kernel": "fused", "tile_rows": 4, "tile_kz": 16},
]


def _cache_path() -> str:
    return os.environ.get("FDTD_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fdtd_tune.json"))


def signature(specs: Sequence, dtype: str, adjoint: bool) -> str:
    h = hashlib.sha256()
    for s in specs:
        lor = [(L.lo, L.hi, [p.kind for p in L.pole_list()]) for L in s.lorentz]
        src = [(x.kind, x.comp, tuple(x.pos)) for x in s.sources]
        h.update(repr((s.shape, tuple(s.pml), s.eps_kind, s.eps_box, lor, src, s.grad_box,
                       tuple(getattr(s, "periodic", (0, 0, 0))))).encode())
    dev = "unknown"
    try:
        import torch
        dev = torch.cuda.get_device_name(0)
    except Exception:
        pass
    return f"{dtype}|{dev}|{'adj' if adjoint else 'fwd'}|{h.hexdigest()[:16]}"


def _burst(sim, n, chunk):
    """n stepping launches in chunks, resetting to rest before the run would
    pass the step capacity (source samples beyond it are simply zero)."""
    done = 0
    while done < n:
        c = min(chunk, n - done)
        if sim.steps[0] + c > sim.max_steps:
            sim.reset()
        sim.step(c, record=False)
        done += c


def _time(specs, dtype, cand, steps, adjoint, stream, min_ms) -> float:
    """Average stepping time per time step (ms): a short probe sizes the run so
    that at least min_ms of kernel time is measured (clocks need a sustained
    load before they settle; a handful of launches under-reports)."""
    cap = max(steps + 4, 64)
    try:
        sim = Simulation(specs, dtype=dtype, stream=stream, max_steps=cap, **cand)
    except B.FdtdError as e:
        if e.code != B.FDTD_E_INVALID:
            raise
        return float("inf")                 # a shape this workload does not admit (e.g. periodic + fused)
    try:
        sim.step(2, record=False)
        sim.timing(1)
        sim.step(steps, record=False)
        ms, n = sim.timing(2)
        per = ms / max(n, 1)
        need = max(steps, int(min_ms / max(per, 1e-4)))
        _burst(sim, need // 4, 32)          # settle
        sim.timing(1)
        _burst(sim, need, 32)
        ms, n = sim.timing(2)
        total = ms / max(n, 1)
        if adjoint and any(s.grad_box is not None for s in specs):
            t = sim.steps[0]
            sim.timing(1)
            for _ in range(max(steps, min(need, 200))):
                sim.adjoint_begin(t + 1)
                sim.step_adjoint(1)
            ms, n = sim.timing(2)
            total += ms / max(n, 1)
        return total
    finally:
        sim.close()


def tune(specs, dtype: str = "f32", adjoint: bool = False, steps: int = 6, stream: Optional[int] = None,
         use_cache: bool = True, candidates: Optional[List[Dict]] = None, log=None, min_ms: float = 40.0) -> Dict:
    """Best launch shape {kernel, tile_rows, tile_kz} for this workload."""
    if not isinstance(specs, (list, tuple)):
        specs = [specs]
    cands = candidates or CANDIDATES
    # the key also names the candidate list, so a changed list is measured afresh
    key = signature(specs, dtype, adjoint) + "|" + hashlib.sha256(repr(cands).encode()).hexdigest()[:8]
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return dict(cache[key]["best"])
    results = []
    for cand in cands:
        ms = _time(specs, dtype, cand, steps, adjoint, stream, min_ms)
        results.append((ms, cand))
        if log:
            log(f"tune {cand}: {ms * 1e3:.1f} us/step")
    results.sort(key=lambda x: x[0])
    best = dict(results[0][1])
    cache[key] = {"best": best, "us_per_step": [(round(m * 1e3, 2), c) for m, c in results]}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(cache, fh, indent=1)
        except OSError:
            pass
    return best
