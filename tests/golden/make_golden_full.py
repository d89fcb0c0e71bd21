"""Write the full-length reference records under tests/golden/ from the FP64 oracle.

Every number comes from ``oracle/`` run on the seeded inputs of
``paper_2609_30039_amd.workloads``; nothing is taken from the GPU path.  The
runs take about an hour on an 8-core host, so they live apart from
``make_golden.py``.  Run from the repository root:

    python tests/golden/make_golden_full.py [lorentz_flux_1000] [anisotropic_reduced] [design_patch_full]

Records (compressed ``.npz``, FP64, loaded with ``numpy.load`` and no pickle):

lorentz_flux_1000
    The 148^3 one-pole Lorentz workload (128^3 + 10-cell CPML), 1000 steps:
    the six fields on a strided sample of nodes, each field's whole-grid L2
    norm, and the flux per frequency (Section 2.4).  Also the floor that
    float32 state storage alone sets: the same run with the whole state
    rounded to float32 after every step (FP64 arithmetic), as relative L2
    errors per field (whole grid and on the sample) and relative flux errors.
anisotropic_reduced
    The 536^3 anisotropic workload scaled down with its structure kept:
    128^3 + 12-cell CPML, diagonal eps with each component in [1,5]
    (seed 1005), a central 32^3 Lorentz box, Ex sheet, Ex patch 32x32 over 8
    frequencies, 1000 steps.  Fields on a strided sample, the float32-storage
    floor, the patch spectra, J = sum |Ex(w)|^2 and dJ/deps per component
    (discrete adjoint, Eq. 3) on every 4th cell of the interior box, with the
    whole-box L2 norm per component.
design_patch_full
    The 212^3 design workload (192^3 + 10-cell CPML, 64^3 design box, seed
    1003), 2000 steps: J and dJ/deps over the whole design box (isotropic eps:
    the three component terms summed), and at the generator's 20 cells.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O                      # noqa: E402
from paper_2609_30039_amd import workloads as W     # noqa: E402

# field sample: every 6th node along each axis starting at 3 ([nz][ny][nx])
FIELD_SAMPLE = (3, 6)
# gradient sample of the reduced anisotropic workload: every 4th cell of the box from offset 2
GRAD_SAMPLE = (2, 4)
T0 = time.time()


def log(msg):
    print(f"[{time.time() - T0:7.1f} s] {msg}", flush=True)


def field_sample(f):
    a, s = FIELD_SAMPLE
    return f[a::s, a::s, a::s]


def rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def forward_pair(spec, n_steps):
    """FP64 run and the float32-storage run of the same spec."""
    ref = O.OracleSim(spec)
    for t0 in range(0, n_steps, 250):
        ref.step(min(250, n_steps - t0))
        log(f"  fp64 step {ref.t}")
    f32 = O.OracleSim(spec)
    for t0 in range(0, n_steps, 250):
        f32.step(min(250, n_steps - t0), store_f32=True)
        log(f"  f32-storage step {f32.t}")
    out = {
        "fields_sample": np.stack([field_sample(ref.field(q)) for q in range(6)]),
        "field_norm": np.array([np.linalg.norm(ref.field(q)) for q in range(6)]),
        "f32store_rel_whole": np.array([rel(f32.field(q), ref.field(q)) for q in range(6)]),
        "f32store_rel_sample": np.array([rel(field_sample(f32.field(q)), field_sample(ref.field(q)))
                                         for q in range(6)]),
        "field_sample_spec": np.array(FIELD_SAMPLE),
    }
    return ref, f32, out


def lorentz_flux_1000():
    spec = W.lorentz_flux()
    ref, f32, out = forward_pair(spec, 1000)
    fl = O.OracleSim.flux_from_spectra(ref.spectra(0))
    fl32 = O.OracleSim.flux_from_spectra(f32.spectra(0))
    out["flux"] = fl
    out["f32store_flux_rel"] = np.abs(fl32 - fl) / np.abs(fl)
    out["description"] = np.array("148^3 one-pole Lorentz workload, 1000 FP64 oracle steps: field sample, norms, "
                                  "flux; float32-storage floor")
    return out


def anisotropic_reduced_spec():
    return W.anisotropic_lorentz(interior=128, pml=12, lorentz=32, patch=32, n_steps=1000)


def anisotropic_reduced():
    spec = anisotropic_reduced_spec()
    ref, f32, out = forward_pair(spec, spec.n_steps)
    sp = ref.spectra(0)
    out["spectra"] = sp
    out["f32store_spectra_rel"] = np.array(rel(f32.spectra(0), sp))
    out["J"] = np.array(float(np.sum(np.abs(sp) ** 2)))
    del f32
    log("  gradient (bisection replay)")
    g = ref.gradient({0: 2.0 * sp}, spec.n_steps)
    (i0, j0, k0), (i1, j1, k1) = spec.grad_box
    box = g[:, k0:k1, j0:j1, i0:i1]
    a, s = GRAD_SAMPLE
    out["grad_sample"] = np.ascontiguousarray(box[:, a::s, a::s, a::s])
    out["grad_norm"] = np.array([np.linalg.norm(box[c]) for c in range(3)])
    out["grad_sample_spec"] = np.array(GRAD_SAMPLE)
    out["description"] = np.array("128^3+12 CPML anisotropic workload with a 32^3 Lorentz box, 1000 FP64 oracle "
                                  "steps: field sample, floor, patch spectra, J, dJ/deps per component sampled")
    return out


def design_patch_full():
    spec, cells = W.design_patch()
    sim = O.OracleSim(spec)
    for t0 in range(0, spec.n_steps, 250):
        sim.step(min(250, spec.n_steps - t0))
        log(f"  fp64 step {sim.t}")
    sp = sim.spectra(0)
    log("  gradient (bisection replay)")
    g = sim.gradient({0: 2.0 * sp}, spec.n_steps).sum(axis=0)
    (i0, j0, k0), (i1, j1, k1) = spec.grad_box
    return {
        "J": np.array(float(np.sum(np.abs(sp) ** 2))),
        "grad": np.ascontiguousarray(g[k0:k1, j0:j1, i0:i1]),
        "cells_ijk": np.array(cells, dtype=np.int64),
        "grad_cells": np.array([g[k, j, i] for (i, j, k) in cells]),
        "description": np.array("212^3 design workload, 2000 FP64 oracle steps: J and dJ/deps over the design box "
                                "(component terms summed)"),
    }


RECORDS = {"lorentz_flux_1000": lorentz_flux_1000, "anisotropic_reduced": anisotropic_reduced,
           "design_patch_full": design_patch_full}


def path(name):
    return os.path.join(HERE, name + ".npz")


def read(name):
    with np.load(path(name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    O.build()
    names = sys.argv[1:] or list(RECORDS)
    for name in names:
        log(f"{name}: start")
        data = RECORDS[name]()
        np.savez_compressed(path(name), **data)
        log(f"{name}: wrote {path(name)}")
