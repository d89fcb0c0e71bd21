"""Write the stored expected values under tests/golden/ from the FP64 oracle.

Every number in the fixtures comes from ``oracle/`` run on the seeded inputs
of ``paper_2609_30039_amd.workloads``; nothing is taken from the GPU path.
Run from the repository root:

    python tests/golden/make_golden.py

The fixtures are regression records of the oracle at full precision (17
significant digits): the CPU tests check that the oracle still reproduces
them, the GPU tests compare the FP64 HIP path with them.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O                      # noqa: E402
from paper_2609_30039_amd import workloads as W     # noqa: E402

FIXTURES = {
    # name: (description, builder)
    "pec_cavity_probe": (
        "32^3 PEC cavity, per-cell eps in [1,4] (seed 1001), Ez point source at the centre, 200 FP64 steps: "
        "Ez probe trace (point samples, Section 2.4) and the L2 norm of each field at the end (Eq. 1)",
        lambda: W.pec_cavity(32, 200)),
    "cpml_lorentz_flux": (
        "70x23x41 cells, 6-cell CPML (Section 2.2), 8^3 one-pole Lorentz block (Section 2.3), Ex sheet source, "
        "160 FP64 steps: Poynting flux per frequency of the far z-plane monitor (Section 2.4)",
        lambda: W.lorentz_flux(pml=6, lorentz=8, n_steps=160, n_f=6, shape=(70, 23, 41))),
    "design_patch_gradient": (
        "46x27x39 cells, 6-cell CPML, 12^3 random design box (seed 1003), |DFT Ez|^2 patch objective, 120 FP64 "
        "steps: dJ/deps (discrete adjoint, Eq. 3; isotropic eps, so the sum of the three component terms) at the "
        "design cells drawn by the workload generator",
        lambda: W.design_patch(pml=6, design=12, patch=10, n_steps=120, n_f=3, shape=(46, 27, 39))),
}


def compute(name):
    spec = FIXTURES[name][1]()
    if name == "design_patch_gradient":
        spec, cells = spec
        sim = O.OracleSim(spec)
        sim.step(spec.n_steps)
        cot = {0: 2.0 * sim.spectra(0)}
        # isotropic eps: one scalar per cell feeds all three E components, so
        # dJ/deps is the sum of the three per-component terms
        g = sim.gradient(cot, spec.n_steps).sum(axis=0)
        return {"J": [float(np.sum(np.abs(sim.spectra(0)) ** 2))],
                "cells_ijk": [c for cell in cells for c in cell],
                "dJ_deps": [float(g[k, j, i]) for (i, j, k) in cells]}
    sim = O.OracleSim(spec)
    sim.step(spec.n_steps)
    if name == "pec_cavity_probe":
        return {"Ez_probe": [float(v) for v in sim.probe(0)[:spec.n_steps]],
                "field_l2": [float(np.linalg.norm(sim.field(q))) for q in range(6)]}
    return {"flux": [float(v) for v in O.OracleSim.flux_from_spectra(sim.spectra(0))]}


def write(name, data):
    path = os.path.join(HERE, name + ".txt")
    with open(path, "w") as fh:
        fh.write(f"# {FIXTURES[name][0]}\n")
        fh.write("# written by tests/golden/make_golden.py from the FP64 oracle\n")
        for key, vals in data.items():
            fh.write(f"{key} " + " ".join(repr(v) for v in vals) + "\n")


def read(name):
    out = {}
    with open(os.path.join(HERE, name + ".txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            out[key] = np.array([float(v) for v in vals])
    return out


if __name__ == "__main__":
    O.build()
    for name in FIXTURES:
        write(name, compute(name))
        print("wrote", name)
