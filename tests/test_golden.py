"""Stored oracle results (tests/golden/, written by tests/golden/make_golden.py):
the CPU test checks that the oracle still reproduces them, so any later
change of the oracle's arithmetic shows up here; the GPU test compares the
FP64 HIP path with the same numbers."""
import os

import numpy as np
import pytest

from paper_2609_30039_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read(name):
    out = {}
    with open(os.path.join(GOLDEN, name + ".txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            out[key] = np.array([float(v) for v in vals])
    return out


def _specs():
    return {
        "pec_cavity_probe": W.pec_cavity(32, 200),
        "cpml_lorentz_flux": W.lorentz_flux(pml=6, lorentz=8, n_steps=160, n_f=6, shape=(70, 23, 41)),
        "design_patch_gradient": W.design_patch(pml=6, design=12, patch=10, n_steps=120, n_f=3, shape=(46, 27, 39)),
    }


def _cells(g):
    c = g["cells_ijk"].astype(int)
    return [tuple(c[3 * m:3 * m + 3]) for m in range(len(c) // 3)]


def test_oracle_reproduces_golden():
    from oracle import oracle as O
    O.build()
    specs = _specs()
    g = read("pec_cavity_probe")
    sim = O.OracleSim(specs["pec_cavity_probe"])
    sim.step(200)
    np.testing.assert_allclose(sim.probe(0)[:200], g["Ez_probe"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose([np.linalg.norm(sim.field(q)) for q in range(6)], g["field_l2"], rtol=1e-12)
    g = read("cpml_lorentz_flux")
    sim = O.OracleSim(specs["cpml_lorentz_flux"])
    sim.step(160)
    np.testing.assert_allclose(O.OracleSim.flux_from_spectra(sim.spectra(0)), g["flux"], rtol=1e-12)
    g = read("design_patch_gradient")
    spec, cells = specs["design_patch_gradient"]
    assert [tuple(c) for c in cells] == _cells(g)
    sim = O.OracleSim(spec)
    sim.step(120)
    grad = sim.gradient({0: 2.0 * sim.spectra(0)}, 120).sum(axis=0)   # isotropic eps: sum of the components
    np.testing.assert_allclose([grad[k, j, i] for (i, j, k) in cells], g["dJ_deps"], rtol=1e-11)


@pytest.mark.gpu
def test_hip_fp64_matches_golden():
    from paper_2609_30039_amd.sim import Simulation
    from paper_2609_30039_amd import adjoint as A
    specs = _specs()
    g = read("pec_cavity_probe")
    sim = Simulation(specs["pec_cavity_probe"], dtype="f64")
    sim.step(200)
    np.testing.assert_allclose(sim.probe(0)[:200], g["Ez_probe"], rtol=1e-10, atol=1e-12 * np.abs(g["Ez_probe"]).max())
    np.testing.assert_allclose([np.linalg.norm(sim.field(q)) for q in range(6)], g["field_l2"], rtol=1e-10)
    g = read("cpml_lorentz_flux")
    sim = Simulation(specs["cpml_lorentz_flux"], dtype="f64")
    sim.step(160)
    np.testing.assert_allclose(sim.flux(0), g["flux"], rtol=1e-10)
    g = read("design_patch_gradient")
    spec, cells = specs["design_patch_gradient"]
    sim = Simulation(spec, dtype="f64", n_ckpt=9)
    grad = A.gradient(sim, 120, 9, lambda s: {(0, 0): 2.0 * s.spectra(0)})[0][0]
    (lo, _) = spec.grad_box
    vals = [grad[k - lo[2], j - lo[1], i - lo[0]] for (i, j, k) in cells]
    np.testing.assert_allclose(vals, g["dJ_deps"], rtol=1e-9, atol=1e-12 * np.abs(g["dJ_deps"]).max())
