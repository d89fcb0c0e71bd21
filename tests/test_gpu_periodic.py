"""Bloch-periodic boundaries (x and y, real factor +1 or -1) on the GPU
against the oracle, and the lossless-slab check of Eq. 5 (Section 6.1)
through the library's flux planes."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_30039_amd import workloads as W
from paper_2609_30039_amd.sim import Simulation
from tests.gpu_util import rel
from tests.test_oracle_pins import eq5_T, slab_spec, slab_TR

pytestmark = pytest.mark.gpu


def _periodic_spec(signs, n_steps=120):
    """A cell periodic in x and y with 6 absorbing cells at each z end, a
    random permittivity box across both seams, a Lorentz box on the x seam,
    an Ex sheet and an Ey point source, a flux plane: every seam path of the
    split kernels (plain, absorbing, dispersive columns) is used."""
    nx, ny, nz = 37, 23, 30
    rng = np.random.Generator(np.random.PCG64(31))
    eps = 1.0 + 3.0 * rng.random((1, nz - 12, ny, nx))
    return W.DomainSpec(
        shape=(nx, ny, nz), courant=W.courant_3d(), pml=(0, 0, 0, 0, 6, 6), eps_kind="iso",
        eps_box=((0, 0, 6), (nx, ny, nz - 6)), eps=eps,
        lorentz=[W.LorentzSpec((0, 3, 10), (5, 12, 18), 1.5, 0.3, 0.02)],
        sources=[W.SourceSpec("plane_z", 0, (0, 0, 8), W.gaussian_sine(n_steps, 0.3, 10.0, 30.0)),
                 W.SourceSpec("point", 1, (0, 0, 14), W.gaussian_sine(n_steps, 0.5, 6.0, 20.0))],
        monitors=[W.MonitorSpec("flux_z", pos=(0, 0, 20), rect=(0, nx, 0, ny), omega_dt=W.freq_grid(4, 0.2, 0.5))],
        n_steps=n_steps, periodic=(1, 1, 0), bloch_sign=(signs[0], signs[1], 1))


@pytest.mark.parametrize("signs", [(1, 1), (-1, 1), (1, -1)])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_bloch_periodic_fields_and_flux(signs, dtype, tol):
    spec = _periodic_spec(signs)
    o = O.OracleSim(spec)
    o.step(spec.n_steps)
    g = Simulation(spec, dtype=dtype, kernel="split")
    g.step(spec.n_steps)
    for q in range(6):
        r = rel(g.field(q), o.field(q))
        assert r < tol, (W.COMP_NAMES[q], r)
    assert rel(g.spectra(0), o.spectra(0)) < tol
    # E tangential to the periodic axes' first planes is free there (no wall)
    assert np.abs(g.field(2)[:, 0, 0]).max() > 0


def test_lossless_slab_eq5_on_the_gpu():
    """The Eq. 5 slab through the FP64 library: spectra equal the oracle's,
    and T, R match the analytic slab transmission to the oracle's accuracy."""
    out_g, out_o = [], []
    for e in (1.0, 2.25):
        spec, lam = slab_spec(e)
        g = Simulation(spec, dtype="f64", kernel="split")
        g.step(spec.n_steps)
        out_g.append((g.spectra(0), g.spectra(1)))
        o = O.OracleSim(spec)
        o.step(spec.n_steps)
        out_o.append((o.spectra(0), o.spectra(1)))
        for m in range(2):
            assert rel(out_g[-1][m], out_o[-1][m]) < 1e-11
    T, R = slab_TR(out_g[0], out_g[1])
    Ta = eq5_T(lam)
    eT, eR = np.max(np.abs(T - Ta)), np.max(np.abs(R - (1.0 - Ta)))
    print(f"Eq. 5 slab on the GPU: max |T - T_eq5| {eT:.3e}, max |R - R_eq5| {eR:.3e}, "
          f"max |R + T - 1| {np.max(np.abs(R + T - 1)):.3e}", flush=True)
    assert eT < 2e-3 and eR < 2e-3 and np.max(np.abs(R + T - 1.0)) < 2e-5


def test_periodic_refusals():
    from paper_2609_30039_amd import binding as B
    spec = _periodic_spec((1, 1))
    with pytest.raises(B.FdtdError):
        Simulation(spec, dtype="f32", kernel="fused")
    spec.grad_box = ((5, 5, 10), (20, 15, 20))
    with pytest.raises(B.FdtdError):
        Simulation(spec, dtype="f32")
