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
    """Periodic axes need the split kernels; with a gradient, no reversible mode."""
    from paper_2609_30039_amd import binding as B
    spec = _periodic_spec((1, 1))
    with pytest.raises(B.FdtdError):
        Simulation(spec, dtype="f32", kernel="fused")
    spec.grad_box = ((5, 5, 10), (20, 15, 20))
    with pytest.raises(B.FdtdError):
        Simulation(spec, dtype="f32", reversible=True, max_steps=10)


# ---------------------------------------------------------------- the adjoint
def _cot(mi, m, sp):
    """Cotangents of J = sum Re flux + sum |patch|^2 + sum probe^2."""
    sp = np.asarray(sp)
    if m.kind == "flux_z":
        g = np.zeros_like(sp)
        g[:, 0], g[:, 3], g[:, 1], g[:, 2] = sp[:, 3], sp[:, 0], -sp[:, 2], -sp[:, 1]
        return g
    return 2.0 * sp


def _periodic_grad_spec(signs, n_steps=100):
    """A cell periodic in x and y (ragged against the 64-wide blocks), 6
    absorbing cells at each z end, diagonal eps across both seams, an Ex
    sheet and an Ey point source on the seam corner, a flux plane, an Ez
    patch across the x seam and an Hy probe; the gradient box spans both
    seams and reaches into the z faces."""
    nx, ny, nz = 37, 23, 30
    rng = np.random.Generator(np.random.PCG64(32))
    eps = 1.0 + 3.0 * rng.random((3, nz - 12, ny, nx))
    return W.DomainSpec(
        shape=(nx, ny, nz), courant=W.courant_3d(), pml=(0, 0, 0, 0, 6, 6), eps_kind="diag",
        eps_box=((0, 0, 6), (nx, ny, nz - 6)), eps=eps,
        sources=[W.SourceSpec("plane_z", 0, (0, 0, 8), W.gaussian_sine(n_steps, 0.3, 10.0, 30.0)),
                 W.SourceSpec("point", 1, (0, 0, 14), W.gaussian_sine(n_steps, 0.5, 6.0, 20.0))],
        monitors=[W.MonitorSpec("flux_z", pos=(0, 0, 20), rect=(0, nx, 0, ny), omega_dt=W.freq_grid(4, 0.2, 0.5)),
                  W.MonitorSpec("patch_z", comp=2, pos=(0, 0, 17), rect=(30, 37, 2, 20),
                                omega_dt=W.freq_grid(3, 0.2, 0.4)),
                  W.MonitorSpec("probe", comp=4, pos=(36, 22, 19))],
        n_steps=n_steps, periodic=(1, 1, 0), bloch_sign=(signs[0], signs[1], 1),
        grad_box=((0, 0, 2), (nx, ny, nz - 2)))


_ORC = {}


def _oracle_grad(signs):
    if signs not in _ORC:
        from tests.gpu_util import oracle_gradient
        spec = _periodic_grad_spec(signs)
        _, g = oracle_gradient(spec, _cot)
        (i0, j0, k0), (i1, j1, k1) = spec.grad_box
        _ORC[signs] = g[:, k0:k1, j0:j1, i0:i1].copy()
    return _ORC[signs]


@pytest.mark.parametrize("signs", [(1, 1), (-1, 1), (1, -1)])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_periodic_gradient_matches_oracle(signs, dtype, tol):
    """dJ/deps per component across the seams against the oracle's transposed sweep."""
    from tests.gpu_util import gpu_gradient_store_all
    spec = _periodic_grad_spec(signs)
    _, g, _ = gpu_gradient_store_all(spec, dtype, _cot, kernel="split")
    ref = _oracle_grad(signs)
    errs = [rel(g[c], ref[c]) for c in range(3)]
    print(f"periodic gradient signs={signs} {dtype}: per-component rel L2 "
          f"{', '.join(f'{e:.2e}' for e in errs)}", flush=True)
    assert max(errs) < tol
    assert np.abs(g[:, :, 0, :]).max() > 0 and np.abs(g[:, :, :, 0]).max() > 0   # seam planes carry gradient


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_periodic_and_walled_domains_gradients_in_one_batch(dtype, tol):
    """A periodic domain (its own per-node adjoint launches) beside a walled
    diagonal domain with a Lorentz box (the tiled passes), both with
    gradients, in one handle: each gradient equals that of the domain alone."""
    from tests.gpu_util import gpu_gradient_store_all
    p = _periodic_grad_spec((-1, 1), n_steps=60)
    d = W.anisotropic_lorentz(pml=5, lorentz=8, patch=10, n_steps=60, n_f=4, shape=(38, 26, 34))
    alone = [gpu_gradient_store_all(s, dtype, _cot, kernel="split")[1] for s in (p, d)]
    N = 60
    sim = Simulation([p, d], dtype=dtype, kernel="split", n_ckpt=N + 1, max_steps=N)
    sim.save(0)
    for n in range(N):
        sim.step(1)
        sim.save(n + 1)
    for dom, s in enumerate((p, d)):
        for mi, m in enumerate(s.monitors):
            sim.set_cotangent(mi, _cot(mi, m, sim.spectra(mi, dom)), domain=dom)
    sim.adjoint_begin(N)
    for m_ in range(N, 0, -1):
        sim.restore(m_ - 1)
        sim.step_adjoint(1)
    for dom in range(2):
        r = rel(sim.grad(dom), alone[dom])
        print(f"batch {dtype} domain {dom}: rel L2 vs alone {r:.2e}", flush=True)
        assert r < tol
    sim.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-9)])
def test_streamed_periodic_gradient_equals_resident(dtype, tol):
    """The host-streamed reverse sweep of the periodic domain (three z slabs)
    against the resident sweep."""
    from paper_2609_30039_amd.sim import StreamedSimulation
    from tests.gpu_util import gpu_gradient_store_all
    spec = _periodic_grad_spec((1, -1), n_steps=60)
    N = spec.n_steps
    _, g_res, _ = gpu_gradient_store_all(spec, dtype, _cot, kernel="split")
    s = StreamedSimulation(spec, 10, 2, dtype=dtype)
    s.step(N)
    for mi, m in enumerate(spec.monitors):
        sp = s.spectra(mi)
        s.set_cotangent(mi, _cot(mi, m, sp[:N] if m.kind == "probe" else sp))
    s.reverse()
    g = s.grad()
    info = s.info()
    s.close()
    r = rel(g, g_res)
    print(f"streamed periodic gradient {dtype} ({info['n_slabs']} slabs): rel L2 vs resident {r:.2e}", flush=True)
    assert info["n_slabs"] == 3
    assert r < tol


def test_eq5_slab_index_derivative_f64():
    """The Eq. 5 slab cell (periodic x and y, absorbing z ends): the
    derivative of the transmitted flux summed over the band with respect to
    the slab's permittivity, from the adjoint (the gradient summed over the
    slab cells), against central differences of two FP64 solves (the paper
    checks a Bloch-periodic slab's index derivative this way)."""
    from paper_2609_30039_amd import adjoint as ADJ
    spec, _ = slab_spec(2.25, n_steps=1200)
    spec.monitors = spec.monitors[1:]                 # the back plane
    nz = spec.shape[2]
    spec.grad_box = ((0, 0, 60), (spec.shape[0], spec.shape[1], 68))
    N = spec.n_steps

    def J_of(eps_slab):
        e = spec.eps.copy()
        e[0, 60:68] = eps_slab
        s = W.DomainSpec(**{**spec.__dict__, "eps": e, "grad_box": None})
        sim = Simulation(s, dtype="f64", kernel="split")
        sim.step(N)
        J = float(np.sum(O.OracleSim.flux_from_spectra(sim.spectra(0))))
        sim.close()
        return J

    sim = Simulation(spec, dtype="f64", kernel="split", n_ckpt=24, max_steps=N)
    g = ADJ.gradient(sim, N, 24, lambda s_: {(0, 0): _cot(0, spec.monitors[0], s_.spectra(0))})[0]
    sim.close()
    dJ = float(g.sum())
    h = 1e-4
    fd = (J_of(2.25 + h) - J_of(2.25 - h)) / (2 * h)
    print(f"Eq. 5 slab: dJ/deps_slab adjoint {dJ:.10e}, central differences {fd:.10e}, "
          f"rel {abs(dJ - fd) / abs(fd):.2e}", flush=True)
    assert abs(dJ - fd) <= 1e-6 * abs(fd)
    assert nz == 132


@pytest.mark.parametrize("signs", [(1, 1), (-1, 1)])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_periodic_dispersive_gradient_matches_oracle(signs, dtype, tol):
    """The periodic cell with its Lorentz box on the x seam (the pole
    histories' transposes next to the seam) and the gradient box over the
    box, across both seams and into the z faces: dJ/deps against the oracle."""
    from tests.gpu_util import gpu_gradient_store_all, oracle_gradient
    spec = _periodic_spec(signs, n_steps=100)
    nx, ny, nz = spec.shape
    spec.grad_box = ((0, 0, 3), (nx, ny, nz - 3))
    _, g, _ = gpu_gradient_store_all(spec, dtype, _cot, kernel="split")
    _, ref = oracle_gradient(spec, _cot)
    (i0, j0, k0), (i1, j1, k1) = spec.grad_box
    ref = ref[:, k0:k1, j0:j1, i0:i1].sum(axis=0)
    r = rel(g[0], ref)
    L = spec.lorentz[0]
    rl = rel(g[0][L.lo[2] - k0:L.hi[2] - k0, L.lo[1]:L.hi[1], L.lo[0]:L.hi[0]],
             ref[L.lo[2] - k0:L.hi[2] - k0, L.lo[1]:L.hi[1], L.lo[0]:L.hi[0]])
    print(f"periodic dispersive gradient signs={signs} {dtype}: rel L2 {r:.2e} (dispersive box {rl:.2e})", flush=True)
    assert r < tol and rl < 5 * tol
