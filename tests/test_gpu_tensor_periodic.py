"""Symmetric tensor media on Bloch-periodic axes (Sections 2.2, 2.3 and
3.1) on the GPU against the FP64 oracle.

Across a seam the assembly pass reads the edges at the other end times the
real Bloch factor and the node tensors there unchanged; the adjoint's E-node
pass gathers the same way and its H-node pass is the periodic one.  Covered:
x and y periodic with each sign pattern, absorbing faces in z holding
admitted tensors; a tensor box over the whole grid and one that meets only
the low side of the x seam (the node past the last column is inside the box,
the last column outside); fields, spectra and the gradient of all six
entries; a batch with a walled tensor domain; the host-streamed sweep.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_30039_amd import workloads as W
from paper_2609_30039_amd.sim import Simulation, StreamedSimulation
from tests.gpu_util import gpu_gradient_store_all, oracle_gradient, rel
from tests.test_gpu_tensor_adjoint import _cot, grad_tensor_spec

pytestmark = pytest.mark.gpu

SHAPE = (37, 29, 33)   # ragged against the 64-wide blocks and the 8-plane chunks
PML = 6


def _z_face_tensors(rng, shape, pml):
    """Rotated tensors between the z slabs; in them z is a principal axis
    with the largest eigenvalue and the x-y pair rotated (admitted)."""
    nx, ny, nz = shape
    eps = W.random_spd_tensors(rng, nx * ny * nz).reshape(6, nz, ny, nx)
    for ks in (slice(0, pml), slice(nz - pml, nz)):
        m = eps[:, ks].shape[1:]
        th = rng.uniform(0, np.pi, m)
        l1, l2 = 1.0 + 2.0 * rng.random(m), 1.0 + 2.0 * rng.random(m)
        cs, sn = np.cos(th), np.sin(th)
        eps[0, ks] = cs * cs * l1 + sn * sn * l2
        eps[1, ks] = sn * sn * l1 + cs * cs * l2
        eps[2, ks] = 3.5 + rng.random(m)
        eps[3, ks] = cs * sn * (l1 - l2)
        eps[4, ks] = 0.0
        eps[5, ks] = 0.0
    return eps


def periodic_tensor_spec(signs, box="full", n_steps=100, seed=53):
    """x and y periodic with Bloch factors signs, absorbing faces in z; node
    tensors over the whole grid (box="full") or over x in [0, nx - 5),
    y in [3, ny), between the z slabs (box="part"); an Ex sheet, an Ez
    point source on the x seam, a flux plane, an Ey patch across both seams
    and a probe of Hy on the y seam."""
    nx, ny, nz = SHAPE
    rng = np.random.Generator(np.random.PCG64(seed))
    if box == "full":
        lo, hi = (0, 0, 0), SHAPE
        eps = _z_face_tensors(rng, SHAPE, PML)
    else:
        lo, hi = (0, 3, PML), (nx - 5, ny, nz - PML)
        b = (hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2])
        eps = W.random_spd_tensors(rng, b[0] * b[1] * b[2]).reshape(6, b[2], b[1], b[0])
    return W.DomainSpec(
        shape=SHAPE, courant=W.courant_3d(), pml=(0, 0, 0, 0, PML, PML), eps_kind="tensor", eps_box=(lo, hi),
        eps=eps, eps_bg=1.5,
        sources=[W.SourceSpec("plane_z", 0, (0, 0, PML + 2), W.gaussian_sine(n_steps, 0.3, 10.0, 30.0)),
                 W.SourceSpec("point", 2, (0, ny // 3, nz // 2), W.gaussian_sine(n_steps, 0.5, 6.0, 20.0))],
        monitors=[W.MonitorSpec("flux_z", pos=(0, 0, nz - PML - 3), rect=(0, nx, 0, ny),
                                omega_dt=W.freq_grid(4, 0.2, 0.5)),
                  W.MonitorSpec("patch_z", comp=1, pos=(0, 0, nz // 2 + 2), rect=(0, nx, 0, ny),
                                omega_dt=W.freq_grid(3, 0.2, 0.4)),
                  W.MonitorSpec("probe", comp=4, pos=(nx // 2, 0, nz - 9))],
        grad_box=((0, 0, 0), SHAPE), n_steps=n_steps, periodic=(1, 1, 0), bloch_sign=(signs[0], signs[1], 1))


@pytest.mark.parametrize("box", ["full", "part"])
@pytest.mark.parametrize("signs", [(1, 1), (-1, 1), (1, -1)])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_periodic_tensor_fields_match_oracle(signs, box, dtype, tol):
    spec = periodic_tensor_spec(signs, box)
    spec.grad_box = None
    o = O.OracleSim(spec)
    o.step(spec.n_steps)
    g = Simulation(spec, dtype=dtype, kernel="split")
    g.step(spec.n_steps)
    errs = [rel(g.field(q), o.field(q)) for q in range(6)]
    sp = [rel(g.spectra(m), o.spectra(m)) for m in range(2)]
    print(f"periodic tensor signs={signs} box={box} {dtype}: fields {max(errs):.2e}, spectra {max(sp):.2e}",
          flush=True)
    assert max(errs) < tol and max(sp) < tol
    # E tangential to the periodic axes' first planes is free there (no wall)
    assert np.abs(g.field(2)[:, 0, 0]).max() > 0
    g.close()


@pytest.mark.parametrize("rows,kz,chunk", [(4, 8, 16), (8, 3, 32), (4, 5, 0)])
def test_periodic_tensor_launch_shapes_and_graph_chunks(rows, kz, chunk):
    """Both split block widths (64 columns by 4 rows, 32 by 8), ragged z
    chunks, and captured step chunks replayed several times: bit for bit the
    run of the default launch shape with eager steps, and the oracle's."""
    spec = periodic_tensor_spec((-1, 1), "part")
    spec.grad_box = None
    ref = Simulation(spec, dtype="f64", kernel="split", tile_rows=8, tile_kz=8)
    ref.step(spec.n_steps)
    g = Simulation(spec, dtype="f64", kernel="split", tile_rows=rows, tile_kz=kz, graph_chunk=chunk)
    g.step(spec.n_steps)
    for q in range(6):
        assert np.array_equal(g.field(q), ref.field(q)), W.COMP_NAMES[q]
    o = O.OracleSim(spec)
    o.step(spec.n_steps)
    assert max(rel(g.field(q), o.field(q)) for q in range(6)) < 1e-11
    g.close()
    ref.close()


_ORC = {}


def _oracle_grad(signs, box):
    key = (signs, box)
    if key not in _ORC:
        _ORC[key] = oracle_gradient(periodic_tensor_spec(signs, box), _cot)[1]
    return _ORC[key]


@pytest.mark.parametrize("signs,box", [((-1, 1), "full"), ((1, -1), "part"), ((-1, -1), "full")])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_periodic_tensor_gradient_matches_oracle(signs, box, dtype, tol):
    spec = periodic_tensor_spec(signs, box)
    _, g, _ = gpu_gradient_store_all(spec, dtype, _cot, kernel="split")
    ref = _oracle_grad(signs, box)
    assert g.shape == ref.shape == (6,) + SHAPE[::-1]
    errs = [rel(g[q], ref[q]) for q in range(6)]
    print(f"periodic tensor gradient signs={signs} box={box} {dtype}: per-entry "
          f"{', '.join(f'{e:.2e}' for e in errs)}; whole {rel(g, ref):.2e}", flush=True)
    assert rel(g, ref) < tol
    assert max(errs) < 5 * tol
    # the seam planes carry gradient of their own
    assert np.abs(ref[:, :, :, 0]).max() > 1e-3 * np.abs(ref).max()
    assert np.abs(ref[:, :, 0, :]).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_periodic_and_walled_tensor_domains_in_one_batch(dtype, tol):
    """A periodic tensor domain and a walled one in one handle, both with
    gradients: monitor spectra and gradients equal those of each domain
    alone (one assembly launch serves both; the adjoint's H-node pass is the
    periodic one for the first, the tiled one for the second)."""
    N = 60
    p = periodic_tensor_spec((-1, 1), "full", n_steps=N)
    w = grad_tensor_spec(False, n_steps=N)
    alone = []
    for s in (p, w):
        sim, g, cots = gpu_gradient_store_all(s, dtype, _cot, kernel="split")
        alone.append((cots, g))
        sim.close()
    sim = Simulation([p, w], dtype=dtype, kernel="split", n_ckpt=N + 1, max_steps=N)
    sim.save(0)
    for n in range(N):
        sim.step(1)
        sim.save(n + 1)
    worst = 0.0
    for dom, s in enumerate((p, w)):
        for mi, m in enumerate(s.monitors):
            c = _cot(mi, m, sim.spectra(mi, dom))
            worst = max(worst, rel(c, alone[dom][0][mi]))
            sim.set_cotangent(mi, c, domain=dom)
    sim.adjoint_begin(N)
    for m_ in range(N, 0, -1):
        sim.restore(m_ - 1)
        sim.step_adjoint(1)
    for dom in range(2):
        rg = rel(sim.grad(dom), alone[dom][1])
        print(f"batch {dtype} domain {dom}: spectra {worst:.2e}, gradient {rg:.2e} vs alone", flush=True)
        assert worst < tol and rg < tol
    sim.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-9)])
def test_streamed_periodic_tensor_gradient_equals_resident(dtype, tol):
    """The host-streamed reverse sweep (three 12-plane slabs, 3 steps per
    visit) of a periodic tensor domain against the resident sweep."""
    spec = periodic_tensor_spec((-1, 1), "full", n_steps=60)
    N = spec.n_steps
    sim, g_res, _ = gpu_gradient_store_all(spec, dtype, _cot, kernel="split")
    sim.close()
    s = StreamedSimulation(spec, 12, 3, dtype=dtype)
    s.step(N)
    for mi, m in enumerate(spec.monitors):
        sp = s.spectra(mi)
        s.set_cotangent(mi, _cot(mi, m, sp[:N] if m.kind == "probe" else sp))
    s.reverse()
    g = s.grad()
    info = s.info()
    s.close()
    r = rel(g, g_res)
    print(f"streamed periodic tensor gradient {dtype} ({info['n_slabs']} slabs): rel L2 vs resident {r:.2e}",
          flush=True)
    assert info["n_slabs"] == 3
    assert r < tol
