"""Parity at the full sizes of the benchmark workloads, in the launch shapes
the autotuner picks there (split kernels, 8-row blocks, z chunks of 2, 3, 4
or 8 planes) and with captured step chunks where the benchmark uses them.

The oracle is too slow for whole full-size runs, so these tests take few steps
from a seeded random state in all six fields: every node then carries data,
every absorber memory and Lorentz history becomes nonzero after the first
step, and each output is compared element by element with the oracle started
from the same state.  The adjoint is checked at full size through a property
that holds at any size: the dot-product identity <A x, y> = <x, A^T y> for the
linear step A (sources removed) and random x, y.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_30039_amd import workloads as W
from paper_2609_30039_amd import adjoint as A
from paper_2609_30039_amd.sim import Simulation
from tests.gpu_util import rel

pytestmark = pytest.mark.gpu


def _random_fields(shape, seed):
    """Six seeded N(0,1) fields [nz][ny][nx]; E_c is zero where the index along
    c+1 or c+2 is 0 (the PEC nodes, which are not degrees of freedom)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    k, j, i = np.ogrid[:nz, :ny, :nx]
    idx = (i, j, k)
    out = []
    for q in range(6):
        f = rng.standard_normal((nz, ny, nx))
        if q < 3:
            f[np.broadcast_to((idx[(q + 1) % 3] == 0) | (idx[(q + 2) % 3] == 0), f.shape)] = 0.0
        out.append(f)
    return out


def _start(spec, fields, dtype, **kw):
    sim = Simulation(spec, dtype=dtype, **kw)
    for q in range(6):
        sim.set_field(q, fields[q])
    return sim


def _oracle(spec, fields, n, record):
    o = O.OracleSim(spec)
    for q in range(6):
        o.field(q)[...] = fields[q]
    o.step(n, record=record)
    return o


@pytest.fixture(scope="module")
def flux148():
    spec = W.lorentz_flux()
    fields = _random_fields(spec.shape, 7001)
    o = _oracle(spec, fields, 64, True)
    return spec, fields, o


@pytest.mark.parametrize("shape", [(8, 2), (8, 3), (8, 4), (8, 8)])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_headline_148_fields_and_spectra(flux148, shape, dtype, tol):
    """148^3 + Lorentz box + sheet source + 16-frequency flux plane, 64 steps in
    two captured chunks of 32: six fields and the flux spectra."""
    spec, fields, o = flux148
    sim = _start(spec, fields, dtype, kernel="split", tile_rows=shape[0], tile_kz=shape[1], graph_chunk=32)
    sim.step(64, record=True)
    for q in range(6):
        r = rel(sim.field(q), o.field(q))
        assert r < tol, (W.COMP_NAMES[q], r)
    assert rel(sim.spectra(0), o.spectra(0)) < tol
    sim.close()


def test_anisotropic_536_fields():
    """536^3 (512^3 + 12-cell CPML, diagonal eps, 128^3 Lorentz box), 3 steps
    from a random state, FP64 and FP32 at the tuned shape, every node."""
    spec = W.anisotropic_lorentz()
    fields = _random_fields(spec.shape, 7002)
    o = _oracle(spec, fields, 3, False)
    for dtype, tol in (("f64", 1e-12), ("f32", 3e-6)):
        sim = _start(spec, fields, dtype, kernel="split", tile_rows=8, tile_kz=2)
        sim.step(3, record=False)
        for q in range(6):
            r = rel(sim.field(q), o.field(q))
            assert r < tol, (dtype, W.COMP_NAMES[q], r)
        sim.close()
        del sim
    del o


def _inner(a, b):
    return sum(float(np.dot(a[q].ravel().astype(np.float64), b[q].ravel().astype(np.float64))) for q in range(6))


def _norm(a):
    return np.sqrt(sum(float(np.sum(np.square(a[q].astype(np.float64)))) for q in range(6)))


@pytest.mark.parametrize("shape", [(8, 2), (8, 3), (8, 8)])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_design_patch_212_adjoint_dot_product(shape, dtype, tol):
    """212^3 + CPML with the 64^3 random-eps design box, gradient box on: one
    adjoint step (every tile class of both passes) is the transpose of one
    forward step, <A x, y> = <x, A^T y>, relative to |A x| |y|."""
    spec, _ = W.design_patch()
    spec.sources = []
    x = _random_fields(spec.shape, 7003)
    y = _random_fields(spec.shape, 7004)
    sim = _start(spec, x, dtype, kernel="split", tile_rows=shape[0], tile_kz=shape[1], n_ckpt=1)
    sim.save(0)
    sim.step(1, record=False)
    ax = [sim.field(q) for q in range(6)]
    sim.restore(0)
    sim.adjoint_begin(1)
    for q in range(6):
        sim.set_field(q, y[q], adjoint=True)
    sim.step_adjoint(1)
    aty = [sim.field(q, adjoint=True) for q in range(6)]
    lhs, rhs = _inner(ax, y), _inner(x, aty)
    scale = _norm(ax) * _norm(y)
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs, scale)
    sim.close()


def test_batch_48_domains_sampled():
    """The 48 ragged domains in one launch (tuned shape, captured chunks),
    32 steps from rest: the smallest, the largest and a middle domain against
    the oracle, fields and flux spectra."""
    specs = W.batch_domains()
    cells = [s.ncells for s in specs]
    pick = sorted({int(np.argmin(cells)), int(np.argmax(cells)), len(specs) // 2})
    sim = Simulation(specs, dtype="f64", kernel="split", tile_rows=8, tile_kz=2, graph_chunk=32)
    sim.step(32, record=True)
    for d in pick:
        o = O.OracleSim(specs[d])
        o.step(32, record=True)
        for q in range(6):
            r = rel(sim.field(q, domain=d), o.field(q))
            assert r < 1e-12, (d, W.COMP_NAMES[q], r)
        assert rel(sim.spectra(0, domain=d), o.spectra(0)) < 1e-12
    sim.close()


def test_design_patch_212_gradient_vs_central_differences():
    """The full design workload (212^3, 2000 steps, 24 binomial slots): the FP32
    adjoint gradient at the generator's 20 seeded design cells against central
    differences of J = sum |DFT Ez|^2 from FP64 solves, eps -> eps (1 +- 1e-3)
    at one cell.  Cells whose gradient is below 1e-3 of the largest among them
    are compared in absolute terms."""
    spec, cells = W.design_patch()
    N = spec.n_steps
    shape = dict(kernel="split", tile_rows=8, tile_kz=3)
    sim32 = Simulation(spec, dtype="f32", n_ckpt=24, graph_chunk=32, **shape)
    g = A.gradient(sim32, N, 24, lambda s_: {(0, 0): 2.0 * s_.spectra(0)})[0][0]
    sim32.close()
    lo, _ = spec.eps_box
    sim64 = Simulation(spec, dtype="f64", graph_chunk=32, **shape)

    def J(eps):
        sim64.reset()
        sim64.set_eps(eps)
        sim64.step(N, record=True)
        return float(np.sum(np.abs(sim64.spectra(0)) ** 2))

    fd, ad = [], []
    for (i, j, k) in cells:
        c = (k - lo[2], j - lo[1], i - lo[0])
        e0 = spec.eps[(0,) + c]
        d = 1e-3 * e0
        ep, em = spec.eps.copy(), spec.eps.copy()
        ep[(0,) + c] = e0 + d
        em[(0,) + c] = e0 - d
        fd.append((J(ep) - J(em)) / (2 * d))
        ad.append(g[c])
    sim64.close()
    fd, ad = np.array(fd), np.array(ad)
    big = np.abs(fd).max()
    err = np.abs(ad - fd) / np.maximum(np.abs(fd), 1e-3 * big)
    assert err.max() < 1e-3, (err, fd, ad)


# two Lorentz poles and a Drude pole
POLES = [W.PoleSpec("lorentz", 0.9, 0.45, 0.05), W.PoleSpec("lorentz", 0.6, 0.7, 0.1),
         W.PoleSpec("drude", 0.0, 0.35, 0.08)]


def _float32_storage_error(spec, fields, n):
    """Per-field relative error of the FP64 oracle whose whole state is rounded
    to float32 after every step, against the plain FP64 oracle: what storing
    the state in FP32 costs by itself."""
    a, b = _oracle(spec, fields, 0, False), _oracle(spec, fields, 0, False)
    b.u[...] = b.u.astype(np.float32)
    for _ in range(n):
        a.step(1, record=False)
        b.step(1, record=False)
        b.u[...] = b.u.astype(np.float32)
    return [rel(b.field(q), a.field(q)) for q in range(6)], a


def test_headline_148_several_poles():
    """148^3 with the 48^3 dispersive box holding two Lorentz poles and a Drude
    pole (its cells updated by the leading blocks of the E launch), 32 steps
    from a random state in one captured chunk, tuned shape, every node.  FP64
    to 1e-11; FP32 to 3x the float32 storage error, never below 2e-5."""
    spec = W.lorentz_flux()
    L = spec.lorentz[0]
    spec.lorentz = [W.LorentzSpec(L.lo, L.hi, 0.0, 0.0, 0.0, poles=POLES)]
    fields = _random_fields(spec.shape, 7005)
    store_err, o = _float32_storage_error(spec, fields, 32)
    for dtype in ("f64", "f32"):
        sim = _start(spec, fields, dtype, kernel="split", tile_rows=8, tile_kz=3, graph_chunk=32)
        sim.step(32, record=False)
        for q in range(6):
            tol = 1e-11 if dtype == "f64" else max(2e-5, 3.0 * store_err[q])
            r = rel(sim.field(q), o.field(q))
            assert r < tol, (dtype, W.COMP_NAMES[q], r, tol)
        sim.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_design_patch_212_several_poles_adjoint_dot_product(dtype, tol):
    """212^3 with a 24^3 box of two Lorentz poles and a Drude pole across a
    corner of the gradient box (dielectric, dispersive, in-box and out-of-box
    gradient cells): three adjoint steps are the transpose of three forward
    steps, <A^3 x, y> = <x, (A^T)^3 y>.  x and y live in the six fields; the
    first step fills every pole's history, so the later steps carry all the
    pole terms both ways."""
    spec, _ = W.design_patch()
    spec.sources = []
    lo, _ = spec.grad_box
    blo = tuple(c - 12 for c in lo)
    spec.lorentz = [W.LorentzSpec(blo, tuple(c + 24 for c in blo), 0.0, 0.0, 0.0, poles=POLES)]
    x = _random_fields(spec.shape, 7006)
    y = _random_fields(spec.shape, 7007)
    sim = _start(spec, x, dtype, kernel="split", tile_rows=8, tile_kz=3, n_ckpt=3)
    for t in range(3):
        sim.save(t)
        sim.step(1, record=False)
    ax = [sim.field(q) for q in range(6)]
    sim.adjoint_begin(3)
    for q in range(6):
        sim.set_field(q, y[q], adjoint=True)
    for m in range(3, 0, -1):
        sim.restore(m - 1)
        sim.step_adjoint(1)
    aty = [sim.field(q, adjoint=True) for q in range(6)]
    lhs, rhs = _inner(ax, y), _inner(x, aty)
    scale = _norm(ax) * _norm(y)
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs, scale)
    sim.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12)])
def test_anisotropic_tensor_536_local_windows(dtype, tol):
    """The 536^3 tensor workload (a rotated tensor at every interior node) at
    full size, 3 steps from a random state in the tuned launch shape, checked
    on three 20^3 windows spread over the interior (near the low corner, the
    centre, near the high corner: different tiles, XCD runs and large
    offsets).  The oracle steps each window with a margin of 5 planes: a
    window's faces act as walls, whose error moves one plane per step, so the
    inner 20^3 is exact after 3 steps."""
    spec = W.anisotropic_tensor(n_steps=4)
    spec.sources = []
    fields = _random_fields(spec.shape, 7003)
    sim = _start(spec, fields, dtype, kernel="split", tile_rows=8, tile_kz=8)
    sim.step(3, record=False)
    got = [sim.field(q) for q in range(6)]
    sim.close()
    del sim
    (bx0, by0, bz0), _ = spec.eps_box
    m, w, n = 5, 20, 3
    for c in ((40, 45, 50), (268, 261, 270), (494, 500, 497)):
        lo = [c[a] - w // 2 - m for a in range(3)]
        hi = [c[a] + w // 2 + m for a in range(3)]
        shape = tuple(hi[a] - lo[a] for a in range(3))
        win = W.DomainSpec(shape=shape, courant=spec.courant, eps_kind="tensor", eps_box=((0, 0, 0), shape),
                           eps=np.ascontiguousarray(spec.eps[:, lo[2] - bz0:hi[2] - bz0, lo[1] - by0:hi[1] - by0,
                                                            lo[0] - bx0:hi[0] - bx0]), eps_bg=1.0)
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        o = O.OracleSim(win)
        for q in range(6):
            o.field(q)[...] = fields[q][sl]
        o.step(n, record=False)
        inner = (slice(m, m + w),) * 3
        for q in range(6):
            r = rel(got[q][sl][inner], o.field(q)[inner])
            assert r < tol, (c, W.COMP_NAMES[q], r)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_anisotropic_tensor_536_adjoint(dtype, tol):
    """The 536^3 tensor workload with the gradient over its whole interior,
    one step from random forward and cotangent states in the tuned launch
    shape: the dot-product identity <A x, y> = <x, A^T y> over the whole
    grid, and (FP64) the new cotangent fields and the node-tensor gradient
    element by element on three 20^3 windows against the oracle's adjoint
    step on the window with a 5-plane margin (a window's faces perturb one
    plane per step, the tensor's assembly one more)."""
    spec = W.anisotropic_tensor(n_steps=4)
    spec.sources = []
    spec.monitors = []
    spec.grad_box = spec.eps_box
    x = _random_fields(spec.shape, 7005)
    y = _random_fields(spec.shape, 7006)
    sim = _start(spec, x, dtype, kernel="split", tile_rows=8, tile_kz=8, n_ckpt=1, max_steps=1)
    sim.save(0)
    sim.step(1, record=False)
    ax = [sim.field(q) for q in range(6)]
    sim.restore(0)
    sim.adjoint_begin(1)
    for q in range(6):
        sim.set_field(q, y[q], adjoint=True)
    sim.step_adjoint(1)
    aty = [sim.field(q, adjoint=True) for q in range(6)]
    lhs, rhs = _inner(ax, y), _inner(x, aty)
    scale = _norm(ax) * _norm(y)
    print(f"tensor 536^3 {dtype}: dot-product defect {abs(lhs - rhs) / scale:.2e}", flush=True)
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs, scale)
    del ax
    if dtype != "f64":
        sim.close()
        return
    g = sim.grad()
    sim.close()
    del sim
    (bx0, by0, bz0), _ = spec.eps_box
    m, w = 5, 20
    for c in ((40, 45, 50), (268, 261, 270), (494, 500, 497)):
        lo = [c[a] - w // 2 - m for a in range(3)]
        hi = [c[a] + w // 2 + m for a in range(3)]
        shape = tuple(hi[a] - lo[a] for a in range(3))
        win = W.DomainSpec(shape=shape, courant=spec.courant, eps_kind="tensor", eps_box=((0, 0, 0), shape),
                           eps=np.ascontiguousarray(spec.eps[:, lo[2] - bz0:hi[2] - bz0, lo[1] - by0:hi[1] - by0,
                                                            lo[0] - bx0:hi[0] - bx0]), eps_bg=1.0)
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        o = O.OracleSim(win)
        u = np.zeros_like(o.u)
        a = np.zeros_like(o.u)
        for q in range(6):
            u[O.F0 + q] = x[q][sl].reshape(-1)
            a[O.F0 + q] = y[q][sl].reshape(-1)
        gw = np.zeros((6, o.N))
        o.adjoint_step_state(a, u, gw)
        gw = o._tensor_eps_gradient(gw).reshape((6,) + o.shape3)
        inner = (slice(m, m + w),) * 3
        gsl = (slice(lo[2] - bz0 + m, lo[2] - bz0 + m + w), slice(lo[1] - by0 + m, lo[1] - by0 + m + w),
               slice(lo[0] - bx0 + m, lo[0] - bx0 + m + w))
        for q in range(6):
            r = rel(aty[q][sl][inner], a[O.F0 + q].reshape(o.shape3)[inner])
            assert r < 1e-12, (c, "cotangent", W.COMP_NAMES[q], r)
            r = rel(g[(q,) + gsl], gw[q][inner])
            assert r < 1e-12, (c, "gradient entry", q, r)
        print(f"tensor 536^3 window at {c}: cotangents and gradient match the oracle", flush=True)
