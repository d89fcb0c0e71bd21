"""The single-pass family (interior blocks advance E and H in one z-marching
launch, the split kernels take the blocks that meet a slab, a wall or a
dispersive box, state ping-ponged between the working sets) against the
split family: bitwise equal fields, spectra, probe traces and gradients, over
launch shapes, captured chunks, sources and monitors in interior blocks, and
a ragged batch; and against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_30039_amd import adjoint as A
from paper_2609_30039_amd import workloads as W
from paper_2609_30039_amd.sim import Simulation
from tests.gpu_util import gpu_gradient_store_all, rel

pytestmark = pytest.mark.gpu


def _spec(n_steps=80):
    """160 x 80 x 72, 6 absorbing cells on every face, diagonal eps, a Lorentz
    box, an Ex sheet and two Ez point sources, a flux plane, an Hy patch and an
    Ex probe, the sources and monitors on interior blocks of both block
    widths (32 and 64 columns)."""
    nx, ny, nz = 160, 80, 72
    rng = np.random.Generator(np.random.PCG64(61))
    lo, hi = (6, 6, 6), (nx - 6, ny - 6, nz - 6)
    eps = 1.0 + 3.0 * rng.random((3, hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]))
    return W.DomainSpec(
        shape=(nx, ny, nz), courant=W.courant_3d(), pml=(6,) * 6, eps_kind="diag", eps_box=(lo, hi), eps=eps,
        lorentz=[W.LorentzSpec((60, 20, 30), (76, 40, 50), 1.2, 0.35, 0.02)],
        sources=[W.SourceSpec("plane_z", 0, (0, 0, 14), W.gaussian_sine(n_steps, 0.3, 10.0, 30.0)),
                 W.SourceSpec("point", 2, (40, 33, 27), W.gaussian_sine(n_steps, 0.5, 6.0, 20.0)),
                 W.SourceSpec("point", 1, (100, 35, 29), W.gaussian_sine(n_steps, 0.4, 8.0, 25.0))],
        monitors=[W.MonitorSpec("flux_z", pos=(0, 0, 50), rect=(10, 150, 10, 70), omega_dt=W.freq_grid(4, 0.2, 0.5)),
                  W.MonitorSpec("patch_z", comp=4, pos=(0, 0, 33), rect=(20, 140, 15, 55),
                                omega_dt=W.freq_grid(3, 0.2, 0.4)),
                  W.MonitorSpec("probe", comp=0, pos=(100, 41, 40))],
        grad_box=((20, 20, 20), (140, 60, 55)), n_steps=n_steps)


def _run(spec, dtype, **kw):
    g = Simulation(spec, dtype=dtype, **kw)
    g.step(spec.n_steps)
    out = [g.field(q) for q in range(6)] + [g.spectra(m) for m in range(len(spec.monitors))]
    g.close()
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("rows,kz,chunk", [(8, 8, 0), (8, 16, 32), (0, 16, 0), (0, 5, 32), (8, 3, 0)])
def test_onepass_equals_split_bitwise(dtype, rows, kz, chunk):
    spec = _spec()
    ref = _run(spec, dtype, kernel="split", tile_rows=rows, tile_kz=kz)
    got = _run(spec, dtype, kernel="onepass", tile_rows=rows, tile_kz=kz, graph_chunk=chunk)
    for q, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a, b), (q, rel(a, b))


def test_onepass_matches_oracle():
    spec = _spec()
    got = _run(spec, "f64", kernel="onepass", tile_rows=8, tile_kz=8)
    o = O.OracleSim(spec)
    o.step(spec.n_steps)
    for q in range(6):
        assert rel(got[q], o.field(q)) < 1e-11
    for m in range(2):
        assert rel(got[6 + m], o.spectra(m)) < 1e-11


def test_onepass_gradient_equals_split():
    """Forward replays of the reverse sweep in the single-pass family give the
    split family's gradient bit for bit."""
    spec = _spec(40)

    def cot(mi, m, sp):
        return sp if m.kind == "probe" else 2.0 * sp
    _, g1, _ = gpu_gradient_store_all(spec, "f32", cot, kernel="split", tile_rows=8, tile_kz=8)
    _, g2, _ = gpu_gradient_store_all(spec, "f32", cot, kernel="onepass", tile_rows=8, tile_kz=8)
    assert np.array_equal(g1, g2)
    sim = Simulation(spec, dtype="f32", n_ckpt=4, kernel="onepass", tile_rows=8, tile_kz=8, graph_chunk=8)
    g3 = A.gradient(sim, spec.n_steps, 4, lambda s_: {(0, m): cot(m, mm, s_.spectra(m))
                                                      for m, mm in enumerate(spec.monitors)})[0]
    assert rel(g3, g1) < 1e-6


def test_onepass_batch_bitwise():
    specs = W.batch_domains(n_domains=4, sizes=(48, 64, 96), pml=6, n_steps=30, n_f=3, seed=9)
    a = Simulation(specs, dtype="f32", kernel="split", tile_rows=8, tile_kz=8)
    b = Simulation(specs, dtype="f32", kernel="onepass", tile_rows=8, tile_kz=8, graph_chunk=10)
    a.step(30)
    b.step(30)
    for d in range(len(specs)):
        for q in range(6):
            assert np.array_equal(a.field(q, d), b.field(q, d)), (d, q)
        assert rel(a.spectra(0, d), b.spectra(0, d)) == 0.0
