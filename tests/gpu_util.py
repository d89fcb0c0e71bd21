"""Helpers shared by the GPU tests: oracle runs and HIP runs of the same spec."""
import numpy as np

from oracle import oracle as O
from paper_2609_30039_amd.sim import Simulation


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def oracle_forward(spec, n=None):
    sim = O.OracleSim(spec)
    sim.step(spec.n_steps if n is None else n)
    return sim


def gpu_forward(spec, dtype="f64", n=None, **kw):
    sim = Simulation(spec, dtype=dtype, **kw)
    sim.step(spec.n_steps if n is None else n)
    return sim


def patch_objective(sp):
    """J = sum |X|^2 over a patch spectrum, and its cotangent dJ/dRe + i dJ/dIm."""
    return float(np.sum(np.abs(sp) ** 2)), 2.0 * sp


def flux_objective(sp):
    """J = sum_f Re sum (Ex Hy* - Ey Hx*) and its cotangents."""
    J = float(np.sum(np.real(sp[:, 0] * np.conj(sp[:, 3]) - sp[:, 1] * np.conj(sp[:, 2]))))
    g = np.zeros_like(sp)
    g[:, 0] = sp[:, 3]
    g[:, 3] = sp[:, 0]
    g[:, 1] = -sp[:, 2]
    g[:, 2] = -sp[:, 1]
    return J, g


def gpu_gradient_store_all(spec, dtype, cot_fn, n=None, **kw):
    """Adjoint on the HIP path with every forward state kept in a slot (kw:
    launch options such as the kernel family)."""
    N = spec.n_steps if n is None else n
    sim = Simulation(spec, dtype=dtype, n_ckpt=N + 1, max_steps=N, **kw)
    sim.save(0)
    for t in range(N):
        sim.step(1)
        sim.save(t + 1)
    cots = {}
    for mi, m in enumerate(spec.monitors):
        sp = sim.spectra(mi)
        cots[mi] = cot_fn(mi, m, sp)
        sim.set_cotangent(mi, cots[mi])
    sim.adjoint_begin(N)
    for m_ in range(N, 0, -1):
        sim.restore(m_ - 1)
        sim.step_adjoint(1)
    return sim, sim.grad(), cots


def oracle_gradient(spec, cot_fn, n=None):
    """Oracle adjoint with cotangents from the oracle's own spectra."""
    N = spec.n_steps if n is None else n
    sim = O.OracleSim(spec)
    sim.step(N)
    cots = {}
    for mi, m in enumerate(spec.monitors):
        sp = sim.probe(mi) if m.kind == "probe" else sim.spectra(mi)
        cots[mi] = cot_fn(mi, m, sp)
    g = sim.gradient(cots, N)
    return sim, g
