"""The reversible mode (Section 3.2, absorbing-face variant) on the GPU.

The forward fields of the lossless box between the absorbing slabs are rebuilt
by stepping Eq. 1 backward, with the interface fields recorded during the
forward sweep, so the reverse sweep reads no checkpoint.  The result must be
the discrete adjoint's gradient: the oracle's (bisection replay) up to the
round-off of the backward steps.  Also: the backward steps undo the forward
ones, several objectives from one forward run (the retained backward pass),
and the admissibility rule.
"""
import numpy as np
import pytest

from paper_2609_30039_amd import adjoint as A
from paper_2609_30039_amd import binding as B
from paper_2609_30039_amd import workloads as W
from paper_2609_30039_amd.sim import Simulation
from tests.gpu_util import gpu_gradient_store_all, oracle_gradient, rel

pytestmark = pytest.mark.gpu


def _spec(n_steps=90):
    spec, _ = W.design_patch(pml=6, design=12, patch=10, n_steps=n_steps, n_f=3, shape=(40, 34, 38))
    return spec


def _cot(mi, m, sp):
    return 2.0 * sp


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_reversible_gradient_matches_oracle(dtype, tol):
    """|DFT Ez|^2 patch objective, 6-cell CPML on every face, a random design
    box: dJ/deps from the reversible sweep against the oracle adjoint."""
    spec = _spec()
    N = spec.n_steps
    sim = Simulation(spec, dtype=dtype, reversible=True, max_steps=N)
    g = A.reversible_gradient(sim, N, lambda s: {(0, 0): 2.0 * s.spectra(0)})[0]
    _, g_orc = oracle_gradient(spec, _cot)
    (i0, j0, k0), (i1, j1, k1) = spec.grad_box
    r = rel(g[0], g_orc.sum(axis=0)[k0:k1, j0:j1, i0:i1])
    print(f"reversible {dtype}: gradient rel L2 vs oracle {r:.3e}", flush=True)
    assert r < tol, r


def test_reversible_equals_checkpointed_f64():
    """The same gradient as the adjoint over stored forward states, FP64, to
    the round-off of 90 backward steps."""
    spec = _spec()
    N = spec.n_steps
    sim = Simulation(spec, dtype="f64", reversible=True, max_steps=N)
    g = A.reversible_gradient(sim, N, lambda s: {(0, 0): 2.0 * s.spectra(0)})[0]
    _, g_ref, _ = gpu_gradient_store_all(spec, "f64", _cot)
    assert rel(g, g_ref) < 1e-11


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-4)])
def test_backward_steps_undo_forward_steps(dtype, tol):
    """From a seeded random state, 60 forward steps then 60 backward steps
    give back the starting fields inside the lossless box (outside it the
    state is left undefined), with sources on."""
    spec = _spec(60)
    nx, ny, nz = spec.shape
    rng = np.random.default_rng(5)
    k, j, i = np.ogrid[:nz, :ny, :nx]
    idx = (i, j, k)
    f0 = []
    for q in range(6):
        f = rng.standard_normal((nz, ny, nx))
        if q < 3:
            f[np.broadcast_to((idx[(q + 1) % 3] == 0) | (idx[(q + 2) % 3] == 0), f.shape)] = 0.0
        f0.append(f)
    sim = Simulation(spec, dtype=dtype, reversible=True, max_steps=60)
    for q in range(6):
        sim.set_field(q, f0[q])
    sim.step(60, record=False)
    moved = max(rel(sim.field(q), f0[q]) for q in range(6))
    sim.step_reverse(60)
    assert sim.steps[0] == 0
    L = 6
    box = (slice(L, nz - L), slice(L, ny - L), slice(L, nx - L))
    errs = [rel(sim.field(q)[box], f0[q][box]) for q in range(6)]
    print(f"{dtype}: fields moved by {moved:.2f} over 60 steps; after reversal {max(errs):.3e}", flush=True)
    assert moved > 0.5
    assert max(errs) < tol, errs


def test_retained_backward_pass_serves_two_objectives():
    """One forward run, two objectives (|Ez|^2 on the patch and the real part
    of the summed spectrum): each gradient equals its own forward+reverse run
    bitwise."""
    spec = _spec()
    N = spec.n_steps
    objectives = [lambda s: {(0, 0): 2.0 * s.spectra(0)},
                  lambda s: {(0, 0): np.ones_like(s.spectra(0))}]
    sim = Simulation(spec, dtype="f64", reversible=True, max_steps=N, n_ckpt=1)
    both = A.retained_gradients(sim, N, objectives)
    for k, fn in enumerate(objectives):
        solo = Simulation(spec, dtype="f64", reversible=True, max_steps=N)
        g = A.reversible_gradient(solo, N, fn)[0]
        assert np.array_equal(both[k][0], g), k
    assert rel(both[0][0], both[1][0]) > 0.1


def test_reverse_needs_reversible_mode_and_a_record():
    spec = _spec(20)
    sim = Simulation(spec, dtype="f32", max_steps=20)
    sim.step(5)
    with pytest.raises(B.FdtdError) as e:
        sim.step_reverse(1)
    assert e.value.code == B.FDTD_E_STATE
    sim = Simulation(spec, dtype="f32", reversible=True, max_steps=20)
    sim.step(5)
    sim.set_field(0, np.zeros(spec.shape[::-1], dtype=np.float32))   # another trajectory from here
    with pytest.raises(B.FdtdError) as e:
        sim.step_reverse(1)
    assert e.value.code == B.FDTD_E_STATE
