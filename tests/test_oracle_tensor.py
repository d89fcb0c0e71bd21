"""Pins of the oracle's symmetric-tensor media (Section 2.3; Appendix A's
anisotropic-media checks).

The E update of a tensor medium applies the node assembly
(1/8) sum_s R_s^T eps^-1 R_s to the curl, with eps sampled at the grid nodes.
The oracle applies it edge by edge; here it is rebuilt from its definition by
enumerating, at every node, the eight octants (one x, one y and one z edge
meeting at the node) and summing their 3x3 forms, and one step is compared
with that matrix times an independently computed curl, and the discrete
energy with that matrix's inverse in place of eps is conserved.  Then the
properties the paper records: unit spectral radius of the lossless one-step operator for
admitted tensors, growth for a tensor whose eigenvalue lies below one, and,
inside an absorbing face, unit spectral radius when the face normal is a
principal axis with a non-intermediate eigenvalue and growth for the
rejected cases (an intermediate normal eigenvalue, principal axes rotated
against the normal).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_30039_amd import workloads as W

COMP = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def _rot(rng):
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return q


def _pack(m):
    return np.array([m[a, b] for (a, b) in COMP])


def random_tensors(rng, box_shape, lo=1.0, hi=4.0):
    """[6][bz][by][bx] rotated symmetric tensors with eigenvalues in [lo, hi]."""
    bx, by, bz = box_shape
    out = np.zeros((6, bz, by, bx))
    for k in range(bz):
        for j in range(by):
            for i in range(bx):
                R = _rot(rng)
                out[:, k, j, i] = _pack(R @ np.diag(lo + (hi - lo) * rng.random(3)) @ R.T)
    return out


def uniform_tensor(shape, m):
    nx, ny, nz = shape
    return np.broadcast_to(_pack(m)[:, None, None, None], (6, nz, ny, nx)).copy()


def _one_step_matrix(sim):
    dof = sim.dof_mask().reshape(-1)
    idx = np.nonzero(dof)[0]
    M = np.zeros((len(idx), len(idx)))
    for col, q in enumerate(idx):
        u = np.zeros(sim.u.size)
        u[q] = 1.0
        u = u.reshape(sim.u.shape)
        sim.step_state(u, 0, sources=False)
        M[:, col] = u.reshape(-1)[idx]
    return M


def _radius(spec):
    return np.abs(np.linalg.eigvals(_one_step_matrix(O.OracleSim(spec)))).max()


def _assembly_by_octants(spec):
    """The assembled operator [3N][3N] (rows and columns: edge component c,
    then [nz][ny][nx]) from its definition: at each node v = (i, j, k),
    0 <= v_a <= n_a, and each octant s, R_s picks the x, y and z edges that
    meet at v on the octant's side (an edge that leaves v or one that arrives
    at it); an edge outside the grid or tangential to a wall is absent
    (zero).  eps^-1 at v from the node arrays, the background past them."""
    nx, ny, nz = spec.shape
    n = (nx, ny, nz)
    N = nx * ny * nz
    en = spec.eps_nodes()

    def einv(v):
        if any(v[a] >= n[a] for a in range(3)):
            return np.eye(3) / spec.eps_bg
        m = np.zeros((3, 3))
        for q, (a, b) in enumerate(COMP):
            m[a, b] = m[b, a] = en[q, v[2], v[1], v[0]]
        return np.linalg.inv(m)

    def edge(b, start):
        if any(start[a] < 0 or start[a] >= n[a] for a in range(3)):
            return None
        if start[(b + 1) % 3] == 0 or start[(b + 2) % 3] == 0:    # tangential to a PEC wall
            return None
        return b * N + (start[2] * ny + start[1]) * nx + start[0]

    M = np.zeros((3 * N, 3 * N))
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                v = (i, j, k)
                A = einv(v)
                for s in range(8):
                    rows = []
                    for b in range(3):
                        st = list(v)
                        st[b] -= (s >> b) & 1          # 1: the edge arriving at v along b
                        rows.append(edge(b, st))
                    for a in range(3):
                        for b in range(3):
                            if rows[a] is not None and rows[b] is not None:
                                M[rows[a], rows[b]] += A[a, b] / 8.0
    return M


def _curl_minus(H):
    """Backward-difference curl of H [3][nz][ny][nx] at the E edges, H zero
    before the first node."""
    def dm(f, axis):   # axis in array order: 0 z, 1 y, 2 x
        g = np.zeros_like(f)
        sl = [slice(None)] * 3
        sl[axis] = slice(1, None)
        lo = [slice(None)] * 3
        lo[axis] = slice(None, -1)
        g[tuple(sl)] = f[tuple(sl)] - f[tuple(lo)]
        g[tuple([slice(0, 1) if a == axis else slice(None) for a in range(3)])] = \
            f[tuple([slice(0, 1) if a == axis else slice(None) for a in range(3)])]
        return g
    hx, hy, hz = H
    return np.stack([dm(hz, 1) - dm(hy, 0), dm(hx, 0) - dm(hz, 2), dm(hy, 2) - dm(hx, 1)])


def test_tensor_step_is_the_octant_assembly():
    """One step from E = 0 and a random H: E^1 = S M C^-(H) on the unmasked
    edges, with M built octant by octant; a random rotated tensor on a box
    that leaves background nodes on every side (eps_bg = 1.5)."""
    rng = np.random.Generator(np.random.PCG64(21))
    shape = (5, 4, 6)
    nx, ny, nz = shape
    box = ((1, 0, 2), (4, 3, 5))
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(), eps_kind="tensor", eps_box=box,
                        eps=random_tensors(rng, (3, 3, 3)), eps_bg=1.5)
    sim = O.OracleSim(spec)
    H = rng.standard_normal((3, nz, ny, nx))
    for c in range(3):
        sim.u[O.F0 + 3 + c] = H[c].reshape(-1)
    sim.step(1, record=False)
    M = _assembly_by_octants(spec)
    dof = sim.dof_mask()[:3].reshape(-1)
    c = _curl_minus(H).reshape(-1) * dof
    want = spec.courant * (M @ c) * dof
    got = np.concatenate([sim.field(q).reshape(-1) for q in range(3)])
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # the assembly is symmetric and, with every eigenvalue >= 1, below the identity
    Md = M[np.ix_(dof, dof)]
    assert np.array_equal(Md, Md.T) or np.max(np.abs(Md - Md.T)) < 1e-15
    w = np.linalg.eigvalsh(0.5 * (Md + Md.T))
    assert w.min() > 0.0 and w.max() <= 1.0 + 1e-12


def test_isotropic_tensor_is_the_scalar_medium():
    """eps = e I at every node (background e too) is the scalar medium e."""
    rng = np.random.Generator(np.random.PCG64(22))
    shape = (6, 5, 7)
    nx, ny, nz = shape
    e = 2.25
    t = W.DomainSpec(shape=shape, courant=W.courant_3d(), eps_kind="tensor", eps_box=((0, 0, 0), shape),
                     eps=uniform_tensor(shape, e * np.eye(3)), eps_bg=e)
    s = W.DomainSpec(shape=shape, courant=W.courant_3d(), eps_kind="iso", eps_box=((0, 0, 0), shape),
                     eps=np.full((1, nz, ny, nx), e), eps_bg=e)
    a, b = O.OracleSim(t), O.OracleSim(s)
    u0 = rng.standard_normal(a.u.shape) * a.dof_mask()
    u0[O.PSIE0:] = 0.0
    a.u[:] = u0
    b.u[:] = u0
    a.step(40, record=False)
    b.step(40, record=False)
    assert np.max(np.abs(a.u - b.u)) <= 1e-12 * np.max(np.abs(b.u))


def test_spectral_radius_admitted_rotated_tensors():
    """Lossless PEC box, random rotated tensors with eigenvalues in [1, 4] at
    every node: every eigenvalue of the one-step operator is on the unit
    circle (Appendix A records one to nine decimals)."""
    rng = np.random.Generator(np.random.PCG64(11))
    shape = (4, 5, 4)
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(0.99), eps_kind="tensor",
                        eps_box=((0, 0, 0), shape), eps=random_tensors(rng, shape))
    lam = np.abs(np.linalg.eigvals(_one_step_matrix(O.OracleSim(spec))))
    assert np.max(np.abs(lam - 1.0)) < 1e-12


def test_spectral_radius_tensor_below_one():
    """An eigenvalue below one breaks the vacuum step bound: 0.9 I grows as
    the scalar 0.9 medium does."""
    shape = (7, 6, 8)
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(0.99), eps_kind="tensor",
                        eps_box=((0, 0, 0), shape), eps=uniform_tensor(shape, 0.9 * np.eye(3)), eps_bg=0.9)
    assert _radius(spec) > 1.3


def _rz(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rx(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


FACE_SHAPE = (6, 6, 14)
FACE_PML = (0, 0, 0, 0, 4, 4)
ADMITTED = {
    "isotropic": 2.0 * np.eye(3),
    "normal eigenvalue largest, xy rotated": _rz(0.6) @ np.diag([1.5, 4.0, 6.0]) @ _rz(0.6).T,
    "normal eigenvalue smallest, xy rotated": _rz(0.6) @ np.diag([1.5, 4.0, 1.0]) @ _rz(0.6).T,
}
REJECTED = {
    "normal eigenvalue intermediate": (np.diag([1.0, 4.0, 2.0]), FACE_SHAPE, 1e-3),
    "normal eigenvalue intermediate, contrast 16": (np.diag([1.0, 16.0, 4.0]), FACE_SHAPE, 5e-3),
    "principal axes rotated 45 degrees about x": (_rx(math.pi / 4) @ np.diag([1.0, 16.0, 1.0]) @ _rx(math.pi / 4).T,
                                                  (5, 6, 12), 1e-4),
}


def _face_spec(m, shape):
    return W.DomainSpec(shape=shape, courant=W.courant_3d(0.99), pml=FACE_PML, eps_kind="tensor",
                        eps_box=((0, 0, 0), shape), eps=uniform_tensor(shape, m))


@pytest.mark.parametrize("name", sorted(ADMITTED))
def test_absorbing_face_admitted_tensor(name):
    """A tensor filling both z faces whose normal (z) is a principal axis with
    the largest or smallest eigenvalue: the one-step operator of the absorbing
    box has spectral radius 1 (its static modes) to round-off."""
    assert _radius(_face_spec(ADMITTED[name], FACE_SHAPE)) <= 1.0 + 1e-12


@pytest.mark.parametrize("name", sorted(REJECTED))
def test_absorbing_face_rejected_tensor_grows(name):
    """The cases the admission rule refuses: inside the z faces the stretched
    formulation grows (Appendix A records radii 1.0049 to 1.0089 on its Bloch
    grids; these PEC-walled grids give 1.0003 to 1.011)."""
    m, shape, bar = REJECTED[name]
    assert _radius(_face_spec(m, shape)) > 1.0 + bar


def test_discrete_energy_invariant_rotated_tensor():
    """Lossless PEC box with random rotated tensors: the quadratic form
    <E, M^-1 E> + <H^{n-1/2}, H^{n+1/2}>, with M the octant assembly on the
    unmasked edges, is conserved to round-off over 300 steps (the Yee energy
    with eps replaced by the assembled operator)."""
    rng = np.random.Generator(np.random.PCG64(23))
    shape = (5, 4, 6)
    nx, ny, nz = shape
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(0.99), eps_kind="tensor", eps_box=((0, 0, 0), shape),
                        eps=random_tensors(rng, shape), eps_bg=1.3)
    sim = O.OracleSim(spec)
    dof = sim.dof_mask()
    sim.u[:] = rng.standard_normal(sim.u.shape) * dof
    sim.u[O.PSIE0:] = 0.0
    M = _assembly_by_octants(spec)
    edof = dof[:3].reshape(-1)
    Minv = np.linalg.inv(M[np.ix_(edof, edof)])

    def energy(h_prev):
        e = np.concatenate([sim.field(c).reshape(-1) for c in range(3)])[edof]
        hh = sum(np.sum(h_prev[c] * sim.field(3 + c)) for c in range(3))
        return e @ Minv @ e + hh

    hist = []
    for n in range(300):
        h_prev = [sim.field(3 + c).copy() for c in range(3)]
        sim.step(1, record=False)
        hist.append(energy(h_prev))
    hist = np.asarray(hist)
    assert np.max(np.abs(hist - hist[0])) / abs(hist[0]) < 1e-11
