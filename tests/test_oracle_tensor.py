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

On Bloch grids (x and y periodic with real factors): the octant assembly
across the seams, unit radii for admitted tensors, growth for the rejected
ones in absorbing z faces, the energy invariant, the adjoint's dot product
and central differences at seam nodes.

The adjoint (Section 3.1 with the tensor of Section 2.3): the dot-product
identity of the step map with admitted tensors in absorbing faces; the
one-step eps^-1 gradient against the derivative of the octant-built
assembly; dJ/deps of the stored entries against fourth-order central
differences of whole solves and a Taylor remainder falling as h^2; and an
isotropic tensor's gradient against the scalar medium's.
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


# ------------------------------------------------------------ the adjoint
def _tensor_adjoint_case(seed):
    """Absorbing faces on every side holding admitted tensors (z faces: the
    normal a principal axis with the largest eigenvalue; x and y faces: the
    isotropic background), random rotated tensors inside, PEC walls."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (10, 9, 12)
    nx, ny, nz = shape
    pml = (2, 2, 2, 3, 3, 2)
    box = ((2, 2, 0), (8, 6, 12))           # inside the x and y faces, through both z faces
    bx, by, bz = 6, 4, 12
    eps = random_tensors(rng, (bx, by, bz), 1.0, 3.0)
    face = _pack(_rz(0.4) @ np.diag([1.5, 2.5, 4.0]) @ _rz(0.4).T)
    eps[:, :3] = face[:, None, None, None]
    eps[:, -2:] = face[:, None, None, None]
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(), pml=pml, eps_kind="tensor", eps_box=box, eps=eps,
                        eps_bg=1.2)
    sim = O.OracleSim(spec)
    dof = sim.dof_mask()
    x = rng.standard_normal(sim.u.shape) * dof
    y = rng.standard_normal(sim.u.shape) * dof
    return sim, x, y


@pytest.mark.parametrize("nsteps", [1, 40])
def test_tensor_adjoint_dot_product(nsteps):
    """<A x, y> = <x, A^T y> for the source-free step map of a tensor medium
    with absorbing faces, to round-off: the transposed assembly, the curl
    and absorber transposes around it (Section 3.1)."""
    sim, x, y = _tensor_adjoint_case(31)
    ax = x.copy()
    for t in range(nsteps):
        sim.step_state(ax, t, sources=False)
    aty = y.copy()
    for t in range(nsteps):
        sim.adjoint_step_state(aty, x, None)
    dof = sim.dof_mask()
    lhs = np.sum(ax * y * dof)
    rhs = np.sum(x * aty * dof)
    scale = np.linalg.norm(ax * dof) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    assert np.all(aty[~dof] == 0.0)


def test_tensor_gradient_one_step_is_the_octant_outer_product():
    """One step from a random state: the eps^-1 gradient the adjoint step
    accumulates equals, at every node, 1/8 sum over its octants of the
    outer product of S Ebar and the curl on the octant's edges, built here
    from the assembled matrix's definition: d<Ebar, S M c>/dA_v with M
    differentiated through the octant enumeration (finite differences of
    the exactly linear map M(A) are exact up to rounding)."""
    rng = np.random.Generator(np.random.PCG64(33))
    shape = (5, 4, 6)
    nx, ny, nz = shape
    box = ((0, 0, 0), shape)
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(), eps_kind="tensor", eps_box=box,
                        eps=random_tensors(rng, shape), eps_bg=1.4)
    sim = O.OracleSim(spec)
    dof = sim.dof_mask()
    u = np.zeros_like(sim.u)
    u[O.F0 + 3:O.F0 + 6] = rng.standard_normal((3, sim.N))
    a = rng.standard_normal(sim.u.shape) * dof
    a[O.F0 + 3:] = 0.0                        # E cotangents only: the H transpose adds nothing
    ebar = np.concatenate([a[O.F0 + c] for c in range(3)])
    g = np.zeros((6, sim.N))
    sim.adjoint_step_state(a.copy(), u, g)
    H = np.stack([u[O.F0 + 3 + c].reshape(sim.shape3) for c in range(3)])
    edof = dof[:3].reshape(-1)
    curl = _curl_minus(H).reshape(-1) * edof
    base = spec.eps_nodes()
    S = spec.courant
    for (i, j, k) in [(0, 0, 0), (2, 1, 3), (4, 3, 5), (3, 0, 2)]:
        p = (k * ny + j) * nx + i
        for q, (ca, cb) in enumerate(COMP):
            # J(A) = <Ebar, S M(A) c> is linear in A_v: its derivative along the
            # stored entry q (both matrix entries for q >= 3) is a difference
            def J(delta):
                inv = sim.einvT.copy()
                inv[q].reshape(-1)[p] += delta
                s2 = W.DomainSpec(**{**spec.__dict__})
                M = _assembly_from_inverse(s2, inv)
                return ebar @ (S * (M @ curl) * edof)
            want = (J(0.5) - J(-0.5)) / 1.0
            assert abs(g[q, p] - want) <= 1e-12 * (1.0 + abs(want)), (i, j, k, q, g[q, p], want)


def _assembly_from_inverse(spec, inv):
    """The octant assembly with eps^-1 at the in-grid nodes taken from inv
    [6][N] (the background past the arrays)."""
    nx, ny, nz = spec.shape
    n = (nx, ny, nz)
    N = nx * ny * nz
    inv = inv.reshape(6, N)

    def einv(v):
        if any(v[a] >= n[a] for a in range(3)):
            return np.eye(3) / spec.eps_bg
        p = (v[2] * ny + v[1]) * nx + v[0]
        m = np.zeros((3, 3))
        for q, (a, b) in enumerate(COMP):
            m[a, b] = m[b, a] = inv[q, p]
        return m

    def edge(b, start):
        if any(start[a] < 0 or start[a] >= n[a] for a in range(3)):
            return None
        if start[(b + 1) % 3] == 0 or start[(b + 2) % 3] == 0:
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
                        st[b] -= (s >> b) & 1
                        rows.append(edge(b, st))
                    for a in range(3):
                        for b in range(3):
                            if rows[a] is not None and rows[b] is not None:
                                M[rows[a], rows[b]] += A[a, b] / 8.0
    return M


def _tensor_fd_problem():
    """A tensor design box in a domain with absorbing faces, a sheet and a
    point source, a patch spectrum, a flux plane and a probe."""
    rng = np.random.Generator(np.random.PCG64(41))
    pml = 4
    shape = (10 + 2 * pml, 9 + 2 * pml, 12 + 2 * pml)
    nx, ny, nz = shape
    lo, hi = (pml + 1, pml + 1, pml + 3), (nx - pml - 1, ny - pml - 1, nz - pml - 3)
    bx = [hi[a] - lo[a] for a in range(3)]
    nsteps = 50
    spec = W.DomainSpec(
        shape=shape, courant=W.courant_3d(), pml=(pml,) * 6, eps_kind="tensor", eps_box=(lo, hi),
        eps=random_tensors(rng, tuple(bx), 1.0, 3.0), eps_bg=1.0,
        sources=[W.SourceSpec("plane_z", 0, (0, 0, pml + 1), W.gaussian_sine(nsteps, 0.6, 6.0, 18.0)),
                 W.SourceSpec("point", 1, (nx // 2, ny // 2, pml + 2), W.gaussian_sine(nsteps, 0.5, 5.0, 15.0))],
        monitors=[W.MonitorSpec("patch_z", comp=1, pos=(0, 0, nz - pml - 2), rect=(5, 13, 5, 12),
                                omega_dt=np.array([0.4, 0.55, 0.7])),
                  W.MonitorSpec("flux_z", pos=(0, 0, nz - pml - 3), rect=(0, nx, 0, ny),
                                omega_dt=np.array([0.5, 0.6])),
                  W.MonitorSpec("probe", comp=0, pos=(nx // 2, ny // 2 + 1, nz - pml - 4))],
        n_steps=nsteps)
    return spec


def _objective(sim):
    """J = sum |E_y patch|^2 + sum_f flux_f + sum probe^2 and its monitor cotangents."""
    sp0, sp1, pr = sim.spectra(0), sim.spectra(1), sim.probe(2)
    J = np.sum(np.abs(sp0) ** 2) + np.sum(O.OracleSim.flux_from_spectra(sp1)) + np.sum(pr ** 2)
    g1 = np.zeros_like(sp1)
    g1[:, 0], g1[:, 3], g1[:, 1], g1[:, 2] = sp1[:, 3], sp1[:, 0], -sp1[:, 2], -sp1[:, 1]
    return J, {0: 2.0 * sp0, 1: g1, 2: 2.0 * pr}


def _run_J(spec):
    sim = O.OracleSim(spec)
    sim.step(spec.n_steps)
    return _objective(sim)[0]


def test_tensor_gradient_central_differences():
    """dJ/deps for the stored tensor entries (an off-diagonal entry moves both
    matrix entries) from the transposed sweep equals fourth-order central
    differences of the full solve, for every entry at three nodes."""
    spec = _tensor_fd_problem()
    sim = O.OracleSim(spec)
    sim.step(spec.n_steps)
    J, cot = _objective(sim)
    g = sim.gradient(cot, spec.n_steps)
    assert g.shape == (6,) + sim.shape3
    (i0, j0, k0), _ = spec.eps_box
    for (li, lj, lk) in [(1, 2, 1), (4, 5, 3), (7, 3, 5)]:
        i, j, k = i0 + li, j0 + lj, k0 + lk
        for q in range(6):
            h = 2e-3
            vals = {}
            for m in (-2, -1, 1, 2):
                e = spec.eps.copy()
                e[q, lk, lj, li] += m * h
                vals[m] = _run_J(W.DomainSpec(**{**spec.__dict__, "eps": e}))
            fd = (8.0 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12.0 * h)
            ad = g[q, k, j, i]
            assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(J), (i, j, k, q, ad, fd)


def test_tensor_gradient_taylor_remainder():
    """Along a random symmetric direction over the whole box the remainder
    J(eps + h d) - J(eps) - h <g, d> falls as h^2."""
    spec = _tensor_fd_problem()
    sim = O.OracleSim(spec)
    sim.step(spec.n_steps)
    J0, cot = _objective(sim)
    g = sim.gradient(cot, spec.n_steps)
    (i0, j0, k0), (i1, j1, k1) = spec.eps_box
    gb = g[:, k0:k1, j0:j1, i0:i1]
    rng = np.random.Generator(np.random.PCG64(12))
    d = rng.standard_normal(spec.eps.shape)
    rem = []
    for h in (1e-2, 5e-3, 2.5e-3):
        s2 = W.DomainSpec(**{**spec.__dict__, "eps": spec.eps + h * d})
        rem.append(abs(_run_J(s2) - J0 - h * np.sum(gb * d)))
    rem = np.asarray(rem)
    r = rem[:-1] / rem[1:]
    assert np.all(r > 3.5) and np.all(r < 4.5), (rem, r)


def test_isotropic_tensor_gradient_is_the_scalar_gradient():
    """eps = e I over the whole grid with background e: the derivative of J
    along a uniform change of e is the same whether e is the scalar medium's
    (the sum of its edge gradient) or every node tensor's (the sum of the
    diagonal node gradients, the high-wall background nodes moved too: their
    share is the derivative with the background fixed subtracted, by central
    differences of the background alone)."""
    rng = np.random.Generator(np.random.PCG64(24))
    shape = (7, 6, 8)
    nx, ny, nz = shape
    e = 2.0
    nsteps = 30
    common = dict(shape=shape, courant=W.courant_3d(), pml=(2,) * 6, eps_box=((0, 0, 0), shape), eps_bg=e,
                  sources=[W.SourceSpec("point", 2, (3, 3, 3), W.gaussian_sine(nsteps, 0.6, 5.0, 12.0))],
                  monitors=[W.MonitorSpec("probe", comp=1, pos=(4, 2, 5))], n_steps=nsteps)
    t = W.DomainSpec(eps_kind="tensor", eps=uniform_tensor(shape, e * np.eye(3)), **common)
    s = W.DomainSpec(eps_kind="iso", eps=np.full((1, nz, ny, nx), e), **common)
    out = []
    for spec in (t, s):
        sim = O.OracleSim(spec)
        sim.step(nsteps)
        pr = sim.probe(0)
        g = sim.gradient({0: 2.0 * pr}, nsteps)
        out.append((np.sum(pr ** 2), g))
    (Jt, gt), (Js, gs) = out
    assert abs(Jt - Js) <= 1e-12 * abs(Js)
    d_scalar = gs.sum()
    h = 1e-4
    jb = [_run_probe_J(W.DomainSpec(**{**t.__dict__, "eps_bg": e + m * h})) for m in (-1, 1)]
    d_bg = (jb[1] - jb[0]) / (2 * h)
    d_tensor = gt[:3].sum() + d_bg
    assert abs(d_tensor - d_scalar) <= 1e-7 * abs(d_scalar), (d_tensor, d_scalar, d_bg)


def _run_probe_J(spec):
    sim = O.OracleSim(spec)
    sim.step(spec.n_steps)
    return np.sum(sim.probe(0) ** 2)


# ------------------------------------------------------------ Bloch-periodic tensor media
def _assembly_by_octants_bloch(spec):
    """The assembled operator of a domain periodic in x and/or y: the node
    set is 0..n-1 along a periodic axis (node n is node 0), the edges seen
    from a node across the seam are the edges at the other end times the
    Bloch factor, and both factors enter the node's 3x3 form."""
    nx, ny, nz = spec.shape
    n = (nx, ny, nz)
    N = nx * ny * nz
    per = tuple(int(p) for p in spec.periodic)
    sign = tuple(float(s) for s in spec.bloch_sign)
    en = spec.eps_nodes()

    def einv(v):
        w = list(v)
        for a in range(3):
            if w[a] >= n[a]:
                if not per[a]:
                    return np.eye(3) / spec.eps_bg
                w[a] -= n[a]
        m = np.zeros((3, 3))
        for q, (a, b) in enumerate(COMP):
            m[a, b] = m[b, a] = en[q, w[2], w[1], w[0]]
        return np.linalg.inv(m)

    def edge(b, start):
        w = list(start)
        f = 1.0
        for a in range(3):
            if 0 <= w[a] < n[a]:
                continue
            if not per[a]:
                return None, 0.0
            w[a] += n[a] if w[a] < 0 else -n[a]
            f *= sign[a]
        masked = any(w[(b + t) % 3] == 0 and not per[(b + t) % 3] for t in (1, 2))
        if masked:
            return None, 0.0
        return b * N + (w[2] * ny + w[1]) * nx + w[0], f

    M = np.zeros((3 * N, 3 * N))
    ranges = [range(n[a]) if per[a] else range(n[a] + 1) for a in range(3)]
    for k in ranges[2]:
        for j in ranges[1]:
            for i in ranges[0]:
                v = (i, j, k)
                A = einv(v)
                for s in range(8):
                    rows = []
                    for b in range(3):
                        st = list(v)
                        st[b] -= (s >> b) & 1
                        rows.append(edge(b, st))
                    for a in range(3):
                        for b in range(3):
                            (ra, fa), (rb, fb) = rows[a], rows[b]
                            if ra is not None and rb is not None:
                                M[ra, rb] += A[a, b] * fa * fb / 8.0
    return M


@pytest.mark.parametrize("signs", [(1, 1), (-1, 1), (-1, -1)])
def test_tensor_step_is_the_octant_assembly_bloch(signs):
    """One step from E = 0 and a random H on a cell periodic in x and y: the
    tensor update equals S M C^-(H) with M built octant by octant across the
    seams (the curl's own seam taken from the oracle's scalar step, which the
    scalar pins fix); M is symmetric with eigenvalues in (0, 1]."""
    rng = np.random.Generator(np.random.PCG64(25))
    shape = (5, 4, 6)
    nx, ny, nz = shape
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(), eps_kind="tensor", eps_box=((0, 0, 0), shape),
                        eps=random_tensors(rng, shape), eps_bg=1.0, periodic=(1, 1, 0),
                        bloch_sign=(signs[0], signs[1], 1))
    sim = O.OracleSim(spec)
    H = rng.standard_normal((3, nz, ny, nx))
    for c in range(3):
        sim.u[O.F0 + 3 + c] = H[c].reshape(-1)
    sim.step(1, record=False)
    # the curl by the scalar oracle: eps = 1 everywhere, one step from the same H
    iso = W.DomainSpec(shape=shape, courant=W.courant_3d(), eps_kind="iso", eps_box=((0, 0, 0), shape),
                       eps=np.ones((1, nz, ny, nx)), periodic=(1, 1, 0), bloch_sign=(signs[0], signs[1], 1))
    si = O.OracleSim(iso)
    for c in range(3):
        si.u[O.F0 + 3 + c] = H[c].reshape(-1)
    si.step(1, record=False)
    curl = np.concatenate([si.field(c).reshape(-1) for c in range(3)]) / spec.courant
    M = _assembly_by_octants_bloch(spec)
    dof = sim.dof_mask()[:3].reshape(-1)
    want = spec.courant * (M @ (curl * dof)) * dof
    got = np.concatenate([sim.field(q).reshape(-1) for q in range(3)])
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    Md = M[np.ix_(dof, dof)]
    assert np.max(np.abs(Md - Md.T)) < 1e-15
    w = np.linalg.eigvalsh(0.5 * (Md + Md.T))
    assert w.min() > 0.0 and w.max() <= 1.0 + 1e-12


@pytest.mark.parametrize("signs", [(1, 1), (-1, 1), (-1, -1)])
def test_spectral_radius_admitted_tensors_bloch_grid(signs):
    """On small Bloch grids (x and y periodic, z walled) with random rotated
    tensors at every node, every eigenvalue of the one-step operator lies on
    the unit circle (Appendix A: one to nine decimals)."""
    rng = np.random.Generator(np.random.PCG64(13))
    shape = (4, 4, 5)
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(0.99), eps_kind="tensor", eps_box=((0, 0, 0), shape),
                        eps=random_tensors(rng, shape), periodic=(1, 1, 0), bloch_sign=(signs[0], signs[1], 1))
    lam = np.abs(np.linalg.eigvals(_one_step_matrix(O.OracleSim(spec))))
    assert np.max(np.abs(lam - 1.0)) < 1e-12


def _face_spec_bloch(m, shape):
    return W.DomainSpec(shape=shape, courant=W.courant_3d(0.99), pml=FACE_PML, eps_kind="tensor",
                        eps_box=((0, 0, 0), shape), eps=uniform_tensor(shape, m), periodic=(1, 1, 0))


@pytest.mark.parametrize("name", sorted(ADMITTED))
def test_absorbing_face_admitted_tensor_bloch(name):
    """A Bloch grid (x, y periodic) with absorbing z faces filled by an
    admitted tensor: spectral radius 1 to round-off."""
    assert _radius(_face_spec_bloch(ADMITTED[name], FACE_SHAPE)) <= 1.0 + 1e-12


@pytest.mark.parametrize("name", sorted(REJECTED))
def test_absorbing_face_rejected_tensor_grows_bloch(name):
    """The rejected tensors in the absorbing z faces of a Bloch grid grow
    (measured 1.0028, 1.0132 and 1.0082 here; the paper's Bloch grids: radii
    1.0049 to 1.0089)."""
    m, shape, bar = REJECTED[name]
    r = _radius(_face_spec_bloch(m, shape))
    assert r > 1.0 + bar, r


def test_tensor_energy_invariant_bloch():
    """A lossless Bloch cell (x anti-periodic, y periodic, z walled) with
    random rotated tensors: <E, M^-1 E> + <H^{n-1/2}, H^{n+1/2}> with M the
    octant assembly across the seams is conserved over 300 steps."""
    rng = np.random.Generator(np.random.PCG64(27))
    shape = (5, 4, 6)
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(0.99), eps_kind="tensor", eps_box=((0, 0, 0), shape),
                        eps=random_tensors(rng, shape), periodic=(1, 1, 0), bloch_sign=(-1, 1, 1))
    sim = O.OracleSim(spec)
    dof = sim.dof_mask()
    sim.u[:] = rng.standard_normal(sim.u.shape) * dof
    sim.u[O.PSIE0:] = 0.0
    M = _assembly_by_octants_bloch(spec)
    edof = dof[:3].reshape(-1)
    Minv = np.linalg.inv(M[np.ix_(edof, edof)])

    def energy(h_prev):
        e = np.concatenate([sim.field(c).reshape(-1) for c in range(3)])[edof]
        return e @ Minv @ e + sum(np.sum(h_prev[c] * sim.field(3 + c)) for c in range(3))

    hist = []
    for _ in range(300):
        h_prev = [sim.field(3 + c).copy() for c in range(3)]
        sim.step(1, record=False)
        hist.append(energy(h_prev))
    hist = np.asarray(hist)
    assert np.max(np.abs(hist - hist[0])) / abs(hist[0]) < 1e-11


@pytest.mark.parametrize("nsteps", [1, 30])
def test_tensor_adjoint_dot_product_bloch(nsteps):
    """The dot-product identity of the step map of a Bloch cell (x
    anti-periodic, y periodic) with random tensors inside and admitted ones
    in its absorbing z faces."""
    rng = np.random.Generator(np.random.PCG64(35))
    shape = (6, 5, 12)
    nx, ny, nz = shape
    eps = random_tensors(rng, shape, 1.0, 3.0)
    face = _pack(_rz(0.4) @ np.diag([1.5, 2.5, 4.0]) @ _rz(0.4).T)
    eps[:, :3] = face[:, None, None, None]
    eps[:, -3:] = face[:, None, None, None]
    spec = W.DomainSpec(shape=shape, courant=W.courant_3d(), pml=(0, 0, 0, 0, 3, 3), eps_kind="tensor",
                        eps_box=((0, 0, 0), shape), eps=eps, periodic=(1, 1, 0), bloch_sign=(-1, 1, 1))
    sim = O.OracleSim(spec)
    dof = sim.dof_mask()
    x = rng.standard_normal(sim.u.shape) * dof
    y = rng.standard_normal(sim.u.shape) * dof
    ax = x.copy()
    for t in range(nsteps):
        sim.step_state(ax, t, sources=False)
    aty = y.copy()
    for t in range(nsteps):
        sim.adjoint_step_state(aty, x, None)
    lhs, rhs = np.sum(ax * y * dof), np.sum(x * aty * dof)
    scale = np.linalg.norm(ax * dof) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    assert np.all(aty[~dof] == 0.0)


def test_tensor_gradient_central_differences_bloch():
    """dJ/deps of node tensors on both seams of a Bloch cell (x
    anti-periodic) against fourth-order central differences."""
    rng = np.random.Generator(np.random.PCG64(43))
    nx, ny, nz = 6, 5, 30
    shape = (nx, ny, nz)
    n_steps = 60
    lo, hi = (0, 0, 10), (nx, ny, 20)
    spec = W.DomainSpec(
        shape=shape, courant=W.courant_3d(), pml=(0, 0, 0, 0, 6, 6), eps_kind="tensor", eps_box=(lo, hi),
        eps=random_tensors(rng, (nx, ny, 10), 1.0, 3.0), eps_bg=1.0, periodic=(1, 1, 0), bloch_sign=(-1, 1, 1),
        sources=[W.SourceSpec("plane_z", 0, (0, 0, 7), W.gaussian_sine(n_steps, 0.5, 8.0, 24.0)),
                 W.SourceSpec("point", 1, (0, 2, 8), W.gaussian_sine(n_steps, 0.6, 6.0, 18.0))],
        monitors=[W.MonitorSpec("flux_z", pos=(0, 0, 22), rect=(0, nx, 0, ny), omega_dt=np.array([0.45, 0.6]))],
        n_steps=n_steps)

    def run(sp):
        sim = O.OracleSim(sp)
        sim.step(sp.n_steps)
        f = sim.spectra(0)
        g = np.zeros_like(f)
        g[:, 0], g[:, 3], g[:, 1], g[:, 2] = f[:, 3], f[:, 0], -f[:, 2], -f[:, 1]
        return sim, float(np.sum(O.OracleSim.flux_from_spectra(f))), g

    sim, J, cot = run(spec)
    g = sim.gradient({0: cot}, n_steps)
    for (i, j, k) in [(0, 2, 12), (5, 0, 15), (3, 4, 18)]:
        for q in range(6):
            h = 2e-3
            vals = {}
            for m in (-2, -1, 1, 2):
                e = spec.eps.copy()
                e[q, k - lo[2], j, i] += m * h
                vals[m] = run(W.DomainSpec(**{**spec.__dict__, "eps": e}))[1]
            fd = (8.0 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12.0 * h)
            assert abs(g[q, k, j, i] - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(J), (i, j, k, q, g[q, k, j, i], fd)
