"""Seeded synthetic workloads for the FDTD hot path.

This module only *describes* problems: grid sizes, absorbing-layer depths and
grading constants, permittivity arrays drawn from seeded generators, dispersive
boxes, source waveforms, monitor placements and frequencies.  It performs none
of the method's arithmetic (no curls, no absorber coefficients, no dispersion
coefficients, no transforms), so that the CPU oracle and the HIP library can
both consume the same inputs without sharing any numerical code.

Index conventions (used by both consumers):
  * every field-like array is ``[nz][ny][nx]`` (x fastest);
  * ``lo``/``hi`` boxes are half-open ``[lo, hi)`` triples ``(i, j, k)``;
  * component codes: 0,1,2 = Ex,Ey,Ez ; 3,4,5 = Hx,Hy,Hz.

The workloads follow the shapes of the paper's scenes (Section 6-7: dielectric
scatterers in absorbing boxes, dispersive slabs, plane monitors); no dataset
is read.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

Box = Tuple[Tuple[int, int, int], Tuple[int, int, int]]

EX, EY, EZ, HX, HY, HZ = range(6)
COMP_NAMES = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


@dataclass
class PoleSpec:
    """One pole of a dispersive medium.  kind 'lorentz': strength delta_eps,
    resonance omega_dt = omega_0 dt; kind 'drude': plasma omega_dt = omega_p dt
    (delta_eps unused).  gamma_dt = damping gamma dt."""
    kind: str
    delta_eps: float
    omega_dt: float
    gamma_dt: float


@dataclass
class LorentzSpec:
    """Dispersive medium on a box; eps_inf is the cell's permittivity.  One
    Lorentz pole (delta_eps, omega0_dt, gamma_dt), or, when ``poles`` is given,
    those poles (up to 16) instead."""
    lo: Tuple[int, int, int]
    hi: Tuple[int, int, int]
    delta_eps: float
    omega0_dt: float
    gamma_dt: float
    poles: Optional[List[PoleSpec]] = None

    def pole_list(self) -> List[PoleSpec]:
        if self.poles:
            return list(self.poles)
        return [PoleSpec("lorentz", self.delta_eps, self.omega0_dt, self.gamma_dt)]


@dataclass
class SourceSpec:
    """Soft electric source.  ``kind`` is 'point' or 'plane_z' (whole z-plane).

    ``waveform[t]`` is the increment added at forward step t (the step that
    produces E at time (t+1)*dt); steps past the end add nothing.
    """
    kind: str
    comp: int
    pos: Tuple[int, int, int]
    waveform: np.ndarray


@dataclass
class MonitorSpec:
    """Observation.

    kind 'probe'   : comp at pos, one sample per forward step.
    kind 'flux_z'  : z-plane pos[2], rectangle rect=(i0,i1,j0,j1); records
                     Ex, Ey and Hx, Hy averaged over planes k and k-1.
    kind 'patch_z' : one component comp on z-plane pos[2], rectangle rect.
    """
    kind: str
    comp: int = 0
    pos: Tuple[int, int, int] = (0, 0, 0)
    rect: Tuple[int, int, int, int] = (0, 0, 0, 0)
    omega_dt: np.ndarray = field(default_factory=lambda: np.zeros(0))


@dataclass
class DomainSpec:
    shape: Tuple[int, int, int]                 # (nx, ny, nz), absorbing cells included
    courant: float                              # S = c dt / h
    pml: Tuple[int, int, int, int, int, int] = (0, 0, 0, 0, 0, 0)   # xlo,xhi,ylo,yhi,zlo,zhi
    pml_m: float = 3.0
    pml_kappa_max: float = 5.0
    pml_sigma_max: float = 3.2
    pml_alpha_max: float = 0.05
    eps_kind: str = "iso"                       # 'iso', 'diag' or 'tensor'
    eps_box: Optional[Box] = None               # where ``eps`` is given; eps_bg outside
    eps: Optional[np.ndarray] = None            # [ncomp][bz][by][bx]; tensor: 6 components
    #                                             xx, yy, zz, xy, xz, yz at the grid nodes
    eps_bg: float = 1.0
    lorentz: List[LorentzSpec] = field(default_factory=list)
    sources: List[SourceSpec] = field(default_factory=list)
    monitors: List[MonitorSpec] = field(default_factory=list)
    grad_box: Optional[Box] = None
    n_steps: int = 0
    periodic: Tuple[int, int, int] = (0, 0, 0)  # 1: Bloch-periodic axis (x or y), no absorber on it
    bloch_sign: Tuple[int, int, int] = (1, 1, 1)  # real Bloch factor exp(i k L) of each periodic axis: +1 or -1

    @property
    def ncells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def eps_nodes(self) -> np.ndarray:
        """Tensor media: the dense node tensor [6][nz][ny][nx] (xx, yy, zz, xy,
        xz, yz), eps_bg times the identity outside the box."""
        assert self.eps_kind == "tensor"
        nx, ny, nz = self.shape
        out = np.zeros((6, nz, ny, nx))
        out[:3] = float(self.eps_bg)
        if self.eps is not None:
            (i0, j0, k0), (i1, j1, k1) = self.eps_box
            out[:, k0:k1, j0:j1, i0:i1] = self.eps
        return out

    def eps_full(self) -> np.ndarray:
        """Dense per-component permittivity [3][nz][ny][nx] (float64); tensor
        media have none per E node (eps_bg throughout)."""
        nx, ny, nz = self.shape
        if self.eps_kind == "tensor":
            return np.full((3, nz, ny, nx), float(self.eps_bg))
        out = np.full((3, nz, ny, nx), float(self.eps_bg))
        if self.eps is not None:
            (i0, j0, k0), (i1, j1, k1) = self.eps_box
            e = self.eps
            for c in range(3):
                out[c, k0:k1, j0:j1, i0:i1] = e[0] if e.shape[0] == 1 else e[c]
        return out


# --------------------------------------------------------------------------
# waveforms and frequency grids (inputs, not method arithmetic)
# --------------------------------------------------------------------------

def gaussian_sine(n_steps: int, omega_c_dt: float, tau: float, n0: float) -> np.ndarray:
    """s(n) = sin(w_c dt (n-n0)) exp(-((n-n0)/tau)^2 / 2), sampled at n=1..n_steps.

    Entry t of the result is s(t+1), the increment of forward step t."""
    n = np.arange(1, n_steps + 1, dtype=np.float64)
    x = n - n0
    return np.sin(omega_c_dt * x) * np.exp(-0.5 * (x / tau) ** 2)


def freq_grid(n_f: int, lo: float = 0.10, hi: float = 0.20) -> np.ndarray:
    return np.linspace(lo, hi, n_f)


def courant_3d(eta: float = 0.99) -> float:
    """Uniform-mesh Courant number S = eta / sqrt(3)."""
    return eta / math.sqrt(3.0)


def _centered_box(n: Sequence[int], size: Sequence[int]) -> Box:
    lo = tuple((n[a] - size[a]) // 2 for a in range(3))
    hi = tuple(lo[a] + size[a] for a in range(3))
    return lo, hi


# --------------------------------------------------------------------------
# the five workloads and their reduced parity-size relatives
# --------------------------------------------------------------------------

def pec_cavity(n: int = 32, n_steps: int = 200, seed: int = 1001, src=None, probe=None) -> DomainSpec:
    """3D Yee FP64 PEC box with per-cell eps in [1,4], Ez point dipole, Ez probe."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = 1.0 + 3.0 * rng.random((n, n, n))
    c = n // 2
    src = src or (c, c, c)
    probe = probe or (min(n - 2, c + n // 4), c, c)
    return DomainSpec(
        shape=(n, n, n), courant=courant_3d(), eps_kind="iso",
        eps_box=((0, 0, 0), (n, n, n)), eps=eps[None], eps_bg=1.0,
        sources=[SourceSpec("point", EZ, src, gaussian_sine(n_steps, 0.2 * math.pi, 20.0, 80.0))],
        monitors=[MonitorSpec("probe", comp=EZ, pos=probe)],
        n_steps=n_steps,
    )


def pole_set(n: int) -> List[PoleSpec]:
    """Pole lists for a dispersive box: 3 = two Lorentz poles and a Drude pole;
    16 (the maximum a box takes) = ten Lorentz poles spread over resonance and
    damping and six Drude poles."""
    if n == 3:
        return [PoleSpec("lorentz", 0.9, 0.45, 0.05), PoleSpec("lorentz", 0.6, 0.7, 0.1),
                PoleSpec("drude", 0.0, 0.35, 0.08)]
    if n == 16:
        return ([PoleSpec("lorentz", 0.05 + 0.03 * p, 0.2 + 0.05 * p, 0.01 + 0.01 * p) for p in range(10)] +
                [PoleSpec("drude", 0.0, 0.05 + 0.02 * p, 0.02 + 0.02 * p) for p in range(6)])
    raise ValueError("pole sets: 3 or 16")


def with_poles(spec: "DomainSpec", poles: List[PoleSpec]) -> "DomainSpec":
    """The same domain with every dispersive box holding ``poles``."""
    spec.lorentz = [LorentzSpec(L.lo, L.hi, 0.0, 0.0, 0.0, poles=list(poles)) for L in spec.lorentz]
    return spec


def lorentz_flux(interior: int = 128, pml: int = 10, lorentz: int = 48, n_steps: int = 1000,
                 n_f: int = 16, shape: Optional[Tuple[int, int, int]] = None) -> DomainSpec:
    """FP32 forward: interior^3 + CPML, central Lorentz block, z-sheet source, far flux plane."""
    if shape is None:
        shape = (interior + 2 * pml,) * 3
    nx, ny, nz = shape
    lo, hi = _centered_box(shape, (lorentz,) * 3)
    eps = np.full((1, lorentz, lorentz, lorentz), 2.0)
    ks = pml + 5
    kf = nz - pml - 6
    return DomainSpec(
        shape=shape, courant=courant_3d(), pml=(pml,) * 6, eps_kind="iso",
        eps_box=(lo, hi), eps=eps, eps_bg=1.0,
        lorentz=[LorentzSpec(lo, hi, 1.5, 0.15, 0.01)],
        sources=[SourceSpec("plane_z", EX, (0, 0, ks), gaussian_sine(n_steps, 0.15, 30.0, 120.0))],
        monitors=[MonitorSpec("flux_z", pos=(0, 0, kf), rect=(0, nx, 0, ny), omega_dt=freq_grid(n_f))],
        n_steps=n_steps,
    )


def design_patch(interior: int = 192, pml: int = 10, design: int = 64, patch: int = 32,
                 n_steps: int = 2000, n_f: int = 8, seed: int = 1003, n_fd: int = 20,
                 shape: Optional[Tuple[int, int, int]] = None):
    """FP32 adjoint: random eps_r in [1,6] on a centred design box; |DFT Ez|^2 on a patch.

    Returns (spec, fd_cells) where fd_cells are (i,j,k) inside the design box
    drawn from the same generator after eps."""
    if shape is None:
        shape = (interior + 2 * pml,) * 3
    nx, ny, nz = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = _centered_box(shape, (design,) * 3)
    eps = 1.0 + 5.0 * rng.random((design, design, design))
    cells = rng.integers(0, design, size=(n_fd, 3))
    fd_cells = [tuple(int(lo[a] + cells[m, a]) for a in range(3)) for m in range(n_fd)]
    kp = nz - pml - 10
    p0 = ((nx - patch) // 2, (ny - patch) // 2)
    spec = DomainSpec(
        shape=shape, courant=courant_3d(), pml=(pml,) * 6, eps_kind="iso",
        eps_box=(lo, hi), eps=eps[None], eps_bg=1.0,
        sources=[SourceSpec("plane_z", EX, (0, 0, pml + 5), gaussian_sine(n_steps, 0.15, 30.0, 120.0))],
        monitors=[MonitorSpec("patch_z", comp=EZ, pos=(0, 0, kp),
                              rect=(p0[0], p0[0] + patch, p0[1], p0[1] + patch), omega_dt=freq_grid(n_f))],
        grad_box=(lo, hi), n_steps=n_steps,
    )
    return spec, fd_cells


def batch_domains(n_domains: int = 48, sizes: Sequence[int] = (48, 64, 96, 128, 160), pml: int = 10,
                  n_steps: int = 800, n_f: int = 4, seed: int = 1004) -> List[DomainSpec]:
    """Ragged ensemble: per-axis interior sizes drawn from ``sizes`` (Cartesian product)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    picks = rng.integers(0, len(sizes), size=(n_domains, 3))
    out = []
    for d in range(n_domains):
        inner = tuple(int(sizes[picks[d, a]]) for a in range(3))
        shape = tuple(inner[a] + 2 * pml for a in range(3))
        nx, ny, nz = shape
        eps = 1.0 + 3.0 * rng.random((inner[2], inner[1], inner[0]))
        lo = (pml, pml, pml)
        hi = (nx - pml, ny - pml, nz - pml)
        c = (nx // 2, ny // 2, nz // 2)
        kf = nz - pml - 3
        out.append(DomainSpec(
            shape=shape, courant=courant_3d(), pml=(pml,) * 6, eps_kind="iso",
            eps_box=(lo, hi), eps=eps[None], eps_bg=1.0,
            sources=[SourceSpec("point", EZ, c, gaussian_sine(n_steps, 0.15, 30.0, 120.0))],
            monitors=[MonitorSpec("flux_z", pos=(0, 0, kf), rect=(0, nx, 0, ny), omega_dt=freq_grid(n_f))],
            grad_box=(lo, hi) if d % 2 == 0 else None, n_steps=n_steps,
        ))
    return out


def anisotropic_lorentz(interior: int = 512, pml: int = 12, lorentz: int = 128, patch: int = 64,
                        n_steps: int = 4000, n_f: int = 8, seed: int = 1005,
                        shape: Optional[Tuple[int, int, int]] = None) -> DomainSpec:
    """FP32 adjoint: diagonal eps (each in [1,5]) on the interior, central Lorentz box."""
    if shape is None:
        shape = (interior + 2 * pml,) * 3
    nx, ny, nz = shape
    inner = (nx - 2 * pml, ny - 2 * pml, nz - 2 * pml)
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = np.empty((3, inner[2], inner[1], inner[0]))
    for c in range(3):
        eps[c] = 1.0 + 4.0 * rng.random((inner[2], inner[1], inner[0]))
    lo = (pml, pml, pml)
    hi = (nx - pml, ny - pml, nz - pml)
    llo, lhi = _centered_box(shape, (lorentz,) * 3)
    kp = nz - pml - 5
    p0 = ((nx - patch) // 2, (ny - patch) // 2)
    return DomainSpec(
        shape=shape, courant=courant_3d(), pml=(pml,) * 6, eps_kind="diag",
        eps_box=(lo, hi), eps=eps, eps_bg=1.0,
        lorentz=[LorentzSpec(llo, lhi, 1.5, 0.15, 0.01)],
        sources=[SourceSpec("plane_z", EX, (0, 0, pml + 5), gaussian_sine(n_steps, 0.15, 30.0, 120.0))],
        monitors=[MonitorSpec("patch_z", comp=EX, pos=(0, 0, kp),
                              rect=(p0[0], p0[0] + patch, p0[1], p0[1] + patch), omega_dt=freq_grid(n_f))],
        grad_box=(lo, hi), n_steps=n_steps,
    )


def random_spd_tensors(rng: np.random.Generator, n: int, lo: float = 1.0, hi: float = 5.0,
                       chunk: int = 1 << 22) -> np.ndarray:
    """[6][n] symmetric tensors R diag(l) R^T (xx, yy, zz, xy, xz, yz) with
    eigenvalues l uniform in [lo, hi] and R a uniformly random rotation (a
    normalised Gaussian quaternion), drawn chunk by chunk."""
    out = np.empty((6, n))
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for s0 in range(0, n, chunk):
        m = min(chunk, n - s0)
        w, x, y, z = rng.standard_normal((4, m))
        r = np.sqrt(w * w + x * x + y * y + z * z)
        w, x, y, z = w / r, x / r, y / r, z / r
        R = ((1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)),
             (2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)),
             (2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)))
        lam = lo + (hi - lo) * rng.random((3, m))
        for q, (a, b) in enumerate(pairs):
            out[q, s0:s0 + m] = R[a][0] * R[b][0] * lam[0] + R[a][1] * R[b][1] * lam[1] + R[a][2] * R[b][2] * lam[2]
    return out


def anisotropic_tensor(interior: int = 512, pml: int = 12, patch: int = 64, n_steps: int = 4000, n_f: int = 8,
                       seed: int = 1006, shape: Optional[Tuple[int, int, int]] = None,
                       block: int = 64) -> DomainSpec:
    """Full symmetric tensor media (Section 2.3): a randomly rotated tensor
    with eigenvalues in [1, 5] at every node between the absorbing slabs,
    vacuum in the slabs; the x-polarised plane source and Ex patch monitor of
    the diagonal anisotropic workload; forward only.  A block of block^3
    independent node tensors repeats across the interior (drawing 1.3e8
    rotations one by one would dominate the set-up)."""
    if shape is None:
        shape = (interior + 2 * pml,) * 3
    nx, ny, nz = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = (pml, pml, pml)
    hi = (nx - pml, ny - pml, nz - pml)
    bx, by, bz = hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]
    cb = (min(block, bz), min(block, by), min(block, bx))
    cell = random_spd_tensors(rng, cb[0] * cb[1] * cb[2]).reshape((6,) + cb)
    eps = np.empty((6, bz, by, bx))
    for z0 in range(0, bz, cb[0]):
        for y0 in range(0, by, cb[1]):
            for x0 in range(0, bx, cb[2]):
                dz, dy, dx = min(cb[0], bz - z0), min(cb[1], by - y0), min(cb[2], bx - x0)
                eps[:, z0:z0 + dz, y0:y0 + dy, x0:x0 + dx] = cell[:, :dz, :dy, :dx]
    kp = nz - pml - 5
    p0 = ((nx - patch) // 2, (ny - patch) // 2)
    return DomainSpec(
        shape=shape, courant=courant_3d(), pml=(pml,) * 6, eps_kind="tensor",
        eps_box=(lo, hi), eps=eps, eps_bg=1.0,
        sources=[SourceSpec("plane_z", EX, (0, 0, pml + 5), gaussian_sine(n_steps, 0.15, 30.0, 120.0))],
        monitors=[MonitorSpec("patch_z", comp=EX, pos=(0, 0, kp),
                              rect=(p0[0], p0[0] + patch, p0[1], p0[1] + patch), omega_dt=freq_grid(n_f))],
        n_steps=n_steps,
    )


def bloch_cell(nxy: int = 512, nz: int = 536, pml: int = 12, layer: int = 64, n_steps: int = 4000, n_f: int = 8,
               seed: int = 1007, sign_x: int = -1) -> DomainSpec:
    """A Bloch-periodic cell at the headline's size (Section 2.2; the slab
    set-up of Section 6.1): x and y periodic with the real factors (sign_x,
    +1), absorbing cells at the z ends only, a patterned layer of `layer`
    planes with diagonal eps in [1, 5] over the whole cross-section (the
    gradient box), an Ex sheet below it and a flux plane above it."""
    shape = (nxy, nxy, nz)
    rng = np.random.Generator(np.random.PCG64(seed))
    z0 = (nz - layer) // 2
    eps = 1.0 + 4.0 * rng.random((3, layer, nxy, nxy))
    box = ((0, 0, z0), (nxy, nxy, z0 + layer))
    return DomainSpec(
        shape=shape, courant=courant_3d(), pml=(0, 0, 0, 0, pml, pml), eps_kind="diag", eps_box=box, eps=eps,
        eps_bg=1.0,
        sources=[SourceSpec("plane_z", EX, (0, 0, pml + 5), gaussian_sine(n_steps, 0.15, 30.0, 120.0))],
        monitors=[MonitorSpec("flux_z", pos=(0, 0, nz - pml - 5), rect=(0, nxy, 0, nxy), omega_dt=freq_grid(n_f))],
        grad_box=box, n_steps=n_steps, periodic=(1, 1, 0), bloch_sign=(sign_x, 1, 1),
    )


def random_state_like(spec: DomainSpec, seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# Full-size named workloads, for the benchmark, profiling and sampled
# full-size parity.
WORKLOADS = {
    "pec_cavity": lambda: pec_cavity(32, 200),
    "lorentz_flux": lambda: lorentz_flux(),
    "design_patch": lambda: design_patch()[0],
    "batch_domains": lambda: batch_domains(),
    "anisotropic_lorentz": lambda: anisotropic_lorentz(),
    "anisotropic_tensor": lambda: anisotropic_tensor(),
    "bloch_cell": lambda: bloch_cell(),
}
