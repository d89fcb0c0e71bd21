"""FP64 CPU oracle of the differentiable FDTD hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never does.

Numerics live in ``fdtd_oracle.c`` (plain loops).  This file holds what the
paper leaves to the driver:

* absorber profiles (Section 2.2): polynomial grading of sigma and kappa,
  linear alpha; the coefficients b and c of the recursive convolution;
* the step driver with soft sources (Section 2.4) and monitors (Section 2.4:
  point samples, plane spectra with the magnetic half-step phase, Poynting
  flux);
* the adjoint driver (Eq. 3, Section 3.1) with seeds dJ/du^n from the
  observation transposes, and a bisection checkpoint schedule: a plain
  recursive replay whose correctness is evident by inspection.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdtd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# state layout: 21 + 6 P full-grid arrays for P dispersive poles (27 for one):
# fields, E- and H-side absorber memories, E^{n-1}, then W^n of each pole
# (3 components each) and W^{n-1} of each pole
F0 = 0                      # Ex Ey Ez Hx Hy Hz
PSI_PAIRS = [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)]   # (component, derivative axis)
PSIE0 = 6
PSIH0 = 12
EOLD0, W0, WOLD0 = 18, 21, 24   # one pole
NSTATE = 27                     # one pole
MAXP = 16


def state_layout(npole: int):
    """(index of W^n of pole 0, index of W^{n-1} of pole 0, state arrays) for
    npole poles; pole p, component c sit at base + 3 p + c."""
    w0 = 21
    return w0, w0 + 3 * npole, w0 + 6 * npole


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("S", C.c_double),
                ("bE", C.c_void_p * 3), ("cE", C.c_void_p * 3), ("kiE", C.c_void_p * 3),
                ("bH", C.c_void_p * 3), ("cH", C.c_void_p * 3), ("kiH", C.c_void_p * 3),
                ("slab", C.c_void_p * 3), ("eps", C.c_void_p * 3), ("lor", C.c_void_p),
                ("npole", C.c_int), ("pkind", C.c_int * MAXP), ("pdeps", C.c_double * MAXP),
                ("pwdt", C.c_double * MAXP), ("pgdt", C.c_double * MAXP),
                ("per", C.c_int * 3), ("bsign", C.c_double * 3),
                ("einvT", C.c_void_p * 6), ("einv_bg", C.c_double)]


class _State(C.Structure):
    _fields_ = [("F", C.c_void_p * 6), ("psiE", C.c_void_p * 9), ("psiH", C.c_void_p * 9),
                ("Eold", C.c_void_p * 3), ("W", C.c_void_p * (3 * MAXP)), ("Wold", C.c_void_p * (3 * MAXP))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.orc_step.argtypes = [C.POINTER(_Params), C.POINTER(_State), C.c_int, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        _lib.orc_step.restype = None
        _lib.orc_adjoint_step.argtypes = [C.POINTER(_Params), C.POINTER(_State), C.POINTER(_State),
                                          C.c_void_p, C.c_void_p]
        _lib.orc_adjoint_step.restype = None
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# --------------------------------------------------------------------------
# absorber profiles (Section 2.2, Roden-Gedney recursive convolution)
# --------------------------------------------------------------------------

def cpml_axis(n: int, l0: int, l1: int, S: float, m: float, kmax: float, smax: float, amax: float,
              half: bool):
    """Tables along one axis.  Node i sits at x = i (E-update derivatives) or
    x = i + 1/2 (H-update derivatives).  Depth into a face d in [0,1] is 0 at
    the interface and 1 at the outer wall; sigma = smax d^m,
    kappa = 1 + (kmax-1) d^m, alpha = amax (1-d);
    b = exp(-(sigma/kappa + alpha) dt), c = sigma (b-1) / (sigma kappa + kappa^2 alpha)."""
    b = np.ones(n)
    c = np.zeros(n)
    ki = np.ones(n)
    slab = np.zeros(n, dtype=np.uint8)
    for i in range(n):
        x = i + (0.5 if half else 0.0)
        d = None
        if l0 > 0 and i < l0:
            d = max(0.0, (l0 - x) / l0)
        elif l1 > 0 and i >= n - l1:
            d = max(0.0, (x - (n - l1)) / l1)
        if d is None:
            continue
        slab[i] = 1
        sig = smax * d ** m
        kap = 1.0 + (kmax - 1.0) * d ** m
        alp = amax * (1.0 - d)
        b[i] = math.exp(-(sig / kap + alp) * S)
        c[i] = sig * (b[i] - 1.0) / (sig * kap + kap * kap * alp) if sig > 0 else 0.0
        ki[i] = 1.0 / kap
    return b, c, ki, slab


class OracleSim:
    """One domain advanced by the FP64 oracle."""

    def __init__(self, spec):
        _load()
        self.spec = spec
        nx, ny, nz = spec.shape
        self.shape3 = (nz, ny, nx)
        self.N = nx * ny * nz
        S = spec.courant
        self._keep = []
        P = _Params()
        P.n[0], P.n[1], P.n[2] = nx, ny, nz
        P.S = S
        self.per = tuple(int(v) for v in getattr(spec, "periodic", (0, 0, 0)))
        for a in range(3):
            P.per[a] = self.per[a]
            P.bsign[a] = float(getattr(spec, "bloch_sign", (1, 1, 1))[a])
        self.tabE, self.tabH = [], []
        for a in range(3):
            n = spec.shape[a]
            l0, l1 = spec.pml[2 * a], spec.pml[2 * a + 1]
            tE = cpml_axis(n, l0, l1, S, spec.pml_m, spec.pml_kappa_max, spec.pml_sigma_max,
                           spec.pml_alpha_max, half=False)
            tH = cpml_axis(n, l0, l1, S, spec.pml_m, spec.pml_kappa_max, spec.pml_sigma_max,
                           spec.pml_alpha_max, half=True)
            self.tabE.append(tE)
            self.tabH.append(tH)
            assert np.array_equal(tE[3], tH[3])
            P.bE[a], P.cE[a], P.kiE[a] = _ptr(tE[0]), _ptr(tE[1]), _ptr(tE[2])
            P.bH[a], P.cH[a], P.kiH[a] = _ptr(tH[0]), _ptr(tH[1]), _ptr(tH[2])
            P.slab[a] = _ptr(tE[3])
            self._keep += list(tE) + list(tH)
        self.eps = np.ascontiguousarray(spec.eps_full())
        for c in range(3):
            P.eps[c] = _ptr(self.eps[c])
        self.tensor = spec.eps_kind == "tensor"
        if self.tensor:
            # Section 2.3: the symmetric tensor at each node, inverted there
            assert not spec.lorentz, "tensor media: no dispersive box"
            en = spec.eps_nodes()
            m = np.empty(en.shape[1:] + (3, 3))
            for q, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
                m[..., a, b] = m[..., b, a] = en[q]
            inv = np.linalg.inv(m)
            self.einvT = np.ascontiguousarray(
                np.stack([inv[..., a, b] for (a, b) in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))]))
            for q in range(6):
                P.einvT[q] = _ptr(self.einvT[q])
            P.einv_bg = 1.0 / float(spec.eps_bg)
        self.lor = None
        self.npole = 1
        if spec.lorentz:
            assert len(spec.lorentz) == 1
            L = spec.lorentz[0]
            self.lor = np.zeros(self.shape3, dtype=np.uint8)
            (i0, j0, k0), (i1, j1, k1) = L.lo, L.hi
            self.lor[k0:k1, j0:j1, i0:i1] = 1
            P.lor = _ptr(self.lor)
            poles = L.pole_list()
            assert 1 <= len(poles) <= MAXP
            self.npole = len(poles)
            P.npole = len(poles)
            for q, pl in enumerate(poles):
                P.pkind[q] = {"lorentz": 0, "drude": 1}[pl.kind]
                P.pdeps[q], P.pwdt[q], P.pgdt[q] = pl.delta_eps, pl.omega_dt, pl.gamma_dt
        else:
            P.lor = None
            P.npole = 0
            self.npole = 0
        # (a domain without dispersive cells keeps the one-pole layout, unused)
        self.W0, self.WOLD0, self.NSTATE = state_layout(max(self.npole, 1))
        self.P = P
        self.u = np.zeros((self.NSTATE, self.N))
        self.work = np.zeros((7 if self.tensor else 4, self.N))
        self.t = 0
        # sources: flattened node lists
        self.src_comp, self.src_idx, self.src_wave = [], [], []
        for s_id, s in enumerate(spec.sources):
            if s.kind == "point":
                i, j, k = s.pos
                idx = [(k * ny + j) * nx + i]
            elif s.kind == "plane_z":
                k = s.pos[2]
                idx = list(k * nx * ny + np.arange(nx * ny))
            else:
                raise ValueError(s.kind)
            self.src_idx += idx
            self.src_comp += [s.comp] * len(idx)
            self.src_wave += [s_id] * len(idx)
        self.src_idx = np.asarray(self.src_idx, dtype=np.int64)
        self.src_comp = np.asarray(self.src_comp, dtype=np.int32)
        self.src_wave = np.asarray(self.src_wave, dtype=np.int64)
        self.reset_monitors()

    # ---------------- state helpers ----------------
    def _state_struct(self, u: np.ndarray) -> _State:
        st = _State()
        N = self.N
        base = _ptr(u)
        for q in range(6):
            st.F[q] = base + 8 * N * (F0 + q)
        for r, (c, a) in enumerate(PSI_PAIRS):
            st.psiE[3 * c + a] = base + 8 * N * (PSIE0 + r)
            st.psiH[3 * c + a] = base + 8 * N * (PSIH0 + r)
        for c in range(3):
            st.Eold[c] = base + 8 * N * (EOLD0 + c)
            for q in range(self.npole):
                st.W[MAXP * c + q] = base + 8 * N * (self.W0 + 3 * q + c)
                st.Wold[MAXP * c + q] = base + 8 * N * (self.WOLD0 + 3 * q + c)
        return st

    def field(self, q: int, u: Optional[np.ndarray] = None) -> np.ndarray:
        u = self.u if u is None else u
        return u[F0 + q].reshape(self.shape3)

    def dof_mask(self) -> np.ndarray:
        """Boolean [NSTATE][N]: entries of the state that are degrees of freedom."""
        nz, ny, nx = self.shape3
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        x = (i, j, k)
        m = np.zeros((self.NSTATE,) + self.shape3, dtype=bool)
        for c in range(3):
            a1, a2 = (c + 1) % 3, (c + 2) % 3
            m[F0 + c] = ~(((x[a1] == 0) & (not self.per[a1])) | ((x[a2] == 0) & (not self.per[a2])))
            m[F0 + 3 + c] = True
        for r, (c, a) in enumerate(PSI_PAIRS):
            sl = self.tabE[a][3][x[a]].astype(bool)
            m[PSIE0 + r] = sl & m[F0 + c]
            m[PSIH0 + r] = sl
        if self.lor is not None:
            for c in range(3):
                bases = [EOLD0] + [self.W0 + 3 * q for q in range(self.npole)] + \
                        [self.WOLD0 + 3 * q for q in range(self.npole)]
                for base in bases:
                    m[base + c] = self.lor.astype(bool) & m[F0 + c]
        return m.reshape(self.NSTATE, self.N)

    # ---------------- stepping ----------------
    def _src_amps(self, t: int) -> np.ndarray:
        amps = np.zeros(len(self.src_idx))
        for s_id, s in enumerate(self.spec.sources):
            v = s.waveform[t] if t < len(s.waveform) else 0.0
            amps[self.src_wave == s_id] = v
        return amps

    def step_state(self, u: np.ndarray, t: int, sources: bool = True):
        st = self._state_struct(u)
        if sources and len(self.src_idx):
            amps = self._src_amps(t)
            _lib.orc_step(C.byref(self.P), C.byref(st), len(self.src_idx), _ptr(self.src_comp),
                          _ptr(self.src_idx), _ptr(amps), _ptr(self.work))
        else:
            _lib.orc_step(C.byref(self.P), C.byref(st), 0, None, None, None, _ptr(self.work))

    def step(self, n: int = 1, record: bool = True, store_f32: bool = False):
        """Advance n steps.  store_f32 rounds the whole state to float32 after
        every step while the arithmetic stays FP64: a model of float32 state
        storage alone, used to measure the error floor any float32-state
        solver carries (it is not part of the method)."""
        for _ in range(n):
            self.step_state(self.u, self.t)
            if store_f32:
                if getattr(self, "_u32", None) is None:
                    self._u32 = np.zeros(self.u.shape, dtype=np.float32)
                np.copyto(self._u32, self.u, casting="same_kind")   # round to nearest
                np.copyto(self.u, self._u32)
            self.t += 1
            if record:
                self._record(self.u, self.t)

    def adjoint_step_state(self, a: np.ndarray, u: np.ndarray, g: Optional[np.ndarray]):
        sa = self._state_struct(a)
        su = self._state_struct(u)
        if g is not None:
            gp = (C.c_void_p * len(g))(*[_ptr(g[q]) for q in range(len(g))])
            _lib.orc_adjoint_step(C.byref(self.P), C.byref(sa), C.byref(su), C.cast(gp, C.c_void_p),
                                  _ptr(self.work))
        else:
            _lib.orc_adjoint_step(C.byref(self.P), C.byref(sa), C.byref(su), None, _ptr(self.work))

    # ---------------- monitors (Section 2.4) ----------------
    def reset_monitors(self):
        self.mon = []
        for m in self.spec.monitors:
            if m.kind == "probe":
                self.mon.append([])
            elif m.kind == "flux_z":
                i0, i1, j0, j1 = m.rect
                self.mon.append(np.zeros((len(m.omega_dt), 4, j1 - j0, i1 - i0), dtype=np.complex128))
            elif m.kind == "patch_z":
                i0, i1, j0, j1 = m.rect
                self.mon.append(np.zeros((len(m.omega_dt), 1, j1 - j0, i1 - i0), dtype=np.complex128))
            else:
                raise ValueError(m.kind)

    def _plane_samples(self, m, u):
        """Samples of one monitor from state u (E at time n, H at n+1/2)."""
        k = m.pos[2]
        i0, i1, j0, j1 = m.rect
        F = [self.field(q, u) for q in range(6)]
        if m.kind == "flux_z":
            hx = F[3][k, j0:j1, i0:i1] + (F[3][k - 1, j0:j1, i0:i1] if k > 0 else 0.0)
            hy = F[4][k, j0:j1, i0:i1] + (F[4][k - 1, j0:j1, i0:i1] if k > 0 else 0.0)
            return [(F[0][k, j0:j1, i0:i1], False), (F[1][k, j0:j1, i0:i1], False),
                    (0.5 * hx, True), (0.5 * hy, True)]
        return [(F[m.comp][k, j0:j1, i0:i1], m.comp >= 3)]

    def _record(self, u, n: int):
        for mi, m in enumerate(self.spec.monitors):
            if m.kind == "probe":
                i, j, k = m.pos
                self.mon[mi].append(self.field(m.comp, u)[k, j, i])
                continue
            for q, (val, is_h) in enumerate(self._plane_samples(m, u)):
                tph = n + (0.5 if is_h else 0.0)
                ph = np.exp(-1j * m.omega_dt * tph)          # e^{-i w t}
                self.mon[mi][:, q] += ph[:, None, None] * val[None]

    def spectra(self, mi: int) -> np.ndarray:
        return self.mon[mi]

    def probe(self, mi: int) -> np.ndarray:
        return np.asarray(self.mon[mi])

    @staticmethod
    def flux_from_spectra(sp: np.ndarray) -> np.ndarray:
        """F(w) = Re sum [Ex Hy* - Ey Hx*] over the plane, +z positive."""
        return np.real(np.sum(sp[:, 0] * np.conj(sp[:, 3]) - sp[:, 1] * np.conj(sp[:, 2]), axis=(1, 2)))

    # ---------------- adjoint (Eq. 3) ----------------
    def _add_seeds(self, a: np.ndarray, n: int, cot: Dict[int, np.ndarray]):
        """a += dJ/du^n.  cot[mi] holds dJ/dRe + i dJ/dIm of monitor mi's
        spectra (or dJ/dsample for a probe).  Seed of a sample taken with
        phase e^{-i w t}: Re sum_f cot_f e^{+i w_f t}."""
        if n < 1:
            return
        for mi, G in cot.items():
            m = self.spec.monitors[mi]
            if m.kind == "probe":
                if n - 1 < len(G):
                    i, j, k = m.pos
                    self.field(m.comp, a)[k, j, i] += G[n - 1]
                continue
            k = m.pos[2]
            i0, i1, j0, j1 = m.rect
            if m.kind == "flux_z":
                comps = [(0, False, [k]), (1, False, [k]), (3, True, [k, k - 1]), (4, True, [k, k - 1])]
            else:
                comps = [(m.comp, m.comp >= 3, [k])]
            for q, (fq, is_h, planes) in enumerate(comps):
                tph = n + (0.5 if is_h else 0.0)
                ph = np.exp(1j * m.omega_dt * tph)
                seed = np.real(np.sum(G[:, q] * ph[:, None, None], axis=0))
                w = 0.5 if m.kind == "flux_z" and is_h else 1.0
                for kk in planes:
                    if kk >= 0:
                        self.field(fq, a)[kk, j0:j1, i0:i1] += w * seed

    def gradient(self, cot: Dict[int, np.ndarray], n_steps: int, u0: Optional[np.ndarray] = None,
                 return_adjoint: bool = False):
        """dJ/deps per component [3][nz][ny][nx] for an objective whose
        cotangents w.r.t. the monitors are ``cot``, after n_steps from u0.
        Tensor media: [6][nz][ny][nx], dJ/deps for the stored entries xx yy zz
        xy xz yz of the node tensors, an off-diagonal entry being one
        parameter for both of its matrix entries.

        Forward states are regenerated by recursive bisection: to reverse
        steps [lo, hi) from u^lo, advance a copy to the midpoint, reverse the
        upper half, then the lower half from u^lo."""
        u_start = np.zeros_like(self.u) if u0 is None else u0.copy()
        a = np.zeros_like(self.u)
        g = np.zeros((6 if self.tensor else 3, self.N))
        self._add_seeds(a, n_steps, cot)
        # one state buffer per recursion depth, reused: a fresh copy per
        # bisection would page in a whole new state every time
        bufs: List[np.ndarray] = []

        def buffer(depth: int) -> np.ndarray:
            while len(bufs) <= depth:
                bufs.append(np.zeros_like(self.u))
            return bufs[depth]

        def reverse(lo: int, hi: int, ulo: np.ndarray, depth: int):
            if hi - lo == 1:
                self.adjoint_step_state(a, ulo, g)
                self._add_seeds(a, lo, cot)
                return
            mid = (lo + hi) // 2
            um = buffer(depth)
            np.copyto(um, ulo)
            for t in range(lo, mid):
                self.step_state(um, t)
            reverse(mid, hi, um, depth + 1)
            # um is no longer needed: the lower half may reuse its buffer
            reverse(lo, mid, ulo, depth)

        if n_steps > 0:
            reverse(0, n_steps, u_start, 0)
        if self.tensor:
            g = self._tensor_eps_gradient(g)
        g = g.reshape((len(g),) + self.shape3)
        return (g, a) if return_adjoint else g

    def _tensor_eps_gradient(self, gp: np.ndarray) -> np.ndarray:
        """From dJ/dp of the stored entries of A = eps^-1 to those of eps.
        As symmetric matrices under <X, Y> = tr(XY), the gradient of A is G
        with G_aa = dJ/dp_aa and G_ab = dJ/dp_ab / 2; dA = -A deps A gives
        the gradient of eps Q = -A G A, whose stored entries are Q_aa and
        2 Q_ab."""
        N = self.N
        G = np.zeros((N, 3, 3))
        A = np.zeros((N, 3, 3))
        for q, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
            w = 1.0 if a == b else 0.5
            G[:, a, b] = G[:, b, a] = w * gp[q]
            A[:, a, b] = A[:, b, a] = self.einvT[q].reshape(-1)
        Q = -np.matmul(np.matmul(A, G), A)
        return np.stack([(1.0 if a == b else 2.0) * Q[:, a, b]
                         for (a, b) in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])


def run_forward(spec, n_steps: Optional[int] = None) -> OracleSim:
    sim = OracleSim(spec)
    sim.step(spec.n_steps if n_steps is None else n_steps)
    return sim
