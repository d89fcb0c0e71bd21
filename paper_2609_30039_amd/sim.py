"""Convenience layer over the C-ABI handle: numpy in, numpy out."""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import binding as B


class Simulation:
    """Owns one libfdtd handle advancing ``specs`` (one or more domains)."""

    def __init__(self, specs, dtype: str = "f32", n_ckpt: int = 0, ckpt_storage: Optional[str] = None,
                 ckpt_checksum: bool = False, max_steps: Optional[int] = None, kernel: str = "auto",
                 dft_block: int = 0, graph_chunk: int = 0, stream: Optional[int] = None,
                 mem_budget_bytes: float = 0.0, tile_rows: int = 0, tile_kz: int = 0, reversible: bool = False,
                 torch_pool: bool = False):
        if not isinstance(specs, (list, tuple)):
            specs = [specs]
        self.specs = list(specs)
        self.dtype = np.float32 if dtype == "f32" else np.float64
        dt = B.FDTD_F32 if dtype == "f32" else B.FDTD_F64
        storage = {None: dt, "f32": B.FDTD_F32, "f64": B.FDTD_F64, "bf16": B.FDTD_BF16}[ckpt_storage]
        kern = {"auto": B.FDTD_KERNEL_AUTO, "split": B.FDTD_KERNEL_SPLIT, "fused": B.FDTD_KERNEL_FUSED,
                "onepass": B.FDTD_KERNEL_ONEPASS}[kernel]
        if max_steps is None:
            max_steps = max(max(s.n_steps for s in self.specs), 1)
        self.max_steps = max_steps
        # bumped by every reset and permittivity upload: a recorded forward
        # sweep is valid for a backward pass only while it is unchanged
        self.generation = 0
        # torch_pool: the device pool comes from torch's caching allocator
        self._alloc = B.torch_allocator() if torch_pool else None
        self.h = B.fdtd_create(self.specs, dt, n_ckpt, storage, ckpt_checksum, max_steps, kern, dft_block,
                               graph_chunk, stream, mem_budget_bytes, tile_rows, tile_kz, reversible, self._alloc)

    def close(self):
        if self.h is not None:
            B.fdtd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------- stepping ----------------
    def step(self, n: int = 1, record: bool = True):
        B.fdtd_step_forward(self.h, n, B.FDTD_RECORD if record else B.FDTD_REPLAY)

    def adjoint_begin(self, n_total: int):
        B.fdtd_adjoint_begin(self.h, n_total)

    def step_adjoint(self, n: int = 1):
        B.fdtd_step_adjoint(self.h, n)

    def step_reverse(self, n: int = 1):
        """Reversible mode: n backward steps of the lossless box (the forward
        state there goes from u^m to u^{m-n})."""
        B.fdtd_step_reverse(self.h, n)

    def save(self, slot: int):
        B.fdtd_checkpoint_save(self.h, slot)

    def restore(self, slot: int):
        B.fdtd_checkpoint_restore(self.h, slot)

    def reset(self):
        self.generation += 1
        B.fdtd_reset(self.h)

    @property
    def steps(self):
        return B.fdtd_get_step(self.h)

    # ---------------- data ----------------
    def field(self, comp: int, domain: int = 0, adjoint: bool = False) -> np.ndarray:
        nx, ny, nz = self.specs[domain].shape
        out = np.empty((nz, ny, nx), dtype=self.dtype)
        B.fdtd_get_field(self.h, domain, comp + (B.FDTD_ADJ if adjoint else 0), out)
        return out

    def set_field(self, comp: int, values: np.ndarray, domain: int = 0, adjoint: bool = False):
        B.fdtd_set_field(self.h, domain, comp + (B.FDTD_ADJ if adjoint else 0),
                         np.ascontiguousarray(values, dtype=self.dtype))

    def _mon_shape(self, domain: int, monitor: int):
        m = self.specs[domain].monitors[monitor]
        i0, i1, j0, j1 = m.rect
        nc = 4 if m.kind == "flux_z" else 1
        return (len(m.omega_dt), nc, j1 - j0, i1 - i0)

    def spectra(self, monitor: int, domain: int = 0) -> np.ndarray:
        m = self.specs[domain].monitors[monitor]
        if m.kind == "probe":
            out = np.zeros(self.max_steps)
            B.fdtd_monitor_dft(self.h, domain, monitor, B.FDTD_MON_GET, out)
            return out
        buf = np.zeros(self._mon_shape(domain, monitor) + (2,))
        B.fdtd_monitor_dft(self.h, domain, monitor, B.FDTD_MON_GET, buf)
        return buf[..., 0] + 1j * buf[..., 1]

    def probe(self, monitor: int, domain: int = 0, n: Optional[int] = None) -> np.ndarray:
        tr = self.spectra(monitor, domain)
        return tr if n is None else tr[:n]

    def flux(self, monitor: int, domain: int = 0) -> np.ndarray:
        nf = len(self.specs[domain].monitors[monitor].omega_dt)
        out = np.zeros(nf)
        B.fdtd_monitor_dft(self.h, domain, monitor, B.FDTD_MON_FLUX, out)
        return out

    def set_cotangent(self, monitor: int, g: np.ndarray, domain: int = 0):
        m = self.specs[domain].monitors[monitor]
        if m.kind == "probe":
            buf = np.zeros(self.max_steps)
            g = np.asarray(g, dtype=np.float64).ravel()
            buf[:len(g)] = g[:self.max_steps]
        else:
            g = np.asarray(g, dtype=np.complex128).reshape(self._mon_shape(domain, monitor))
            buf = np.ascontiguousarray(np.stack([g.real, g.imag], axis=-1))
        B.fdtd_monitor_dft(self.h, domain, monitor, B.FDTD_MON_SET_COTANGENT, buf)

    def reset_monitor(self, monitor: int, domain: int = 0):
        B.fdtd_monitor_dft(self.h, domain, monitor, B.FDTD_MON_RESET, None)

    def grad(self, domain: int = 0) -> np.ndarray:
        s = self.specs[domain]
        lo, hi = s.grad_box
        nc = {"diag": 3, "tensor": 6}.get(s.eps_kind, 1)
        out = np.zeros((nc, hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]))
        B.fdtd_get_grad(self.h, domain, out)
        return out

    def set_eps(self, eps: np.ndarray, domain: int = 0):
        self.generation += 1
        B.fdtd_set_eps(self.h, domain, eps)

    def timing(self, op: int):
        """1: enable and clear, 0: disable, 2: (total kernel ms, launches)."""
        return B.fdtd_kernel_timing(self.h, op)

    def memory_bytes(self) -> float:
        return B.fdtd_get_memory(self.h)

    def field_energy(self, domain: int = 0) -> float:
        """Sum of squares of the six fields (the watchdog: raises FdtdError
        with FDTD_E_UNSTABLE when the state holds a NaN or an infinity)."""
        return B.fdtd_field_energy(self.h, domain)


class StreamedSimulation:
    """One domain advanced by host-streamed causal slabs (the libfdtd
    fdtd_stream_* calls): its state in pinned host banks, slabs of at most
    ``slab_planes`` z planes stepped ``steps_per_pass`` steps per visit in a
    device workspace."""

    def __init__(self, spec, slab_planes: int, steps_per_pass: int, dtype: str = "f32",
                 max_steps: Optional[int] = None, tile_rows: int = 0, tile_kz: int = 0,
                 stream: Optional[int] = None, mem_budget_bytes: float = 0.0, host_budget_bytes: float = 0.0,
                 overlap: bool = True, local_slots: int = 0, host_banks: int = 0):
        self.spec = spec
        self.dtype = np.float32 if dtype == "f32" else np.float64
        self.max_steps = max(spec.n_steps, 1) if max_steps is None else max_steps
        self.h = B.fdtd_stream_create(spec, B.FDTD_F32 if dtype == "f32" else B.FDTD_F64, slab_planes,
                                      steps_per_pass, self.max_steps, tile_rows, tile_kz, stream,
                                      mem_budget_bytes, host_budget_bytes, overlap, local_slots, host_banks)

    def close(self):
        if self.h is not None:
            B.fdtd_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        B.fdtd_stream_step(self.h, n)

    def reset(self):
        B.fdtd_stream_reset(self.h)

    def info(self) -> dict:
        return B.fdtd_stream_get_info(self.h)

    def field(self, comp: int) -> np.ndarray:
        nx, ny, nz = self.spec.shape
        out = np.empty((nz, ny, nx), dtype=self.dtype)
        B.fdtd_stream_get_field(self.h, comp, out)
        return out

    def spectra(self, monitor: int) -> np.ndarray:
        m = self.spec.monitors[monitor]
        if m.kind == "probe":
            out = np.zeros(self.max_steps)
            B.fdtd_stream_monitor(self.h, monitor, B.FDTD_MON_GET, out)
            return out
        i0, i1, j0, j1 = m.rect
        buf = np.zeros((len(m.omega_dt), 4 if m.kind == "flux_z" else 1, j1 - j0, i1 - i0, 2))
        B.fdtd_stream_monitor(self.h, monitor, B.FDTD_MON_GET, buf)
        return buf[..., 0] + 1j * buf[..., 1]

    def flux(self, monitor: int) -> np.ndarray:
        out = np.zeros(len(self.spec.monitors[monitor].omega_dt))
        B.fdtd_stream_monitor(self.h, monitor, B.FDTD_MON_FLUX, out)
        return out

    def set_cotangent(self, monitor: int, g: np.ndarray):
        m = self.spec.monitors[monitor]
        if m.kind == "probe":
            buf = np.zeros(self.max_steps)
            g = np.asarray(g, dtype=np.float64).ravel()
            buf[:len(g)] = g[:self.max_steps]
        else:
            i0, i1, j0, j1 = m.rect
            shape = (len(m.omega_dt), 4 if m.kind == "flux_z" else 1, j1 - j0, i1 - i0)
            g = np.asarray(g, dtype=np.complex128).reshape(shape)
            buf = np.ascontiguousarray(np.stack([g.real, g.imag], axis=-1))
        B.fdtd_stream_set_cotangent(self.h, monitor, buf)

    def reverse(self):
        """The reverse sweep over the forward steps done since the reset."""
        B.fdtd_stream_reverse(self.h)

    def grad(self) -> np.ndarray:
        s = self.spec
        lo, hi = s.grad_box
        nc = {"diag": 3, "tensor": 6}.get(s.eps_kind, 1)
        out = np.zeros((nc, hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]))
        B.fdtd_stream_get_grad(self.h, out)
        return out
