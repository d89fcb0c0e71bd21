"""Thin ctypes binding of libfdtd (include/fdtd.h): same names, argument
marshalling only.  Every step of the hot path runs in the HIP library; if the
library is missing or fails to load this module raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

FDTD_OK, FDTD_E_INVALID, FDTD_E_UNSTABLE, FDTD_E_NOMEM, FDTD_E_DEVICE, FDTD_E_STATE, FDTD_E_RANGE = \
    0, -1, -2, -3, -4, -5, -6
FDTD_F32, FDTD_F64, FDTD_BF16 = 0, 1, 2
FDTD_EPS_ISO, FDTD_EPS_DIAG, FDTD_EPS_TENSOR = 0, 1, 2
FDTD_SRC_POINT, FDTD_SRC_PLANE_Z = 0, 1
FDTD_MON_PROBE, FDTD_MON_FLUX_Z, FDTD_MON_PATCH_Z = 0, 1, 2
FDTD_ADJ = 6
FDTD_RECORD, FDTD_REPLAY = 1, 2
FDTD_MON_GET, FDTD_MON_FLUX, FDTD_MON_SET_COTANGENT, FDTD_MON_RESET = 0, 1, 2, 3
FDTD_KERNEL_AUTO, FDTD_KERNEL_SPLIT, FDTD_KERNEL_FUSED, FDTD_KERNEL_ONEPASS = 0, 1, 2, 3
FDTD_MAX_SOURCES, FDTD_MAX_MONITORS = 4, 8

ERROR_NAMES = {0: "FDTD_OK", -1: "FDTD_E_INVALID", -2: "FDTD_E_UNSTABLE", -3: "FDTD_E_NOMEM",
               -4: "FDTD_E_DEVICE", -5: "FDTD_E_STATE", -6: "FDTD_E_RANGE"}

EXPORTED = ["fdtd_create", "fdtd_destroy", "fdtd_step_forward", "fdtd_adjoint_begin", "fdtd_step_adjoint",
            "fdtd_step_reverse",
            "fdtd_checkpoint_save", "fdtd_checkpoint_restore", "fdtd_monitor_dft", "fdtd_get_field",
            "fdtd_set_field", "fdtd_get_grad", "fdtd_set_eps", "fdtd_reset", "fdtd_get_step", "fdtd_field_energy",
            "fdtd_probe_trace",
            "fdtd_get_memory", "fdtd_kernel_timing", "fdtd_copy_probe", "fdtd_checkpoint_corrupt",
            "fdtd_flux_reduce", "fdtd_flux_reduce_noalloc", "fdtd_last_error",
            "fdtd_stream_create", "fdtd_stream_destroy", "fdtd_stream_step", "fdtd_stream_get_field",
            "fdtd_stream_monitor", "fdtd_stream_reset", "fdtd_stream_get_info", "fdtd_stream_last_error",
            "fdtd_stream_set_cotangent", "fdtd_stream_reverse", "fdtd_stream_get_grad"]

FDTD_FLUX_POINTS_PER_BLOCK, FDTD_FLUX_MAX_BLOCKS = 4096, 256
FDTD_FLUX_SCRATCH_BYTES = 65536


def flux_workspace_bytes(n_freq: int, n_pts: int) -> int:
    """FDTD_FLUX_WORKSPACE_BYTES of the header."""
    nb = min(FDTD_FLUX_MAX_BLOCKS, max(1, -(-n_pts // FDTD_FLUX_POINTS_PER_BLOCK)))
    return n_freq * nb * 8


class FdtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


FDTD_MAX_POLES = 16
FDTD_POLE_LORENTZ, FDTD_POLE_DRUDE = 0, 1


class PoleDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("delta_eps", C.c_double), ("omega_dt", C.c_double),
                ("gamma_dt", C.c_double)]


class LorentzDesc(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3), ("n_poles", C.c_int32),
                ("poles", PoleDesc * FDTD_MAX_POLES)]


class SourceDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("comp", C.c_int32), ("pos", C.c_int32 * 3),
                ("waveform", C.POINTER(C.c_double)), ("n_waveform", C.c_int32)]


class MonitorDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("comp", C.c_int32), ("pos", C.c_int32 * 3), ("rect", C.c_int32 * 4),
                ("omega_dt", C.POINTER(C.c_double)), ("n_freq", C.c_int32)]


class DomainDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("courant", C.c_double), ("pml", C.c_int32 * 6),
                ("pml_m", C.c_double), ("pml_kappa_max", C.c_double), ("pml_sigma_max", C.c_double),
                ("pml_alpha_max", C.c_double), ("eps_kind", C.c_int32), ("eps_lo", C.c_int32 * 3),
                ("eps_hi", C.c_int32 * 3), ("eps", C.POINTER(C.c_double)), ("eps_bg", C.c_double),
                ("n_lorentz", C.c_int32), ("lorentz", LorentzDesc), ("n_sources", C.c_int32),
                ("sources", SourceDesc * FDTD_MAX_SOURCES), ("n_monitors", C.c_int32),
                ("monitors", MonitorDesc * FDTD_MAX_MONITORS), ("grad", C.c_int32),
                ("grad_lo", C.c_int32 * 3), ("grad_hi", C.c_int32 * 3),
                ("periodic", C.c_int32 * 3), ("bloch_sign", C.c_int32 * 3)]


class Options(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("n_ckpt", C.c_int32), ("ckpt_storage", C.c_int32),
                ("ckpt_checksum", C.c_int32), ("max_steps", C.c_int32), ("kernel", C.c_int32),
                ("dft_block", C.c_int32), ("graph_chunk", C.c_int32), ("tile_rows", C.c_int32),
                ("tile_kz", C.c_int32), ("stream", C.c_void_p),
                ("mem_budget_bytes", C.c_double), ("reversible", C.c_int32),
                ("alloc", C.c_void_p), ("release", C.c_void_p), ("alloc_ctx", C.c_void_p)]


# the optional pool allocator of fdtd_options
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def torch_allocator(device: int = 0):
    """(alloc, release) callbacks that take the pool from torch's caching
    allocator on `device` (so torch.cuda.memory_allocated counts it).  Keep
    the returned pair alive as long as the handle."""
    import torch

    def alloc(ctx, nbytes):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:
            return None

    def release(ctx, p):
        torch.cuda.caching_allocator_delete(p)

    return ALLOC_FN(alloc), RELEASE_FN(release)


class StreamOptions(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("slab_planes", C.c_int32), ("steps_per_pass", C.c_int32),
                ("max_steps", C.c_int32), ("tile_rows", C.c_int32), ("tile_kz", C.c_int32),
                ("stream", C.c_void_p), ("mem_budget_bytes", C.c_double), ("host_budget_bytes", C.c_double),
                ("overlap", C.c_int32), ("local_slots", C.c_int32), ("host_banks", C.c_int32)]


class StreamInfo(C.Structure):
    _fields_ = [("n_slabs", C.c_int32), ("halo", C.c_int32), ("max_extent", C.c_int32), ("step", C.c_int32),
                ("device_bytes", C.c_double), ("host_bytes", C.c_double), ("resident_bytes", C.c_double),
                ("materials_resident", C.c_int32), ("replay_passes", C.c_int32)]


_lib = None


def lib():
    """Load libfdtd.so from the package directory (built by build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libfdtd.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname as the system
        # one libfdtd links against; whichever loads first serves the process.
        # Load torch's first, so that torch's device memory and streams and
        # this library share one runtime whatever the import order.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_size_t
        L.fdtd_create.argtypes = [C.POINTER(DomainDesc), i32, C.POINTER(Options), C.POINTER(vp)]
        L.fdtd_destroy.argtypes = [vp]
        L.fdtd_step_forward.argtypes = [vp, i32, u32]
        L.fdtd_adjoint_begin.argtypes = [vp, i32]
        L.fdtd_step_adjoint.argtypes = [vp, i32]
        L.fdtd_step_reverse.argtypes = [vp, i32]
        L.fdtd_checkpoint_save.argtypes = [vp, i32]
        L.fdtd_checkpoint_restore.argtypes = [vp, i32]
        L.fdtd_monitor_dft.argtypes = [vp, i32, i32, i32, vp, sz]
        L.fdtd_get_field.argtypes = [vp, i32, i32, vp, sz]
        L.fdtd_set_field.argtypes = [vp, i32, i32, vp, sz]
        L.fdtd_get_grad.argtypes = [vp, i32, vp, sz]
        L.fdtd_set_eps.argtypes = [vp, i32, vp, sz]
        L.fdtd_reset.argtypes = [vp]
        L.fdtd_get_step.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.fdtd_get_memory.argtypes = [vp, C.POINTER(C.c_double)]
        L.fdtd_field_energy.argtypes = [vp, i32, C.POINTER(C.c_double)]
        L.fdtd_probe_trace.argtypes = [vp, i32, i32, vp, i32]
        L.fdtd_kernel_timing.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.fdtd_checkpoint_corrupt.argtypes = [vp, i32, sz, u32]
        L.fdtd_copy_probe.argtypes = [sz, i32, C.POINTER(C.c_double)]
        L.fdtd_flux_reduce.argtypes = [vp, i32, C.c_int64, vp, vp, sz, vp]
        L.fdtd_flux_reduce_noalloc.argtypes = [vp, i32, C.c_int64, vp, vp]
        L.fdtd_last_error.argtypes = [vp]
        L.fdtd_last_error.restype = C.c_char_p
        L.fdtd_stream_create.argtypes = [C.POINTER(DomainDesc), C.POINTER(StreamOptions), C.POINTER(vp)]
        L.fdtd_stream_destroy.argtypes = [vp]
        L.fdtd_stream_step.argtypes = [vp, i32]
        L.fdtd_stream_get_field.argtypes = [vp, i32, vp, sz]
        L.fdtd_stream_monitor.argtypes = [vp, i32, i32, vp, sz]
        L.fdtd_stream_reset.argtypes = [vp]
        L.fdtd_stream_get_info.argtypes = [vp, C.POINTER(StreamInfo)]
        L.fdtd_stream_set_cotangent.argtypes = [vp, i32, vp, sz]
        L.fdtd_stream_reverse.argtypes = [vp]
        L.fdtd_stream_get_grad.argtypes = [vp, vp, sz]
        L.fdtd_stream_last_error.argtypes = [vp]
        L.fdtd_stream_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if not name.endswith("last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _chk(rc: int, h=None):
    if rc != FDTD_OK:
        msg = lib().fdtd_last_error(h)
        raise FdtdError(rc, msg.decode() if msg else "")
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def domain_desc(spec, keep: list) -> DomainDesc:
    """Marshal a workloads.DomainSpec into the C descriptor (arrays kept alive in `keep`)."""
    d = DomainDesc()
    for a in range(3):
        d.n[a] = spec.shape[a]
    for a in range(3):
        d.periodic[a] = int(getattr(spec, "periodic", (0, 0, 0))[a])
        d.bloch_sign[a] = int(getattr(spec, "bloch_sign", (1, 1, 1))[a])
    d.courant = spec.courant
    for q in range(6):
        d.pml[q] = spec.pml[q]
    d.pml_m, d.pml_kappa_max = spec.pml_m, spec.pml_kappa_max
    d.pml_sigma_max, d.pml_alpha_max = spec.pml_sigma_max, spec.pml_alpha_max
    d.eps_kind = {"iso": FDTD_EPS_ISO, "diag": FDTD_EPS_DIAG, "tensor": FDTD_EPS_TENSOR}[spec.eps_kind]
    d.eps_bg = spec.eps_bg
    if spec.eps is not None:
        (lo, hi) = spec.eps_box
        e = np.ascontiguousarray(spec.eps, dtype=np.float64)
        keep.append(e)
        for a in range(3):
            d.eps_lo[a], d.eps_hi[a] = lo[a], hi[a]
        d.eps = _dptr(e)
    d.n_lorentz = len(spec.lorentz)
    if spec.lorentz:
        L = spec.lorentz[0]
        for a in range(3):
            d.lorentz.lo[a], d.lorentz.hi[a] = L.lo[a], L.hi[a]
        poles = L.pole_list()
        if len(poles) > FDTD_MAX_POLES:
            raise ValueError(f"at most {FDTD_MAX_POLES} poles")
        d.lorentz.n_poles = len(poles)
        for q, pl in enumerate(poles):
            pd = d.lorentz.poles[q]
            pd.kind = {"lorentz": FDTD_POLE_LORENTZ, "drude": FDTD_POLE_DRUDE}[pl.kind]
            pd.delta_eps, pd.omega_dt, pd.gamma_dt = pl.delta_eps, pl.omega_dt, pl.gamma_dt
    d.n_sources = len(spec.sources)
    for q, s in enumerate(spec.sources):
        w = np.ascontiguousarray(s.waveform, dtype=np.float64)
        keep.append(w)
        d.sources[q].kind = FDTD_SRC_POINT if s.kind == "point" else FDTD_SRC_PLANE_Z
        d.sources[q].comp = s.comp
        for a in range(3):
            d.sources[q].pos[a] = s.pos[a]
        d.sources[q].waveform = _dptr(w)
        d.sources[q].n_waveform = len(w)
    d.n_monitors = len(spec.monitors)
    kinds = {"probe": FDTD_MON_PROBE, "flux_z": FDTD_MON_FLUX_Z, "patch_z": FDTD_MON_PATCH_Z}
    for q, m in enumerate(spec.monitors):
        md = d.monitors[q]
        md.kind = kinds[m.kind]
        md.comp = m.comp
        for a in range(3):
            md.pos[a] = m.pos[a]
        for a in range(4):
            md.rect[a] = m.rect[a]
        om = np.ascontiguousarray(m.omega_dt, dtype=np.float64)
        keep.append(om)
        md.omega_dt = _dptr(om) if len(om) else None
        md.n_freq = len(om)
    if spec.grad_box is not None:
        d.grad = 1
        lo, hi = spec.grad_box
        for a in range(3):
            d.grad_lo[a], d.grad_hi[a] = lo[a], hi[a]
    return d


# ---------------------------------------------------------------- C-ABI names
def fdtd_create(specs: Sequence, dtype: int = FDTD_F32, n_ckpt: int = 0, ckpt_storage: Optional[int] = None,
                ckpt_checksum: bool = False, max_steps: int = 0, kernel: int = FDTD_KERNEL_AUTO,
                dft_block: int = 0, graph_chunk: int = 0, stream: Optional[int] = None,
                mem_budget_bytes: float = 0.0, tile_rows: int = 0, tile_kz: int = 0, reversible: bool = False,
                allocator=None):
    """allocator: None (hipMalloc) or an (alloc, release) pair of ctypes
    callbacks (torch_allocator()) that the caller keeps alive."""
    keep: list = []
    arr = (DomainDesc * len(specs))()
    for q, s in enumerate(specs):
        arr[q] = domain_desc(s, keep)
    o = Options()
    o.dtype = dtype
    o.n_ckpt = n_ckpt
    o.ckpt_storage = dtype if ckpt_storage is None else ckpt_storage
    o.ckpt_checksum = int(bool(ckpt_checksum))
    o.max_steps = max_steps
    o.reversible = int(bool(reversible))
    o.kernel = kernel
    o.dft_block = dft_block
    o.graph_chunk = graph_chunk
    o.tile_rows = tile_rows
    o.tile_kz = tile_kz
    o.stream = stream
    o.mem_budget_bytes = mem_budget_bytes
    if allocator is not None:
        o.alloc = C.cast(allocator[0], C.c_void_p)
        o.release = C.cast(allocator[1], C.c_void_p)
    h = C.c_void_p()
    _chk(lib().fdtd_create(arr, len(specs), C.byref(o), C.byref(h)))
    return h


def fdtd_destroy(h):
    return _chk(lib().fdtd_destroy(h), None)


def fdtd_step_forward(h, n_steps: int, flags: int = FDTD_RECORD):
    return _chk(lib().fdtd_step_forward(h, n_steps, flags), h)


def fdtd_adjoint_begin(h, n_total: int):
    return _chk(lib().fdtd_adjoint_begin(h, n_total), h)


def fdtd_step_adjoint(h, n_steps: int = 1):
    return _chk(lib().fdtd_step_adjoint(h, n_steps), h)


def fdtd_step_reverse(h, n_steps: int = 1):
    return _chk(lib().fdtd_step_reverse(h, n_steps), h)


def fdtd_checkpoint_save(h, slot: int):
    return _chk(lib().fdtd_checkpoint_save(h, slot), h)


def fdtd_checkpoint_restore(h, slot: int):
    return _chk(lib().fdtd_checkpoint_restore(h, slot), h)


def fdtd_monitor_dft(h, domain: int, monitor: int, op: int, buf: Optional[np.ndarray]):
    ptr = None if buf is None else buf.ctypes.data
    nbytes = 0 if buf is None else buf.nbytes
    return _chk(lib().fdtd_monitor_dft(h, domain, monitor, op, ptr, nbytes), h)


def fdtd_get_field(h, domain: int, comp: int, out: np.ndarray):
    return _chk(lib().fdtd_get_field(h, domain, comp, out.ctypes.data, out.nbytes), h)


def fdtd_set_field(h, domain: int, comp: int, src: np.ndarray):
    src = np.ascontiguousarray(src)
    return _chk(lib().fdtd_set_field(h, domain, comp, src.ctypes.data, src.nbytes), h)


def fdtd_get_grad(h, domain: int, out: np.ndarray):
    return _chk(lib().fdtd_get_grad(h, domain, out.ctypes.data, out.nbytes), h)


def fdtd_set_eps(h, domain: int, eps: np.ndarray):
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    return _chk(lib().fdtd_set_eps(h, domain, eps.ctypes.data, eps.nbytes), h)


def fdtd_reset(h):
    return _chk(lib().fdtd_reset(h), h)


def fdtd_get_step(h):
    n, m = C.c_int32(), C.c_int32()
    _chk(lib().fdtd_get_step(h, C.byref(n), C.byref(m)), h)
    return n.value, m.value


def fdtd_get_memory(h) -> float:
    b = C.c_double()
    _chk(lib().fdtd_get_memory(h, C.byref(b)), h)
    return b.value


def fdtd_kernel_timing(h, op: int):
    ms, n = C.c_double(), C.c_int64()
    _chk(lib().fdtd_kernel_timing(h, op, C.byref(ms), C.byref(n)), h)
    return ms.value, n.value


def fdtd_copy_probe(nbytes: int, reps: int) -> float:
    ms = C.c_double()
    _chk(lib().fdtd_copy_probe(nbytes, reps, C.byref(ms)), None)
    return ms.value


def fdtd_flux_reduce(spectra_ptr: int, n_freq: int, n_pts: int, flux_ptr: int, workspace_ptr=None,
                     workspace_bytes: int = 0, stream=None):
    """Device pointers in, device pointer out (see include/fdtd.h)."""
    return _chk(lib().fdtd_flux_reduce(spectra_ptr, n_freq, n_pts, flux_ptr, workspace_ptr, workspace_bytes,
                                       stream), None)


def fdtd_flux_reduce_noalloc(spectra_ptr: int, n_freq: int, n_pts: int, flux_ptr: int, stream=None):
    """fdtd_flux_reduce with the library's fixed device scratch (no allocation)."""
    return _chk(lib().fdtd_flux_reduce_noalloc(spectra_ptr, n_freq, n_pts, flux_ptr, stream), None)


def fdtd_checkpoint_corrupt(h, slot: int, word: int, value: int):
    return _chk(lib().fdtd_checkpoint_corrupt(h, slot, word, value), h)


def fdtd_last_error(h=None) -> str:
    s = lib().fdtd_last_error(h)
    return s.decode() if s else ""


# ---------------------------------------------------------------- streamed slabs
def _schk(rc: int, h=None):
    if rc != FDTD_OK:
        msg = lib().fdtd_stream_last_error(h)
        raise FdtdError(rc, msg.decode() if msg else "")
    return rc


def fdtd_stream_create(spec, dtype: int, slab_planes: int, steps_per_pass: int, max_steps: int = 0,
                       tile_rows: int = 0, tile_kz: int = 0, stream: Optional[int] = None,
                       mem_budget_bytes: float = 0.0, host_budget_bytes: float = 0.0, overlap: bool = True,
                       local_slots: int = 0, host_banks: int = 0):
    keep: list = []
    d = domain_desc(spec, keep)
    o = StreamOptions()
    o.dtype, o.slab_planes, o.steps_per_pass, o.max_steps = dtype, slab_planes, steps_per_pass, max_steps
    o.tile_rows, o.tile_kz = tile_rows, tile_kz
    o.stream = stream
    o.mem_budget_bytes, o.host_budget_bytes = mem_budget_bytes, host_budget_bytes
    o.overlap = 1 if overlap else 0
    o.local_slots = local_slots
    o.host_banks = host_banks
    h = C.c_void_p()
    _schk(lib().fdtd_stream_create(C.byref(d), C.byref(o), C.byref(h)), None)
    return h


def fdtd_stream_destroy(h):
    return _schk(lib().fdtd_stream_destroy(h), None)


def fdtd_stream_step(h, n_steps: int):
    return _schk(lib().fdtd_stream_step(h, n_steps), h)


def fdtd_stream_get_field(h, comp: int, out: np.ndarray):
    return _schk(lib().fdtd_stream_get_field(h, comp, out.ctypes.data, out.nbytes), h)


def fdtd_stream_monitor(h, monitor: int, op: int, out: np.ndarray):
    return _schk(lib().fdtd_stream_monitor(h, monitor, op, out.ctypes.data, out.nbytes), h)


def fdtd_stream_reset(h):
    return _schk(lib().fdtd_stream_reset(h), h)


def fdtd_stream_get_info(h) -> dict:
    i = StreamInfo()
    _schk(lib().fdtd_stream_get_info(h, C.byref(i)), h)
    return {k: getattr(i, k) for k, _ in StreamInfo._fields_}


def fdtd_stream_set_cotangent(h, monitor: int, buf: np.ndarray):
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    return _schk(lib().fdtd_stream_set_cotangent(h, monitor, buf.ctypes.data, buf.nbytes), h)


def fdtd_stream_reverse(h):
    return _schk(lib().fdtd_stream_reverse(h), h)


def fdtd_stream_get_grad(h, out: np.ndarray):
    return _schk(lib().fdtd_stream_get_grad(h, out.ctypes.data, out.nbytes), h)


def fdtd_field_energy(h, domain: int) -> float:
    e = C.c_double()
    _chk(lib().fdtd_field_energy(h, domain, C.byref(e)), h)
    return e.value


def fdtd_probe_trace(h, domain: int, probe: int, n: int) -> np.ndarray:
    out = np.zeros(max(n, 1))
    _chk(lib().fdtd_probe_trace(h, domain, probe, out.ctypes.data, n), h)
    return out[:n]
