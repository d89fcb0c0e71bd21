"""The C-ABI library loads, exports every entry point of include/fdtd.h, and
refuses bad descriptors on the host before touching the device."""
import os
import re

import numpy as np
import pytest

from paper_2609_30039_amd import binding as B
from paper_2609_30039_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "fdtd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtd_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = B.lib()
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTED)


def _spec(**kw):
    s = W.pec_cavity(8, 10)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _refused(spec, code, **kw):
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([spec], B.FDTD_F32, mem_budget_bytes=1e12, **kw)
    assert e.value.code == code, str(e.value)


def test_cfl_bound_refused():
    _refused(_spec(courant=0.995 / np.sqrt(3.0)), B.FDTD_E_UNSTABLE)


def test_nonpositive_eps_refused():
    s = _spec()
    s.eps = s.eps.copy()
    s.eps[0, 1, 2, 3] = -1.0
    _refused(s, B.FDTD_E_UNSTABLE)
    s.eps[0, 1, 2, 3] = np.nan
    _refused(s, B.FDTD_E_UNSTABLE)


def test_eps_below_one_refused():
    """Eq. 2's step bound is the vacuum one: a permittivity below 1 in the
    box or in the background is refused (the oracle's one-step operator grows
    at 0.9), and 1 itself passes validation (then the tiny budget refuses)."""
    s = _spec()
    s.eps = s.eps.copy()
    s.eps[0, 1, 2, 3] = 0.99
    _refused(s, B.FDTD_E_UNSTABLE)
    _refused(_spec(eps_bg=0.5), B.FDTD_E_UNSTABLE)
    s.eps[0, 1, 2, 3] = 1.0
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([s], B.FDTD_F32, mem_budget_bytes=1.0)
    assert e.value.code == B.FDTD_E_NOMEM


def test_lorentz_resonance_bound_refused():
    """A Lorentz pole with omega_0 dt >= 2 is refused (its recursion has a
    root outside the unit disc; the oracle's operator grows at 2.01 and keeps
    radius 1 at 1.99); a Drude pole has no such bound."""
    def with_pole(p):
        return _spec(lorentz=[W.LorentzSpec((2, 2, 2), (5, 5, 5), 0.0, 0.0, 0.0, poles=[p])])
    _refused(with_pole(W.PoleSpec("lorentz", 1.0, 2.0, 0.05)), B.FDTD_E_UNSTABLE)
    _refused(with_pole(W.PoleSpec("lorentz", 1.0, 3.0, 0.0)), B.FDTD_E_UNSTABLE)
    for p in (W.PoleSpec("lorentz", 1.0, 1.99, 0.0), W.PoleSpec("drude", 0.0, 3.0, 0.05)):
        with pytest.raises(B.FdtdError) as e:
            B.fdtd_create([with_pole(p)], B.FDTD_F32, mem_budget_bytes=1.0)
        assert e.value.code == B.FDTD_E_NOMEM


def test_tensor_rule_in_absorbing_face():
    """Diagonal eps inside an absorbing face whose normal eigenvalue is the
    intermediate one is refused (Section 2.3); a non-intermediate one passes
    validation (and is then refused only by the tiny memory budget)."""
    n = 10
    eps = np.ones((3, n, n, n))
    eps[0, 5, 5, 0] = 2.0      # eps_xx = 2 at x = 0 (x face), eps_yy = 1, eps_zz = 3 -> intermediate
    eps[2, 5, 5, 0] = 3.0
    s = W.DomainSpec(shape=(n, n, n), courant=W.courant_3d(), pml=(3, 3, 0, 0, 0, 0), eps_kind="diag",
                     eps_box=((0, 0, 0), (n, n, n)), eps=eps)
    _refused(s, B.FDTD_E_UNSTABLE)
    eps[0, 5, 5, 0] = 4.0      # largest eigenvalue along the normal: admitted
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([s], B.FDTD_F32, mem_budget_bytes=1.0)
    assert e.value.code == B.FDTD_E_NOMEM


def test_memory_budget_refused_before_allocation():
    _refused_small = _spec()
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([_refused_small], B.FDTD_F32, mem_budget_bytes=1024.0)
    assert e.value.code == B.FDTD_E_NOMEM
    assert "budget" in str(e.value)


def test_bad_positions_refused():
    s = _spec()
    s.sources[0].pos = (8, 1, 1)
    _refused(s, B.FDTD_E_RANGE)
    s = _spec()
    s.monitors[0].comp = 7
    _refused(s, B.FDTD_E_RANGE)
    s = _spec()
    s.monitors.append(W.MonitorSpec("flux_z", pos=(0, 0, 3), rect=(0, 9, 0, 8), omega_dt=np.array([0.1])))
    _refused(s, B.FDTD_E_RANGE)
    s = _spec(pml=(5, 5, 0, 0, 0, 0))
    _refused(s, B.FDTD_E_INVALID)


def test_bf16_needs_fp32():
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([_spec()], B.FDTD_F64, ckpt_storage=B.FDTD_BF16, mem_budget_bytes=1e12)
    assert e.value.code == B.FDTD_E_INVALID


def test_launch_shape_options_checked():
    """Split blocks take 4 or 8 rows, fused tiles 2, 4 or 8 rows per wave;
    captured chunks hold at most 64 steps."""
    _refused(_spec(), B.FDTD_E_INVALID, kernel=B.FDTD_KERNEL_SPLIT, tile_rows=2)
    _refused(_spec(), B.FDTD_E_INVALID, kernel=B.FDTD_KERNEL_FUSED, tile_rows=3)
    _refused(_spec(), B.FDTD_E_INVALID, graph_chunk=65)
    _refused(_spec(), B.FDTD_E_INVALID, tile_kz=-1)


def test_pole_descriptors_checked():
    """1 to 16 poles of a known kind, omega > 0, gamma >= 0, Lorentz delta_eps >= 0."""
    def with_poles(poles):
        return _spec(lorentz=[W.LorentzSpec((2, 2, 2), (5, 5, 5), 0.0, 0.0, 0.0, poles=poles)])
    ok = W.PoleSpec("lorentz", 1.0, 0.3, 0.05)
    with pytest.raises(ValueError):
        B.fdtd_create([with_poles([ok] * 17)], B.FDTD_F32, mem_budget_bytes=1e12)
    _refused(with_poles([W.PoleSpec("drude", 0.0, 0.0, 0.05)]), B.FDTD_E_UNSTABLE)
    _refused(with_poles([ok, W.PoleSpec("lorentz", -1.0, 0.3, 0.05)]), B.FDTD_E_UNSTABLE)
    _refused(with_poles([W.PoleSpec("lorentz", 1.0, 0.3, -0.1)]), B.FDTD_E_UNSTABLE)


    class NoPoles(W.LorentzSpec):
        def pole_list(self):
            return []

    _refused(_spec(lorentz=[NoPoles((2, 2, 2), (5, 5, 5), 0.0, 0.0, 0.0)]), B.FDTD_E_INVALID)


def test_reversible_mode_admissibility():
    """The reversible mode needs a lossless interior around the gradient box
    (Section 3.2): a dispersive box, a gradient box inside an absorbing slab
    or max_steps 0 are refused before any allocation; an admissible domain
    passes validation (then the tiny budget refuses)."""
    spec, _ = W.design_patch(pml=6, design=12, patch=10, n_steps=20, n_f=2, shape=(40, 34, 38))
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([spec], B.FDTD_F32, max_steps=20, reversible=True, mem_budget_bytes=1.0)
    assert e.value.code == B.FDTD_E_NOMEM
    _refused(spec, B.FDTD_E_INVALID, max_steps=0, reversible=True)
    bad, _ = W.design_patch(pml=6, design=12, patch=10, n_steps=20, n_f=2, shape=(40, 34, 38))
    bad.grad_box = ((6, 14, 14), (20, 26, 26))      # touches the low x slab's neighbour row
    _refused(bad, B.FDTD_E_INVALID, max_steps=20, reversible=True)
    lor = W.lorentz_flux(pml=6, lorentz=8, n_steps=20, n_f=2, shape=(40, 30, 36))
    lor.grad_box = ((10, 10, 10), (30, 20, 26))
    _refused(lor, B.FDTD_E_INVALID, max_steps=20, reversible=True)
    from paper_2609_30039_amd import adjoint as A
    assert A.reversible_admissible(spec) and not A.reversible_admissible(bad) and not A.reversible_admissible(lor)


def test_periodic_descriptor_checked():
    """Periodic axes: x and y only, no absorbing cells on them, a Bloch sign of
    +1 or -1, split kernels; a gradient (with a dispersive box too) but not
    the reversible mode; an admissible one passes validation (the tiny budget
    then refuses)."""
    def spec(**kw):
        s = W.DomainSpec(shape=(8, 8, 12), courant=W.courant_3d(), pml=(0, 0, 0, 0, 3, 3), eps_kind="iso",
                         eps_box=((0, 0, 0), (8, 8, 12)), eps=np.ones((1, 12, 8, 8)), periodic=(1, 1, 0))
        for k, v in kw.items():
            setattr(s, k, v)
        return s
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([spec()], B.FDTD_F32, mem_budget_bytes=1.0)
    assert e.value.code == B.FDTD_E_NOMEM
    _refused(spec(periodic=(1, 1, 1)), B.FDTD_E_INVALID)
    _refused(spec(pml=(2, 2, 0, 0, 3, 3)), B.FDTD_E_INVALID)
    _refused(spec(bloch_sign=(2, 1, 1)), B.FDTD_E_INVALID)
    _refused(spec(), B.FDTD_E_INVALID, kernel=B.FDTD_KERNEL_FUSED)
    g = ((2, 2, 4), (6, 6, 8))
    _passes_validation(spec(grad_box=g))
    _passes_validation(spec(grad_box=g, lorentz=[W.LorentzSpec((2, 2, 4), (5, 5, 7), 1.0, 0.3, 0.01)]))
    _refused(spec(grad_box=g), B.FDTD_E_INVALID, reversible=True, max_steps=4)


def _tensor_spec(m_node, n=10, pml=(0, 0, 0, 0, 3, 3), **kw):
    """A tensor domain whose node (5, 5, 1) (inside the low z face) holds m_node."""
    from tests.test_oracle_tensor import uniform_tensor
    eps = uniform_tensor((n, n, n), 2.0 * np.eye(3))
    eps[:, 1, 5, 5] = [m_node[0, 0], m_node[1, 1], m_node[2, 2], m_node[0, 1], m_node[0, 2], m_node[1, 2]]
    s = W.DomainSpec(shape=(n, n, n), courant=W.courant_3d(), pml=pml, eps_kind="tensor",
                     eps_box=((0, 0, 0), (n, n, n)), eps=eps)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _passes_validation(spec, **kw):
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_create([spec], B.FDTD_F32, mem_budget_bytes=1.0, **kw)
    assert e.value.code == B.FDTD_E_NOMEM, str(e.value)


def test_tensor_admission_node_by_node():
    """Section 2.3's rule for tensor media, checked at every node: eigenvalues
    of at least 1; inside an absorbing face the normal is a principal axis
    with the largest or smallest eigenvalue.  The refused cases are those whose
    one-step operator grows in the oracle (tests/test_oracle_tensor.py)."""
    import math
    c, s_ = math.cos(0.6), math.sin(0.6)
    rz = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])
    cx, sx = math.cos(math.pi / 4), math.sin(math.pi / 4)
    rx = np.array([[1.0, 0.0, 0.0], [0.0, cx, -sx], [0.0, sx, cx]])
    # admitted in the z face: normal eigenvalue largest / smallest with the transverse block rotated
    _passes_validation(_tensor_spec(rz @ np.diag([1.5, 4.0, 6.0]) @ rz.T))
    _passes_validation(_tensor_spec(rz @ np.diag([1.5, 4.0, 1.0]) @ rz.T))
    # refused in the face: intermediate normal eigenvalue, axes rotated against the normal
    _refused(_tensor_spec(np.diag([1.0, 4.0, 2.0])), B.FDTD_E_UNSTABLE)
    _refused(_tensor_spec(rx @ np.diag([1.0, 16.0, 1.0]) @ rx.T), B.FDTD_E_UNSTABLE)
    # the same rotated tensor outside every face is admitted
    _passes_validation(_tensor_spec(rx @ np.diag([1.0, 16.0, 1.0]) @ rx.T, pml=(0,) * 6))
    # an eigenvalue below one anywhere, or a non-finite entry
    r = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))[0]
    _refused(_tensor_spec(r @ np.diag([0.95, 2.0, 3.0]) @ r.T, pml=(0,) * 6), B.FDTD_E_UNSTABLE)
    bad = np.diag([2.0, 2.0, np.nan])
    _refused(_tensor_spec(bad, pml=(0,) * 6), B.FDTD_E_UNSTABLE)


def test_tensor_media_combinations_refused():
    """The tensor path is nondispersive and split, and has no reversible
    mode; a gradient over its node tensors is admitted, and so are
    Bloch-periodic x and y axes (with a gradient too)."""
    m = 2.0 * np.eye(3)
    _refused(_tensor_spec(m, lorentz=[W.LorentzSpec((2, 2, 2), (5, 5, 5), 1.0, 0.3, 0.01)]), B.FDTD_E_INVALID)
    _refused(_tensor_spec(m), B.FDTD_E_INVALID, kernel=B.FDTD_KERNEL_FUSED)
    _refused(_tensor_spec(m, grad_box=((2, 2, 4), (6, 6, 8))), B.FDTD_E_INVALID, reversible=1)
    _passes_validation(_tensor_spec(m, grad_box=((2, 2, 4), (6, 6, 8))))
    per = dict(pml=(0, 0, 0, 0, 3, 3), periodic=(1, 1, 0), bloch_sign=(-1, 1, 1))
    _passes_validation(_tensor_spec(m, **per))
    _passes_validation(_tensor_spec(m, grad_box=((0, 0, 4), (8, 8, 8)), **per))
    _refused(_tensor_spec(m, pml=(3, 3, 0, 0, 3, 3), periodic=(1, 0, 0)), B.FDTD_E_INVALID)
    _refused(_tensor_spec(m, **per), B.FDTD_E_INVALID, kernel=B.FDTD_KERNEL_FUSED)


def _stream_refused(spec, code, **kw):
    args = dict(dtype=B.FDTD_F32, slab_planes=16, steps_per_pass=4, max_steps=10, mem_budget_bytes=1e12,
                host_budget_bytes=1e12)
    args.update(kw)
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_stream_create(spec, **args)
    assert e.value.code == code, str(e.value)
    return str(e.value)


def test_stream_admission():
    """Host-streamed slabs: the domain is validated as a resident handle
    would be, a gradient needs max_steps, a slab whose extent would
    cut an absorbing z face is refused, and the device workspace and the host
    banks are admitted against their budgets before anything is allocated."""
    spec = W.lorentz_flux(pml=6, lorentz=8, n_steps=10, n_f=2, shape=(24, 20, 60))
    _stream_refused(spec, B.FDTD_E_INVALID, slab_planes=0)
    _stream_refused(spec, B.FDTD_E_INVALID, steps_per_pass=0)
    g = W.lorentz_flux(pml=6, lorentz=8, n_steps=10, n_f=2, shape=(24, 20, 60))
    g.grad_box = ((8, 8, 8), (16, 12, 40))
    _stream_refused(g, B.FDTD_E_INVALID, max_steps=0)          # a gradient needs the step count
    # with a gradient the host keeps a bank per pass boundary: 10 steps of 4 -> 4 banks + 2 cotangent banks
    msg = _stream_refused(g, B.FDTD_E_NOMEM, host_budget_bytes=5.5 * 24 * 20 * 60 * 4 * 6)
    assert "host budget" in msg
    # cores of 8 planes, halo 5: slab 1 starts at plane 3, cutting the low face
    msg = _stream_refused(spec, B.FDTD_E_INVALID, slab_planes=8, steps_per_pass=4)
    assert "absorbing z face" in msg
    bad = W.lorentz_flux(pml=6, lorentz=8, n_steps=10, n_f=2, shape=(24, 20, 60))
    bad.courant = 0.995 / np.sqrt(3.0)
    _stream_refused(bad, B.FDTD_E_UNSTABLE)
    msg = _stream_refused(spec, B.FDTD_E_NOMEM, mem_budget_bytes=1e5)
    assert "device budget" in msg
    msg = _stream_refused(spec, B.FDTD_E_NOMEM, host_budget_bytes=1e5)
    assert "host budget" in msg
    # bounded forward banks: fewer than 4 refused; 4 banks pass a host budget that one bank per pass
    # boundary (40 steps of 4 -> 11 banks) exceeds, and are then refused only by the device budget
    g40 = W.lorentz_flux(pml=6, lorentz=8, n_steps=40, n_f=2, shape=(24, 20, 60))
    g40.grad_box = ((8, 8, 8), (16, 12, 40))
    bank = 24 * 20 * 60 * 4 * 6
    _stream_refused(g40, B.FDTD_E_INVALID, max_steps=40, host_banks=3)
    msg = _stream_refused(g40, B.FDTD_E_NOMEM, max_steps=40, host_budget_bytes=9 * bank)
    assert "host budget" in msg
    msg = _stream_refused(g40, B.FDTD_E_NOMEM, max_steps=40, host_budget_bytes=9 * bank, host_banks=4,
                          mem_budget_bytes=1e5)
    assert "device budget" in msg
