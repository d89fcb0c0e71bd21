"""The device reduction of the Poynting flux (Section 2.4) through the C-ABI:
fdtd_flux_reduce on caller-owned device spectra, and the FLUX op of a flux
monitor, which runs the same reduction.  The reference is the oracle's flux of
the same spectra in FP64; the device sums in another order, so the bar is a
few ulp of the sum of magnitudes."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_30039_amd import binding as B
from paper_2609_30039_amd import workloads as W
from paper_2609_30039_amd.sim import Simulation

pytestmark = pytest.mark.gpu


def _spectra(nf, npts, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((nf, 4, npts)) + 1j * rng.standard_normal((nf, 4, npts))


def _bound(sp):
    """Round-off bound of a sum of 4 n products: n * 2^-50 times the sum of |terms|."""
    mag = np.sum(np.abs(sp[:, 0]) * np.abs(sp[:, 3]) + np.abs(sp[:, 1]) * np.abs(sp[:, 2]), axis=1)
    return 4.0 * sp.shape[2] * 2.0 ** -52 * mag


def _device_flux(sp, workspace=False):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(sp)).cuda()
    out = torch.empty(sp.shape[0], dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    if workspace:
        nb = B.flux_workspace_bytes(sp.shape[0], sp.shape[2])
        ws = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
        B.fdtd_flux_reduce(d.data_ptr(), sp.shape[0], sp.shape[2], out.data_ptr(), ws.data_ptr(), nb, stream)
    else:
        B.fdtd_flux_reduce(d.data_ptr(), sp.shape[0], sp.shape[2], out.data_ptr(), None, 0, stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("nf,npts", [(1, 1), (3, 4095), (16, 21904), (7, 4096 * 256 + 17)])
def test_flux_reduce_matches_oracle(nf, npts):
    """Sizes below one block, one block short, the headline plane (148^2)
    and past the block cap (every block then takes more than 4096 points)."""
    sp = _spectra(nf, npts, 11 + nf)
    ref = O.OracleSim.flux_from_spectra(sp[:, :, None, :])
    got = _device_flux(sp)
    assert np.all(np.abs(got - ref) <= _bound(sp)), (got - ref, _bound(sp))
    # a caller-owned workspace gives the same bits as the library's own
    assert np.array_equal(_device_flux(sp, workspace=True), got)


def test_flux_reduce_refuses_bad_arguments():
    import torch
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_flux_reduce(d.data_ptr(), 0, 1, d.data_ptr())
    assert e.value.code == B.FDTD_E_INVALID
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_flux_reduce(d.data_ptr(), 1, 1, d.data_ptr(), d.data_ptr(), 4)
    assert e.value.code == B.FDTD_E_RANGE


def test_monitor_flux_op_is_the_device_reduction():
    """FLUX of a flux monitor equals fdtd_flux_reduce of its GET spectra
    bitwise, and the oracle's flux of the same spectra to round-off."""
    spec = W.lorentz_flux(pml=6, lorentz=8, n_steps=120, n_f=5, shape=(70, 23, 41))
    sim = Simulation(spec, dtype="f64")
    sim.step(spec.n_steps)
    sp = sim.spectra(0)
    fl = sim.flux(0)
    flat = sp.reshape(sp.shape[0], 4, -1)
    assert np.array_equal(fl, _device_flux(flat))
    ref = O.OracleSim.flux_from_spectra(sp)
    assert np.all(np.abs(fl - ref) <= _bound(flat))
