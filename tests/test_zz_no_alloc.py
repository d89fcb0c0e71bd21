"""fdtd_flux_reduce_noalloc against fdtd_flux_reduce through the C-ABI: the
allocation-free entry point keeps its partial sums in the library's fixed
device scratch array and must give the same bits as the workspace entry
point, on two calls in a row (the second with a smaller input, so stale
partials of the first would show), and refuse sizes beyond its scratch."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_30039_amd import binding as B

pytestmark = pytest.mark.gpu


def _spectra(nf, npts, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((nf, 4, npts)) + 1j * rng.standard_normal((nf, 4, npts))


def _run(sp, noalloc):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(sp)).cuda()
    out = torch.full((sp.shape[0],), np.nan, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        B.fdtd_flux_reduce_noalloc(d.data_ptr(), sp.shape[0], sp.shape[2], out.data_ptr(), stream)
    else:
        B.fdtd_flux_reduce(d.data_ptr(), sp.shape[0], sp.shape[2], out.data_ptr(), None, 0, stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_equals_workspace_entry_point_on_two_calls():
    # first call: 12 frequencies x 64 blocks (a quarter of the scratch);
    # second: 5 frequencies x 3 blocks, fewer partials than the first left
    for nf, npts, seed in [(12, 64 * 4096, 1), (5, 2 * 4096 + 9, 2)]:
        sp = _spectra(nf, npts, seed)
        a = _run(sp, noalloc=True)
        b = _run(sp, noalloc=False)
        assert np.array_equal(a, b), (nf, npts, a - b)
        ref = O.OracleSim.flux_from_spectra(sp[:, :, None, :])
        mag = np.sum(np.abs(sp[:, 0]) * np.abs(sp[:, 3]) + np.abs(sp[:, 1]) * np.abs(sp[:, 2]), axis=1)
        assert np.all(np.abs(a - ref) <= 4.0 * npts * 2.0 ** -52 * mag)


def test_noalloc_at_the_scratch_limit_and_beyond():
    # 32 frequencies x 256 blocks fill the 64 KiB exactly; 33 do not fit
    import torch
    npts = 256 * 4096
    assert B.flux_workspace_bytes(32, npts) == B.FDTD_FLUX_SCRATCH_BYTES
    g = torch.Generator(device="cuda").manual_seed(3)
    d = torch.randn(32 * 4 * npts * 2, dtype=torch.float64, device="cuda", generator=g)
    outs = []
    for noalloc in (True, False):
        out = torch.full((32,), np.nan, dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        if noalloc:
            B.fdtd_flux_reduce_noalloc(d.data_ptr(), 32, npts, out.data_ptr(), stream)
        else:
            B.fdtd_flux_reduce(d.data_ptr(), 32, npts, out.data_ptr(), None, 0, stream)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    assert np.all(np.isfinite(outs[0])) and np.array_equal(outs[0], outs[1])
    with pytest.raises(B.FdtdError) as e:
        B.fdtd_flux_reduce_noalloc(d.data_ptr(), 33, npts, d.data_ptr())
    assert e.value.code == B.FDTD_E_RANGE
