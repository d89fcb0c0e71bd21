"""Algorithmic byte counts of one time step (the minimum the method must move).

Per cell and step the Yee update reads and writes the six field components
once (12 words).  Add eps^-1 where it is stored (1 word per cell of the eps
box, 3 for a diagonal tensor, 6 per node of a symmetric tensor's box; the
tensor path's curl scratch, written and read once per step, is an
implementation cost and not counted), 8 words per absorbing-face cell (two E and two
H memories read and written), 15 words per Lorentz cell (per component read
E^{n-1}, W^n, W^{n-1}; write E^{n-1}, W^{n+1}).  Halo re-reads, the second
copy of W^{n-1} that ping-ponged state writes, and padding are not counted.
The adjoint step moves the same cotangent state plus, inside the gradient
box, the forward H (3 words) and the FP64 accumulator (read + write, 16 B
per accumulator).
"""
from __future__ import annotations

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, vendor figure


def _box_cells(box):
    if box is None:
        return 0
    lo, hi = box
    n = 1
    for a in range(3):
        n *= max(0, hi[a] - lo[a])
    return n


def face_cells(spec) -> int:
    nx, ny, nz = spec.shape
    cross = (ny * nz, nx * nz, nx * ny)
    return sum(spec.pml[2 * a + s] * cross[a] for a in range(3) for s in range(2))


def forward_bytes(spec, word: int) -> int:
    n = spec.ncells
    per = {"iso": 1, "diag": 3, "tensor": 6}[spec.eps_kind]
    neps = _box_cells(spec.eps_box) * per if spec.eps is not None else 0
    # dispersive cells, per component: read E^{n-1} and each pole's W^n, W^{n-1};
    # write E^{n-1} and each pole's W^{n+1} (2 + 3 P words; 5 for one pole)
    lor_words = sum(_box_cells((L.lo, L.hi)) * 3 * (2 + 3 * len(L.pole_list())) for L in spec.lorentz)
    return word * (12 * n + neps + 8 * face_cells(spec) + lor_words)


def adjoint_bytes(spec, word: int) -> int:
    gb = _box_cells(spec.grad_box) if spec.grad_box is not None else 0
    nacc = {"diag": 3, "tensor": 6}.get(spec.eps_kind, 1)
    return forward_bytes(spec, word) + gb * (3 * word + 16 * nacc)
