"""The single-precision parity tests let the oracle take the kernel's column
decision for a volume whose position rounds across a cell face.  This CPU
test checks that the handoff accepts only such volumes: a column decision
off by one cell for a volume away from the face, or a column that is not a
neighbour, must fail."""
import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W
from helpers import check_flips_at_faces, oracle_deposit_with_kernel_decisions


def _setup(orc):
    w = W.make_c1(n_rays=256)
    bg = orc.Background.from_workload(w)
    rs = orc.RaySet(w.rays)
    orc.keys(bg, rs)
    return w, bg, rs


def test_flip_at_a_face_is_accepted(orc):
    w, bg, rs = _setup(orc)
    i = 7
    # put volume i a hair below the x face between its column and the next
    ci = int(rs["col"][i]) % w.nx
    rs.a["x"][i] = (ci + 1) * w.dx * (1.0 - 1e-9)
    orc.keys(bg, rs)
    snap = rs.snapshot()
    cols = rs["col"].copy()
    cols[i] = cols[i] - ci + (ci + 1) % w.nx  # the kernel put it just across the face
    gpu = {k: snap[k] for k in ("id", "x", "y")}
    assert check_flips_at_faces(bg, rs, gpu, cols, 2e-6) < 2e-6
    flux, flips, nset = oracle_deposit_with_kernel_decisions(orc, bg, rs, gpu, cols)
    assert flips == 1 and nset == 0


@pytest.mark.parametrize("shift", [1, 2])
def test_planted_column_error_fails(orc, shift):
    w, bg, rs = _setup(orc)
    snap = rs.snapshot()
    gx = (snap["x"] - w.x0) / w.dx
    mid = np.nonzero(np.abs(gx - np.floor(gx) - 0.5) < 0.3)[0]
    i = int(mid[0])
    cols = rs["col"].copy()
    ci = int(cols[i]) % w.nx
    cols[i] = cols[i] - ci + (ci + shift) % w.nx  # an off-by-shift column key
    gpu = {k: snap[k] for k in ("id", "x", "y")}
    with pytest.raises(AssertionError):
        check_flips_at_faces(bg, rs, gpu, cols, 2e-6)
    with pytest.raises(AssertionError):
        oracle_deposit_with_kernel_decisions(orc, bg, rs, gpu, cols)
