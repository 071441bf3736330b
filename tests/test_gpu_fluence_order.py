"""The dose of a plan (vmat_dose) forms the plan's fluence in the order of
the tiled layout's beamlet lists and stages it with one contiguous read; the
same fluence given in beamlet order (vmat_dose_fluence) takes the gather
path.  The two give the same bits in every storage format, in the plain
layout too, and at the prostate case's full size (many work items per
block)."""
import numpy as np
import pytest

from _cases import preset_case, small_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402


def _plan(c, rng):
    N, R, C = c.n_beams, c.n_rows, c.n_cols
    occ = (rng.random(N) < 0.7).astype(np.uint8)
    l = rng.integers(0, C + 1, size=(N, R)).astype(np.int32)
    r = np.minimum(C, l + rng.integers(0, C + 1, size=(N, R))).astype(np.int32)
    y = rng.random(N) * 2.0
    return y, l, r, occ


def _fluence(c, y, l, r, occ):
    """x_i = y_k when beamlet i (beam k, row rho, column c) lies in the open
    interval [l, r) of an occupied beam's row, else 0 (beamlet-major)."""
    cols = np.arange(c.n_cols)
    open_ = (cols[None, None, :] >= l[..., None]) & (cols[None, None, :] < r[..., None]) & (occ[:, None, None] > 0)
    return np.where(open_, y[:, None, None], 0.0).reshape(-1)


def _check(prob, c, seed, plans):
    rng = np.random.default_rng(seed)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    for _ in range(plans):
        y, l, r, occ = _plan(c, rng)
        z_plan = prob.dose(dev(y), dev(l.reshape(-1)), dev(r.reshape(-1)), dev(occ)).cpu().numpy()
        z_flu = prob.dose_fluence(dev(_fluence(c, y, l, r, occ))).cpu().numpy()
        np.testing.assert_array_equal(z_plan, z_flu)
        assert np.abs(z_plan).max() > 0


@pytest.mark.parametrize("layout", ["tiled", "plain"])
@pytest.mark.parametrize("d_store", ["f32", "bf16", "fp8"])
def test_plan_dose_equals_fluence_dose(d_store, layout):
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    prob = P.Problem.from_case(c, d_store=d_store, layout=layout)
    try:
        assert prob.layout()["tiled"] == (layout == "tiled")
        _check(prob, c, 5, 3)
    finally:
        prob.close()


def test_plan_dose_equals_fluence_dose_prostate():
    c = preset_case("prostate180")
    prob = P.Problem.from_case(c)
    try:
        assert prob.layout()["tiled"] == 1
        _check(prob, c, 9, 2)
    finally:
        prob.close()
