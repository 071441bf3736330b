"""Mixed voxel resolution (Sec. 3): the plan optimised on the mixed case
matches the FP64 oracle in lockstep on the same case, and its dose evaluated at
full resolution (one extra dose product) matches the reference dose."""
import numpy as np
import pytest

import casegen
import oracle as O
from _cases import oracle_D, preset_case
from _lockstep import lockstep

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402


def _opts(mode):
    o = P.vmat.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = mode
    o.master = P.master_opts()
    return o


@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_resolution_plan_and_full_evaluation(mode):
    c = casegen.make_case(casegen.tiny_case(n_beams=8, n_rows=4, n_cols=8, grid=(16, 16, 10)))
    m, owner = casegen.mixed_resolution(c)
    Dm = oracle_D(m)
    pm = P.Problem.from_case(m)
    try:
        l, r, occ, y = pm.empty_plan()
        rep, tr = pm.solve(l, r, occ, y, _opts(mode))
    finally:
        pm.close()
    assert rep.cg_iters == m.n_beams
    log = lockstep(m, Dm, tr, l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy(), master_every=1,
                   name=f"mixed/mode {mode}")
    assert log.checked == m.n_beams
    pf = P.Problem.from_case(c)
    try:
        zf = pf.dose(y, l, r, occ).cpu().numpy().astype(np.float64)
    finally:
        pf.close()
    Df = oracle_D(c)
    z_ref = O.dose(Df, O.fluence(y.cpu().numpy(), l.cpu().numpy(), r.cpu().numpy(), occ.cpu().numpy(),
                                 c.n_rows, c.n_cols))
    assert np.abs(zf - z_ref).max() <= 1e-6 * np.abs(z_ref).max()
    # the mixed dose is the group average of the full-resolution dose
    zm_ref = O.dose(Dm, O.fluence(y.cpu().numpy(), l.cpu().numpy(), r.cpu().numpy(), occ.cpu().numpy(),
                                  m.n_rows, m.n_cols))
    avg = np.bincount(owner, weights=z_ref) / np.bincount(owner)
    np.testing.assert_allclose(zm_ref, avg, rtol=1e-5, atol=1e-9 * np.abs(z_ref).max())


def test_mixed_resolution_prostate():
    """Prostate-shaped case: the mixed problem has fewer voxels and non-zeros;
    the plan's full-resolution cost (F + gamma G) stays within 10% of the
    plan optimised at full resolution."""
    c = preset_case("prostate180")
    m, owner = casegen.mixed_resolution(c)
    assert m.n_voxels < 0.2 * c.n_voxels and m.nnz < 0.3 * c.nnz
    pm = P.Problem.from_case(m)
    try:
        l, r, occ, y = pm.empty_plan()
        pm.solve(l, r, occ, y, _opts(1), want_trace=False)
    finally:
        pm.close()
    pf = P.Problem.from_case(c)
    try:
        cm = pf.grad(y, l, r, occ, want=())["cost"].cpu().numpy()
        F_mixed = float(cm[0] + cm[1])
        l2, r2, occ2, y2 = pf.empty_plan()
        rep, _ = pf.solve(l2, r2, occ2, y2, _opts(1), want_trace=False)
    finally:
        pf.close()
    full = rep.F + rep.gG
    print(f"prostate mixed: nv {c.n_voxels} -> {m.n_voxels}, nnz {c.nnz} -> {m.nnz}; full-resolution cost "
          f"{F_mixed:.6g} (mixed plan) vs {full:.6g} (full plan)")
    assert 0.9 * full <= F_mixed <= 1.10 * full
