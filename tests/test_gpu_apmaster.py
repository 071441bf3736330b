"""Column generation with the master over stored aperture doses
(master_mode 1): resuming a stopped plan, graph replay against direct
launches, and the store reserved at a size no plan exceeds.  The plans themselves are
checked against the oracle in lockstep (test_gpu_lockstep.py,
test_gpu_fullsize.py)."""
import numpy as np
import pytest

from _cases import hand_case, preset_case, small_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402

CASES = [("small", lambda: small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))),
         ("small_open", lambda: small_case(n_beams=10, n_rows=3, n_cols=8, grid=(14, 14, 8), circular=0,
                                           max_leaf_step=-1, seed=3)),
         ("hand", lambda: hand_case(1)),
         ("tiny36", lambda: preset_case("tiny36"))]


def _opts(mode, max_cg_iter=0, tol_rel=1e-5, max_iter=200):
    o = P.vmat.SolveOpts()
    o.max_cg_iter = max_cg_iter
    o.master_mode = mode
    o.master = P.master_opts(max_iter=max_iter, tol_rel=tol_rel)
    return o


def test_aperture_master_resume_from_partial_plan():
    """A plan stopped after a few apertures and resumed in mode 1 (stored
    doses rebuilt for the occupied beams) ends where an uninterrupted run ends."""
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    prob = P.Problem.from_case(c)
    try:
        l, r, occ, y = prob.empty_plan()
        rep_a, tr_a = prob.solve(l, r, occ, y, _opts(1))
        l2, r2, occ2, y2 = prob.empty_plan()
        rep_b1, tr_b1 = prob.solve(l2, r2, occ2, y2, _opts(1, max_cg_iter=3))
        o = _opts(1)
        o.master.kkt_ref = rep_b1.kkt_ref   # the scale the uninterrupted run uses
        rep_b2, tr_b2 = prob.solve(l2, r2, occ2, y2, o)
    finally:
        prob.close()
    assert rep_b1.cg_iters == 3 and rep_b2.cg_iters == c.n_beams - 3
    np.testing.assert_array_equal(np.concatenate([tr_b1["beam"], tr_b2["beam"]]), tr_a["beam"])
    assert rep_b2.F + rep_b2.gG == pytest.approx(rep_a.F + rep_a.gG, rel=1e-6)
    np.testing.assert_array_equal(l2.cpu().numpy(), l.cpu().numpy())
    np.testing.assert_array_equal(r2.cpu().numpy(), r.cpu().numpy())


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", ["small", "prostate"])
def test_graph_replay_matches_direct_launches(mode, name, monkeypatch):
    """Master iterations replayed from a captured graph give the same bits as
    the same kernels launched one by one (every replay is compared through the
    per-iteration costs, the plan and the final intensities)."""
    c = dict(CASES)["small"]() if name == "small" else preset_case("prostate180")
    iters = 0 if name == "small" else 12
    prob = P.Problem.from_case(c)
    try:
        out = []
        for no_graph in (False, True, False):
            if no_graph:
                monkeypatch.setenv("VMAT_NO_GRAPH", "1")
            else:
                monkeypatch.delenv("VMAT_NO_GRAPH", raising=False)
            l, r, occ, y = prob.empty_plan()
            rep, tr = prob.solve(l, r, occ, y, _opts(mode, max_cg_iter=iters))
            out.append((tr, y.cpu().numpy(), l.cpu().numpy(), r.cpu().numpy(), rep.master_iters))
    finally:
        prob.close()
    for tr, y, l, r, mi in out[1:]:
        assert mi == out[0][4]
        np.testing.assert_array_equal(tr["cost"], out[0][0]["cost"])
        np.testing.assert_array_equal(tr["beam"], out[0][0]["beam"])
        np.testing.assert_array_equal(y, out[0][1])
        np.testing.assert_array_equal(l, out[0][2])
        np.testing.assert_array_equal(r, out[0][3])


def _beam_voxel_bound(c):
    """Sum over beams of the voxels each beam reaches (non-zero D), counted on
    the host from the case's CSR."""
    RC = c.n_rows * c.n_cols
    rows = np.repeat(np.arange(c.row_ptr.size - 1), np.diff(c.row_ptr))
    keep = c.val != 0
    key = (rows[keep] // RC).astype(np.int64) * c.n_voxels + c.col[keep]
    return int(np.unique(key).size)


@pytest.mark.parametrize("name", ["small", "hand", "tiny36"])
def test_reserved_store_holds_every_plan(name):
    """vmat_reserve_solve sizes the store at U + nv entries (U: voxels each
    beam reaches, summed over beams; 28 bytes per entry), and a full plan in
    mode 1 allocates nothing more."""
    c = dict(CASES)[name]()
    U = _beam_voxel_bound(c)
    prob = P.Problem.from_case(c)
    try:
        b0 = prob.device_bytes()
        prob.reserve_solve()
        b1 = prob.device_bytes()
        nv, N = c.n_voxels, c.n_beams
        entries = 28 * (U + nv)
        assert entries <= b1 - b0 <= entries + 16 * (nv + 1) + 4 * ((nv + 1023) // 1024 + 2) + 24 * (N + 1) + 64
        prob.reserve_solve()   # once per handle
        assert prob.device_bytes() == b1
        l, r, occ, y = prob.empty_plan()
        rep, _ = prob.solve(l, r, occ, y, _opts(1))
        assert rep.cg_iters == c.n_beams
        assert prob.device_bytes() == b1
    finally:
        prob.close()
