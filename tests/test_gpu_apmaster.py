"""Column generation with the master over stored aperture doses
(master_mode 1): resuming a stopped plan, graph replay against direct
launches, and a store that grows during a plan.  The plans themselves are
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


def test_aperture_store_growth_keeps_results(monkeypatch):
    """A store that starts at its smallest capacity (one dose vector) has to
    grow during the plan, each time copying the stored entries to larger
    arrays; the plan is the same, bit for bit, as with the default capacity."""
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    out = []
    for small in (False, True):
        if small:
            monkeypatch.setenv("VMAT_AP_MIN_CAP", "1")
        else:
            monkeypatch.delenv("VMAT_AP_MIN_CAP", raising=False)
        prob = P.Problem.from_case(c)
        try:
            b0 = prob.device_bytes()
            l, r, occ, y = prob.empty_plan()
            rep, tr = prob.solve(l, r, occ, y, _opts(1))
            b1 = prob.device_bytes()
            out.append((tr, y.cpu().numpy(), l.cpu().numpy(), r.cpu().numpy(), rep.F + rep.gG, b1 - b0))
        finally:
            prob.close()
    (t0, y0, l0, r0, f0, s0), (t1, y1, l1, r1, f1, s1) = out
    # the smaller store: the hook took effect, so the appends after the first
    # found it full (one dose vector ahead of the stored entries) and grew it
    assert s1 < s0
    assert len(t1["beam"]) == c.n_beams > 1
    np.testing.assert_array_equal(t1["beam"], t0["beam"])
    np.testing.assert_array_equal(t1["cost"], t0["cost"])
    np.testing.assert_array_equal(y1, y0)
    np.testing.assert_array_equal(l1, l0)
    np.testing.assert_array_equal(r1, r0)
    assert f1 == f0
