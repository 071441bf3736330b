"""Column generation with the master over stored aperture doses
(master_mode 1): the same plans as the FP64 reference, and as the master that
streams D (mode 0) at full size."""
import numpy as np
import pytest

import oracle as O
from _cases import compare_plan, hand_case, oracle_D, preset_case, small_case

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


@pytest.mark.parametrize("name", [n for n, _ in CASES])
@pytest.mark.parametrize("layout", ["tiled", "plain"])
def test_aperture_master_solve_matches_oracle(name, layout):
    c = dict(CASES)[name]()
    D = oracle_D(c)
    ref = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step)
    prob = P.Problem.from_case(c, layout=layout)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, _opts(1))
        matched = compare_plan(c, ref, tr, l.cpu().numpy(), r.cpu().numpy(), rep)
        # D products: one forward per opened aperture, one adjoint per pricing
        assert rep.n_forward == c.n_beams and rep.n_adjoint == c.n_beams
    finally:
        prob.close()
    print(f"{name}/{layout}: matched {matched} of {c.n_beams}")
    assert matched >= min(10, c.n_beams)


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_aperture_master_reduced_precision(fmt):
    """With reduced-precision D both master modes use the same stored D: the
    plans agree with each other (costs within 1e-6)."""
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    prob = P.Problem.from_case(c, d_store=fmt)
    try:
        out = []
        for mode in (0, 1):
            l, r, occ, y = prob.empty_plan()
            rep, tr = prob.solve(l, r, occ, y, _opts(mode))
            out.append((tr, rep))
    finally:
        prob.close()
    (t0, r0), (t1, r1) = out
    np.testing.assert_array_equal(t0["beam"], t1["beam"])
    np.testing.assert_allclose(t1["cost"], t0["cost"], rtol=1e-6)


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


def test_aperture_master_prostate_matches_streaming_master():
    """Both master modes with tight masters (KKT 1e-9 of the first price), so
    that the pricing decisions do not hinge on where a master stops."""
    c = preset_case("prostate180")
    prob = P.Problem.from_case(c)
    try:
        res = {}
        for mode in (0, 1):
            l, r, occ, y = prob.empty_plan()
            rep, tr = prob.solve(l, r, occ, y, _opts(mode, tol_rel=1e-9, max_iter=5000))
            res[mode] = (rep, tr, l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy())
    finally:
        prob.close()
    (r0, t0, l0, rr0, y0), (r1, t1, l1, rr1, y1) = res[0], res[1]
    R = c.n_rows
    matched = 0
    for t in range(c.n_beams):
        k = t0["beam"][t]
        same = t1["beam"][t] == k and np.array_equal(l1[k * R:(k + 1) * R], l0[k * R:(k + 1) * R]) \
            and np.array_equal(rr1[k * R:(k + 1) * R], rr0[k * R:(k + 1) * R])
        if not same:
            eps = 1e-5 * abs(t0["price"][t])
            assert t0["margin"][t] <= eps or t0["row_margin"][t] <= eps, t
            break
        matched += 1
    print(f"prostate: modes agree on {matched} of {c.n_beams} apertures; costs {r0.F + r0.gG} / {r1.F + r1.gG}; "
          f"D products {r0.n_forward}+{r0.n_adjoint} vs {r1.n_forward}+{r1.n_adjoint}")
    assert matched >= 20
    if matched == c.n_beams:
        assert r1.F + r1.gG == pytest.approx(r0.F + r0.gG, rel=1e-6)
        np.testing.assert_allclose(t1["cost"], t0["cost"], rtol=1e-6)
    assert np.all(t1["cost"][1:] <= t1["cost"][:-1] * (1 + 1e-12))


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


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
@pytest.mark.parametrize("mode", [0, 1])
def test_reduced_precision_plan_matches_oracle_on_stored_d(fmt, mode):
    """A plan computed with D stored in BF16 / FP8 matches the FP64 reference
    plan of the same rounded D (the plan is exact for what is stored)."""
    c = preset_case("tiny36")
    if fmt == "bf16":
        vals = O.bf16_round(c.val)
    else:
        s_, q_ = O.fp8_quantise(c.row_ptr, c.val)
        vals = O.fp8_dequantise(c.row_ptr, s_, q_)
    D = oracle_D(c, vals)
    ref = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step)
    prob = P.Problem.from_case(c, d_store=fmt)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, _opts(mode))
        matched = compare_plan(c, ref, tr, l.cpu().numpy(), r.cpu().numpy(), rep)
    finally:
        prob.close()
    print(f"{fmt}/mode {mode}: matched {matched} of {c.n_beams}")
    assert matched >= 10


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
