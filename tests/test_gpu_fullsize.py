"""Full plans at the prostate-shaped size (288,000 beamlets, 1,048,576 voxels,
1.09e8 non-zeros), checked where the FP64 reference can follow: the first
apertures against the reference's first column-generation iterations, the
final plan's cost and KKT conditions re-evaluated by the reference at the
plan the GPU returns, and the invariants of column generation."""
import numpy as np
import pytest

import oracle as O
from _cases import oracle_D, preset_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402

FIRST = 3


@pytest.fixture(scope="module")
def prostate_ref():
    c = preset_case("prostate180")
    D = oracle_D(c)
    ref = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step, max_cg_iter=FIRST)
    return c, D, ref


@pytest.mark.parametrize("mode", [0, 1])
def test_prostate_full_plan(prostate_ref, mode):
    c, D, ref = prostate_ref
    o = P.vmat.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = mode
    o.master = P.master_opts()
    prob = P.Problem.from_case(c)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, o)
        lg, rg, og, yg = l.cpu().numpy(), r.cpu().numpy(), occ.cpu().numpy(), y.cpu().numpy()
    finally:
        prob.close()
    N, R = c.n_beams, c.n_rows
    # the first apertures are the reference's
    for t in range(FIRST):
        k = ref.order[t]
        assert tr["beam"][t] == k
        np.testing.assert_array_equal(lg[k * R:(k + 1) * R], ref.apertures[t][0])
        np.testing.assert_array_equal(rg[k * R:(k + 1) * R], ref.apertures[t][1])
        assert abs(tr["price"][t] - ref.prices[t]) <= 1e-4 * abs(ref.prices[0])
    np.testing.assert_allclose(tr["cost"][:FIRST + 1], ref.costs[:FIRST + 1], rtol=1e-6)
    # the final plan, re-evaluated by the reference
    assert rep.cg_iters == N and og.all()
    F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), yg, lg, rg, og, c.gamma, c.theta_deg,
                                        c.circular, R, c.n_cols)
    assert rep.F + rep.gG == pytest.approx(F + gG, rel=1e-6)
    kkt = np.abs(np.minimum(yg, grad)).max()
    assert kkt <= 2e-5 * rep.kkt_ref
    assert np.all(yg >= 0)
    cost = tr["cost"]
    assert np.all(cost[1:] <= cost[:-1] * (1 + 1e-12))
    L, Rr = lg.reshape(N, R), rg.reshape(N, R)
    assert np.all(L <= Rr)
    for a in range(N):
        b = (a + 1) % N
        assert np.all(np.abs(L[a] - L[b]) <= c.max_leaf_step)
        assert np.all(np.abs(Rr[a] - Rr[b]) <= c.max_leaf_step)
    print(f"mode {mode}: cost {rep.F + rep.gG:.9g}, reference re-evaluation {F + gG:.9g}, KKT {kkt:.3g} "
          f"(tolerance {1e-5 * rep.kkt_ref:.3g})")


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_headneck_full_plan(fmt):
    """Head-and-neck-shaped plan (432,000 beamlets, 3,538,944 voxels, 3.7e8
    non-zeros), FP32 and BF16 storage: the first aperture against the
    reference on the same stored D, the final cost and KKT conditions
    re-evaluated by the reference, and the invariants."""
    c = preset_case("headneck180")
    vals = c.val if fmt == "f32" else O.bf16_round(c.val)
    D = oracle_D(c, vals)
    ref = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step, max_cg_iter=1)
    o = P.vmat.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = 1
    o.master = P.master_opts()
    prob = P.Problem.from_case(c, d_store=fmt)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, o)
        lg, rg, og, yg = l.cpu().numpy(), r.cpu().numpy(), occ.cpu().numpy(), y.cpu().numpy()
    finally:
        prob.close()
    N, R = c.n_beams, c.n_rows
    k = ref.order[0]
    assert tr["beam"][0] == k
    np.testing.assert_array_equal(lg[k * R:(k + 1) * R], ref.apertures[0][0])
    np.testing.assert_array_equal(rg[k * R:(k + 1) * R], ref.apertures[0][1])
    np.testing.assert_allclose(tr["cost"][:2], ref.costs[:2], rtol=1e-6)
    assert rep.cg_iters == N and og.all()
    F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), yg, lg, rg, og, c.gamma, c.theta_deg,
                                        c.circular, R, c.n_cols)
    assert rep.F + rep.gG == pytest.approx(F + gG, rel=1e-6)
    assert np.abs(np.minimum(yg, grad)).max() <= 2e-5 * rep.kkt_ref
    cost = tr["cost"]
    assert np.all(cost[1:] <= cost[:-1] * (1 + 1e-12))
    print(f"head-and-neck {fmt}: cost {rep.F + rep.gG:.9g}, reference re-evaluation {F + gG:.9g}")
