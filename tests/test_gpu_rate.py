"""Dose-rate feasibility of a final plan (gamma continuation) against the FP64
reference: same number of rounds, same final gamma, same intensities."""
import numpy as np
import pytest

import oracle as O
from _cases import oracle_D, preset_case, small_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402


def T(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("name,frac,factor", [("small", 0.3, 10.0), ("small", 0.6, 3.0), ("tiny36", 0.4, 10.0)])
def test_enforce_rate_matches_oracle(name, frac, factor):
    c = small_case(n_beams=8, n_rows=3, n_cols=6, grid=(12, 12, 8)) if name == "small" else preset_case("tiny36")
    D = oracle_D(c)
    sol = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step)
    rate0 = O.max_rate(sol.y, c.theta_deg, c.circular)
    rate_max = frac * rate0
    mo = O.MasterOpts(tol_rel=1e-10, max_iter=2000)
    ref = O.enforce_rate(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                         sol.l, sol.r, sol.occ, sol.y, rate_max, factor=factor, opts=mo)
    prob = P.Problem.from_case(c)
    try:
        y = T(sol.y, torch.float64)
        rep = prob.enforce_rate(T(sol.l, torch.int32), T(sol.r, torch.int32), T(sol.occ, torch.uint8), y,
                                rate_max, factor=factor, master=P.master_opts(max_iter=2000, tol_rel=1e-10))
        yg = y.cpu().numpy()
    finally:
        prob.close()
    assert rep.rounds == ref.rounds and bool(rep.feasible) == ref.feasible
    assert rep.gamma == pytest.approx(ref.gamma, rel=1e-12)
    assert np.abs(yg - ref.y).max() <= 1e-6 * np.abs(ref.y).max()
    assert rep.rate == pytest.approx(ref.rate, rel=1e-5, abs=1e-9 * rate0)
    if ref.costs:
        assert rep.F + rep.gG == pytest.approx(ref.costs[-1], rel=1e-8)
    assert prob is not None


def test_enforce_rate_feasible_plan_unchanged():
    c = small_case(n_beams=8, n_rows=3, n_cols=6, grid=(12, 12, 8))
    D = oracle_D(c)
    sol = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step)
    rate0 = O.max_rate(sol.y, c.theta_deg, c.circular)
    prob = P.Problem.from_case(c)
    try:
        y = T(sol.y, torch.float64)
        rep = prob.enforce_rate(T(sol.l, torch.int32), T(sol.r, torch.int32), T(sol.occ, torch.uint8), y,
                                2.0 * rate0)
        assert rep.rounds == 0 and rep.feasible == 1 and rep.gamma == c.gamma
        assert np.array_equal(y.cpu().numpy(), sol.y)
        assert rep.rate == pytest.approx(rate0, rel=1e-12)
    finally:
        prob.close()


def test_enforce_rate_prostate_after_plan():
    """Full prostate-shaped plan on the GPU, then the continuation to half the
    plan's largest rate: the returned plan is feasible (or the round cap is
    reported) and the rate never rises."""
    c = preset_case("prostate180")
    prob = P.Problem.from_case(c)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, _ = prob.solve(l, r, occ, y, want_trace=False)
        rate0 = O.max_rate(y.cpu().numpy(), c.theta_deg, c.circular)
        rr = prob.enforce_rate(l, r, occ, y, 0.5 * rate0, factor=10.0, max_rounds=6)
        yg = y.cpu().numpy()
    finally:
        prob.close()
    print(f"prostate: rate {rate0:.4g} -> {rr.rate:.4g} in {rr.rounds} rounds, gamma {rr.gamma:.3g}, "
          f"master iterations {rr.master_iters}")
    assert rr.rounds >= 1
    assert rr.rate <= rate0
    assert rr.feasible == (rr.rate <= 0.5 * rate0)
    assert rr.feasible or rr.rounds == 6
    assert rr.rate == pytest.approx(O.max_rate(yg, c.theta_deg, c.circular), rel=1e-12)
