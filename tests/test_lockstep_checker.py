"""The lockstep plan checker itself (tests/_lockstep.py), on the CPU: a plan
the oracle made passes with every decision identical, and plans with a
planted mistake (a wrong beam, a moved leaf, a wrong cost, wrong intensities)
are rejected.  The plans here come from the oracle only."""
import numpy as np
import pytest

import oracle as O
from _cases import oracle_D, small_case
from _lockstep import deliverable, lockstep


@pytest.fixture(scope="module")
def oracle_plan():
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    D = oracle_D(c)
    ref = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step)
    tr = {"beam": np.array(ref.order), "price": np.array(ref.prices), "margin": np.array(ref.margins),
          "row_margin": np.array(ref.row_margins), "cost": np.array(ref.costs), "y": np.array(ref.priced_y)}
    return c, D, ref, tr


def _copy(tr):
    return {k: np.array(v, copy=True) for k, v in tr.items()}


def test_oracle_plan_passes(oracle_plan):
    c, D, ref, tr = oracle_plan
    log = lockstep(c, D, tr, ref.l, ref.r, ref.y, master_every=1, log_fn=None)
    assert log.checked == c.n_beams and log.matched == c.n_beams and not log.excused
    assert log.masters == c.n_beams
    # the oracle's own plan carries its dose from step to step; the checker
    # recomputes it from the intensities: rounding-level differences only
    assert log.max_price_dev <= 1e-12 * abs(ref.prices[0]) * 100 and log.max_master_dev <= 1e-10
    deliverable(c, ref.l, ref.r)


def test_checked_range_and_stride(oracle_plan):
    c, D, ref, tr = oracle_plan
    p0 = abs(ref.prices[0])
    log = lockstep(c, D, tr, ref.l, ref.r, ref.y, t_begin=3, check_every=2, kkt_ref=p0, log_fn=None)
    # iterations 4, 6 and the last (7)
    assert log.checked == 3 and log.matched == 3


def test_wrong_beam_is_rejected(oracle_plan):
    c, D, ref, tr = oracle_plan
    # the iteration with the clearest beam choice: a swap there is no near-tie
    t = int(np.argmax(np.array(ref.margins[:-1]) / np.abs(ref.prices[:-1])))
    bad = _copy(tr)
    bad["beam"][t], bad["beam"][t + 1] = tr["beam"][t + 1], tr["beam"][t]
    with pytest.raises(AssertionError, match=f"iteration {t}: GPU beam"):
        lockstep(c, D, bad, ref.l, ref.r, ref.y, log_fn=None)


def test_moved_leaf_is_rejected(oracle_plan):
    c, D, ref, tr = oracle_plan
    R, C = c.n_rows, c.n_cols
    # the first iteration and row whose right leaf can move by one within the window
    for t, k in enumerate(ref.order):
        occ = np.zeros(c.n_beams, np.uint8)
        occ[ref.order[:t]] = 1
        lb = O.leaf_bounds(k, ref.l, ref.r, occ, R, C, c.max_leaf_step, c.circular)
        for rho in range(R):
            i = k * R + rho
            rr = ref.r[i] + 1
            if rr <= min(C, lb[3][rho]):
                r_bad = ref.r.copy()
                r_bad[i] = rr
                with pytest.raises(AssertionError, match=f"iteration {t}: beam {k} row {rho}"):
                    lockstep(c, D, tr, ref.l, r_bad, ref.y, log_fn=None)
                return
    pytest.fail("no movable leaf found")


def test_wrong_cost_is_rejected(oracle_plan):
    c, D, ref, tr = oracle_plan
    bad = _copy(tr)
    bad["cost"][4] *= 1 + 1e-5
    with pytest.raises(AssertionError, match="iteration 4: GPU cost"):
        lockstep(c, D, bad, ref.l, ref.r, ref.y, log_fn=None)


def test_wrong_intensities_are_rejected(oracle_plan):
    c, D, ref, tr = oracle_plan
    bad = _copy(tr)
    bad["y"][3] *= 1.01
    with pytest.raises(AssertionError, match="iteration 3"):
        lockstep(c, D, bad, ref.l, ref.r, ref.y, log_fn=None)


def test_unconverged_master_is_rejected(oracle_plan):
    """A GPU master that stopped early: the oracle's master from the same state
    reaches a lower cost, and the oracle's KKT residual at the GPU's
    intensities exceeds the tolerance."""
    c, D, ref, tr = oracle_plan
    bad = _copy(tr)
    t = 5
    # the intensities after master t halfway between the state before and after
    bad["y"][t + 1] = 0.5 * (tr["y"][t] + tr["y"][t + 1])
    F, dF = O.penalty(O.dose(D, O.fluence(bad["y"][t + 1], ref.l, ref.r,
                                          np.isin(np.arange(c.n_beams), ref.order[:t + 1]).astype(np.uint8),
                                          c.n_rows, c.n_cols)), c.alpha, c.beta, c.T)
    G, _ = O.smoothing(bad["y"][t + 1], c.theta_deg, c.circular)
    bad["cost"][t + 1] = F + c.gamma * G      # consistent with the (wrong) intensities
    with pytest.raises(AssertionError, match=f"iteration {t}: GPU master cost"):
        lockstep(c, D, bad, ref.l, ref.r, ref.y, master_every=1, log_fn=None)
