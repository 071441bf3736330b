"""Lockstep comparison of a GPU column-generation plan with the FP64 oracle.

Column generation (Sec. 2.2) opens one aperture per iteration and never
changes it afterwards, so the GPU's final leaf pairs, its beam order and the
intensities each pricing saw (``trace["y"]``) give the GPU's plan state at
every iteration.  At each checked iteration t the oracle takes that state,
computes the dose, F'(z), the beamlet prices and the pricing problem in FP64
from it, and the GPU's decision must be the oracle's:

* the beam: identical, unless the oracle's beam margin (second-best price
  minus best) is at most eps = eps_rel * |p*| and the oracle prices the GPU's
  beam within eps of the best;
* every leaf pair of the chosen beam: identical to the oracle's best pair for
  that row (of that beam), unless that row's margin (least gap between its
  best sum and any feasible pair with a different sum) is at most eps and the
  GPU's pair sums to within eps of the best;
* the GPU's reported price within ``price_tol`` of the oracle's (when the
  beam matches), and its reported cost after every master within ``cost_rel``
  of the objective the oracle evaluates at the GPU's intensities.

Both sides then continue from the GPU's decision (the plan the GPU made), so
one excused near-tie does not end the comparison.  On checked iterations the
oracle can also run its own master from the GPU's state plus the new aperture
(``master_every``): the cost it reaches must match the GPU's within
``cost_rel``, and the oracle's KKT residual at the GPU's intensities must meet
the master's tolerance (with ``kkt_slack`` for FP32 rounding of F').

Expected values all come from ``oracle/``; the GPU side supplies only the plan
being checked.
"""
from __future__ import annotations

import dataclasses
import numpy as np

import oracle as O


@dataclasses.dataclass
class LockstepLog:
    checked: int = 0          # iterations re-priced by the oracle
    matched: int = 0          # of those, decisions identical to the oracle's
    excused: list = dataclasses.field(default_factory=list)   # (t, what, margin, eps)
    masters: int = 0          # oracle master solves compared
    max_price_dev: float = 0.0
    max_cost_dev: float = 0.0     # relative, GPU cost vs objective at the GPU's state
    max_master_dev: float = 0.0   # relative, GPU cost vs the oracle master's cost
    max_kkt_ratio: float = 0.0    # oracle KKT at the GPU's y / (tol * ref)

    def summary(self, name=""):
        ex = ", ".join(f"t={t} {w} margin {m:.3g} <= {e:.3g}" for t, w, m, e in self.excused)
        return (f"{name}: {self.matched}/{self.checked} decisions identical, {len(self.excused)} excused"
                f"{' (' + ex + ')' if ex else ''}; {self.masters} masters; max |dp| {self.max_price_dev:.3g}, "
                f"cost rel {self.max_cost_dev:.3g}, master cost rel {self.max_master_dev:.3g}, "
                f"KKT/tol {self.max_kkt_ratio:.3g}")


def _objective(c, D, y, l, r, occ):
    """F(z(y)) and gamma G(y) with F'(z) and dG/dy (eq. 1-3), FP64."""
    z = O.dose(D, O.fluence(y, l, r, occ, c.n_rows, c.n_cols))
    F, dF = O.penalty(z, c.alpha, c.beta, c.T)
    G, dG = O.smoothing(y, c.theta_deg, c.circular)
    return F, c.gamma * G, dF, dG


def _row_check(c, g, k, lk, rk, l, r, occ, eps, log, t):
    """Every leaf pair the GPU chose for beam k against the oracle's best pair
    of that row; a different pair is excused only by a row margin <= eps."""
    R, C = c.n_rows, c.n_cols
    Llo, Lhi, Rlo, Rhi = O.leaf_bounds(k, l, r, occ, R, C, c.max_leaf_step, c.circular)
    gk = np.asarray(g).reshape(c.n_beams, R, C)[k]
    same = True
    for rho in range(R):
        S, ll, rr = O.price_row(gk[rho], Llo[rho], Lhi[rho], Rlo[rho], Rhi[rho])
        if ll == lk[rho] and rr == rk[rho]:
            continue
        same = False
        # the GPU's pair must be feasible for the oracle's window and as good
        # as the best within eps, and the row must be a near-tie
        assert Llo[rho] <= lk[rho] <= Lhi[rho] and Rlo[rho] <= rk[rho] <= Rhi[rho] and lk[rho] <= rk[rho], \
            f"iteration {t}: beam {k} row {rho}: GPU pair ({lk[rho]}, {rk[rho]}) outside the leaf window"
        S_gpu = float(np.sum(gk[rho, lk[rho]:rk[rho]]))
        m = O.row_margin(gk[rho], Llo[rho], Lhi[rho], Rlo[rho], Rhi[rho], S)
        assert m <= eps and S_gpu - S <= eps, \
            (f"iteration {t}: beam {k} row {rho}: GPU ({lk[rho]}, {rk[rho]}) vs oracle ({ll}, {rr}), "
             f"row margin {m} > eps {eps} or GPU sum {S_gpu} vs {S}")
        log.excused.append((t, f"row {rho}", m, eps))
    return same


def lockstep(c, D, tr, l_fin, r_fin, y_fin, *, eps_rel=1e-5, price_tol=None, cost_rel=1e-6,
             check_every=1, master_every=0, master_opts=None, kkt_slack=2.0, t_begin=0, t_end=None,
             kkt_ref=None, log_fn=print, name=""):
    """Check a GPU plan (trace ``tr`` with ``y``, final plan l/r/y as host
    arrays) iteration by iteration against the oracle; returns a LockstepLog.

    check_every: re-price every n-th iteration (and the last); master_every:
    run the oracle's master on every n-th checked iteration (0: never);
    price_tol: absolute tolerance on the reported price (default 1e-6 |p_0|);
    t_begin, t_end: check only iterations in [t_begin, t_end) (the state
    before t_begin is rebuilt from the GPU's decisions without checking);
    kkt_ref: the master's KKT scale when t_begin > 0 (|p| of the first
    pricing; by default the oracle's own first price).
    """
    N, R = c.n_beams, c.n_rows
    order = np.asarray(tr["beam"])
    n = len(order)
    ys = np.asarray(tr["y"])
    l_fin = np.asarray(l_fin).astype(np.int64)
    r_fin = np.asarray(r_fin).astype(np.int64)
    t_end = n if t_end is None else min(t_end, n)
    mo = master_opts or O.MasterOpts()
    occ = np.zeros(N, np.uint8)
    l = np.zeros(N * R, np.int64)
    r = np.zeros(N * R, np.int64)
    log = LockstepLog()
    p0 = ref = kkt_ref
    for t in range(t_end):
        k = int(order[t])
        y_t = ys[t].copy()
        lk, rk = l_fin[k * R:(k + 1) * R], r_fin[k * R:(k + 1) * R]
        assert not occ[k], f"iteration {t}: beam {k} opened twice"
        assert np.all(y_t[occ == 0] == 0.0), f"iteration {t}: unoccupied beam with y != 0"
        assert np.all(y_t >= 0.0) and np.all(np.isfinite(y_t))
        checked = t >= t_begin and (t % check_every == 0 or t == n - 1)
        if checked:
            F, gG, dF, dG = _objective(c, D, y_t, l, r, occ)
            # the cost the GPU reported for this state (cost[0]: the empty plan)
            dev = abs(tr["cost"][t] - (F + gG)) / max(abs(F + gG), 1e-300)
            log.max_cost_dev = max(log.max_cost_dev, dev)
            assert dev <= cost_rel, f"iteration {t}: GPU cost {tr['cost'][t]} vs oracle {F + gG}"
            g = D @ dF
            pr = O.price(g, y_t, l, r, occ, c.theta_deg, c.gamma, R, c.n_cols, c.max_leaf_step, c.circular,
                         with_margins=False)
            if p0 is None:
                p0 = ref = abs(pr.price) if pr.price != 0.0 else 1.0
            eps = eps_rel * abs(pr.price)
            ptol = price_tol if price_tol is not None else 1e-6 * p0
            same_beam = pr.beam == k
            if not same_beam:
                cand = [kk for kk in range(N) if not occ[kk]]
                second = min(pr.beam_prices[kk] for kk in cand if kk != pr.beam)
                margin = second - pr.price
                assert margin <= eps and pr.beam_prices[k] - pr.price <= eps, \
                    (f"iteration {t}: GPU beam {k} vs oracle {pr.beam}: margin {margin} > eps {eps} "
                     f"or GPU beam priced {pr.beam_prices[k]} vs best {pr.price}")
                log.excused.append((t, f"beam {k} vs {pr.beam}", margin, eps))
            same_rows = _row_check(c, g, k, lk, rk, l, r, occ, eps, log, t)
            if same_beam and same_rows:
                log.matched += 1
                dp = abs(tr["price"][t] - pr.price)
                log.max_price_dev = max(log.max_price_dev, dp)
                assert dp <= ptol, f"iteration {t}: GPU price {tr['price'][t]} vs oracle {pr.price}"
            log.checked += 1
        # continue from the GPU's decision
        occ[k] = 1
        l[k * R:(k + 1) * R] = lk
        r[k * R:(k + 1) * R] = rk
        y_next = ys[t + 1] if t + 1 < n else np.asarray(y_fin, np.float64)
        if checked and master_every and (log.checked - 1) % master_every == 0 and ref is not None:
            m = O.master(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, R, c.n_cols, l, r, occ,
                         y_t, dataclasses.replace(mo, kkt_ref=ref))
            dev = abs(tr["cost"][t + 1] - (m.F + m.gG)) / max(abs(m.F + m.gG), 1e-300)
            log.max_master_dev = max(log.max_master_dev, dev)
            assert dev <= cost_rel, f"iteration {t}: GPU master cost {tr['cost'][t + 1]} vs oracle {m.F + m.gG}"
            # KKT of the GPU's intensities, evaluated by the oracle
            F, gG, dF, dG = _objective(c, D, y_next, l, r, occ)
            grad = O.beam_sums(D @ dF, l, r, occ, R, c.n_cols) + c.gamma * dG
            v = np.abs(np.minimum(y_next, grad))[occ.astype(bool)]
            kkt = float(v.max()) if v.size else 0.0
            ratio = kkt / (mo.tol_rel * ref)
            log.max_kkt_ratio = max(log.max_kkt_ratio, ratio)
            assert ratio <= kkt_slack, f"iteration {t}: oracle KKT {kkt} at the GPU's y, tol {mo.tol_rel * ref}"
            log.masters += 1
    # the final plan's cost
    if n and t_end == n:
        F, gG, dF, dG = _objective(c, D, np.asarray(y_fin, np.float64), l, r, occ)
        dev = abs(tr["cost"][n] - (F + gG)) / max(abs(F + gG), 1e-300)
        log.max_cost_dev = max(log.max_cost_dev, dev)
        assert dev <= cost_rel, f"final cost {tr['cost'][n]} vs oracle {F + gG}"
    cost = np.asarray(tr["cost"])
    assert np.all(cost[1:] <= cost[:-1] * (1 + 1e-12)), "cost increased across column generation"
    if log_fn:
        log_fn(log.summary(name))
    return log


def deliverable(c, l, r):
    """Row-convex leaf pairs within delta of the neighbouring beam's (the
    invariant column generation keeps when every beam is occupied)."""
    N, R = c.n_beams, c.n_rows
    L = np.asarray(l).reshape(N, R)
    Rr = np.asarray(r).reshape(N, R)
    assert np.all(L <= Rr) and np.all(L >= 0) and np.all(Rr <= c.n_cols)
    if c.max_leaf_step < 0:
        return
    pairs = [(k, k + 1) for k in range(N - 1)] + ([(N - 1, 0)] if c.circular else [])
    for a, b in pairs:
        assert np.all(np.abs(L[a] - L[b]) <= c.max_leaf_step)
        assert np.all(np.abs(Rr[a] - Rr[b]) <= c.max_leaf_step)

