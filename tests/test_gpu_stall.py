"""Line-search passes per captured master iteration: with one pass per
replay nearly every iteration's search outlasts its replay, stalls it and
goes on in the next one; the results are the same bits as with three (and
with five or seven)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_1005_4396_amd as P
from _cases import random_plan, small_case

pytestmark = pytest.mark.gpu


def _t(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _run(c, passes, monkeypatch, mode):
    monkeypatch.setenv("VMAT_LS_PASSES", str(passes))
    prob = P.Problem.from_case(c)
    try:
        out = []
        if mode == 0:
            l, r, occ, y0 = random_plan(c, 61, p_occ=0.9)
            y = _t(y0, torch.float64)
            rep = prob.master(_t(l, torch.int32), _t(r, torch.int32), _t(occ, torch.uint8), y,
                              P.master_opts(max_iter=300, tol_rel=1e-7))
            out += [y.cpu().numpy(), np.array([rep.iters, rep.n_ls_evals, rep.F, rep.gG, rep.kkt])]
        o = P.vmat.SolveOpts()
        o.max_cg_iter = 0
        o.master_mode = mode
        o.master = P.master_opts()
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, o)
        out += [l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy(), tr["cost"],
                np.array([rep.F, rep.gG, rep.master_iters, rep.n_ls_evals])]
        return out
    finally:
        prob.close()
        monkeypatch.delenv("VMAT_LS_PASSES", raising=False)


@pytest.mark.parametrize("mode", [0, 1])
def test_stalled_replays_give_the_same_bits(monkeypatch, mode):
    """1, 5 and 7 passes against the default 3; an even count (2) is not
    accepted (the step kernel would read the state buffer it writes) and runs
    the default."""
    c = small_case(n_beams=7, n_rows=4, n_cols=9, grid=(16, 14, 10), seed=5)
    b = _run(c, 3, monkeypatch, mode)
    for passes in (1, 2, 5, 7):
        a = _run(c, passes, monkeypatch, mode)
        for u, v in zip(a, b):
            assert np.array_equal(u, v), passes
