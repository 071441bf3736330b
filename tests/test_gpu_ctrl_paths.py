"""The single-workgroup gradient/direction step of the master in its two
forms (per-beam vectors in LDS, or read and written in global memory between
its phases) gives the same bits, for both masters."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_1005_4396_amd as P
from _cases import random_plan, small_case

pytestmark = pytest.mark.gpu


def _t(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _run(c, global_form, monkeypatch, mode):
    if global_form:
        monkeypatch.setenv("VMAT_GRAD_DIR_GLOBAL", "1")
    else:
        monkeypatch.delenv("VMAT_GRAD_DIR_GLOBAL", raising=False)
    prob = P.Problem.from_case(c)
    try:
        out = []
        if mode == 0:
            l, r, occ, y0 = random_plan(c, 51, p_occ=0.9)
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
        out += [l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy(), tr["cost"], np.array([rep.F, rep.gG])]
        return out
    finally:
        prob.close()
        monkeypatch.delenv("VMAT_GRAD_DIR_GLOBAL", raising=False)


@pytest.mark.parametrize("mode", [0, 1])
def test_lds_and_global_control_forms_agree_bitwise(monkeypatch, mode):
    c = small_case(n_beams=7, n_rows=4, n_cols=9, grid=(16, 14, 10), seed=5)
    a = _run(c, False, monkeypatch, mode)
    b = _run(c, True, monkeypatch, mode)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
