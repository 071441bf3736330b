"""Degenerate problems against the FP64 reference: an empty D, a single
beamlet, leaves that may not move between angles, and an objective whose
optimum is no dose at all.  Both master modes."""
import dataclasses

import numpy as np
import pytest

import casegen
import oracle as O
from _cases import oracle_D, small_case
from _lockstep import deliverable, lockstep

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


def _empty_d():
    c = small_case(n_beams=6, n_rows=3, n_cols=5, grid=(10, 10, 6))
    return dataclasses.replace(c, row_ptr=np.zeros_like(c.row_ptr), col=np.zeros(0, np.int32),
                               val=np.zeros(0, np.float32))


def _single_beamlet():
    return casegen.make_case(casegen.tiny_case(n_beams=1, n_rows=1, n_cols=1, grid=(8, 8, 6), thr=0.2))


def _frozen_leaves():
    return small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8), max_leaf_step=0, seed=5)


def _no_dose_wanted():
    c = small_case(n_beams=6, n_rows=3, n_cols=6, grid=(12, 12, 8))
    return dataclasses.replace(c, alpha=np.zeros_like(c.alpha), T=np.zeros_like(c.T),
                               beta=np.full_like(c.beta, 0.5))


CASES = [("empty_d", _empty_d), ("single_beamlet", _single_beamlet), ("frozen_leaves", _frozen_leaves),
         ("no_dose_wanted", _no_dose_wanted)]


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", [n for n, _ in CASES])
def test_degenerate_plans_match_oracle(name, mode):
    c = dict(CASES)[name]()
    D = oracle_D(c)
    prob = P.Problem.from_case(c)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, _opts(mode))
        lg, rg, yg = l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy()
        z = prob.dose(y, l, r, occ).cpu().numpy().astype(np.float64)
    finally:
        prob.close()
    assert rep.cg_iters == c.n_beams
    log = lockstep(c, D, tr, lg, rg, yg, master_every=1, name=f"{name}/mode {mode}")
    assert log.checked == c.n_beams
    deliverable(c, lg, rg)
    z_ref = O.dose(D, O.fluence(yg, lg, rg, np.ones(c.n_beams, np.uint8), c.n_rows, c.n_cols))
    assert np.abs(z - z_ref).max() <= 1e-6 * max(np.abs(z_ref).max(), 1e-300)
    if name in ("empty_d", "no_dose_wanted"):
        np.testing.assert_array_equal(yg, np.zeros(c.n_beams))
        assert not z.any()
    if name == "frozen_leaves":
        L, Rr = lg.reshape(c.n_beams, c.n_rows), rg.reshape(c.n_beams, c.n_rows)
        assert np.all(L == L[0]) and np.all(Rr == Rr[0])
