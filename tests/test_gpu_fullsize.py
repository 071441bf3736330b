"""Full plans at the prostate-shaped size (288,000 beamlets, 1,048,576 voxels,
1.09e8 non-zeros) and the head-and-neck-shaped size (432,000 beamlets,
3,538,944 voxels, 3.7e8 non-zeros), checked in lockstep by the FP64 oracle
(Sec. 2.2): the oracle re-prices the GPU's state at every prostate iteration
(both master modes) and at every tenth head-and-neck iteration (FP32 and BF16
storage, the oracle on the same rounded D); it re-runs its own master from
the GPU's state at the start of each checked range; the final plans' costs
and KKT conditions are re-evaluated by the oracle."""
import numpy as np
import pytest

import oracle as O
from _cases import oracle_D, preset_case
from _lockstep import deliverable, lockstep

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402

CHUNKS = [(0, 45), (45, 90), (90, 135), (135, 180)]


def _opts(mode):
    o = P.vmat.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = mode
    o.master = P.master_opts()
    return o


def _first_price(c, D):
    """|p| of the empty plan's best aperture (the master's KKT scale)."""
    N = c.n_beams
    _, dF = O.penalty(np.zeros(c.n_voxels), c.alpha, c.beta, c.T)
    pr = O.price(D @ dF, np.zeros(N), np.zeros(N * c.n_rows, np.int64), np.zeros(N * c.n_rows, np.int64),
                 np.zeros(N, np.uint8), c.theta_deg, c.gamma, c.n_rows, c.n_cols, c.max_leaf_step, c.circular,
                 with_margins=False)
    return abs(pr.price)


def _plan(c, mode, d_store="f32"):
    prob = P.Problem.from_case(c, d_store=d_store)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, _opts(mode))
        return rep, tr, l.cpu().numpy(), r.cpu().numpy(), occ.cpu().numpy(), y.cpu().numpy()
    finally:
        prob.close()


def _final_checks(c, D, rep, l, r, occ, y):
    F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), y, l, r, occ, c.gamma, c.theta_deg,
                                        c.circular, c.n_rows, c.n_cols)
    assert rep.cg_iters == c.n_beams and occ.all()
    assert rep.F + rep.gG == pytest.approx(F + gG, rel=1e-6)
    kkt = np.abs(np.minimum(y, grad)).max()
    assert kkt <= 2e-5 * rep.kkt_ref
    assert np.all(y >= 0)
    deliverable(c, l, r)
    return F + gG, kkt


@pytest.fixture(scope="module")
def prostate():
    c = preset_case("prostate180")
    D = oracle_D(c)
    plans = {mode: _plan(c, mode) for mode in (0, 1)}
    return c, D, plans, _first_price(c, D)


@pytest.mark.parametrize("chunk", CHUNKS, ids=lambda v: f"{v[0]}-{v[1]}")
@pytest.mark.parametrize("mode", [0, 1])
def test_prostate_plan_lockstep(prostate, mode, chunk):
    c, D, plans, p0 = prostate
    rep, tr, l, r, occ, y = plans[mode]
    a, b = chunk
    log = lockstep(c, D, tr, l, r, y, t_begin=a, t_end=b, kkt_ref=p0, master_every=b - a,
                   name=f"prostate mode {mode} iterations {a}-{b}")
    assert log.checked == b - a and log.masters == 1
    if b == c.n_beams:
        cost, kkt = _final_checks(c, D, rep, l, r, occ, y)
        print(f"prostate mode {mode}: cost {rep.F + rep.gG:.9g}, oracle re-evaluation {cost:.9g}, KKT {kkt:.3g} "
              f"(tolerance {1e-5 * rep.kkt_ref:.3g})")


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_headneck_plan_lockstep(fmt):
    """Head-and-neck-shaped plan with the aperture-dose master: every tenth
    iteration re-priced by the oracle on the same stored D."""
    c = preset_case("headneck180")
    vals = c.val if fmt == "f32" else O.bf16_round(c.val)
    D = oracle_D(c, vals)
    rep, tr, l, r, occ, y = _plan(c, 1, d_store=fmt)
    log = lockstep(c, D, tr, l, r, y, check_every=10, kkt_ref=_first_price(c, D), master_every=0,
                   name=f"head-and-neck {fmt}")
    assert log.checked == 19
    cost, kkt = _final_checks(c, D, rep, l, r, occ, y)
    print(f"head-and-neck {fmt}: cost {rep.F + rep.gG:.9g}, oracle re-evaluation {cost:.9g}")
