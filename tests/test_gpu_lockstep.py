"""Column-generation plans on the GPU (through the C ABI), checked in lockstep
by the FP64 oracle (Sec. 2.2): at every iteration the oracle re-prices the
GPU's own state and every decision must be the oracle's or an excused
near-tie; the GPU's costs must match the objective at its intensities, and the
oracle's own master from the GPU's state must reach the GPU's cost (1e-6).

Cases: small seeded and hand-built cases, an open chain, both layouts, both
master modes; the tiny parity case (36 beams) with D stored FP32, BF16 and
FP8 (the oracle on the same rounded D); three batched variants."""
import dataclasses

import numpy as np
import pytest

import casegen
import oracle as O
from _cases import hand_case, oracle_D, preset_case, small_case
from _lockstep import deliverable, lockstep

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402


def T(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def solve_opts(mode, max_cg_iter=0):
    o = P.vmat.SolveOpts()
    o.max_cg_iter = max_cg_iter
    o.master_mode = mode
    o.master = P.master_opts()
    return o


def gpu_plan(c, opts, d_store="f32", layout="auto"):
    prob = P.Problem.from_case(c, d_store=d_store, layout=layout)
    try:
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, opts)
        return rep, tr, l.cpu().numpy(), r.cpu().numpy(), occ.cpu().numpy(), y.cpu().numpy()
    finally:
        prob.close()


def rounded_values(c, fmt):
    """The D values the library stores in format fmt (the oracle's rounding)."""
    if fmt == "f32":
        return c.val
    if fmt == "bf16":
        return O.bf16_round(c.val)
    s_, q_ = O.fp8_quantise(c.row_ptr, c.val)
    return O.fp8_dequantise(c.row_ptr, s_, q_)


SMALL = [
    ("hand", lambda: hand_case()),
    ("small8", lambda: small_case()),
    ("wide64", lambda: small_case(n_beams=5, n_rows=3, n_cols=64, grid=(20, 18, 9))),
    ("open_chain", lambda: small_case(n_beams=9, n_rows=5, n_cols=7, circular=0, max_leaf_step=1, seed=3)),
    ("open_free", lambda: small_case(n_beams=10, n_rows=3, n_cols=8, grid=(14, 14, 8), circular=0,
                                     max_leaf_step=-1, seed=3)),
]


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("layout", ["tiled", "plain"])
@pytest.mark.parametrize("name", [n for n, _ in SMALL])
def test_small_plans_lockstep(name, layout, mode):
    c = dict(SMALL)[name]()
    D = oracle_D(c)
    rep, tr, l, r, occ, y = gpu_plan(c, solve_opts(mode), layout=layout)
    assert rep.cg_iters == c.n_beams and occ.all()
    log = lockstep(c, D, tr, l, r, y, master_every=1, name=f"{name}/{layout}/mode {mode}")
    assert log.checked == c.n_beams and log.masters == c.n_beams
    deliverable(c, l, r)
    if mode == 1:
        # one forward per opened aperture, one adjoint per pricing
        assert rep.n_forward == c.n_beams and rep.n_adjoint == c.n_beams


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("mode", [0, 1])
def test_tiny36_lockstep(mode, fmt):
    """The tiny parity plan (36 beams at 10 degrees, 32^3 voxels, ~1e6 nnz), all
    36 iterations in lockstep, with the oracle working on the D the library
    stores (FP32 as given, or rounded to BF16 / FP8 with per-beamlet scales)."""
    c = preset_case("tiny36")
    D = oracle_D(c, rounded_values(c, fmt))
    rep, tr, l, r, occ, y = gpu_plan(c, solve_opts(mode), d_store=fmt)
    assert rep.cg_iters == c.n_beams
    log = lockstep(c, D, tr, l, r, y, master_every=1, name=f"tiny36/{fmt}/mode {mode}")
    assert log.checked == c.n_beams and log.masters == c.n_beams
    deliverable(c, l, r)
    if fmt == "f32" and mode == 0:
        # free-running comparison, reported: the oracle's own plan from the
        # empty state, first divergence and final-cost gap
        ref = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                      c.max_leaf_step)
        R = c.n_rows
        first = next((t for t in range(c.n_beams)
                      if ref.order[t] != tr["beam"][t]
                      or not np.array_equal(ref.apertures[t][0], l[ref.order[t] * R:(ref.order[t] + 1) * R])
                      or not np.array_equal(ref.apertures[t][1], r[ref.order[t] * R:(ref.order[t] + 1) * R])),
                     None)
        gap = (rep.F + rep.gG - ref.costs[-1]) / ref.costs[-1]
        print(f"tiny36 free-running: first divergence at iteration {first}, final cost gap {gap:.3g}")


def _variant_case(c, tab, b):
    w = tab[b][np.minimum(c.label, tab.shape[1] - 1)].astype(np.float32)
    return dataclasses.replace(c, alpha=w[:, 0].copy(), beta=w[:, 1].copy(), T=w[:, 2].copy())


@pytest.mark.parametrize("name,B", [("small", 5), ("tiny36", 3)])
def test_batched_plans_lockstep(name, B):
    """Batched column generation (variants of eq. 1 sharing D): every variant's
    plan in lockstep with the oracle on that variant's weights."""
    c = small_case(n_beams=6, n_rows=4, n_cols=8, grid=(16, 16, 10)) if name == "small" else preset_case("tiny36")
    D = oracle_D(c)
    tab = casegen.variant_table(c, B, seed=11)
    prob = P.Problem.from_case(c)
    try:
        prob.reserve_batched(B)
        (l, r, occ, y), reps, trs, cnt = prob.solve_batched(T(c.label, torch.uint8), T(tab, torch.float32))
        lg, rg, yg = l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy()
    finally:
        prob.close()
    assert cnt[0] >= 1 and cnt[1] >= 1
    for b in range(B):
        cb = _variant_case(c, tab, b)
        assert reps[b].cg_iters == c.n_beams
        log = lockstep(cb, D, trs[b], lg[b], rg[b], yg[b], master_every=1, name=f"{name} variant {b}")
        assert log.checked == c.n_beams
        deliverable(cb, lg[b], rg[b])
