"""Parity of the HIP library (through the C ABI) with the FP64 reference.

Every expected value comes from ``oracle/`` on the same seeded inputs.
Tolerances: dose, dose derivative and beamlet prices within 1e-6 of the
largest magnitude (FP32 outputs of FP64 accumulations; the only rounding is
the final FP32 store and the FP32 copy of F'(z) gathered by the adjoint);
costs within 1e-9 relative (FP64 throughout); pricing decisions bit-exact on
identical inputs (both sides take them in FP64 with the same summation order).
"""
import math

import numpy as np
import pytest

import oracle as O
from _cases import hand_case, oracle_D, preset_case, random_plan, scatter_case, small_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_ok():
    return torch.cuda.is_available()


if not _gpu_ok():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402


def T(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel_inf(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


SMALL = [
    ("hand", lambda: hand_case()),
    ("small8", lambda: small_case()),
    ("wide64", lambda: small_case(n_beams=5, n_rows=3, n_cols=64, grid=(20, 18, 9))),
    ("open_chain", lambda: small_case(n_beams=9, n_rows=5, n_cols=7, circular=0, max_leaf_step=1, seed=3)),
]


@pytest.fixture(scope="module", params=[(s[0], lay) for s in SMALL for lay in ("tiled", "plain")],
                ids=lambda v: f"{v[0]}-{v[1]}")
def small_prob(request):
    name, layout = request.param
    c = dict(SMALL)[name]()
    prob = P.Problem.from_case(c, layout=layout)
    yield c, oracle_D(c), prob
    prob.close()


# ---------------------------------------------------------------- dose / gradient

def test_dose_matches_oracle(small_prob):
    c, D, prob = small_prob
    for seed in range(4):
        l, r, occ, y = random_plan(c, seed)
        z = prob.dose(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
        zo = O.dose(D, O.fluence(y, l, r, occ, c.n_rows, c.n_cols))
        zg = z.cpu().numpy().astype(np.float64)
        assert rel_inf(zg, zo) <= 1e-6
        assert np.all(np.abs(zg - zo) <= 2.0 ** -24 * np.abs(zo) + 1e-12 * np.abs(zo).max())


def test_dose_fluence_matches_oracle(small_prob):
    c, D, prob = small_prob
    rng = np.random.default_rng(5)
    x = rng.random(c.n_beamlets) * (rng.random(c.n_beamlets) < 0.7)
    z = prob.dose_fluence(T(x, torch.float64)).cpu().numpy()
    assert rel_inf(z, O.dose(D, x)) <= 1e-6


def test_grad_matches_oracle(small_prob):
    c, D, prob = small_prob
    for seed in range(3):
        l, r, occ, y = random_plan(c, 10 + seed)
        out = prob.grad(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
        F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), y, l, r, occ, c.gamma, c.theta_deg,
                                            c.circular, c.n_rows, c.n_cols)
        cost = out["cost"].cpu().numpy()
        assert cost[0] == pytest.approx(F, rel=1e-9, abs=1e-12)
        assert cost[1] == pytest.approx(gG, rel=1e-9, abs=1e-12)
        assert rel_inf(out["z"].cpu().numpy(), z) <= 1e-6
        assert rel_inf(out["dF"].cpu().numpy(), dF) <= 1e-6
        assert rel_inf(out["g"].cpu().numpy(), g) <= 1e-6
        assert rel_inf(out["dfdy"].cpu().numpy(), grad) <= 1e-6


def test_grad_fluence_matches_oracle(small_prob):
    c, D, prob = small_prob
    rng = np.random.default_rng(6)
    x = rng.random(c.n_beamlets) * 2.0
    out = prob.grad_fluence(T(x, torch.float64))
    z = O.dose(D, x)
    F, dF = O.penalty(z, c.alpha, c.beta, c.T)
    assert out["cost"].cpu().numpy()[0] == pytest.approx(F, rel=1e-9)
    assert rel_inf(out["g"].cpu().numpy(), D @ dF) <= 1e-6


def test_runs_are_bitwise_repeatable(small_prob):
    c, D, prob = small_prob
    l, r, occ, y = random_plan(c, 21)
    a = prob.grad(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
    b = prob.grad(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
    for k in ("cost", "z", "dF", "g", "dfdy"):
        assert torch.equal(a[k], b[k])


# ---------------------------------------------------------------- reduced-precision storage

@pytest.mark.parametrize("fmt", ["bf16", "f16", "fp8"])
def test_reduced_precision_dose(fmt):
    c = small_case(n_beams=6, n_rows=4, n_cols=9, grid=(16, 16, 10))
    D = oracle_D(c)
    if fmt == "bf16":
        Dh = oracle_D(c, O.bf16_round(c.val))
    elif fmt == "f16":
        Dh = oracle_D(c, O.fp16_round(c.val))
    else:
        s, q = O.fp8_quantise(c.row_ptr, c.val)
        Dh = oracle_D(c, O.fp8_dequantise(c.row_ptr, s, q))
    prob = P.Problem.from_case(c, d_store=fmt)
    try:
        l, r, occ, y = random_plan(c, 3, p_occ=1.0)
        zg = prob.dose(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
        zg = zg.cpu().numpy().astype(np.float64)
        x = O.fluence(y, l, r, occ, c.n_rows, c.n_cols)
        assert rel_inf(zg, O.dose(Dh, x)) <= 1e-6           # same quantised D: exact up to FP32 store
        z = O.dose(D, x)
        B = O.quantisation_bound(D, Dh, x)
        assert np.all(np.abs(zg - z) <= B + 2.0 ** -23 * np.abs(z) + 1e-12)
        g = prob.grad(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))["g"]
        _, dFh = O.penalty(O.dose(Dh, x), c.alpha, c.beta, c.T)
        assert rel_inf(g.cpu().numpy(), Dh @ dFh) <= 1e-6
    finally:
        prob.close()


# ---------------------------------------------------------------- pricing

def _price_inputs(c, seed):
    rng = np.random.default_rng(seed)
    N, R, C = c.n_beams, c.n_rows, c.n_cols
    g = rng.standard_normal(N * R * C) * (rng.random(N * R * C) < 0.7)   # exact zeros -> ties
    g[rng.random(N * R * C) < 0.1] = -1.0                                  # repeated values
    occ = (rng.random(N) < 0.5).astype(np.uint8)
    l = np.zeros(N * R, np.int32)
    r = np.zeros(N * R, np.int32)
    # a deliverable state: build it by pricing random prices with the reference
    occ_b = np.zeros(N, np.uint8)
    for k in np.flatnonzero(occ):
        pr = O.price(rng.standard_normal(N * R * C), np.zeros(N), l, r, occ_b, c.theta_deg, c.gamma, R, C,
                     c.max_leaf_step, c.circular, with_margins=False)
        kk = pr.beam
        occ_b[kk] = 1
        l[kk * R:(kk + 1) * R], r[kk * R:(kk + 1) * R] = pr.l, pr.r
    y = rng.random(N) * 2 * occ_b
    return g, y, l, r, occ_b


def test_price_bitexact(small_prob):
    c, D, prob = small_prob
    for seed in range(6):
        g, y, l, r, occ = _price_inputs(c, seed)
        if occ.all():
            continue
        ref = O.price(g, y, l, r, occ, c.theta_deg, c.gamma, c.n_rows, c.n_cols, c.max_leaf_step, c.circular)
        out = prob.price(T(g, torch.float64), T(y, torch.float64), T(l, torch.int32), T(r, torch.int32),
                         T(occ, torch.uint8))
        assert out.beam == ref.beam
        np.testing.assert_array_equal(out.l, ref.l)
        np.testing.assert_array_equal(out.r, ref.r)
        assert out.price == ref.price
        assert out.margin == ref.margin
        assert out.row_margin == ref.row_margin
        bp = np.where(occ == 1, np.inf, out.beam_prices)
        np.testing.assert_array_equal(bp, ref.beam_prices)


def test_price_all_occupied_returns_minus_one():
    c = small_case()
    prob = P.Problem.from_case(c)
    try:
        N, R = c.n_beams, c.n_rows
        occ = np.ones(N, np.uint8)
        l = np.zeros(N * R, np.int32)
        r = np.full(N * R, c.n_cols, np.int32)
        out = prob.price(T(np.zeros(c.n_beamlets), torch.float64), T(np.ones(N), torch.float64),
                         T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
        assert out.beam == -1 and math.isinf(out.price)
    finally:
        prob.close()


# ---------------------------------------------------------------- master

def test_master_matches_oracle(small_prob):
    c, D, prob = small_prob
    for seed in range(3):
        l, r, occ, y0 = random_plan(c, 30 + seed, p_occ=0.8)
        opts = O.MasterOpts(max_iter=300, tol_rel=1e-7)
        ref = O.master(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols, l, r, occ,
                       y0, opts)
        yt = T(y0, torch.float64)
        rep = prob.master(T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8), yt,
                          P.master_opts(max_iter=300, tol_rel=1e-7))
        yg = yt.cpu().numpy()
        assert rep.converged == int(ref.converged)
        assert rep.F + rep.gG == pytest.approx(ref.F + ref.gG, rel=1e-9)
        assert rel_inf(yg, ref.y) <= 1e-5
        assert np.all(yg[occ == 0] == 0) and np.all(yg >= 0)
        # KKT of the GPU point, checked by the reference in FP64
        F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), yg, l, r, occ, c.gamma, c.theta_deg,
                                            c.circular, c.n_rows, c.n_cols)
        kkt = np.abs(np.minimum(yg, grad))[occ == 1].max()
        assert kkt <= 1e-7 * rep.kkt_ref * 1.01 + 1e-12
        assert abs(rep.iters - ref.iters) <= 2


def test_master_iteration_cap_reports_not_converged():
    c = small_case()
    prob = P.Problem.from_case(c)
    try:
        l, r, occ, y0 = random_plan(c, 7, p_occ=1.0)
        rep = prob.master(T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8), T(y0, torch.float64),
                          P.master_opts(max_iter=1, tol_rel=1e-14))
        assert rep.converged == 0 and rep.iters == 1
    finally:
        prob.close()


# ---------------------------------------------------------------- full-size case

@pytest.fixture(scope="module")
def prostate():
    c = preset_case("prostate180")
    prob = P.Problem.from_case(c)
    yield c, prob
    prob.close()


def test_prostate_dose_and_gradient_full_size(prostate):
    c, prob = prostate
    D = oracle_D(c)
    l, r, occ, y = random_plan(c, 99, p_occ=1.0, y_scale=1.0)
    out = prob.grad(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
    F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), y, l, r, occ, c.gamma, c.theta_deg,
                                        c.circular, c.n_rows, c.n_cols)
    assert rel_inf(out["z"].cpu().numpy(), z) <= 1e-6
    assert rel_inf(out["g"].cpu().numpy(), g) <= 1e-6
    assert rel_inf(out["dfdy"].cpu().numpy(), grad) <= 1e-6
    cost = out["cost"].cpu().numpy()
    assert cost[0] == pytest.approx(F, rel=1e-9)
    assert cost[1] == pytest.approx(gG, rel=1e-9)


# ---------------------------------------------------------------- tiled layout edge cases

def test_tiled_layout_splits_wide_blocks():
    """12,000 beamlets over 300 voxels: a block of all voxels reaches more
    beamlets than one tile holds, so the builder has to split it."""
    c = scatter_case()
    D = oracle_D(c)
    prob = P.Problem.from_case(c, layout="tiled")
    try:
        for seed in range(2):
            l, r, occ, y = random_plan(c, seed, p_occ=1.0)
            out = prob.grad(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8))
            F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), y, l, r, occ, c.gamma, c.theta_deg,
                                                c.circular, c.n_rows, c.n_cols)
            assert rel_inf(out["z"].cpu().numpy(), z) <= 1e-6
            assert rel_inf(out["g"].cpu().numpy(), g) <= 1e-6
            assert out["cost"].cpu().numpy()[0] == pytest.approx(F, rel=1e-9)
    finally:
        prob.close()


def test_untileable_case_falls_back_or_reports_unsupported():
    """10,000 beamlets onto 64 voxels: no block can fit one tile."""
    c = scatter_case(nb_rows=25, n_cols=40, n_beams=10, nv=64, per_row=1, seed=1)
    with pytest.raises(P.VmatError) as e:
        P.Problem.from_case(c, layout="tiled")
    assert e.value.code == P.vmat.VMAT_ERR_UNSUPPORTED
    prob = P.Problem.from_case(c, layout="auto")       # falls back to the plain layout
    try:
        D = oracle_D(c)
        x = np.random.default_rng(3).random(c.n_beamlets)
        z = prob.dose_fluence(T(x, torch.float64)).cpu().numpy()
        assert rel_inf(z, O.dose(D, x)) <= 1e-6
    finally:
        prob.close()


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
def test_raw_products_tiled_vs_plain(fmt):
    c = small_case(n_beams=7, n_rows=5, n_cols=11, grid=(24, 20, 12), seed=4)
    a = P.Problem.from_case(c, d_store=fmt, layout="tiled")
    b = P.Problem.from_case(c, d_store=fmt, layout="plain")
    try:
        rng = np.random.default_rng(8)
        x = T(rng.random(c.n_beamlets), torch.float64)
        w = T(rng.standard_normal(c.n_voxels).astype(np.float32), torch.float32)
        za, zb = a.forward(x).cpu().numpy(), b.forward(x).cpu().numpy()
        ga, gb = a.adjoint(w).cpu().numpy(), b.adjoint(w).cpu().numpy()
        assert rel_inf(za, zb) <= 1e-13
        assert rel_inf(ga, gb) <= 1e-13
    finally:
        a.close()
        b.close()


# ---------------------------------------------------------------- errors

def test_invalid_data_is_rejected():
    c = small_case()
    val = c.val.copy()
    val[3] = -1.0
    with pytest.raises(P.VmatError) as e:
        P.Problem(c.n_beams, c.n_rows, c.n_cols, c.n_voxels, c.theta_deg, T(c.row_ptr, torch.int64),
                  T(c.col, torch.int32), T(val, torch.float32), T(c.alpha, torch.float32),
                  T(c.beta, torch.float32), T(c.T, torch.float32), c.gamma)
    assert e.value.code == P.vmat.VMAT_ERR_INVALID_ARG
    col = c.col.copy()
    i = int(np.flatnonzero(np.diff(c.row_ptr) >= 2)[0])
    p0 = int(c.row_ptr[i])
    col[p0], col[p0 + 1] = col[p0 + 1], col[p0]
    with pytest.raises(P.VmatError):
        P.Problem(c.n_beams, c.n_rows, c.n_cols, c.n_voxels, c.theta_deg, T(c.row_ptr, torch.int64),
                  T(col, torch.int32), T(c.val, torch.float32), T(c.alpha, torch.float32),
                  T(c.beta, torch.float32), T(c.T, torch.float32), c.gamma)
