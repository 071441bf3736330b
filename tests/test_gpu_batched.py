"""Plan variants sharing one D: products with many right-hand sides and the
batched cost/gradient, against the FP64 reference applied column by column.

Product variants (tile width x rows per wave) change no result: every
variant gives the same bits.
"""
import numpy as np
import pytest

import casegen
import oracle as O
from _cases import oracle_D, preset_case, small_case
from _lockstep import lockstep

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402

VARIANTS = P.vmat.SPMM_VARIANTS


def T(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _inputs(c, B, seed):
    rng = np.random.default_rng(seed)
    X = rng.random((c.n_beamlets, B)).astype(np.float32)
    X[rng.random(c.n_beamlets) < 0.3] = 0.0
    return X


def _reference(D, c, X, tab):
    """Column-by-column eq. 1 with per-variant weights, FP64."""
    B = X.shape[1]
    lab = np.minimum(c.label, tab.shape[1] - 1)
    Z = np.empty((c.n_voxels, B))
    dF = np.empty((c.n_voxels, B))
    cost = np.empty(B)
    for b in range(B):
        Z[:, b] = O.dose(D, X[:, b].astype(np.float64))
        w = tab[b].astype(np.float64)[lab]
        cost[b], dF[:, b] = O.penalty(Z[:, b], w[:, 0], w[:, 1], w[:, 2])
    return Z, dF, cost


CASES = [("small", lambda: small_case(n_beams=6, n_rows=4, n_cols=8, grid=(16, 16, 10))),
         ("tiny36", lambda: preset_case("tiny36"))]


@pytest.mark.parametrize("layout", ["tiled", "plain"])
@pytest.mark.parametrize("name,B", [("small", 1), ("small", 5), ("small", 64), ("tiny36", 64), ("tiny36", 13)])
def test_batched_products_and_cost(name, B, layout):
    c = dict(CASES)[name]()
    D = oracle_D(c)
    X = _inputs(c, B, B)
    tab = casegen.variant_table(c, B, seed=B)
    Z, dF, cost = _reference(D, c, X, tab)
    prob = P.Problem.from_case(c, layout=layout)
    try:
        if layout == "tiled":
            prob.reserve_batched(B)   # the adjoint's slot sums
        out = prob.grad_batched(T(c.label, torch.uint8), T(tab, torch.float32), T(X, torch.float32))
        Zg = out["Z"].cpu().numpy()
        assert rel_inf(Zg, Z) <= 1e-12
        assert np.allclose(out["cost"].cpu().numpy(), cost, rtol=1e-9, atol=0)
        dFg = out["dF"].cpu().numpy().astype(np.float64)
        assert np.abs(dFg - dF).max() <= 2.0 ** -23 * np.abs(dF).max() * 4
        # adjoint of the library's own dF against the reference product
        G_ref = D @ dFg
        assert rel_inf(out["G"].cpu().numpy(), G_ref) <= 1e-12
        # every variant gives the same bits
        Xt, Wt = T(X, torch.float32), out["dF"]
        ref_z, ref_g = None, None
        for v in VARIANTS:
            prob.set_batched_tile(B, v, v)
            z = prob.forward_batched(Xt).cpu().numpy()
            g = prob.adjoint_batched(Wt).cpu().numpy()
            if ref_z is None:
                ref_z, ref_g = z, g
            assert np.array_equal(z, ref_z) and np.array_equal(g, ref_g), v
        fw, aw, times = prob.tune_batched(B, reps=2)
        assert fw in VARIANTS and aw in VARIANTS and fw[0] <= max(B, 1) * 2 and aw[0] <= max(B, 1) * 2
        assert np.isfinite(times["forward"][fw]) and np.isfinite(times["adjoint"][aw])
        assert np.array_equal(prob.forward_batched(Xt).cpu().numpy(), ref_z)
    finally:
        prob.close()


@pytest.mark.parametrize("fmt", ["bf16", "f16", "fp8"])
def test_batched_reduced_precision(fmt):
    """Every product variant on the tiled layout with D stored in fmt (the
    forward variants with 4, 8 or 16 lanes per row take the quads through
    lane broadcasts of the raw 1-, 2- or 4-dword bits): the same bits for all
    variants, within 1e-6 of the FP64 product of the same rounded D."""
    c = small_case(n_beams=6, n_rows=4, n_cols=8, grid=(16, 16, 10))
    if fmt == "fp8":
        s, q = O.fp8_quantise(c.row_ptr, c.val)
        vals = O.fp8_dequantise(c.row_ptr, s, q)
    else:
        vals = O.bf16_round(c.val) if fmt == "bf16" else O.fp16_round(c.val)
    D = oracle_D(c, vals)
    B = 64
    X = _inputs(c, B, 7)
    W = np.random.default_rng(8).standard_normal((c.n_voxels, B)).astype(np.float32)
    prob = P.Problem.from_case(c, d_store=fmt)
    try:
        assert prob.layout()["tiled"] == 1
        prob.reserve_batched(B)   # the tiled adjoint's slot sums
        Xt, Wt = T(X, torch.float32), T(W, torch.float32)
        out = []
        for v in VARIANTS:
            prob.set_batched_tile(B, v, v)
            out.append((v, prob.forward_batched(Xt).cpu().numpy(), prob.adjoint_batched(Wt).cpu().numpy()))
    finally:
        prob.close()
    _, Z0, G0 = out[0]
    assert rel_inf(Z0, D.T @ X.astype(np.float64)) <= 1e-6
    assert rel_inf(G0, D @ W.astype(np.float64)) <= 1e-6
    for v, Zg, Gg in out[1:]:
        assert np.array_equal(Zg, Z0) and np.array_equal(Gg, G0), v


def test_batched_prostate_full_size():
    """64 variants of the prostate-shaped problem: sampled voxel and beamlet
    rows against the reference, costs against the reference on all voxels."""
    c = preset_case("prostate180")
    D = oracle_D(c)
    B = 64
    X = _inputs(c, B, 3)
    tab = casegen.variant_table(c, B, seed=3)
    prob = P.Problem.from_case(c)
    try:
        prob.reserve_batched(B)
        prob.tune_batched(B, reps=2)
        out = prob.grad_batched(T(c.label, torch.uint8), T(tab, torch.float32), T(X, torch.float32))
        Zg, dFg = out["Z"].cpu().numpy(), out["dF"].cpu().numpy().astype(np.float64)
        Gg, cost = out["G"].cpu().numpy(), out["cost"].cpu().numpy()
    finally:
        prob.close()
    rng = np.random.default_rng(4)
    Dt = D.T.tocsr()
    vox = rng.choice(c.n_voxels, 4096, replace=False)
    Zs = Dt[vox] @ X.astype(np.float64)
    assert rel_inf(Zg[vox], Zs) <= 1e-12
    rows = rng.choice(c.n_beamlets, 4096, replace=False)
    Gs = D[rows] @ dFg
    assert rel_inf(Gg[rows], Gs) <= 1e-12
    lab = c.label
    for b in range(0, B, 9):
        w = tab[b].astype(np.float64)[lab]
        Zb = O.dose(D, X[:, b].astype(np.float64))
        Fb, _ = O.penalty(Zb, w[:, 0], w[:, 1], w[:, 2])
        assert cost[b] == pytest.approx(Fb, rel=1e-9)


# ---------------------------------------------------------------- batched solves

def _variant_weights(c, tab, b):
    w = tab[b][np.minimum(c.label, tab.shape[1] - 1)]
    return w[:, 0].copy(), w[:, 1].copy(), w[:, 2].copy()


def test_batched_solve_prostate_first_iterations():
    """Two variants of the prostate-shaped problem, four column-generation
    iterations each, in lockstep with the oracle on each variant's weights."""
    import dataclasses
    c = preset_case("prostate180")
    D = oracle_D(c)
    B, iters = 2, 4
    tab = casegen.variant_table(c, B, seed=12)
    opts = P.vmat.SolveOpts()
    opts.max_cg_iter = iters
    opts.master = P.master_opts()
    prob = P.Problem.from_case(c)
    try:
        prob.reserve_batched(B)
        (l, r, occ, y), reps, trs, cnt = prob.solve_batched(T(c.label, torch.uint8), T(tab, torch.float32), opts)
        lg, rg, yg = l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy()
    finally:
        prob.close()
    for b in range(B):
        al, be, tt = _variant_weights(c, tab, b)
        cb = dataclasses.replace(c, alpha=al.astype(np.float32), beta=be.astype(np.float32), T=tt.astype(np.float32))
        assert reps[b].cg_iters == iters
        log = lockstep(cb, D, trs[b], lg[b], rg[b], yg[b], master_every=2, name=f"prostate variant {b}")
        assert log.checked == iters


def test_batched_solve_graph_replay_matches_direct_launches(monkeypatch):
    """The captured lockstep iterations give the same bits as the same kernels
    launched one by one."""
    c = dict(CASES)["tiny36"]()
    B = 4
    tab = casegen.variant_table(c, B, seed=21)
    prob = P.Problem.from_case(c)
    try:
        prob.reserve_batched(B)
        out = []
        for no_graph in (False, True):
            if no_graph:
                monkeypatch.setenv("VMAT_NO_GRAPH", "1")
            else:
                monkeypatch.delenv("VMAT_NO_GRAPH", raising=False)
            (l, r, occ, y), reps, trs, cnt = prob.solve_batched(T(c.label, torch.uint8), T(tab, torch.float32))
            out.append((y.cpu().numpy(), l.cpu().numpy(), r.cpu().numpy(), trs, cnt))
    finally:
        prob.close()
    (y0, l0, r0, t0, c0), (y1, l1, r1, t1, c1) = out
    assert c0 == c1
    np.testing.assert_array_equal(y0, y1)
    np.testing.assert_array_equal(l0, l1)
    np.testing.assert_array_equal(r0, r1)
    for a, b in zip(t0, t1):
        np.testing.assert_array_equal(a["cost"], b["cost"])
        np.testing.assert_array_equal(a["beam"], b["beam"])


@pytest.mark.parametrize("fmt", ["f32", "fp8"])
def test_batched_tiled_adjoint_after_reserve(fmt):
    """With the batched state reserved, the adjoint runs over the tiled slot
    rows: same result as the reference product up to rounding."""
    c = dict(CASES)["tiny36"]()
    if fmt == "fp8":
        s_, q_ = O.fp8_quantise(c.row_ptr, c.val)
        D = oracle_D(c, O.fp8_dequantise(c.row_ptr, s_, q_))
    else:
        D = oracle_D(c)
    B = 64
    W = np.random.default_rng(31).standard_normal((c.n_voxels, B)).astype(np.float32)
    prob = P.Problem.from_case(c, d_store=fmt)
    try:
        prob.set_batched_tile(B, (64, 4), (64, 4))
        G_plain = prob.adjoint_batched(T(W, torch.float32)).cpu().numpy()
        prob.reserve_batched(B)
        G_tiled = prob.adjoint_batched(T(W, torch.float32)).cpu().numpy()
        G_again = prob.adjoint_batched(T(W, torch.float32)).cpu().numpy()
    finally:
        prob.close()
    ref = D @ W.astype(np.float64)
    assert rel_inf(G_tiled, ref) <= 1e-12
    assert rel_inf(G_tiled, G_plain) <= 1e-13
    assert np.array_equal(G_tiled, G_again)
