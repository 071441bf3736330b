"""Plan contexts (vmat_create_plan): handles that read another handle's
layouts of D and own everything else.  A plan on a context gives the same
bits as the same plan on the handle that owns D, contexts hold no copy of D,
the owner outlives its contexts, and contexts on separate streams run plans
concurrently without touching each other's state."""
import concurrent.futures as cf

import numpy as np
import pytest

import casegen
from _cases import preset_case, small_case

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


def _weights(c, seed):
    """One objective variant of the case (device float32 alpha, beta, T)."""
    tab = casegen.variant_table(c, 1, seed=seed)[0]
    lab = np.minimum(c.label, tab.shape[0] - 1)
    return [torch.as_tensor(np.ascontiguousarray(tab[lab][:, q], dtype=np.float32), device="cuda") for q in range(3)]


def _plan(prob, mode):
    if mode == 1:
        prob.reserve_solve()
    l, r, occ, y = prob.empty_plan()
    rep, tr = prob.solve(l, r, occ, y, _opts(mode))
    return [l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy(), tr["cost"], tr["beam"],
            np.array([rep.F, rep.gG, rep.master_iters])]


def _same(a, b):
    assert len(a) == len(b)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("layout", ["tiled", "plain"])
@pytest.mark.parametrize("mode", [0, 1])
def test_context_plan_matches_owner(mode, layout):
    """A context with a second objective gives the bits the owner gives with
    that objective; the owner's own plan afterwards is unchanged."""
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    src = P.Problem.from_case(c, layout=layout)
    ctx = src.new_plan()
    assert ctx.layout() == src.layout() and src.layout()["tiled"] == (layout == "tiled")
    try:
        base = _plan(src, mode)
        w = _weights(c, 11)
        ctx.set_weights(*w)
        on_ctx = _plan(ctx, mode)
        _same(_plan(src, mode), base)          # the owner's weights are its own
        src.set_weights(*w)
        _same(_plan(src, mode), on_ctx)
    finally:
        ctx.close()
        src.close()


def test_context_products_and_master_match_owner():
    """Single and 64-wide products, the gradient and the master on a context
    against the owner (tiled layout: the slot sums are each handle's own)."""
    c = preset_case("tiny36")
    src = P.Problem.from_case(c)
    ctx = src.new_plan()
    try:
        assert src.layout()["tiled"] == 1 and ctx.layout() == src.layout()
        rng = np.random.default_rng(3)
        x = torch.as_tensor(rng.random(c.n_beamlets), device="cuda")
        w = torch.as_tensor(rng.standard_normal(c.n_voxels).astype(np.float32), device="cuda")
        for p in (src, ctx):
            p.reserve_batched(64)
        X = torch.as_tensor(rng.random((c.n_beamlets, 64)).astype(np.float32), device="cuda")
        W = torch.as_tensor(rng.standard_normal((c.n_voxels, 64)).astype(np.float32), device="cuda")
        out = []
        for p in (src, ctx):
            l, r, occ, y = p.empty_plan()
            occ.fill_(1)
            r.fill_(c.n_cols)
            y.fill_(0.5)
            rep = p.master(l, r, occ, y, P.master_opts(max_iter=50))
            out.append([p.forward(x).cpu().numpy(), p.adjoint(w).cpu().numpy(),
                        p.forward_batched(X).cpu().numpy(), p.adjoint_batched(W).cpu().numpy(),
                        y.cpu().numpy(), np.array([rep.iters, rep.F, rep.gG])])
        _same(out[0], out[1])
    finally:
        ctx.close()
        src.close()


def test_context_holds_no_copy_of_D():
    """On the prostate-shaped case the owner holds D's layouts (over 2 GB);
    a context's bytes are its plan state, and creating it takes about that
    much device memory (allocation granularity and the captured iteration
    aside)."""
    c = preset_case("prostate180")
    src = P.Problem.from_case(c)
    try:
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        ctx = src.new_plan()
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        try:
            nb, nv, S = c.n_beamlets, c.n_voxels, ctx.layout()["slots"]
            b = ctx.device_bytes()
            assert 37 * nv + 16 * nb + 8 * S <= b <= 37 * nv + 16 * nb + 8 * S + 64 * 2**20
            assert src.device_bytes() > 2 * 2**30 and b < src.device_bytes() / 10
            assert free0 - free1 < b + 256 * 2**20
        finally:
            ctx.close()
    finally:
        src.close()


def test_owner_outlives_its_contexts():
    """Destroying the owner while a context (or a context of a context)
    reads its D is refused and frees nothing; once they are gone it works."""
    c = small_case(n_beams=6, n_rows=3, n_cols=5, grid=(10, 10, 6))
    src = P.Problem.from_case(c)
    ctx = src.new_plan()
    ctx2 = ctx.new_plan()
    with pytest.raises(P.vmat.VmatError) as e:
        src.close()
    assert e.value.code == P.vmat.VMAT_ERR_INVALID_ARG
    _same(_plan(ctx2, 0), _plan(src, 0))       # the owner still works
    ctx.close()
    with pytest.raises(P.vmat.VmatError):
        src.close()
    ctx2.close()
    src.close()


def test_contexts_run_plans_concurrently():
    """Four contexts, each with its own objective and stream, run their plans
    (both masters) at the same time: every plan equals the same plan run alone
    on the owner."""
    c = preset_case("tiny36")
    src = P.Problem.from_case(c)
    ctxs = [src.new_plan() for _ in range(4)]
    streams = [torch.cuda.Stream() for _ in ctxs]
    ws = [_weights(c, 20 + t) for t in range(len(ctxs))]
    try:
        alone = []
        for t, w in enumerate(ws):
            src.set_weights(*w)
            alone.append([_plan(src, 0), _plan(src, 1)])
        for p, w in zip(ctxs, ws):
            p.set_weights(*w)
            p.reserve_solve()
        torch.cuda.synchronize()

        def work(t):
            with torch.cuda.stream(streams[t]):
                return [_plan(ctxs[t], 0), _plan(ctxs[t], 1)]
        with cf.ThreadPoolExecutor(len(ctxs)) as ex:
            together = list(ex.map(work, range(len(ctxs))))
        for a, b in zip(together, alone):
            _same(a[0], b[0])
            _same(a[1], b[1])
    finally:
        for p in ctxs:
            p.close()
        src.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_solve_variants_matches_plans_one_by_one(mode):
    """vmat_solve_variants (five variants, three workers) gives each variant
    the plan vmat_solve gives on the owner with that variant's weights, and
    leaves the owner's own weights as they were."""
    c = preset_case("tiny36")
    B = 5
    tab = casegen.variant_table(c, B, seed=7)
    lab = np.minimum(c.label, tab.shape[1] - 1)
    src = P.Problem.from_case(c)
    try:
        before = _plan(src, mode)
        reps, l, r, occ, y = src.solve_variants(torch.as_tensor(c.label, device="cuda"),
                                                torch.as_tensor(tab, device="cuda"), K=3, opts=_opts(mode))
        _same(_plan(src, mode), before)
        for b in range(B):
            src.set_weights(*[torch.as_tensor(np.ascontiguousarray(tab[b][lab][:, q]), device="cuda")
                              for q in range(3)])
            one = _plan(src, mode)
            np.testing.assert_array_equal(l[b].cpu().numpy(), one[0])
            np.testing.assert_array_equal(r[b].cpu().numpy(), one[1])
            np.testing.assert_array_equal(y[b].cpu().numpy(), one[2])
            assert occ[b].cpu().numpy().all()
            assert [reps[b].F, reps[b].gG, reps[b].master_iters] == list(one[5])
    finally:
        src.close()


def test_solve_variants_worker_counts():
    """K outside [1, 16] is rejected; more workers than variants run one
    variant each (default options: the master that streams D)."""
    c = small_case(n_beams=6, n_rows=3, n_cols=5, grid=(10, 10, 6))
    tabn = casegen.variant_table(c, 2, seed=1)
    tab = torch.as_tensor(tabn, device="cuda")
    label = torch.as_tensor(c.label, device="cuda")
    lab = np.minimum(c.label, tabn.shape[1] - 1)
    src = P.Problem.from_case(c)
    try:
        for K in (0, 17):
            with pytest.raises(P.vmat.VmatError) as e:
                src.solve_variants(label, tab, K=K)
            assert e.value.code == P.vmat.VMAT_ERR_INVALID_ARG
        reps, l, r, occ, y = src.solve_variants(label, tab, K=4)
        for b in range(2):
            src.set_weights(*[torch.as_tensor(np.ascontiguousarray(tabn[b][lab][:, q]), device="cuda")
                              for q in range(3)])
            one = _plan(src, 0)
            np.testing.assert_array_equal(y[b].cpu().numpy(), one[2])
            assert reps[b].cg_iters == c.n_beams
    finally:
        src.close()
