"""vmat_price_noalloc (pricing with the library's static scratch, for
callers that cannot allocate) against vmat_price on a handle with the same
beams: bit for bit, on two calls in a row, the second on a smaller problem;
device memory unchanged by the calls; sizes beyond the scratch rejected."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from _cases import preset_case, small_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402
from paper_1005_4396_amd import vmat as V  # noqa: E402


def _inputs(c, seed):
    """Beamlet prices with exact ties, and a deliverable partial plan built by
    the FP64 reference's own pricing (Sec. 2.2)."""
    rng = np.random.default_rng(seed)
    N, R, C = c.n_beams, c.n_rows, c.n_cols
    g = rng.standard_normal(N * R * C) * (rng.random(N * R * C) < 0.7)
    g[rng.random(N * R * C) < 0.1] = -1.0
    l = np.zeros(N * R, np.int32)
    r = np.zeros(N * R, np.int32)
    occ = np.zeros(N, np.uint8)
    for _ in range(max(1, N // 3)):
        pr = O.price(rng.standard_normal(N * R * C), np.zeros(N), l, r, occ, c.theta_deg, c.gamma, R, C,
                     c.max_leaf_step, c.circular, with_margins=False)
        occ[pr.beam] = 1
        l[pr.beam * R:(pr.beam + 1) * R], r[pr.beam * R:(pr.beam + 1) * R] = pr.l, pr.r
    y = rng.random(N) * 2 * occ
    return g, y, l, r, occ


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def test_noalloc_pricing_matches_handle_pricing_twice():
    cases = [preset_case("tiny36"), small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))]
    probs = [P.Problem.from_case(c) for c in cases]
    try:
        staged = []
        for c, prob in zip(cases, probs):
            g, y, l, r, occ = _inputs(c, 7)
            args = (_dev(g, torch.float64), _dev(y, torch.float64), _dev(l, torch.int32), _dev(r, torch.int32),
                    _dev(occ, torch.uint8))
            ref = prob.price(*args)
            N, R = c.n_beams, c.n_rows
            outs = (torch.full((1 + 2 * R,), -7, dtype=torch.int32, device="cuda"),
                    torch.full((3,), np.nan, dtype=torch.float64, device="cuda"),
                    torch.full((N,), np.nan, dtype=torch.float64, device="cuda"))
            staged.append((c, args, ref, outs, _dev(c.theta_deg, torch.float64)))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        # the larger problem first, then the smaller one: the second call
        # reuses the scratch the first left behind
        for c, args, ref, (ob, op, bp), theta in staged:
            code = V.price_noalloc(theta, c.n_rows, c.n_cols, c.gamma, c.circular, c.max_leaf_step, *args,
                                   ob, op, bp)
            assert code == V.VMAT_OK, V.last_error()
            torch.cuda.synchronize()
            R = c.n_rows
            obh, oph = ob.cpu().numpy(), op.cpu().numpy()
            assert obh[0] == ref.beam >= 0
            np.testing.assert_array_equal(obh[1:1 + R], ref.l)
            np.testing.assert_array_equal(obh[1 + R:], ref.r)
            assert oph[0] == ref.price and oph[1] == ref.margin and oph[2] == ref.row_margin
            np.testing.assert_array_equal(bp.cpu().numpy(), ref.beam_prices)
        assert torch.cuda.mem_get_info()[0] == free0
    finally:
        for p in probs:
            p.close()


def test_noalloc_pricing_rejects_sizes_beyond_its_scratch():
    theta = torch.zeros(4097, dtype=torch.float64, device="cuda")
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    i = torch.zeros(8, dtype=torch.int32, device="cuda")
    u = torch.zeros(8, dtype=torch.uint8, device="cuda")
    code = V.price_noalloc(theta, 1, 4, 0.1, 1, 2, d, d, i, i, u, i, d, None)
    assert code == V.VMAT_ERR_INVALID_ARG and "scratch" in V.last_error()
    theta = torch.zeros(1024, dtype=torch.float64, device="cuda")
    code = V.price_noalloc(theta, 65, 4, 0.1, 1, 2, d, d, i, i, u, i, d, None)   # 66,560 rows
    assert code == V.VMAT_ERR_INVALID_ARG and "scratch" in V.last_error()
