"""Plan variants on one handle (vmat_set_weights) and plans on separate
handles at the same time: a handle given new weights plans exactly as a
handle created with them (both masters); invalid weights leave the handle as
it was; two handles solving concurrently in two threads and streams give the
bits each gives alone."""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses

import numpy as np
import pytest

import casegen
from _cases import preset_case, small_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402
from paper_1005_4396_amd import vmat as V  # noqa: E402


def _opts(mode):
    o = V.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = mode
    o.master = P.master_opts()
    return o


def _variant(c, tab_b):
    w = tab_b[np.minimum(c.label, tab_b.shape[0] - 1)]
    return dataclasses.replace(c, alpha=w[:, 0].copy(), beta=w[:, 1].copy(), T=w[:, 2].copy())


def _plan(prob, mode):
    l, r, occ, y = prob.empty_plan()
    rep, tr = prob.solve(l, r, occ, y, _opts(mode))
    return [l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy(), tr["cost"], tr["beam"]]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", ["small", "tiny36"])
def test_set_weights_plans_as_a_new_handle(name, mode):
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8)) if name == "small" else preset_case("tiny36")
    tab = casegen.variant_table(c, 3, seed=11)
    vb = _variant(c, tab[1])
    fresh = P.Problem.from_case(vb)
    try:
        want = _plan(fresh, mode)
    finally:
        fresh.close()
    prob = P.Problem.from_case(c)
    try:
        _plan(prob, mode)                         # the base weights first (graphs captured on them)
        b0 = prob.device_bytes()
        prob.set_weights(_dev(vb.alpha), _dev(vb.beta), _dev(vb.T))
        got = _plan(prob, mode)
        assert prob.device_bytes() == b0
    finally:
        prob.close()
    for u, v in zip(got, want):
        np.testing.assert_array_equal(u, v)


def test_invalid_weights_leave_the_handle_unchanged():
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    prob = P.Problem.from_case(c)
    try:
        want = _plan(prob, 0)
        bad = c.beta.copy()
        bad[5] = -1.0
        with pytest.raises(V.VmatError) as e:
            prob.set_weights(_dev(c.alpha), _dev(bad), _dev(c.T))
        assert e.value.code == V.VMAT_ERR_INVALID_ARG
        nan_t = c.T.copy()
        nan_t[3] = np.nan
        with pytest.raises(V.VmatError):
            prob.set_weights(_dev(c.alpha), _dev(c.beta), _dev(nan_t))
        # more than 256 distinct triples on a handle holding labels
        assert prob.layout()["weight_labels"] > 0
        many = c.T.copy() + np.arange(c.n_voxels, dtype=np.float32) * 1e-3
        with pytest.raises(V.VmatError) as e:
            prob.set_weights(_dev(c.alpha), _dev(c.beta), _dev(many))
        assert e.value.code == V.VMAT_ERR_UNSUPPORTED
        got = _plan(prob, 0)
    finally:
        prob.close()
    for u, v in zip(got, want):
        np.testing.assert_array_equal(u, v)


def test_concurrent_handles_give_their_own_bits():
    c = preset_case("tiny36")
    tab = casegen.variant_table(c, 4, seed=12)
    variants = [_variant(c, tab[b]) for b in range(4)]
    alone = []
    for vb in variants:
        p = P.Problem.from_case(vb)
        try:
            alone.append(_plan(p, 1))
        finally:
            p.close()
    probs = [P.Problem.from_case(c) for _ in range(2)]
    streams = [torch.cuda.Stream() for _ in range(2)]
    try:
        for p in probs:
            p.reserve_solve()

        def work(t):
            out = {}
            with torch.cuda.stream(streams[t]):
                for b in range(t, 4, 2):
                    vb = variants[b]
                    probs[t].set_weights(_dev(vb.alpha), _dev(vb.beta), _dev(vb.T))
                    out[b] = _plan(probs[t], 1)
            return out
        with cf.ThreadPoolExecutor(2) as ex:
            results = {}
            for r in ex.map(work, range(2)):
                results.update(r)
    finally:
        for p in probs:
            p.close()
    for b in range(4):
        for u, v in zip(results[b], alone[b]):
            np.testing.assert_array_equal(u, v)
