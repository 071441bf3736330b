"""Voxel weights of eq. 1 held as one-byte labels into a table of the distinct
(alpha, beta, T) against per-voxel weights: the master and the whole plan give
the same bits, and a case with more distinct triples than labels can hold
uses per-voxel weights and still matches the reference."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
import paper_1005_4396_amd as P
from _cases import oracle_D, random_plan, small_case

pytestmark = pytest.mark.gpu


def _t(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _problem(c, labels, monkeypatch):
    if labels:
        monkeypatch.delenv("VMAT_NO_WEIGHT_LABELS", raising=False)
    else:
        monkeypatch.setenv("VMAT_NO_WEIGHT_LABELS", "1")
    prob = P.Problem.from_case(c)
    monkeypatch.delenv("VMAT_NO_WEIGHT_LABELS", raising=False)
    return prob


def _distinct(c):
    w = np.stack([np.asarray(c.alpha, np.float32), np.asarray(c.beta, np.float32), np.asarray(c.T, np.float32)], 1)
    return np.unique(w.view(np.uint32), axis=0).shape[0]


def test_labels_and_per_voxel_weights_give_identical_bits(monkeypatch):
    c = small_case(n_beams=7, n_rows=4, n_cols=9, grid=(16, 14, 10), seed=5)
    a = _problem(c, True, monkeypatch)
    b = _problem(c, False, monkeypatch)
    try:
        assert a.layout()["weight_labels"] == _distinct(c) > 0
        assert b.layout()["weight_labels"] == 0
        for seed in (41, 42):
            l, r, occ, y0 = random_plan(c, seed, p_occ=0.9)
            ya, yb = _t(y0, torch.float64), _t(y0, torch.float64)
            args = (_t(l, torch.int32), _t(r, torch.int32), _t(occ, torch.uint8))
            ra = a.master(*args, ya, P.master_opts(max_iter=300, tol_rel=1e-7))
            rb = b.master(*args, yb, P.master_opts(max_iter=300, tol_rel=1e-7))
            assert torch.equal(ya, yb)
            assert (ra.iters, ra.n_ls_evals, ra.F, ra.gG) == (rb.iters, rb.n_ls_evals, rb.F, rb.gG)
        plans = []
        for prob in (a, b):
            l, r, occ, y = prob.empty_plan()
            rep, tr = prob.solve(l, r, occ, y)
            plans.append((l.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy(), rep.F, rep.gG, tr["cost"]))
        for u, v in zip(plans[0], plans[1]):
            assert np.array_equal(u, v)
    finally:
        a.close()
        b.close()


def test_many_distinct_weights_use_per_voxel_weights(monkeypatch):
    base = small_case(n_beams=7, n_rows=4, n_cols=9, grid=(16, 14, 10), seed=5)
    T = np.asarray(base.T, np.float32) + np.arange(base.n_voxels, dtype=np.float32) * np.float32(1e-3)
    c = dataclasses.replace(base, T=T)
    assert _distinct(c) > 256
    prob = _problem(c, True, monkeypatch)
    try:
        assert prob.layout()["weight_labels"] == 0
        D = oracle_D(c)
        l, r, occ, y0 = random_plan(c, 43, p_occ=0.9)
        ref = O.master(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols, l, r, occ,
                       y0, O.MasterOpts(max_iter=300, tol_rel=1e-7))
        yt = _t(y0, torch.float64)
        rep = prob.master(_t(l, torch.int32), _t(r, torch.int32), _t(occ, torch.uint8), yt,
                          P.master_opts(max_iter=300, tol_rel=1e-7))
        assert rep.converged == int(ref.converged)
        assert rep.F + rep.gG == pytest.approx(ref.F + ref.gG, rel=1e-9)
        y = yt.cpu().numpy()
        assert np.max(np.abs(y - ref.y)) <= 1e-5 * max(1.0, np.max(np.abs(ref.y)))
    finally:
        prob.close()
