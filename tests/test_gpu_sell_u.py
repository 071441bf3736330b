"""The sliced products with 2, 4 or 8 quads in flight per lane (the handle
picks 4 or 8 by timing at creation; VMAT_SELL_U overrides) give the same
bits: every lane sums its quads in order."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_1005_4396_amd as P
from _cases import small_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d_store", ["f32", "bf16", "fp8"])
def test_quads_in_flight_do_not_change_the_bits(monkeypatch, d_store):
    c = small_case(n_beams=12, n_rows=6, n_cols=10, grid=(20, 18, 12), seed=3)
    prob = P.Problem.from_case(c, d_store=d_store)
    try:
        assert prob.layout()["tiled"] == 1
        rng = np.random.default_rng(5)
        x = torch.from_numpy(rng.random(c.n_beamlets)).cuda()
        w = torch.from_numpy(rng.standard_normal(c.n_voxels).astype(np.float32)).cuda()
        out = {}
        for u in ("2", "4", "8"):
            monkeypatch.setenv("VMAT_SELL_U", u)
            z = torch.empty(c.n_voxels, dtype=torch.float64, device="cuda")
            g = torch.empty(c.n_beamlets, dtype=torch.float64, device="cuda")
            prob.forward(x, z)
            prob.adjoint(w, g)
            torch.cuda.synchronize()
            out[u] = (z.cpu().numpy(), g.cpu().numpy())
        monkeypatch.delenv("VMAT_SELL_U")
        for u in ("2", "8"):
            assert np.array_equal(out[u][0], out["4"][0])
            assert np.array_equal(out[u][1], out["4"][1])
    finally:
        prob.close()
