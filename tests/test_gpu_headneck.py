"""Head-and-neck-shaped case (180 beams, 60x40 beamlets, 192x192x96 voxels,
about 3.7e8 non-zeros): dose with D stored as FP32, BF16 and FP8 E4M3 (per-
beamlet scale), FP64 accumulation, against the FP64 reference.

For each reduced format the GPU dose must equal the reference dose of the
same quantised D (up to the FP32 store of the output), stay inside the exact
per-voxel quantisation bound of the unquantised dose, and its relative error
is printed.  BF16 must stay within 1e-3 relative (L2); FP8 is reported.
"""
import numpy as np
import pytest

import oracle as O
from _cases import oracle_D, preset_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402


def T(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_headneck_dose_by_storage_format():
    c = preset_case("headneck180")
    N, R, C = c.n_beams, c.n_rows, c.n_cols
    occ = np.ones(N, np.uint8)
    l = np.zeros(N * R, np.int32)
    r = np.full(N * R, C, np.int32)
    y = np.random.default_rng(11).random(N) + 0.5
    x = O.fluence(y, l, r, occ, R, C)
    D = oracle_D(c)
    z = O.dose(D, x)
    nz = np.linalg.norm(z)
    errs = {}
    for fmt in ("f32", "bf16", "fp8"):
        prob = P.Problem.from_case(c, d_store=fmt)
        try:
            zg = prob.dose(T(y, torch.float64), T(l, torch.int32), T(r, torch.int32),
                           T(occ, torch.uint8)).cpu().numpy().astype(np.float64)
        finally:
            prob.close()
        err_l2 = float(np.linalg.norm(zg - z) / nz)
        err_inf = float(np.abs(zg - z).max() / np.abs(z).max())
        errs[fmt] = (err_l2, err_inf)
        if fmt == "f32":
            assert err_inf <= 1e-6 and err_l2 <= 1e-6
            continue
        if fmt == "bf16":
            Dh = oracle_D(c, O.bf16_round(c.val))
        else:
            s, q = O.fp8_quantise(c.row_ptr, c.val)
            Dh = oracle_D(c, O.fp8_dequantise(c.row_ptr, s, q))
        zh = O.dose(Dh, x)
        assert np.abs(zg - zh).max() <= 1e-6 * np.abs(zh).max()
        B = O.quantisation_bound(D, Dh, x)
        assert np.all(np.abs(zg - z) <= B + 2.0 ** -23 * np.abs(z) + 1e-9)
        del Dh
    print("head-and-neck dose error vs FP64 reference (rel L2, rel inf):", errs)
    assert errs["bf16"][0] <= 1e-3
