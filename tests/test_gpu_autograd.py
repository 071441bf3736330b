"""Differentiable dose + cost (torch.autograd) against the FP64 reference.

The backward is the library's adjoint product.  Checked against (a) the
reference gradient over all coordinates and (b) central finite differences
of the reference objective (h = 1e-3), evaluated incrementally over the
support of the perturbed coordinate.  F is piecewise quadratic, so central
differences are exact except where the perturbation moves a voxel across
its threshold; for those coordinates the error is bounded analytically.
"""
import numpy as np
import pytest

import oracle as O
from _cases import oracle_D, preset_case, random_plan, small_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1005_4396_amd as P  # noqa: E402

H = 1e-3


def T(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _fd_along(z, a_idx, a_val, alpha, beta, Tt):
    """Central difference of F(z + t a) at t = 0 over the support of a, and an
    analytic bound of its error at threshold crossings."""
    zs = z[a_idx]
    al, be, tt = alpha[a_idx].astype(float), beta[a_idx].astype(float), Tt[a_idx].astype(float)
    Fp, _ = O.penalty(zs + H * a_val, al, be, tt)
    Fm, _ = O.penalty(zs - H * a_val, al, be, tt)
    fd = (Fp - Fm) / (2 * H)
    cross = (np.minimum(zs - H * np.abs(a_val), zs + H * np.abs(a_val)) < tt) & \
            (np.maximum(zs - H * np.abs(a_val), zs + H * np.abs(a_val)) > tt)
    bound = float(np.sum((np.maximum(al, be) * H * a_val ** 2)[cross])) * 2.0
    return fd, bound


def _check_fluence(c, D, prob, n_coords, seed):
    rng = np.random.default_rng(seed)
    x = rng.random(c.n_beamlets) + 0.5
    xt = T(x, torch.float64).requires_grad_(True)
    cost = P.fluence_cost(prob, xt)
    cost.backward()
    g = xt.grad.cpu().numpy()
    z = O.dose(D, x)
    F, dF = O.penalty(z, c.alpha, c.beta, c.T)
    g_ref = D @ dF
    assert float(cost.detach()) == pytest.approx(F, rel=1e-9)
    scale = np.abs(g_ref).max()
    assert np.max(np.abs(g - g_ref)) <= 1e-6 * scale
    rows = rng.choice(np.flatnonzero(np.diff(c.row_ptr) > 0), n_coords, replace=False)
    for i in rows:
        a, b = c.row_ptr[i], c.row_ptr[i + 1]
        fd, bound = _fd_along(z, c.col[a:b], D.data[a:b], c.alpha, c.beta, c.T)
        assert abs(g[i] - fd) <= 1e-6 * scale + bound + 1e-9 * abs(fd), (i, g[i], fd, bound)


def _check_apertures(c, D, prob, seed):
    l, r, occ, y = random_plan(c, seed, p_occ=1.0, y_scale=1.0)
    y = y + 0.5 * occ
    yt = T(y, torch.float64).requires_grad_(True)
    lt, rt, ot = T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8)
    cost = P.aperture_cost(prob, yt, lt, rt, ot)
    cost.backward()
    gy = yt.grad.cpu().numpy()
    F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), y, l, r, occ, c.gamma, c.theta_deg,
                                        c.circular, c.n_rows, c.n_cols)
    assert float(cost.detach()) == pytest.approx(F + gG, rel=1e-9)
    scale = np.abs(grad).max()
    assert np.max(np.abs(gy - grad)) <= 1e-6 * scale
    N, R, C = c.n_beams, c.n_rows, c.n_cols
    mask = O.aperture_mask(l, r, occ, R, C).reshape(N, R * C)
    for k in range(N):
        ak = np.asarray(D[k * R * C:(k + 1) * R * C][mask[k]].sum(axis=0)).ravel()
        idx = np.flatnonzero(ak)
        fd, bound = _fd_along(z, idx, ak[idx], c.alpha, c.beta, c.T)
        e = np.zeros(N)
        e[k] = H
        Gp, _ = O.smoothing(y + e, c.theta_deg, c.circular)
        Gm, _ = O.smoothing(y - e, c.theta_deg, c.circular)
        fd += c.gamma * (Gp - Gm) / (2 * H)
        assert abs(gy[k] - fd) <= 1e-6 * scale + bound + 1e-9 * abs(fd), (k, gy[k], fd, bound)


def test_autograd_small():
    c = small_case(n_beams=6, n_rows=4, n_cols=8, grid=(16, 16, 10))
    D = oracle_D(c)
    prob = P.Problem.from_case(c)
    try:
        _check_fluence(c, D, prob, 40, 1)
        _check_apertures(c, D, prob, 2)
    finally:
        prob.close()


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_autograd_prostate_full_size(fmt):
    """The prostate-shaped problem (288,000 beamlets, 1,048,576 voxels): 256
    random beamlet coordinates and all 180 aperture coordinates, fp32 and
    bf16 storage of D (the reference differentiates the same stored D)."""
    c = preset_case("prostate180")
    vals = c.val if fmt == "f32" else O.bf16_round(c.val)
    D = oracle_D(c, vals)
    prob = P.Problem.from_case(c, d_store=fmt)
    try:
        _check_fluence(c, D, prob, 256, 2)
        _check_apertures(c, D, prob, 3)
    finally:
        prob.close()
