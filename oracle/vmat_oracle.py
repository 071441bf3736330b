"""FP64 reference of the column-generation VMAT optimiser (Men, Romeijn, Jia,
Jiang, "Ultra-fast treatment plan optimization for VMAT").

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the GPU library.

Notation (Sec. 2.1): N beams sorted by angle theta_k; beam k has R leaf rows
of C beamlets; beamlet i = (k*R + rho)*C + c.  D is beamlet-major:
``D[i, j]`` is the dose to voxel j from beamlet i at unit intensity.  An
aperture A_k is one open interval [l_{k,rho}, r_{k,rho}) per leaf row
(l == r: closed row); y_k >= 0 is its intensity.

Readings of points the paper leaves open:
  * Apertures are row-convex leaf intervals; rows are independent (no
    interdigitation or minimum-gap rule).  Closed rows are allowed.
  * eq. 2 smoothing: ``circular=0`` is the literal open chain k=1..N-1;
    ``circular=1`` adds the pair (N, 1) with angle gap theta_1 + 360 - theta_N.
    Angles are in degrees.  Beams without an aperture have y_k = 0 and stay
    in G.
  * Maximum leaf speed (Sec. 2.2): a leaf of a new aperture may differ from the
    same leaf of the nearest occupied beam on each side by at most
    delta * (index distance); delta < 0 means unconstrained.
  * Beamlet price (Sec. 2.2, KKT): g = D F'(z).  Row search (one left-to-right
    pass): for every right end r the best left end maximises the prefix sum
    P[l] (ties: larger l); over r the key (S, r-l, l) is minimised, S = P[r]-P[l].
  * Beam price p_k = sum_rho S*_rho + gamma dG/dy_k at y_k = 0; k* = argmin over
    unoccupied beams, ties to the smallest k.  An aperture is added even when
    p_k* >= 0, so that every angle ends with an aperture.
  * Master (Sec. 2.2, "gradient projection"): steps on the free face of the
    bound y >= 0, steepest descent after every face change and Polak-Ribiere(+)
    conjugate directions while the face holds, each with an exact line search
    (safeguarded Newton on the piecewise-linear phi') up to the first blocking
    bound; stop at max_k |min(y_k, grad_k)| <= tol * ref.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# Problem data (Sec. 2.1)
# --------------------------------------------------------------------------


def dose_matrix(row_ptr, col, val, n_voxels) -> sp.csr_matrix:
    """D as an FP64 sparse matrix, row i = beamlet, column j = voxel (Sec. 2.1)."""
    nb = len(row_ptr) - 1
    return sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)),
                         shape=(nb, int(n_voxels)))


def aperture_mask(l, r, occ, R, C):
    """Indicator of i in A_k over all beamlets (Sec. 2.1: A_k = exposed beamlets).

    l, r: int [N*R] leaf-pair interval [l, r) per row; occ: [N] beam has an aperture.
    """
    N = len(occ)
    c = np.arange(C)
    lk = np.asarray(l).reshape(N, R)[:, :, None]
    rk = np.asarray(r).reshape(N, R)[:, :, None]
    m = (c[None, None, :] >= lk) & (c[None, None, :] < rk) & (np.asarray(occ).astype(bool)[:, None, None])
    return m.reshape(-1)


def fluence(y, l, r, occ, R, C):
    """x_i = y_k if beamlet i of beam k is exposed in A_k, else 0 (eq. 3 constraint)."""
    N = len(occ)
    m = aperture_mask(l, r, occ, R, C).reshape(N, R * C)
    return (m * np.asarray(y, dtype=np.float64)[:, None]).reshape(-1)


def dose(D, x):
    """z_j = sum_i D_ij x_i, i.e. sum_k y_k sum_{i in A_k} D_ij (Sec. 2.1, eq. 3)."""
    return D.T @ np.asarray(x, dtype=np.float64)


def beam_sums(v, l, r, occ, R, C):
    """sum_{i in A_k} v_i for every beam (the transpose of ``fluence``)."""
    N = len(occ)
    m = aperture_mask(l, r, occ, R, C).reshape(N, R * C)
    return (m * np.asarray(v, dtype=np.float64).reshape(N, R * C)).sum(axis=1)


# --------------------------------------------------------------------------
# eq. 1: one-sided quadratic voxel penalty
# --------------------------------------------------------------------------


def penalty(z, alpha, beta, T):
    """F(z) = sum_j alpha_j max(0,T_j-z_j)^2 + beta_j max(0,z_j-T_j)^2 (eq. 1),
    and its derivative F'_j = 2 beta_j max(0,z_j-T_j) - 2 alpha_j max(0,T_j-z_j)."""
    z = np.asarray(z, dtype=np.float64)
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    t = np.asarray(T, dtype=np.float64)
    under = np.maximum(0.0, t - z)
    over = np.maximum(0.0, z - t)
    F = float(np.sum(a * under * under + b * over * over))
    dF = 2.0 * b * over - 2.0 * a * under
    return F, dF


def curvature(z, alpha, beta, T):
    """F''_j: 2 alpha_j below the threshold, 2 beta_j at or above it (eq. 1)."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z < np.asarray(T, dtype=np.float64), 2.0 * np.asarray(alpha, np.float64),
                    2.0 * np.asarray(beta, np.float64))


# --------------------------------------------------------------------------
# eq. 2: dose-rate smoothing
# --------------------------------------------------------------------------


def smoothing_pairs(theta_deg, circular):
    """Neighbour pairs (a, b, theta_b - theta_a) of eq. 2; the wrap pair if circular."""
    th = np.asarray(theta_deg, dtype=np.float64)
    N = len(th)
    pairs = [(k, k + 1, th[k + 1] - th[k]) for k in range(N - 1)]
    if circular and N > 1:
        pairs.append((N - 1, 0, th[0] + 360.0 - th[N - 1]))
    return pairs


def smoothing(y, theta_deg, circular):
    """G(y) = sum (y_b - y_a)^2 / (theta_b - theta_a) over neighbour pairs (eq. 2),
    with its gradient."""
    y = np.asarray(y, dtype=np.float64)
    G = 0.0
    dG = np.zeros_like(y)
    for a, b, w in smoothing_pairs(theta_deg, circular):
        diff = y[b] - y[a]
        G += diff * diff / w
        dG[a] -= 2.0 * diff / w
        dG[b] += 2.0 * diff / w
    return G, dG


def smoothing_curvature(d, theta_deg, circular):
    """d^T (Hessian of G) d = sum 2 (d_b - d_a)^2 / (theta_b - theta_a)."""
    d = np.asarray(d, dtype=np.float64)
    return float(sum(2.0 * (d[b] - d[a]) ** 2 / w for a, b, w in smoothing_pairs(theta_deg, circular)))


# --------------------------------------------------------------------------
# eq. 3 objective and its gradient in y
# --------------------------------------------------------------------------


def objective(D, case_arrays, y, l, r, occ, gamma, theta_deg, circular, R, C):
    """f(y) = F(z(y)) + gamma G(y) (eq. 3).  Returns (F, gamma*G, z, F'(z), g, grad_y)."""
    alpha, beta, T = case_arrays
    z = dose(D, fluence(y, l, r, occ, R, C))
    F, dF = penalty(z, alpha, beta, T)
    g = D @ dF
    G, dG = smoothing(y, theta_deg, circular)
    grad = beam_sums(g, l, r, occ, R, C) + gamma * dG
    return F, gamma * G, z, dF, g, grad


# --------------------------------------------------------------------------
# Pricing (Sec. 2.2)
# --------------------------------------------------------------------------


def nearest_occupied(k, occ, circular):
    """Nearest occupied beam before and after k in angle order: (index, distance) or None."""
    N = len(occ)
    before = after = None
    for dist in range(1, N):
        kk = k - dist
        if kk < 0:
            if not circular:
                break
            kk += N
        if occ[kk]:
            before = (kk, dist)
            break
    for dist in range(1, N):
        kk = k + dist
        if kk >= N:
            if not circular:
                break
            kk -= N
        if occ[kk]:
            after = (kk, dist)
            break
    return before, after


def leaf_bounds(k, l, r, occ, R, C, delta, circular):
    """Per-row windows [L_lo, L_hi], [R_lo, R_hi] for a new aperture in beam k:
    each leaf within delta*(index distance) of the same leaf in the nearest
    occupied beam on either side (Sec. 2.2, maximum leaf motion speed)."""
    Llo = np.zeros(R, dtype=np.int64)
    Lhi = np.full(R, C, dtype=np.int64)
    Rlo = np.zeros(R, dtype=np.int64)
    Rhi = np.full(R, C, dtype=np.int64)
    if delta < 0:
        return Llo, Lhi, Rlo, Rhi
    lk = np.asarray(l).reshape(-1, R)
    rk = np.asarray(r).reshape(-1, R)
    for nb in nearest_occupied(k, occ, circular):
        if nb is None:
            continue
        a, dist = nb
        reach = delta * dist
        Llo = np.maximum(Llo, lk[a] - reach)
        Lhi = np.minimum(Lhi, lk[a] + reach)
        Rlo = np.maximum(Rlo, rk[a] - reach)
        Rhi = np.minimum(Rhi, rk[a] + reach)
    return Llo, Lhi, Rlo, Rhi


def price_row(g_row, Llo, Lhi, Rlo, Rhi):
    """Best leaf pair of one row in one left-to-right pass (Sec. 2.2).

    Minimises S(l, r) = sum_{c=l}^{r-1} g_c over Llo <= l <= Lhi, Rlo <= r <= Rhi,
    l <= r.  P is the running prefix sum; for each right end r the best left
    end is the one with the largest P[l] seen so far (ties: the later l); over r
    the key (S, r - l, l) is minimised.  Returns (S, l, r); (inf, -1, -1) if
    no pair is feasible.
    """
    C = len(g_row)
    P = 0.0
    best_P = -math.inf
    best_l = -1
    best = (math.inf, 0, 0)
    best_lr = (-1, -1)
    for pos in range(C + 1):          # pos is both a candidate l and a candidate r
        if Llo <= pos <= Lhi and P >= best_P:
            best_P, best_l = P, pos
        if Rlo <= pos <= Rhi and best_l >= 0:
            S = P - best_P
            key = (S, pos - best_l, best_l)
            if key < best:
                best, best_lr = key, (best_l, pos)
        if pos < C:
            P = P + float(g_row[pos])
    return best[0], best_lr[0], best_lr[1]


def row_margin(g_row, Llo, Lhi, Rlo, Rhi, S_best):
    """Smallest gap between S_best and any feasible pair with a different S value."""
    C = len(g_row)
    P = np.zeros(C + 1)
    # sequential prefix, to reproduce price_row's arithmetic exactly
    acc = 0.0
    for c in range(C):
        acc = acc + float(g_row[c])
        P[c + 1] = acc
    gap = math.inf
    for rr in range(max(Rlo, 0), min(Rhi, C) + 1):
        for ll in range(max(Llo, 0), min(Lhi, rr) + 1):
            S = P[rr] - P[ll]
            if S != S_best:
                gap = min(gap, S - S_best)
    return gap


@dataclasses.dataclass
class PriceResult:
    beam: int                 # k*, -1 if every beam is occupied
    l: np.ndarray             # [R]
    r: np.ndarray             # [R]
    price: float              # p_k*
    margin: float             # second-best beam price - best (inf if none)
    row_margin: float         # min over rows of k* of the row margin
    beam_prices: np.ndarray   # [N], +inf for occupied beams


def beam_smoothing_price(k, y, theta_deg, circular, gamma):
    """gamma dG/dy_k evaluated with y_k = 0 (the first-order effect of opening beam k)."""
    yy = np.asarray(y, dtype=np.float64).copy()
    yy[k] = 0.0
    _, dG = smoothing(yy, theta_deg, circular)
    return gamma * dG[k]


def price(g, y, l, r, occ, theta_deg, gamma, R, C, delta, circular, with_margins=True):
    """Pricing problem (Sec. 2.2): the most promising deliverable aperture over
    all unoccupied beams, from the beamlet prices g."""
    N = len(occ)
    g = np.asarray(g, dtype=np.float64).reshape(N, R, C)
    prices = np.full(N, math.inf)
    shapes = {}
    for k in range(N):
        if occ[k]:
            continue
        Llo, Lhi, Rlo, Rhi = leaf_bounds(k, l, r, occ, R, C, delta, circular)
        lk = np.zeros(R, dtype=np.int64)
        rk = np.zeros(R, dtype=np.int64)
        Sk = np.zeros(R)
        total = 0.0
        for rho in range(R):
            S, ll, rr = price_row(g[k, rho], Llo[rho], Lhi[rho], Rlo[rho], Rhi[rho])
            lk[rho], rk[rho], Sk[rho] = ll, rr, S
            total = total + S
        prices[k] = total + beam_smoothing_price(k, y, theta_deg, circular, gamma)
        shapes[k] = (lk, rk, Sk, (Llo, Lhi, Rlo, Rhi))
    cand = [k for k in range(N) if not occ[k]]
    if not cand:
        return PriceResult(-1, np.zeros(R, np.int64), np.zeros(R, np.int64), math.inf, math.inf,
                           math.inf, prices)
    kstar = min(cand, key=lambda k: (prices[k], k))
    others = [prices[k] for k in cand if k != kstar]
    margin = (min(others) - prices[kstar]) if others else math.inf
    lk, rk, Sk, (Llo, Lhi, Rlo, Rhi) = shapes[kstar]
    rm = math.inf
    if with_margins:
        for rho in range(R):
            rm = min(rm, row_margin(g[kstar, rho], Llo[rho], Lhi[rho], Rlo[rho], Rhi[rho], Sk[rho]))
    return PriceResult(kstar, lk, rk, float(prices[kstar]), float(margin), float(rm), prices)


# --------------------------------------------------------------------------
# Master problem (Sec. 2.2): gradient projection
# --------------------------------------------------------------------------


@dataclasses.dataclass
class MasterOpts:
    max_iter: int = 200
    tol_rel: float = 1e-5
    kkt_ref: float = 0.0      # <= 0: use max_k |grad_k| at the start point
    ls_max_steps: int = 50


@dataclasses.dataclass
class MasterResult:
    y: np.ndarray
    z: np.ndarray
    dF: np.ndarray
    g: np.ndarray
    grad: np.ndarray
    F: float
    gG: float
    kkt: float
    kkt_ref: float
    iters: int
    converged: bool
    n_forward: int
    n_adjoint: int
    n_ls_evals: int


def line_search(z, dz, alpha, beta, T, gG_slope0, gG_curv, t_max, max_steps=50):
    """Exact minimiser over [0, t_max] of phi(t) = F(z + t dz) + gamma G(y + t d).

    phi'(t) = sum_j dz_j F'_j(z_j + t dz_j) + gG_slope0 + t gG_curv is piecewise
    linear and non-decreasing; phi'' is the matching piecewise constant.
    Safeguarded Newton inside a bracket, from t = 0.  Returns (t, n_evals).
    """
    def ev(t):
        zt = z + t * dz
        _, dF = penalty(zt, alpha, beta, T)
        d1 = float(np.sum(dz * dF)) + gG_slope0 + t * gG_curv
        d2 = float(np.sum(dz * dz * curvature(zt, alpha, beta, T))) + gG_curv
        return d1, d2

    p0, h0 = ev(0.0)
    nev = 1
    if not (p0 < 0.0):
        return 0.0, nev
    lo, hi = 0.0, t_max
    if math.isfinite(hi):
        ph, _ = ev(hi)
        nev += 1
        if ph <= 0.0:
            return hi, nev
    t, p, h = 0.0, p0, h0
    for _ in range(max_steps):
        tn = t - p / h if h > 0.0 else math.nan
        if not (lo < tn < hi):
            tn = 0.5 * (lo + hi) if math.isfinite(hi) else (2.0 * lo if lo > 0.0 else 1.0)
        t = tn
        p, h = ev(t)
        nev += 1
        if p <= 0.0:
            lo = t
        else:
            hi = t
        if abs(p) <= 1e-12 * abs(p0):
            return t, nev
        if math.isfinite(hi) and hi - lo <= 1e-15 * hi:
            break
    return lo, nev


def master(D, alpha, beta, T, theta_deg, gamma, circular, R, C, l, r, occ, y0, opts=MasterOpts(),
           start=None):
    """Solve min F(z) + gamma G(y), y >= 0, over the intensities of the current
    apertures (Sec. 2.2 master problem: model (3) with the A_k fixed) by
    gradient projection.  Unoccupied beams keep y_k = 0.

    Each iteration moves along a direction on the current free face
    W = {k occupied: y_k > 0 or grad_k < 0}: steepest descent -grad_W after
    any change of W (and at the start), otherwise the Polak-Ribiere(+)
    conjugate direction.  The step is the exact minimiser of f along the
    direction up to the first bound that blocks (``line_search``); blocking
    intensities are set to 0.  Stops when max_k |min(y_k, grad_k)| <= tol*ref.

    ``start`` = (z, g) carries the dose and beamlet prices of y0 over from the
    caller (column generation adds an aperture at y = 0, which changes
    neither); without it both are computed from y0.
    """
    occ_b = np.asarray(occ).astype(bool)
    y = np.where(occ_b, np.asarray(y0, dtype=np.float64), 0.0)
    if start is None:
        z = dose(D, fluence(y, l, r, occ, R, C))
        F, dF = penalty(z, alpha, beta, T)
        g = D @ dF
        n_fwd, n_adj = 1, 1
    else:
        z, g = start
        F, dF = penalty(z, alpha, beta, T)
        n_fwd, n_adj = 0, 0
    G, dG = smoothing(y, theta_deg, circular)
    grad = beam_sums(g, l, r, occ, R, C) + gamma * dG
    n_ls = 0

    def kkt_of(y, grad):
        v = np.abs(np.minimum(y, grad))[occ_b]
        return float(v.max()) if v.size else 0.0

    ref = opts.kkt_ref
    if not (ref > 0.0):
        v = np.abs(grad[occ_b])
        ref = float(v.max()) if v.size else 0.0
        if ref == 0.0:
            ref = 1.0
    W_prev = d_prev = grad_prev = None
    it = 0
    converged = False
    while True:
        kkt = kkt_of(y, grad)
        if kkt <= opts.tol_rel * ref:
            converged = True
            break
        if it >= opts.max_iter:
            break
        W = occ_b & ((y > 0.0) | (grad < 0.0))
        d = np.where(W, -grad, 0.0)
        if W_prev is not None and np.array_equal(W, W_prev):
            gp = np.where(W, grad_prev, 0.0)
            den = float(np.dot(gp, gp))
            beta_cg = max(0.0, float(np.dot(np.where(W, grad, 0.0), np.where(W, grad, 0.0) - gp)) / den) \
                if den > 0.0 else 0.0
            dc = np.where(W, -grad + beta_cg * d_prev, 0.0)
            if float(np.dot(dc, grad)) < 0.0:
                d = dc
        blk = d < 0.0
        ratio = np.where(blk, y / np.where(blk, -d, 1.0), math.inf)
        t_max = float(np.min(ratio)) if blk.any() else math.inf
        if not np.any(d != 0.0):
            break
        dz = dose(D, fluence(d, l, r, occ, R, C))
        n_fwd += 1
        _, dGy = smoothing(y, theta_deg, circular)
        slope0 = gamma * float(np.dot(dGy, d))
        curv = gamma * smoothing_curvature(d, theta_deg, circular)
        t, nev = line_search(z, dz, alpha, beta, T, slope0, curv, t_max, opts.ls_max_steps)
        n_ls += nev
        W_prev, d_prev, grad_prev = W, d, grad
        y = np.maximum(0.0, y + t * d)
        if t == t_max:
            y[blk & (ratio == t_max)] = 0.0           # the blocking bounds become active
        z = z + t * dz
        F, dF = penalty(z, alpha, beta, T)
        g = D @ dF
        n_adj += 1
        G, dG = smoothing(y, theta_deg, circular)
        grad = beam_sums(g, l, r, occ, R, C) + gamma * dG
        it += 1
    return MasterResult(y, z, dF, g, grad, F, gamma * G, kkt, ref, it, converged, n_fwd, n_adj, n_ls)


# --------------------------------------------------------------------------
# Column generation (abstract; Sec. 2.2)
# --------------------------------------------------------------------------


@dataclasses.dataclass
class SolveResult:
    y: np.ndarray
    l: np.ndarray
    r: np.ndarray
    occ: np.ndarray
    z: np.ndarray
    order: list          # beam chosen at each iteration
    prices: list
    margins: list
    row_margins: list
    costs: list          # cost_0 (no apertures), then after each master solve
    master_iters: list
    apertures: list      # (l[R], r[R]) chosen at each iteration
    priced_y: list = dataclasses.field(default_factory=list)  # intensities each pricing saw


def solve(D, alpha, beta, T, theta_deg, gamma, circular, R, C, delta, max_cg_iter=None,
          master_opts=MasterOpts(), with_margins=True, on_iter=None):
    """Column generation: price one aperture over the unoccupied beams, add it,
    re-solve the master, until every beam has an aperture (Sec. 2.2; abstract).
    The dose and prices of the current plan carry over from one master solve to
    the next: the new aperture starts at intensity 0.  on_iter (optional) is
    called after every iteration with (iteration, beam, cost), for progress
    reports; it takes no part in the computation."""
    N = len(theta_deg)
    occ = np.zeros(N, dtype=np.uint8)
    l = np.zeros(N * R, dtype=np.int64)
    r = np.zeros(N * R, dtype=np.int64)
    y = np.zeros(N)
    z = np.zeros(D.shape[1])
    F, dF = penalty(z, alpha, beta, T)
    g = D @ dF
    out = SolveResult(y, l, r, occ, z, [], [], [], [], [F], [], [])
    ref = None
    iters = N if max_cg_iter is None else min(N, max_cg_iter)
    for _ in range(iters):
        out.priced_y.append(np.array(y, dtype=np.float64))
        pr = price(g, y, l, r, occ, theta_deg, gamma, R, C, delta, circular, with_margins)
        if pr.beam < 0:
            break
        k = pr.beam
        occ[k] = 1
        l[k * R:(k + 1) * R] = pr.l
        r[k * R:(k + 1) * R] = pr.r
        y[k] = 0.0
        if ref is None:
            ref = abs(pr.price) if pr.price != 0.0 else 1.0
        mo = dataclasses.replace(master_opts, kkt_ref=ref)
        m = master(D, alpha, beta, T, theta_deg, gamma, circular, R, C, l, r, occ, y, mo, start=(z, g))
        y, z, g = m.y, m.z, m.g
        out.order.append(k)
        out.prices.append(pr.price)
        out.margins.append(pr.margin)
        out.row_margins.append(pr.row_margin)
        out.costs.append(m.F + m.gG)
        out.master_iters.append(m.iters)
        out.apertures.append((pr.l.copy(), pr.r.copy()))
        if on_iter is not None:
            on_iter(len(out.order), k, m.F + m.gG)
    out.y, out.l, out.r, out.occ, out.z = y, l, r, occ, z
    return out


# --------------------------------------------------------------------------
# Dose-rate feasibility of the final plan (Sec. 3): the smoothing term is a
# soft constraint; when the final intensities still change too fast between
# neighbouring angles, gamma is raised and the intensities re-optimised with
# the apertures fixed, until the plan is feasible.
# --------------------------------------------------------------------------


def max_rate(y, theta_deg, circular):
    """Largest intensity change per degree over the neighbour pairs of eq. 2."""
    y = np.asarray(y, dtype=np.float64)
    rates = [abs(y[b] - y[a]) / w for a, b, w in smoothing_pairs(theta_deg, circular)]
    return max(rates) if rates else 0.0


@dataclasses.dataclass
class RateResult:
    y: np.ndarray
    gamma: float
    rounds: int           # re-optimisations run
    feasible: bool
    rate: float           # max_rate of the returned y
    costs: list           # F + gamma G after each round (at that round's gamma)
    smoothing: list       # G after each round


def enforce_rate(D, alpha, beta, T, theta_deg, gamma, circular, R, C, l, r, occ, y, rate_max,
                 factor=10.0, max_rounds=8, opts=MasterOpts()):
    """Raise gamma by ``factor`` and re-solve the master (apertures fixed, warm
    start from the previous intensities) until max_rate(y) <= rate_max or
    ``max_rounds`` re-optimisations have run.  The first check is on y as
    given; a feasible y is returned unchanged."""
    y = np.where(np.asarray(occ).astype(bool), np.asarray(y, dtype=np.float64), 0.0)
    g_now = float(gamma)
    rounds = 0
    costs, smooth = [], []
    rate = max_rate(y, theta_deg, circular)
    start = None
    while rate > rate_max and rounds < max_rounds:
        g_now *= factor
        res = master(D, alpha, beta, T, theta_deg, g_now, circular, R, C, l, r, occ, y, opts, start=start)
        y = res.y
        start = (res.z, res.g)
        rounds += 1
        costs.append(res.F + res.gG)
        smooth.append(res.gG / g_now if g_now > 0 else 0.0)
        rate = max_rate(y, theta_deg, circular)
    return RateResult(y=y, gamma=g_now, rounds=rounds, feasible=rate <= rate_max, rate=rate, costs=costs,
                      smoothing=smooth)


# --------------------------------------------------------------------------
# Reduced-precision storage of D (bf16 / fp16 / fp8 E4M3 with per-beamlet scale)
# --------------------------------------------------------------------------


def bf16_round(v):
    """Round float32 values to bfloat16 (round to nearest, ties to even), returned
    as float32.  bfloat16 keeps the upper 16 bits of the float32 encoding."""
    b = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    rb = ((b + 0x7FFF + lsb) >> 16) << 16
    return rb.astype(np.uint32).view(np.float32)


def fp16_round(v):
    return np.asarray(v, dtype=np.float32).astype(np.float16).astype(np.float32)


def e4m3_values():
    """All 256 OCP FP8 E4M3 codes as float64 (NaN for 0x7F/0xFF).  Exponent bias 7,
    3 mantissa bits, subnormals for exponent field 0, no infinities."""
    out = np.empty(256)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 15 and m == 7:
            out[code] = math.nan
        elif e == 0:
            out[code] = s * m * 2.0 ** -9
        else:
            out[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return out


def e4m3_encode(v):
    """Non-negative values (<= 448) to E4M3 codes, round to nearest, ties to even code."""
    table = e4m3_values()[:127]            # codes 0..126, ascending, finite
    v = np.asarray(v, dtype=np.float64)
    if np.any(v < 0) or np.any(v > 448.0):
        raise ValueError("e4m3_encode expects values in [0, 448]")
    hi = np.searchsorted(table, v, side="left")
    hi = np.minimum(hi, 126)
    lo = np.maximum(hi - 1, 0)
    dlo = v - table[lo]
    dhi = table[hi] - v
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(table[hi] == v, hi, code)
    return code.astype(np.uint8)


def fp8_quantise(row_ptr, val):
    """Per-beamlet scale s_i = max_j D_ij / 448 (float32) and codes q_ij with
    D_ij ~ s_i * e4m3(q_ij).  Empty or all-zero rows get scale 1."""
    row_ptr = np.asarray(row_ptr)
    val = np.asarray(val, dtype=np.float32)
    nb = len(row_ptr) - 1
    lens = np.diff(row_ptr)
    rowmax = np.zeros(nb, dtype=np.float32)
    nz = lens > 0
    rowmax[nz] = np.maximum.reduceat(val, row_ptr[:-1][nz])
    scale = np.where(rowmax > 0, rowmax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    rows = np.repeat(np.arange(nb), lens)
    q = e4m3_encode(np.minimum(val.astype(np.float64) / scale[rows].astype(np.float64), 448.0))
    return scale, q


def fp8_dequantise(row_ptr, scale, q):
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(np.asarray(row_ptr)))
    return (e4m3_values()[q] * np.asarray(scale, np.float64)[rows])


def quantisation_bound(D, Dhat, x):
    """Exact per-voxel bound sum_i |Dhat_ij - D_ij| x_i (x >= 0) on the dose change."""
    E = abs(Dhat - D)
    return E.T @ np.abs(np.asarray(x, dtype=np.float64))
