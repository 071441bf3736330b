"""Pins of the FP64 reference against what the paper and mathematics fix.

Each test checks the reference against something other than itself: hand-
worked values of eq. 1 / eq. 2 (tests/golden), brute force on tiny inputs,
textbook special cases (Kadane's maximum subarray), closed forms of the master
problem, an independent exact line search, library conversions for the
reduced-precision formats, and the invariants of column generation.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append([float(v) for v in line.split()])
    return out


# ---------------------------------------------------------------- eq. 1 / eq. 2

def test_eq1_penalty_golden():
    for a, b, T, z, F, dF, d2F in _rows("eq1_penalty.txt"):
        Fo, dFo = O.penalty(np.array([z]), np.array([a]), np.array([b]), np.array([T]))
        assert Fo == F
        assert dFo[0] == dF
        assert O.curvature(np.array([z]), np.array([a]), np.array([b]), np.array([T]))[0] == d2F


def test_eq1_curvature_is_second_difference():
    """Away from the threshold F is a quadratic on each side, so the second
    difference of eq. 1 is exact: it must equal the curvature on both sides."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        a, b = rng.integers(0, 5, 2).astype(float)
        a, b = (a, b) if a != b else (a, b + 1.0)
        T = float(rng.integers(5, 50))
        for z in (T - 2.0 - rng.random(), T + 2.0 + rng.random()):
            h = 0.5
            Fz = [O.penalty(np.array([v]), np.array([a]), np.array([b]), np.array([T]))[0]
                  for v in (z - h, z, z + h)]
            d2 = (Fz[0] - 2 * Fz[1] + Fz[2]) / (h * h)
            assert O.curvature(np.array([z]), np.array([a]), np.array([b]), np.array([T]))[0] == \
                pytest.approx(d2, rel=1e-9, abs=1e-9)


def test_eq1_zero_dose_cost():
    # y = 0 gives z = 0 and F = sum_j alpha_j T_j^2 (eq. 1 with z_j = 0 <= T_j)
    rng = np.random.default_rng(1)
    a, b, T = rng.random(50), rng.random(50), rng.random(50) * 70
    F, _ = O.penalty(np.zeros(50), a, b, T)
    assert F == pytest.approx(float(np.sum(a * T * T)), rel=1e-14)


def test_eq2_smoothing_golden():
    for circ, y1, y2, y3, t1, t2, t3, G, g1, g2, g3 in _rows("eq2_smoothing.txt"):
        Go, dGo = O.smoothing(np.array([y1, y2, y3]), np.array([t1, t2, t3]), int(circ))
        assert Go == pytest.approx(G, rel=1e-15)
        np.testing.assert_allclose(dGo, [g1, g2, g3], rtol=1e-14)


def test_eq2_gradient_and_curvature_fd():
    rng = np.random.default_rng(2)
    th = np.sort(rng.choice(360, 7, replace=False)).astype(float)
    for circ in (0, 1):
        y, d = rng.random(7), rng.standard_normal(7)
        G0, dG = O.smoothing(y, th, circ)
        h = 1e-4
        Gp, _ = O.smoothing(y + h * d, th, circ)
        Gm, _ = O.smoothing(y - h * d, th, circ)
        assert (Gp - Gm) / (2 * h) == pytest.approx(float(dG @ d), rel=1e-8)
        # G is quadratic: second difference is exact up to rounding
        assert (Gp - 2 * G0 + Gm) / h ** 2 == pytest.approx(O.smoothing_curvature(d, th, circ), rel=1e-5)


# ---------------------------------------------------------------- dose model

def test_dose_bruteforce_small_integers():
    """z_j = sum_k y_k sum_{i in A_k} D_ij (Sec. 2.1), by explicit loops, exact on integers."""
    rng = np.random.default_rng(3)
    N, R, C, nv = 4, 3, 5, 17
    nb = N * R * C
    Dd = rng.integers(0, 4, size=(nb, nv)) * (rng.random((nb, nv)) < 0.4)
    y = rng.integers(0, 5, size=N).astype(float)
    occ = np.array([1, 0, 1, 1], dtype=np.uint8)
    l = rng.integers(0, C + 1, size=N * R)
    r = np.maximum(l, rng.integers(0, C + 1, size=N * R))
    z_ref = np.zeros(nv)
    for k in range(N):
        if not occ[k]:
            continue
        for rho in range(R):
            for c in range(l[k * R + rho], r[k * R + rho]):
                i = (k * R + rho) * C + c
                for j in range(nv):
                    z_ref[j] += y[k] * Dd[i, j]
    D = sp.csr_matrix(Dd.astype(float))
    z = O.dose(D, O.fluence(y, l, r, occ, R, C))
    assert np.array_equal(z, z_ref)


def test_dose_adjoint_identity():
    rng = np.random.default_rng(4)
    N, R, C, nv = 5, 4, 6, 200
    nb = N * R * C
    D = sp.random(nb, nv, density=0.1, random_state=5, format="csr")
    y = rng.random(N)
    occ = (rng.random(N) < 0.7).astype(np.uint8)
    l = rng.integers(0, C + 1, N * R)
    r = np.maximum(l, rng.integers(0, C + 1, N * R))
    w = rng.standard_normal(nv)
    lhs = float(O.dose(D, O.fluence(y, l, r, occ, R, C)) @ w)
    rhs = float(y @ O.beam_sums(D @ w, l, r, occ, R, C))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_dose_voxel_permutation_invariance():
    rng = np.random.default_rng(6)
    nb, nv = 30, 40
    D = sp.random(nb, nv, density=0.2, random_state=7, format="csr")
    x = rng.random(nb)
    perm = rng.permutation(nv)
    z = O.dose(D, x)
    zp = O.dose(D[:, perm], x)
    np.testing.assert_allclose(zp, z[perm], rtol=1e-15)


def test_objective_gradient_fd():
    rng = np.random.default_rng(8)
    N, R, C, nv = 6, 2, 4, 60
    nb = N * R * C
    D = sp.random(nb, nv, density=0.3, random_state=9, format="csr")
    alpha = (rng.random(nv) < 0.5) * rng.random(nv)
    beta = rng.random(nv)
    T = rng.random(nv) * 2
    th = np.arange(N) * 60.0
    occ = np.array([1, 1, 0, 1, 1, 1], dtype=np.uint8)
    l = rng.integers(0, 2, N * R)
    r = rng.integers(2, C + 1, N * R)
    y = rng.random(N) * 3 * occ
    F, gG, z, dF, g, grad = O.objective(D, (alpha, beta, T), y, l, r, occ, 0.3, th, 1, R, C)
    for k in np.flatnonzero(occ):
        h = 1e-6
        e = np.zeros(N)
        e[k] = h
        fp = sum(O.objective(D, (alpha, beta, T), y + e, l, r, occ, 0.3, th, 1, R, C)[:2])
        fm = sum(O.objective(D, (alpha, beta, T), y - e, l, r, occ, 0.3, th, 1, R, C)[:2])
        assert (fp - fm) / (2 * h) == pytest.approx(grad[k], rel=1e-5, abs=1e-7)


# ---------------------------------------------------------------- pricing

def _brute_row(g, Llo, Lhi, Rlo, Rhi):
    best = None
    for l in range(Llo, Lhi + 1):
        for r in range(max(l, Rlo), Rhi + 1):
            S = sum(g[l:r])
            key = (S, r - l, l)
            if best is None or key < best[0]:
                best = (key, l, r)
    return best


def test_price_row_exhaustive_small_integer_rows():
    """Every row with g_c in {-2..2} for C <= 5, every window: exact ties included."""
    for C in range(1, 6):
        for g in itertools.product(range(-2, 3), repeat=C):
            g = np.array(g, dtype=float)
            for Llo, Lhi, Rlo, Rhi in ((0, C, 0, C), (1, min(2, C), 1, C), (0, 1, max(0, C - 1), C)):
                if Llo > Lhi or Rlo > Rhi:
                    continue
                S, l, r = O.price_row(g, Llo, Lhi, Rlo, Rhi)
                br = _brute_row(list(g), Llo, Lhi, Rlo, Rhi)
                assert (S, l, r) == (br[0][0], br[1], br[2]), (g, Llo, Lhi, Rlo, Rhi)


def test_price_row_random_bounds_vs_bruteforce():
    rng = np.random.default_rng(10)
    for _ in range(3000):
        C = int(rng.integers(1, 13))
        g = rng.integers(-5, 6, C).astype(float)
        a, b = sorted(rng.integers(0, C + 1, 2))
        c, d = sorted(rng.integers(0, C + 1, 2))
        if a > d:
            continue
        S, l, r = O.price_row(g, a, b, c, d)
        br = _brute_row(list(g), a, b, c, d)
        assert (S, l, r) == (br[0][0], br[1], br[2])


def _kadane(v):
    best = cur = 0.0
    for x in v:
        cur = max(0.0, cur + x)
        best = max(best, cur)
    return best


def test_price_row_unconstrained_is_kadane():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        C = int(rng.integers(1, 40))
        g = rng.integers(-9, 10, C).astype(float)
        S, l, r = O.price_row(g, 0, C, 0, C)
        assert -S == _kadane(-g)
        assert S == g[l:r].sum()


def test_row_margin_bruteforce():
    rng = np.random.default_rng(12)
    for _ in range(300):
        C = int(rng.integers(1, 9))
        g = rng.integers(-3, 4, C).astype(float)
        S, l, r = O.price_row(g, 0, C, 0, C)
        vals = sorted({sum(g[a:b]) for a in range(C + 1) for b in range(a, C + 1)})
        higher = [v for v in vals if v != S]
        m = O.row_margin(g, 0, C, 0, C, S)
        assert m == (min(higher) - S if higher else math.inf)


def test_first_pricing_opens_negative_span():
    """At z = 0 every price is <= 0; each row opens from its first to its last
    strictly negative beamlet (the unique shortest minimiser)."""
    rng = np.random.default_rng(13)
    N, R, C = 5, 6, 9
    g = -1.0 * (rng.random(N * R * C) < 0.4) * rng.random(N * R * C)
    pr = O.price(g, np.zeros(N), np.zeros(N * R, int), np.zeros(N * R, int), np.zeros(N, np.uint8),
                 np.arange(N) * 72.0, 0.1, R, C, 2, 1)
    gk = g.reshape(N, R, C)[pr.beam]
    for rho in range(R):
        neg = np.flatnonzero(gk[rho] < 0)
        if neg.size:
            assert (pr.l[rho], pr.r[rho]) == (neg[0], neg[-1] + 1)
        else:
            assert (pr.l[rho], pr.r[rho]) == (0, 0)
    sums = g.reshape(N, R * C).sum(axis=1)
    assert pr.beam == int(np.argmin(sums))


def test_leaf_bounds_deliverable_against_all_occupied():
    """A priced aperture is within delta*(distance) of every occupied beam's leaves."""
    rng = np.random.default_rng(14)
    N, R, C, delta = 12, 3, 10, 1
    for circ in (0, 1):
        occ = np.zeros(N, np.uint8)
        l = np.zeros(N * R, int)
        r = np.zeros(N * R, int)
        for _ in range(N):
            g = rng.standard_normal(N * R * C)
            pr = O.price(g, np.zeros(N), l, r, occ, np.arange(N) * 30.0, 0.0, R, C, delta, circ)
            k = pr.beam
            for a in np.flatnonzero(occ):
                dist = abs(a - k) if not circ else min(abs(a - k), N - abs(a - k))
                assert np.all(np.abs(pr.l - l[a * R:(a + 1) * R]) <= delta * dist)
                assert np.all(np.abs(pr.r - r[a * R:(a + 1) * R]) <= delta * dist)
            assert np.all(pr.l <= pr.r)
            occ[k] = 1
            l[k * R:(k + 1) * R], r[k * R:(k + 1) * R] = pr.l, pr.r


def _leaf_window_cases():
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "leaf_window.txt")) as f:
        for line in f:
            w = line.split("#")[0].split()
            if not w:
                continue
            if w[0] == "setup":
                N, R, C, delta, circ = (int(v) for v in w[2:])
                cur = dict(name=w[1], N=N, R=R, C=C, delta=delta, circ=circ, occ=np.zeros(N, np.uint8),
                           l=np.zeros(N * R, np.int64), r=np.zeros(N * R, np.int64), win=[])
                cases.append(cur)
            elif w[0] == "occ":
                k, lr = int(w[1]), [int(v) for v in w[2:]]
                cur["occ"][k] = 1
                cur["l"][k * cur["R"]:(k + 1) * cur["R"]] = lr[0::2]
                cur["r"][k * cur["R"]:(k + 1) * cur["R"]] = lr[1::2]
            elif w[0] == "win":
                cur["win"].append(tuple(int(v) for v in w[1:]))
    return cases


def test_leaf_bounds_golden_windows():
    """Hand-worked leaf windows (tests/golden/leaf_window.txt): neighbours at
    distances 1 to 4, open and circular chains, delta 1 and 2, unconstrained,
    and no occupied beam."""
    n = 0
    for cs in _leaf_window_cases():
        for k, rho, Llo, Lhi, Rlo, Rhi in cs["win"]:
            w = O.leaf_bounds(k, cs["l"], cs["r"], cs["occ"], cs["R"], cs["C"], cs["delta"], cs["circ"])
            assert tuple(int(v[rho]) for v in w) == (Llo, Lhi, Rlo, Rhi), (cs["name"], k, rho)
            n += 1
    assert n == 19


def test_leaf_bounds_window_is_every_deliverable_position():
    """Brute force: a leaf position is in the window exactly when, for every
    occupied beam a, it is within delta * d(a) of beam a's leaf, where d(a)
    is the number of beam steps from k to a along the chain in the direction
    in which a is the first occupied beam (every occupied beam is reached from
    k through the nearest one on that side, so this is the reading's rule
    written out over all beams)."""
    rng = np.random.default_rng(15)
    for circ in (0, 1):
        for _ in range(40):
            N, R, C, delta = int(rng.integers(3, 9)), 2, int(rng.integers(3, 9)), int(rng.integers(0, 3))
            occ = np.zeros(N, np.uint8)
            l = np.zeros(N * R, np.int64)
            r = np.zeros(N * R, np.int64)
            for _ in range(int(rng.integers(1, N))):
                g = rng.standard_normal(N * R * C)
                pr = O.price(g, np.zeros(N), l, r, occ, np.arange(N) * (360.0 / N), 0.0, R, C, delta, circ,
                             with_margins=False)
                occ[pr.beam] = 1
                l[pr.beam * R:(pr.beam + 1) * R], r[pr.beam * R:(pr.beam + 1) * R] = pr.l, pr.r
            for k in np.flatnonzero(occ == 0):
                Llo, Lhi, Rlo, Rhi = O.leaf_bounds(k, l, r, occ, R, C, delta, circ)
                # the first occupied beam met walking each way from k, with its step count
                walks = []
                for step in (-1, 1):
                    for dist in range(1, N):
                        kk = k + step * dist
                        if not circ and not 0 <= kk < N:
                            break
                        if occ[kk % N]:
                            walks.append((kk % N, dist))
                            break
                for rho in range(R):
                    for leaf, lo, hi in ((l, Llo, Lhi), (r, Rlo, Rhi)):
                        ok = [p for p in range(C + 1)
                              if all(abs(p - leaf[a * R + rho]) <= delta * dist for a, dist in walks)]
                        if ok:
                            assert (lo[rho], hi[rho]) == (ok[0], ok[-1])
                            assert ok == list(range(ok[0], ok[-1] + 1))
                        else:
                            assert lo[rho] > hi[rho]


def test_beam_price_exact_tie_goes_to_smaller_beam():
    """Two unoccupied beams with identical rows and identical neighbours have
    the same price to the last bit; the smaller beam index is chosen and the
    beam margin is zero."""
    N, R, C = 4, 2, 3
    th = np.array([0.0, 90.0, 180.0, 270.0])
    g = np.zeros((N, R, C))
    g[1] = g[3] = [[-1.0, -2.0, 0.5], [0.25, -0.75, -0.5]]
    g[0] = g[2] = [[-0.5, 0.0, 0.0], [0.0, 0.0, -0.25]]
    for gamma, occ, y in ((0.0, np.zeros(N, np.uint8), np.zeros(N)),
                          (0.3, np.array([1, 0, 1, 0], np.uint8), np.array([1.5, 0.0, 1.5, 0.0]))):
        l = np.zeros(N * R, np.int64)
        r = np.where(np.repeat(occ, R) == 1, C, 0).astype(np.int64)
        gg = g.copy()
        gg[occ == 1] = 0.0
        pr = O.price(gg.reshape(-1), y, l, r, occ, th, gamma, R, C, -1, 1)
        assert pr.beam_prices[1] == pr.beam_prices[3]
        assert pr.beam == 1
        assert pr.margin == 0.0
        assert list(pr.l) == [0, 1] and list(pr.r) == [2, 3]


def test_beam_price_includes_smoothing_derivative():
    # single-row, single-column beams; price = g + gamma dG/dy_k at y_k = 0
    N, R, C = 4, 1, 1
    th = np.array([0.0, 90.0, 180.0, 270.0])
    y = np.array([2.0, 0.0, 0.0, 1.0])
    occ = np.array([1, 0, 0, 1], np.uint8)
    g = np.array([0.0, -1.0, -0.5, 0.0])
    pr = O.price(g, y, np.zeros(4, int), np.ones(4, int), occ, th, 0.5, R, C, -1, 1)
    # beam 1: neighbours y0=2 (gap 90), y2=0 -> -2*0.5*(2/90); beam 2: y3=1 -> -2*0.5*(1/90)
    p1 = -1.0 - 2 * 0.5 * 2 / 90
    p2 = -0.5 - 2 * 0.5 * 1 / 90
    np.testing.assert_allclose(pr.beam_prices[[1, 2]], [p1, p2], rtol=1e-15)
    assert pr.beam == 1 and pr.margin == pytest.approx(p2 - p1)


# ---------------------------------------------------------------- line search / master

def _exact_min_piecewise(z, dz, a, b, T, s0, c, tmax):
    """Independent exact minimiser: split [0, tmax] at every threshold crossing;
    on each piece phi is quadratic, minimise it there in closed form."""
    with np.errstate(divide="ignore", invalid="ignore"):
        bp = (T - z) / dz
    bp = np.sort(bp[np.isfinite(bp) & (bp > 0) & (bp < tmax)])
    edges = np.concatenate([[0.0], bp, [tmax]])

    def phi(t):
        F, _ = O.penalty(z + t * dz, a, b, T)
        return F + s0 * t + 0.5 * c * t * t

    best_t, best_v = 0.0, phi(0.0)
    for lo, hi in zip(edges[:-1], edges[1:]):
        mid = 0.5 * (lo + hi)
        zm = z + mid * dz
        w = np.where(zm < T, a, b)                 # regime on this piece
        q2 = float(np.sum(w * dz * dz)) + 0.5 * c  # phi = q2 t^2 + q1 t + const
        q1 = float(np.sum(2 * w * dz * (z - T))) + s0
        cands = [lo, hi]
        if q2 > 0:
            cands.append(min(max(-q1 / (2 * q2), lo), hi))
        for t in cands:
            v = phi(t)
            if v < best_v:
                best_t, best_v = t, v
    return best_t, best_v


def test_line_search_exact_vs_piecewise():
    rng = np.random.default_rng(15)
    for trial in range(60):
        n = 40
        z = rng.random(n) * 10
        dz = rng.standard_normal(n) * 3
        a = rng.random(n) * (rng.random(n) < 0.6)
        b = rng.random(n)
        T = rng.random(n) * 10
        s0 = rng.standard_normal() * 0.1
        c = rng.random() * 0.1
        tmax = 1.0 if trial % 2 else math.inf
        t, _ = O.line_search(z, dz, a, b, T, s0, c, tmax)
        tt, vv = _exact_min_piecewise(z, dz, a, b, T, s0, c, 1e6 if math.isinf(tmax) else tmax)
        F, _ = O.penalty(z + t * dz, a, b, T)
        v = F + s0 * t + 0.5 * c * t * t
        assert v <= vv + 1e-10 * max(1.0, abs(vv))
        assert t == pytest.approx(tt, rel=1e-7, abs=1e-9) or abs(v - vv) <= 1e-12 * max(1, abs(vv))


def _single_beam_problem(Dval, alpha, T, gamma):
    N, R, C = 3, 1, 1
    D = sp.csr_matrix(np.array([[Dval], [0.0], [0.0]]))
    th = np.array([0.0, 120.0, 240.0])
    return D, th, N, R, C


def test_master_one_beam_one_voxel_closed_form():
    """f = alpha (T - yD)^2 + gamma y^2 (1/dth- + 1/dth+)  =>  y* = alpha D T / (alpha D^2 + gamma (...))."""
    for Dval, alpha, T, gamma in ((0.7, 1.0, 60.0, 0.1), (2.0, 3.0, 10.0, 5.0), (0.3, 0.5, 78.0, 0.0)):
        D, th, N, R, C = _single_beam_problem(Dval, alpha, T, gamma)
        occ = np.array([1, 0, 0], np.uint8)
        m = O.master(D, np.array([alpha]), np.array([1.0]), np.array([T]), th, gamma, 1, R, C,
                     np.zeros(3, int), np.ones(3, int), occ, np.zeros(3), O.MasterOpts(tol_rel=1e-12))
        y_star = alpha * Dval * T / (alpha * Dval ** 2 + gamma * (1 / 120 + 1 / 120))
        assert m.y[0] == pytest.approx(y_star, rel=1e-10)
        assert m.converged


def _enumerate_kkt(Dd, alpha, beta, T, th, gamma, circ, occ):
    """Exact solution of a tiny master problem by enumerating active sets and
    voxel regimes; each candidate is a linear system."""
    N, nv = Dd.shape
    best = None
    occ_idx = [k for k in range(N) if occ[k]]
    pairs = O.smoothing_pairs(th, circ)
    H_G = np.zeros((N, N))
    for a_, b_, w in pairs:
        H_G[a_, a_] += 2 / w
        H_G[b_, b_] += 2 / w
        H_G[a_, b_] -= 2 / w
        H_G[b_, a_] -= 2 / w
    for mask in itertools.product((0, 1), repeat=len(occ_idx)):
        S = [k for k, m in zip(occ_idx, mask) if m]
        for reg in itertools.product((0, 1), repeat=nv):
            w = np.where(np.array(reg) == 1, beta, alpha)   # 1: over-dose regime
            # f = sum_j w_j (z_j - T_j)^2 + gamma/2 y^T H_G y, z = Dd^T y
            H = 2 * (Dd * w) @ Dd.T + gamma * H_G
            rhs = 2 * (Dd * w) @ T
            y = np.zeros(N)
            if S:
                HS = H[np.ix_(S, S)]
                try:
                    y[S] = np.linalg.solve(HS, rhs[S])
                except np.linalg.LinAlgError:
                    continue
            if np.any(y < -1e-12):
                continue
            y = np.maximum(y, 0)
            z = Dd.T @ y
            F, dF = O.penalty(z, alpha, beta, T)
            G, dG = O.smoothing(y, th, circ)
            grad = Dd @ dF + gamma * dG
            if any(grad[k] < -1e-9 for k in occ_idx if k not in S):
                continue
            f = F + gamma * G
            if best is None or f < best[0]:
                best = (f, y)
    return best


def test_master_small_problems_vs_enumeration():
    rng = np.random.default_rng(16)
    for trial in range(25):
        N, nv = 4, 5
        Dd = rng.random((N, nv)) * (rng.random((N, nv)) < 0.8)
        alpha = np.where(rng.random(nv) < 0.5, rng.random(nv) + 0.1, 0.0)
        beta = rng.random(nv) + 0.1
        T = rng.random(nv) * 5
        th = np.array([0.0, 80.0, 170.0, 260.0])
        gamma = 0.05 * trial
        occ = np.array([1, 1, 0, 1], np.uint8) if trial % 3 else np.ones(4, np.uint8)
        best = _enumerate_kkt(Dd, alpha, beta, T, th, gamma, 1, occ)
        D = sp.csr_matrix(Dd)
        m = O.master(D, alpha, beta, T, th, gamma, 1, 1, 1, np.zeros(N, int), np.ones(N, int), occ,
                     np.zeros(N), O.MasterOpts(tol_rel=1e-12, max_iter=2000))
        f = m.F + m.gG
        assert f == pytest.approx(best[0], rel=1e-9, abs=1e-12)


def test_master_kkt_and_monotone_on_generated_case():
    import casegen
    c = casegen.make_case(casegen.tiny_case(n_beams=6, n_rows=3, n_cols=5))
    D = O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels)
    N, R, C = c.n_beams, c.n_rows, c.n_cols
    occ = np.array([1, 0, 1, 1, 0, 1], np.uint8)
    l = np.tile([0, 1, 0], N)
    r = np.tile([5, 4, 3], N)
    m = O.master(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, 1, R, C, l, r, occ, np.zeros(N),
                 O.MasterOpts(tol_rel=1e-9, max_iter=1000))
    assert m.converged
    F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), m.y, l, r, occ, c.gamma,
                                        c.theta_deg, 1, R, C)
    kkt = np.abs(np.minimum(m.y, grad))[occ == 1].max()
    assert kkt <= 1e-9 * m.kkt_ref * 1.0001
    assert np.all(m.y[occ == 0] == 0)


# ---------------------------------------------------------------- column generation

def test_column_generation_invariants():
    import casegen
    for delta, circ in ((2, 1), (1, 0), (-1, 1)):
        c = casegen.make_case(casegen.tiny_case(n_beams=8, n_rows=4, n_cols=6, circular=circ,
                                                max_leaf_step=delta))
        D = O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels)
        N, R, C = c.n_beams, c.n_rows, c.n_cols
        res = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, circ, R, C, delta)
        assert sorted(res.order) == list(range(N))                # one aperture per beam
        costs = res.costs
        assert costs[0] == pytest.approx(float(np.sum(c.alpha.astype(float) * c.T.astype(float) ** 2)))
        for a, b in zip(costs[:-1], costs[1:]):
            assert b <= a * (1 + 1e-12)                           # cost never increases
        lk, rk = res.l.reshape(N, R), res.r.reshape(N, R)
        assert np.all(lk <= rk) and np.all(lk >= 0) and np.all(rk <= C)
        if delta >= 0:
            pairs = [(k, k + 1) for k in range(N - 1)] + ([(N - 1, 0)] if circ else [])
            for a, b in pairs:
                assert np.all(np.abs(lk[a] - lk[b]) <= delta)
                assert np.all(np.abs(rk[a] - rk[b]) <= delta)
        assert np.all(res.y >= 0)


# ---------------------------------------------------------------- reduced precision

def test_bf16_fp16_rounding_match_library():
    import torch
    rng = np.random.default_rng(17)
    v = (rng.random(100000) * 2).astype(np.float32)
    v[:10] = [0.0, 1.0, 1.00390625, 1.005859375, 0.5, 3.0, 1e-3, 0.99609375, 1.0078125, 2.0]
    np.testing.assert_array_equal(O.bf16_round(v), torch.from_numpy(v).to(torch.bfloat16).float().numpy())
    np.testing.assert_array_equal(O.fp16_round(v), torch.from_numpy(v).half().float().numpy())


def test_e4m3_table_and_encoder_match_library():
    import torch
    codes = torch.arange(256, dtype=torch.uint8)
    lib = codes.view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    mine = O.e4m3_values()
    same = (lib == mine) | (np.isnan(lib) & np.isnan(mine))
    assert same.all()
    rng = np.random.default_rng(18)
    v = np.concatenate([rng.random(200000) * 448.0, mine[:127]])
    lib_codes = torch.from_numpy(v.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(O.e4m3_encode(v.astype(np.float32).astype(np.float64)), lib_codes)


def test_fp8_quantisation_error_bound():
    import casegen
    c = casegen.make_case(casegen.tiny_case())
    scale, q = O.fp8_quantise(c.row_ptr, c.val)
    dq = O.fp8_dequantise(c.row_ptr, scale, q)
    rel = np.abs(dq - c.val) / c.val
    assert rel.max() <= 2.0 ** -4 + 1e-12          # 3 mantissa bits: half-ulp <= 2^-4 relative
    D = O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels)
    Dh = O.dose_matrix(c.row_ptr, c.col, dq, c.n_voxels)
    x = np.random.default_rng(19).random(D.shape[0])
    B = O.quantisation_bound(D, Dh, x)
    assert np.all(np.abs(O.dose(Dh, x) - O.dose(D, x)) <= B * (1 + 1e-12) + 1e-300)


# ---------------------------------------------------------------- dose-rate feasibility (Sec. 3)

def _two_beam_problem(T1, T2):
    """Two beams (open chain, 10 degrees apart), one beamlet each, each dosing
    its own voxel with D = 1; alpha = beta = 1, so F = (y1-T1)^2 + (y2-T2)^2 in
    every regime and the master optimum solves
    [1 + g/10, -g/10; -g/10, 1 + g/10] y = (T1, T2):  y2 - y1 = (T2-T1)/(1 + g/5)."""
    D = sp.csr_matrix(np.eye(2))
    th = np.array([0.0, 10.0])
    one = np.ones(2)
    return D, th, one, np.array([T1, T2])


def _two_beam_optimum(T1, T2, g):
    diff = (T2 - T1) / (1.0 + g / 5.0)
    s = T1 + T2
    return np.array([(s - diff) / 2, (s + diff) / 2])


def test_rate_continuation_two_beams_closed_form():
    T1, T2 = 10.0, 20.0
    D, th, one, T = _two_beam_problem(T1, T2)
    l, r, occ = np.zeros(2, int), np.ones(2, int), np.ones(2, np.uint8)
    y0 = _two_beam_optimum(T1, T2, 0.1)
    # rates per degree: 1/(1+g/5) at g = 0.1, 1, 10, 100 -> 0.980, 0.833, 0.333, 0.0476
    res = O.enforce_rate(D, one, one, T, th, 0.1, 0, 1, 1, l, r, occ, y0, rate_max=0.2, factor=10.0,
                         opts=O.MasterOpts(tol_rel=1e-12))
    assert res.rounds == 3 and res.feasible
    assert res.gamma == pytest.approx(100.0, rel=1e-12)
    np.testing.assert_allclose(res.y, _two_beam_optimum(T1, T2, 100.0), rtol=1e-9)
    assert res.rate == pytest.approx(1.0 / 21.0, rel=1e-8)
    # G of each round's optimum: ((T2-T1)/(1+g/5))^2 / 10 for g = 1, 10, 100
    np.testing.assert_allclose(res.smoothing, [(10 / (1 + g / 5)) ** 2 / 10 for g in (1.0, 10.0, 100.0)],
                               rtol=1e-8)


def test_rate_continuation_feasible_plan_untouched_and_round_cap():
    T1, T2 = 10.0, 20.0
    D, th, one, T = _two_beam_problem(T1, T2)
    l, r, occ = np.zeros(2, int), np.ones(2, int), np.ones(2, np.uint8)
    y0 = _two_beam_optimum(T1, T2, 0.1)
    res = O.enforce_rate(D, one, one, T, th, 0.1, 0, 1, 1, l, r, occ, y0, rate_max=1.0)
    assert res.rounds == 0 and res.feasible and res.gamma == 0.1
    np.testing.assert_array_equal(res.y, y0)
    res = O.enforce_rate(D, one, one, T, th, 0.1, 0, 1, 1, l, r, occ, y0, rate_max=1e-6, max_rounds=2)
    assert res.rounds == 2 and not res.feasible and res.gamma == pytest.approx(10.0)


def test_rate_continuation_on_generated_case():
    """After a full plan: G of the re-optimised intensities never increases
    from round to round (the optimum's G is non-increasing in gamma for a
    convex objective), and the last round is a KKT point at its gamma."""
    import casegen
    c = casegen.make_case(casegen.tiny_case(n_beams=8, n_rows=3, n_cols=6, grid=(12, 12, 8), thr=0.3))
    D = O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels)
    sol = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                  c.max_leaf_step)
    G0, _ = O.smoothing(sol.y, c.theta_deg, c.circular)
    rate0 = O.max_rate(sol.y, c.theta_deg, c.circular)
    assert rate0 > 0
    opts = O.MasterOpts(tol_rel=1e-10, max_iter=2000)
    res = O.enforce_rate(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, c.n_rows, c.n_cols,
                         sol.l, sol.r, sol.occ, sol.y, rate_max=0.25 * rate0, factor=4.0, opts=opts)
    assert res.rounds >= 1
    Gs = [G0] + res.smoothing
    assert all(b <= a * (1 + 1e-9) + 1e-12 for a, b in zip(Gs, Gs[1:]))
    assert res.feasible == (res.rate <= 0.25 * rate0)
    F, gG, z, dF, g, grad = O.objective(D, (c.alpha, c.beta, c.T), res.y, sol.l, sol.r, sol.occ, res.gamma,
                                        c.theta_deg, c.circular, c.n_rows, c.n_cols)
    occ = sol.occ.astype(bool)
    kkt = np.abs(np.minimum(res.y, grad))[occ].max()
    assert kkt <= 1e-8 * abs(sol.prices[0])


# ---------------------------------------------------------------- property tests (Hypothesis)

try:
    from hypothesis import given, settings, strategies as st
except ImportError:  # pragma: no cover
    given = None

if given is not None:
    def _brute_row_prefix(g, Llo, Lhi, Rlo, Rhi):
        # every feasible pair; S from prefix sums accumulated in column order
        P = [0.0]
        for v in g:
            P.append(P[-1] + v)
        best = None
        for l in range(Llo, Lhi + 1):
            for r in range(max(l, Rlo), Rhi + 1):
                key = (P[r] - P[l], r - l, l)
                if best is None or key < best[0]:
                    best = (key, l, r)
        return best

    @settings(max_examples=400, deadline=None, derandomize=True)
    @given(st.lists(st.integers(-400, 400), min_size=1, max_size=12), st.data())
    def test_price_row_property_vs_bruteforce(gi, data):
        """Rows of multiples of 1/8 (every prefix sum exact in FP64, so exact
        ties stay ties) and any window: the one-pass search finds the least S
        over every feasible pair, with the (S, r-l, l) tie rule.  (With
        arbitrary reals, rounding can make two different sums equal; the
        one-pass rule then keeps the exactly smaller one.)"""
        g = [v / 8.0 for v in gi]
        C = len(g)
        a = data.draw(st.integers(0, C))
        b = data.draw(st.integers(a, C))
        c = data.draw(st.integers(0, C))
        d = data.draw(st.integers(c, C))
        S, l, r = O.price_row(np.asarray(g, float), a, b, c, d)
        if a > d:
            assert (l, r) == (-1, -1)
            return
        br = _brute_row_prefix(g, a, b, c, d)
        assert (l, r) == (br[1], br[2])
        assert S == br[0][0]

    @settings(max_examples=200, deadline=None, derandomize=True)
    @given(st.lists(st.floats(min_value=0, max_value=100, allow_nan=False), min_size=1, max_size=20),
           st.floats(min_value=0, max_value=5), st.floats(min_value=0, max_value=5),
           st.floats(min_value=0, max_value=100))
    def test_penalty_property_convex_and_derivative(z, alpha, beta, T):
        """eq. 1 per voxel: F >= 0, F = 0 exactly at z = T, F' matches a central
        difference away from the kink, and F is convex along any segment."""
        z = np.asarray(z, float)
        n = len(z)
        a, b, t = np.full(n, alpha), np.full(n, beta), np.full(n, T)
        F, dF = O.penalty(z, a, b, t)
        assert F >= 0
        F0, d0 = O.penalty(t, a, b, t)
        assert F0 == 0 and not d0.any()
        h = 1e-4
        away = np.abs(z - T) > 2 * h
        Fp = np.array([O.penalty(np.array([v + h]), a[:1], b[:1], t[:1])[0] for v in z])
        Fm = np.array([O.penalty(np.array([v - h]), a[:1], b[:1], t[:1])[0] for v in z])
        fd = (Fp - Fm) / (2 * h)
        assert np.allclose(fd[away], dF[away], rtol=1e-6, atol=1e-6)
        mid, _ = O.penalty(0.5 * (z + t[::-1]), a, b, t)
        e1, _ = O.penalty(z, a, b, t)
        e2, _ = O.penalty(t[::-1], a, b, t)
        assert mid <= 0.5 * (e1 + e2) + 1e-9 * (1 + e1 + e2)
