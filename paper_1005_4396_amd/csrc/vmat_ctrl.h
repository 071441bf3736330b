// Control logic of the gradient-projection master (Sec. 2.2), shared by the
// separate-kernel and the fused master pipelines.  Each function runs on one
// workgroup of CTRL threads; scalars are combined with fixed-order reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "vmat_block.h"
#include "vmat_internal.h"

namespace vmat {

struct Pen {
    double F, dF, curv;
};

__device__ __forceinline__ Pen penalty_at(double z, float4 p) {
    const double a = p.x, b = p.y, T = p.z;
    const double under = fmax(0.0, T - z), over = fmax(0.0, z - T);
    Pen r;
    r.F = a * under * under + b * over * over;
    r.dF = 2.0 * b * over - 2.0 * a * under;
    r.curv = z < T ? 2.0 * a : 2.0 * b;
    return r;
}


struct MasterPtrs {
    int N, R, C, circ;
    const double* gamma;  // device scalar
    const double* th;
    double* y;
    const uint8_t* occ;
    const int32_t* l;
    const int32_t* r;
    double* grad;
    double* grad_prev;
    double* d;
    double* d_prev;
    uint8_t* W;
    uint8_t* W_prev;
    double* gF;
    MasterState* ms;
};

inline MasterPtrs master_ptrs(const vmat_ctx* h, double* y, const uint8_t* occ, const int32_t* l, const int32_t* r) {
    MasterPtrs m;
    m.N = h->N; m.R = h->R; m.C = h->C; m.circ = h->circular; m.gamma = h->d_gamma;
    m.th = h->d_theta; m.y = y; m.occ = occ; m.l = l; m.r = r;
    m.grad = h->mgrad; m.grad_prev = h->mgrad_prev; m.d = h->md; m.d_prev = h->md_prev;
    m.W = h->mW; m.W_prev = h->mW_prev; m.gF = h->mgF; m.ms = h->ms;
    return m;
}

// grad = gF + gamma dG/dy; cost; iteration count.  first: 0 after a step,
// 1 at a fresh start, 2 at a carried-over start.
__device__ inline void ctrl_grad(const MasterPtrs& m, double F, int first, double* sh) {
    const int N = m.N;
    double G = smoothing_G_part(m.y, m.th, N, m.circ);
    double ref = 0.0;
    for (int k = threadIdx.x; k < N; k += CTRL) {
        const double gk = m.gF[k] + *m.gamma * dG_at(k, m.y, m.th, N, m.circ);
        m.grad[k] = gk;
        if (m.occ[k]) ref = fmax(ref, fabs(gk));
    }
    bred2<RED_SUM, RED_MAX>(G, ref);
    (void)sh;
    if (threadIdx.x != 0) return;
    MasterState& s = *m.ms;
    s.F = F;
    s.gG = *m.gamma * G;
    if (first != 2) s.n_adj += 1;
    if (first) {
        s.it = 0;
        if (!(s.kkt_ref > 0.0)) s.kkt_ref = ref == 0.0 ? 1.0 : ref;
    } else {
        s.it += 1;
    }
}

// KKT test; if not converged, the direction on the free face (steepest
// descent after a face change, else Polak-Ribiere(+)), the first blocking
// bound and the line-search set-up.  f32_dir: the
// direction is rounded to FP32, the precision in which the batched products
// take it, so that y and the carried dose move by the same step.
__device__ inline void ctrl_dir(const MasterPtrs& m, double* sh, int* shi, bool f32_dir = false) {
    (void)shi;
    auto rnd = [f32_dir](double v) { return f32_dir ? (double)(float)v : v; };
    const int N = m.N;
    MasterState& s0 = *m.ms;
    const double* y = m.y;
    const double* grad = m.grad;
    const double* grad_prev = m.grad_prev;
    double* d = m.d;
    const double* d_prev = m.d_prev;
    uint8_t* W = m.W;
    const uint8_t* W_prev = m.W_prev;
    const uint8_t* occ = m.occ;
    const double* th = m.th;
    const int circ = m.circ;
    const double gamma = *m.gamma;
    if (s0.done) return;
    const int have_prev = s0.have_prev;
    double kkt = 0.0;
    int changed = 0;
    for (int k = threadIdx.x; k < N; k += CTRL) {
        if (occ[k]) kkt = fmax(kkt, fabs(fmin(y[k], grad[k])));
        const uint8_t w = occ[k] && (y[k] > 0.0 || grad[k] < 0.0);
        W[k] = w;
        if (w != W_prev[k]) changed = 1;
        d[k] = w ? rnd(-grad[k]) : 0.0;
    }
    double chg = __any(changed) ? 1.0 : 0.0;
    bred2<RED_MAX, RED_MAX>(kkt, chg);
    changed = chg != 0.0;
    const double tol_abs = s0.tol * s0.kkt_ref;
    if (kkt <= tol_abs || s0.it >= s0.max_iter) {
        __syncthreads();
        if (threadIdx.x == 0) {
            s0.kkt = kkt;
            s0.converged = kkt <= tol_abs;
            s0.done = 1;
        }
        return;
    }
    double b_cg = 0.0;
    if (have_prev && !changed) {
        double den = 0.0, num = 0.0;
        for (int k = threadIdx.x; k < N; k += CTRL) {
            const double gp = W[k] ? grad_prev[k] : 0.0, gw = W[k] ? grad[k] : 0.0;
            den += gp * gp;
            num += gw * (gw - gp);
        }
        bred2<RED_SUM, RED_SUM>(den, num);
        b_cg = den > 0.0 ? fmax(0.0, num / den) : 0.0;
        double slope = 0.0;
        for (int k = threadIdx.x; k < N; k += CTRL) {
            const double dc = W[k] ? -grad[k] + b_cg * d_prev[k] : 0.0;
            slope += dc * grad[k];
        }
        slope = bsum(slope, sh);
        if (slope < 0.0)
            for (int k = threadIdx.x; k < N; k += CTRL) d[k] = W[k] ? rnd(-grad[k] + b_cg * d_prev[k]) : 0.0;
        __syncthreads();
    }
    double tmax = INFINITY, sl = 0.0;
    int any = 0;
    for (int k = threadIdx.x; k < N; k += CTRL) {
        const double dk = d[k];
        if (dk < 0.0) tmax = fmin(tmax, y[k] / (-dk));
        if (dk != 0.0) any = 1;
        sl += dG_at(k, y, th, N, circ) * dk;
    }
    double curv = smoothing_dHd_part(d, th, N, circ);
    double anyd = __any(any) ? 1.0 : 0.0;
    bred4<RED_MIN, RED_MAX, RED_SUM, RED_SUM>(tmax, anyd, sl, curv);
    any = anyd != 0.0;
    if (threadIdx.x != 0) return;
    MasterState& s = s0;
    s.kkt = kkt;
    if (!any) {
        s.done = 1;
        return;
    }
    s.beta_cg = b_cg;
    s.slope0 = gamma * sl;
    s.curv = gamma * curv;
    s.t_max = tmax;
    s.ls_phase = 0;
    s.t_eval = 0.0;
    s.t_eval2 = tmax;
    s.n_eval = isfinite(tmax) ? 2 : 1;
    s.ls_steps = 0;
    s.ls_done = 0;
    s.n_fwd += 1;
}

// One pass of the exact line search that evaluated phi' and phi'' at one or
// two points (thread 0); pa, ha (pb, hb): the voxel sums at t_eval (t_eval2),
// the smoothing part is added here.  The first pass takes t = 0 and the first
// blocking bound t_max.  phi' is piecewise linear and non-decreasing; the
// bracket [lo, hi] keeps phi'(lo) <= 0 < phi'(hi) with phi', phi'' at both
// ends, and each later pass evaluates the Newton points from both ends (a
// Newton step from an end is exact when no breakpoint of phi' lies between it
// and the root), or one Newton point and the midpoint, or the midpoint alone,
// or doubling while no upper end is known.  The stopping tests are those of
// the one-point search: |phi'| <= 1e-12 |phi'(0)| at an evaluated point, a
// bracket narrower than 1e-15 hi, or ls_max passes after the first.
__device__ inline void ctrl_ls_pass(MasterState& s, double pa, double ha, double pb, double hb) {
    const int ne = s.n_eval;
    const double tv[2] = {s.t_eval, s.t_eval2};
    const double pv[2] = {pa + s.slope0 + s.t_eval * s.curv, pb + s.slope0 + s.t_eval2 * s.curv};
    const double hv[2] = {ha + s.curv, hb + s.curv};
    s.n_ls += 1;
    bool fin = false;
    double ts = 0.0;
    if (s.ls_phase == 0) {
        s.p0 = pv[0];
        s.h0 = hv[0];
        if (!(pv[0] < 0.0)) {
            fin = true;
            ts = 0.0;
        } else if (ne == 2 && pv[1] <= 0.0) {
            fin = true;
            ts = s.t_max;
        } else {
            s.lo = 0.0; s.plo = pv[0]; s.hlo = hv[0];
            if (ne == 2) { s.hi = s.t_max; s.phi = pv[1]; s.hhi = hv[1]; }
            else { s.hi = INFINITY; s.phi = 0.0; s.hhi = 0.0; }
            s.ls_phase = 2;
            s.ls_steps = 0;
        }
    } else {
        s.ls_steps += 1;
        for (int i = 0; i < ne && !fin; ++i)
            if (fabs(pv[i]) <= 1e-12 * fabs(s.p0)) { fin = true; ts = tv[i]; }
        if (!fin) {
            for (int i = 0; i < ne; ++i) {
                if (pv[i] <= 0.0) {
                    if (tv[i] > s.lo) { s.lo = tv[i]; s.plo = pv[i]; s.hlo = hv[i]; }
                } else if (tv[i] < s.hi) {
                    s.hi = tv[i]; s.phi = pv[i]; s.hhi = hv[i];
                }
            }
            if (isfinite(s.hi) && s.hi - s.lo <= 1e-15 * s.hi) { fin = true; ts = s.lo; }
            else if (s.ls_steps >= s.ls_max) { fin = true; ts = s.lo; }
        }
    }
    if (fin) {
        s.t_star = ts;
        s.ls_done = 1;
        return;
    }
    const bool bounded = isfinite(s.hi);
    double ta = s.hlo > 0.0 ? s.lo - s.plo / s.hlo : NAN;
    if (!(s.lo < ta && ta < s.hi)) ta = NAN;
    double tb = NAN;
    if (bounded && s.hhi > 0.0) {
        tb = s.hi - s.phi / s.hhi;
        if (!(s.lo < tb && tb < s.hi)) tb = NAN;
    }
    if (isnan(ta)) { ta = tb; tb = NAN; }
    const double mid = bounded ? 0.5 * (s.lo + s.hi) : (s.lo > 0.0 ? 2.0 * s.lo : 1.0);
    if (isnan(ta)) ta = mid;
    else if (isnan(tb) || tb == ta) tb = bounded ? mid : 2.0 * ta;
    if (tb == ta) tb = NAN;
    s.t_eval = ta;
    s.t_eval2 = isnan(tb) ? 0.0 : tb;
    s.n_eval = isnan(tb) ? 1 : 2;
}

// y <- max(0, y + t* d); bounds that block at t* = t_max become exactly 0;
// the direction, gradient and face become the previous ones.
__device__ inline void ctrl_step_vec(const MasterPtrs& m, double t, double tmax) {
    for (int k = threadIdx.x; k < m.N; k += CTRL) {
        const double yo = m.y[k], dk = m.d[k];
        double yn = fmax(0.0, yo + t * dk);
        if (t == tmax && dk < 0.0 && yo / (-dk) == tmax) yn = 0.0;
        m.y[k] = yn;
        m.d_prev[k] = dk;
        m.grad_prev[k] = m.grad[k];
        m.W_prev[k] = m.W[k];
    }
}

__device__ inline void ctrl_step(const MasterPtrs& m) {
    ctrl_step_vec(m, m.ms->t_star, m.ms->t_max);
    if (threadIdx.x == 0) m.ms->have_prev = 1;
}

}  // namespace vmat
