// Hot-path kernels: fluence expansion, the sparse dose product and its adjoint,
// the eq. 1 penalty with its derivative, the exact line search reductions, and
// the single-workgroup control steps of the gradient-projection master.
//
// Determinism: no floating-point atomics anywhere.  Every reduction runs in a
// fixed order (per-lane sequential, fixed shuffle tree, fixed number of blocks
// with a fixed-order final sum), so repeated runs are bitwise identical.
#include <hip/hip_runtime.h>

#include <cmath>

#include "vmat_block.h"
#include "vmat_formats.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"

namespace vmat {

constexpr int BLOCK = 256;

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a 256-thread block; the result is valid on thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double reduce_part(const double* part, int n, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += BLOCK) s += part[i];
    return block_sum(s, sh);
}

// ---------------------------------------------------------------- fluence

__global__ __launch_bounds__(BLOCK) void k_fluence(int64_t nb, int R, int C, const double* __restrict__ v,
                                                   const int32_t* __restrict__ l, const int32_t* __restrict__ r,
                                                   const uint8_t* __restrict__ occ, const float* __restrict__ scale,
                                                   double* __restrict__ x, const int32_t* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= nb) return;
    const int64_t kr = i / C;
    const int c = (int)(i - kr * C);
    const int64_t k = kr / R;
    double xi = 0.0;
    if (occ[k] && c >= l[kr] && c < r[kr]) xi = v[k];
    if (scale) xi *= (double)scale[i];
    x[i] = xi;
}

vmat_status launch_fluence(const vmat_ctx* h, const double* v, const int32_t* l, const int32_t* r,
                           const uint8_t* occ, const float* scale, double* x, const int32_t* skip,
                           hipStream_t st) {
    const unsigned grid = (unsigned)((h->nb + BLOCK - 1) / BLOCK);
    k_fluence<<<grid, BLOCK, 0, st>>>(h->nb, h->R, h->C, v, l, r, occ, scale, x, skip);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// ---------------------------------------------------------------- sparse products
// G lanes cooperate on one row: lane t of the group reads quads t, t+G, ...
// (one 16-byte index load and one value load per quad), gathers the 4 x
// values, and accumulates in FP64; the group then sums with a shuffle tree.

template <int FMT, int G, typename XT>
__global__ __launch_bounds__(BLOCK) void k_spmv(const uint32_t* __restrict__ qptr, const int32_t* __restrict__ col,
                                                const void* __restrict__ val, const float* __restrict__ rscale,
                                                int64_t nrows, const XT* __restrict__ x, double* __restrict__ out,
                                                const int32_t* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t row = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / G;
    const int lane = threadIdx.x & (G - 1);
    double acc = 0.0;
    if (row < nrows) {
        const uint32_t q0 = qptr[row], q1 = qptr[row + 1];
        const i32x4* c4 = reinterpret_cast<const i32x4*>(col);
        for (uint32_t q = q0 + lane; q < q1; q += G) {
            const float4 v = Quad<FMT>::load(val, q);
            const i32x4 c = __builtin_nontemporal_load(c4 + q);
            acc = fma((double)v.x, (double)x[c.x], acc);
            acc = fma((double)v.y, (double)x[c.y], acc);
            acc = fma((double)v.z, (double)x[c.z], acc);
            acc = fma((double)v.w, (double)x[c.w], acc);
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    if (row < nrows && lane == 0) out[row] = rscale ? acc * (double)rscale[row] : acc;
}

template <int FMT, typename XT>
static vmat_status spmv_fmt(const QuadCsr& A, const XT* x, double* out, const int32_t* skip, hipStream_t st) {
    const int G = A.lanes_per_row;
    const unsigned grid = (unsigned)((A.n_rows * G + BLOCK - 1) / BLOCK);
    if (grid == 0) return VMAT_OK;
    switch (G) {
        case 4: k_spmv<FMT, 4, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, skip); break;
        case 8: k_spmv<FMT, 8, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, skip); break;
        case 16: k_spmv<FMT, 16, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, skip); break;
        case 32: k_spmv<FMT, 32, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, skip); break;
        default: k_spmv<FMT, 64, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, skip); break;
    }
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

template <typename XT>
static vmat_status spmv_any(const vmat_ctx* h, const QuadCsr& A, const XT* x, double* out, const int32_t* skip,
                            hipStream_t st) {
    switch (h->d_store) {
        case VMAT_F32: return spmv_fmt<FMT_F32>(A, x, out, skip, st);
        case VMAT_F16: return spmv_fmt<FMT_F16>(A, x, out, skip, st);
        case VMAT_BF16: return spmv_fmt<FMT_BF16>(A, x, out, skip, st);
        default: return spmv_fmt<FMT_FP8>(A, x, out, skip, st);
    }
}

vmat_status launch_spmv(const vmat_ctx* h, const QuadCsr& A, const double* x, double* out, const int32_t* skip,
                        hipStream_t st) {
    return spmv_any(h, A, x, out, skip, st);
}

vmat_status launch_spmv(const vmat_ctx* h, const QuadCsr& A, const float* x, double* out, const int32_t* skip,
                        hipStream_t st) {
    return spmv_any(h, A, x, out, skip, st);
}

// ---------------------------------------------------------------- eq. 1 penalty

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

__global__ __launch_bounds__(BLOCK) void k_penalty(int64_t nv, const double* __restrict__ z,
                                                   const float4* __restrict__ abT, float* __restrict__ rz,
                                                   float* __restrict__ zo, float* __restrict__ dfo,
                                                   double* __restrict__ part) {
    __shared__ double sh[4];
    double F = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < nv; j += (int64_t)gridDim.x * BLOCK) {
        const double zj = z[j];
        const Pen p = penalty_at(zj, abT[j]);
        F += p.F;
        rz[j] = (float)p.dF;
        if (zo) zo[j] = (float)zj;
        if (dfo) dfo[j] = (float)p.dF;
    }
    F = block_sum(F, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = F;
}

vmat_status launch_penalty(const vmat_ctx* h, const double* z, float* z_out, float* dF_out, hipStream_t st) {
    k_penalty<<<h->n_part, BLOCK, 0, st>>>(h->nv, z, h->abT, h->rz, z_out, dF_out, h->part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// ---------------------------------------------------------------- beam sums

__global__ __launch_bounds__(BLOCK) void k_beam_sums(int R, int C, const double* __restrict__ g,
                                                     const int32_t* __restrict__ l, const int32_t* __restrict__ r,
                                                     const uint8_t* __restrict__ occ, double* __restrict__ out,
                                                     const int32_t* __restrict__ skip) {
    __shared__ double sh[4];
    if (skip && *skip) return;
    const int k = blockIdx.x;
    if (!occ[k]) {
        if (threadIdx.x == 0) out[k] = 0.0;
        return;
    }
    const int RC = R * C;
    const double* gk = g + (int64_t)k * RC;
    double s = 0.0;
    for (int e = threadIdx.x; e < RC; e += BLOCK) {
        const int rho = e / C, c = e - rho * C;
        const int64_t kr = (int64_t)k * R + rho;
        if (c >= l[kr] && c < r[kr]) s += gk[e];
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[k] = s;
}

vmat_status launch_beam_sums(const vmat_ctx* h, const double* g, const int32_t* l, const int32_t* r,
                             const uint8_t* occ, double* out, const int32_t* skip, hipStream_t st) {
    k_beam_sums<<<h->N, BLOCK, 0, st>>>(h->R, h->C, g, l, r, occ, out, skip);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// ---------------------------------------------------------------- cost assembly

__global__ __launch_bounds__(CTRL) void k_grad_finish(int N, const double* __restrict__ part, int n_part,
                                                      const double* __restrict__ y, const double* __restrict__ th,
                                                      int circ, double gamma, const double* __restrict__ gF,
                                                      double* __restrict__ cost, double* __restrict__ dfdy,
                                                      int cost_only) {
    __shared__ double sh[4];
    const double F = reduce_part(part, n_part, sh);
    if (cost_only) {
        if (threadIdx.x == 0) cost[0] = F;
        return;
    }
    const double G = smoothing_G(y, th, N, circ, sh);
    if (threadIdx.x == 0) {
        cost[0] = F;
        cost[1] = gamma * G;
    }
    if (dfdy)
        for (int k = threadIdx.x; k < N; k += CTRL) dfdy[k] = gF[k] + gamma * dG_at(k, y, th, N, circ);
}

vmat_status launch_grad_finish(const vmat_ctx* h, const double* y, const double* gF, double* cost, double* dfdy,
                               hipStream_t st) {
    k_grad_finish<<<1, CTRL, 0, st>>>(h->N, h->part, h->n_part, y, h->d_theta, h->circular, h->gamma, gF, cost,
                                     dfdy, 0);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

vmat_status launch_cost_only(const vmat_ctx* h, double* cost, hipStream_t st) {
    k_grad_finish<<<1, CTRL, 0, st>>>(h->N, h->part, h->n_part, nullptr, h->d_theta, h->circular, h->gamma,
                                     nullptr, cost, nullptr, 1);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// ---------------------------------------------------------------- master control (one workgroup)
// All per-beam work is spread over the 256 threads; scalars are combined with
// fixed-order block reductions and written by thread 0.

__global__ __launch_bounds__(CTRL) void k_master_begin(int N, double* __restrict__ y,
                                                       const uint8_t* __restrict__ occ, MasterState* ms,
                                                       int max_iter, int ls_max, double tol, double kkt_ref,
                                                       int fresh) {
    for (int k = threadIdx.x; k < N; k += CTRL)
        if (!occ[k]) y[k] = 0.0;
    if (threadIdx.x == 0) {
        MasterState s = {};
        s.max_iter = max_iter;
        s.ls_max = ls_max;
        s.tol = tol;
        s.kkt_ref = kkt_ref;
        s.n_fwd = fresh ? 1 : 0;
        s.ls_done = 1;
        *ms = s;
    }
}

vmat_status launch_master_begin(const vmat_ctx* h, double* y, const uint8_t* occ, int max_iter, int ls_max,
                                double tol, double kkt_ref, int fresh, hipStream_t st) {
    k_master_begin<<<1, CTRL, 0, st>>>(h->N, y, occ, h->ms, max_iter, ls_max, tol, kkt_ref, fresh);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// After the adjoint: grad = sum over the aperture + gamma dG/dy; cost; iteration count.
__global__ __launch_bounds__(CTRL) void k_master_grad(int N, const double* __restrict__ part, int n_part,
                                                      const double* __restrict__ y, const uint8_t* __restrict__ occ,
                                                      const double* __restrict__ th, int circ, double gamma,
                                                      const double* __restrict__ gF, double* __restrict__ grad,
                                                      MasterState* ms, int first) {
    __shared__ double sh[4];
    if (!first && ms->done) return;
    const double F = reduce_part(part, n_part, sh);
    const double G = smoothing_G(y, th, N, circ, sh);
    double ref = 0.0;
    for (int k = threadIdx.x; k < N; k += CTRL) {
        const double gk = gF[k] + gamma * dG_at(k, y, th, N, circ);
        grad[k] = gk;
        if (occ[k]) ref = fmax(ref, fabs(gk));
    }
    ref = bmax(ref, sh);
    if (threadIdx.x != 0) return;
    MasterState& s = *ms;
    s.F = F;
    s.gG = gamma * G;
    if (first != 2) s.n_adj += 1;
    if (first) {
        s.it = 0;
        if (!(s.kkt_ref > 0.0)) s.kkt_ref = ref == 0.0 ? 1.0 : ref;
    } else {
        s.it += 1;
    }
}

vmat_status launch_master_grad(const vmat_ctx* h, const double* y, const uint8_t* occ, int first, hipStream_t st) {
    k_master_grad<<<1, CTRL, 0, st>>>(h->N, h->part, h->n_part, y, occ, h->d_theta, h->circular, h->gamma, h->mgF,
                                     h->mgrad, h->ms, first);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// KKT test, then the search direction on the free face and the line-search set-up.
__global__ __launch_bounds__(CTRL) void k_master_dir(int N, const double* __restrict__ y,
                                                     const double* __restrict__ grad,
                                                     const double* __restrict__ grad_prev, double* __restrict__ d,
                                                     const double* __restrict__ d_prev, uint8_t* __restrict__ W,
                                                     const uint8_t* __restrict__ W_prev,
                                                     const uint8_t* __restrict__ occ, const double* __restrict__ th,
                                                     int circ, double gamma, MasterState* ms) {
    __shared__ double sh[4];
    __shared__ int shi[4];
    if (ms->done) return;
    const int have_prev = ms->have_prev;
    double kkt = 0.0;
    int changed = 0;
    for (int k = threadIdx.x; k < N; k += CTRL) {
        if (occ[k]) kkt = fmax(kkt, fabs(fmin(y[k], grad[k])));
        const uint8_t w = occ[k] && (y[k] > 0.0 || grad[k] < 0.0);
        W[k] = w;
        if (w != W_prev[k]) changed = 1;
        d[k] = w ? -grad[k] : 0.0;
    }
    kkt = bmax(kkt, sh);
    changed = bor(changed, shi);
    const double tol_abs = ms->tol * ms->kkt_ref;
    if (kkt <= tol_abs || ms->it >= ms->max_iter) {
        __syncthreads();
        if (threadIdx.x == 0) {
            ms->kkt = kkt;
            ms->converged = kkt <= tol_abs;
            ms->done = 1;
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
        den = bsum(den, sh);
        num = bsum(num, sh);
        b_cg = den > 0.0 ? fmax(0.0, num / den) : 0.0;
        double slope = 0.0;
        for (int k = threadIdx.x; k < N; k += CTRL) {
            const double dc = W[k] ? -grad[k] + b_cg * d_prev[k] : 0.0;
            slope += dc * grad[k];
        }
        slope = bsum(slope, sh);
        if (slope < 0.0)
            for (int k = threadIdx.x; k < N; k += CTRL) d[k] = W[k] ? -grad[k] + b_cg * d_prev[k] : 0.0;
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
    tmax = bmin(tmax, sh);
    any = bor(any, shi);
    sl = bsum(sl, sh);
    const double curv = smoothing_dHd(d, th, N, circ, sh);
    if (threadIdx.x != 0) return;
    MasterState& s = *ms;
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
    s.ls_steps = 0;
    s.ls_done = 0;
    s.n_fwd += 1;
}

vmat_status launch_master_dir(const vmat_ctx* h, const double* y, const uint8_t* occ, hipStream_t st) {
    k_master_dir<<<1, CTRL, 0, st>>>(h->N, y, h->mgrad, h->mgrad_prev, h->md, h->md_prev, h->mW, h->mW_prev, occ,
                                    h->d_theta, h->circular, h->gamma, h->ms);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// phi'(t) and phi''(t) partial sums over voxels at t = t_eval.
__global__ __launch_bounds__(BLOCK) void k_ls_eval(int64_t nv, const double* __restrict__ z,
                                                   const double* __restrict__ dz, const float4* __restrict__ abT,
                                                   const MasterState* __restrict__ ms, double* __restrict__ part,
                                                   int n_part) {
    __shared__ double sh[4];
    if (ms->done || ms->ls_done) return;
    const double t = ms->t_eval;
    double p = 0.0, q = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < nv; j += (int64_t)gridDim.x * BLOCK) {
        const double dzj = dz[j];
        const Pen pn = penalty_at(z[j] + t * dzj, abT[j]);
        p += dzj * pn.dF;
        q += dzj * dzj * pn.curv;
    }
    p = block_sum(p, sh);
    q = block_sum(q, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = p;
        part[n_part + blockIdx.x] = q;
    }
}

vmat_status launch_ls_eval(const vmat_ctx* h, hipStream_t st) {
    k_ls_eval<<<h->n_part, BLOCK, 0, st>>>(h->nv, h->z, h->dz, h->abT, h->ms, h->part, h->n_part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// Safeguarded Newton on the piecewise-linear, non-decreasing phi' inside a bracket.
__global__ __launch_bounds__(BLOCK) void k_ls_ctrl(MasterState* ms, const double* __restrict__ part, int n_part) {
    __shared__ double sh[4];
    if (ms->done || ms->ls_done) return;
    const double pF = reduce_part(part, n_part, sh);
    const double hF = reduce_part(part + n_part, n_part, sh);
    if (threadIdx.x != 0) return;
    MasterState& s = *ms;
    const double t = s.t_eval;
    const double p = pF + s.slope0 + t * s.curv;
    const double hh = hF + s.curv;
    s.n_ls += 1;
    bool fin = false;
    double ts = 0.0;
    bool prop = false;
    if (s.ls_phase == 0) {
        s.p0 = p;
        s.h0 = hh;
        if (!(p < 0.0)) {
            fin = true;
            ts = 0.0;
        } else if (isfinite(s.t_max)) {
            s.ls_phase = 1;
            s.t_eval = s.t_max;
        } else {
            s.lo = 0.0; s.hi = INFINITY; s.t = 0.0; s.p = p; s.h = hh;
            s.ls_phase = 2; s.ls_steps = 0;
            prop = true;
        }
    } else if (s.ls_phase == 1) {
        if (p <= 0.0) {
            fin = true;
            ts = s.t_max;
        } else {
            s.lo = 0.0; s.hi = s.t_max; s.t = 0.0; s.p = s.p0; s.h = s.h0;
            s.ls_phase = 2; s.ls_steps = 0;
            prop = true;
        }
    } else {
        s.t = t; s.p = p; s.h = hh;
        s.ls_steps += 1;
        if (p <= 0.0) s.lo = t; else s.hi = t;
        if (fabs(p) <= 1e-12 * fabs(s.p0)) { fin = true; ts = t; }
        else if (isfinite(s.hi) && s.hi - s.lo <= 1e-15 * s.hi) { fin = true; ts = s.lo; }
        else if (s.ls_steps >= s.ls_max) { fin = true; ts = s.lo; }
        else prop = true;
    }
    if (fin) {
        s.t_star = ts;
        s.ls_done = 1;
    } else if (prop) {
        double tn = s.h > 0.0 ? s.t - s.p / s.h : NAN;
        if (!(s.lo < tn && tn < s.hi)) tn = isfinite(s.hi) ? 0.5 * (s.lo + s.hi) : (s.lo > 0.0 ? 2.0 * s.lo : 1.0);
        s.t_eval = tn;
    }
}

vmat_status launch_ls_ctrl(const vmat_ctx* h, hipStream_t st) {
    k_ls_ctrl<<<1, BLOCK, 0, st>>>(h->ms, h->part, h->n_part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// y <- max(0, y + t* d); bounds that block at t* = t_max become exactly 0.
__global__ __launch_bounds__(CTRL) void k_master_step(int N, double* __restrict__ y, const double* __restrict__ d,
                                                      double* __restrict__ d_prev, const double* __restrict__ grad,
                                                      double* __restrict__ grad_prev, const uint8_t* __restrict__ W,
                                                      uint8_t* __restrict__ W_prev, MasterState* ms) {
    if (ms->done) return;
    const double t = ms->t_star, tmax = ms->t_max;
    for (int k = threadIdx.x; k < N; k += CTRL) {
        const double yo = y[k], dk = d[k];
        double yn = fmax(0.0, yo + t * dk);
        if (t == tmax && dk < 0.0 && yo / (-dk) == tmax) yn = 0.0;
        y[k] = yn;
        d_prev[k] = dk;
        grad_prev[k] = grad[k];
        W_prev[k] = W[k];
    }
    if (threadIdx.x == 0) ms->have_prev = 1;
}

vmat_status launch_master_step(const vmat_ctx* h, double* y, hipStream_t st) {
    k_master_step<<<1, CTRL, 0, st>>>(h->N, y, h->md, h->md_prev, h->mgrad, h->mgrad_prev, h->mW, h->mW_prev, h->ms);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// z <- z + t* dz, then F'(z) for the adjoint and the partial sums of F.
__global__ __launch_bounds__(BLOCK) void k_update(int64_t nv, double* __restrict__ z, const double* __restrict__ dz,
                                                  const float4* __restrict__ abT, float* __restrict__ rz,
                                                  const MasterState* __restrict__ ms, double* __restrict__ part) {
    __shared__ double sh[4];
    if (ms->done) return;
    const double t = ms->t_star;
    double F = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < nv; j += (int64_t)gridDim.x * BLOCK) {
        const double zj = z[j] + t * dz[j];
        z[j] = zj;
        const Pen p = penalty_at(zj, abT[j]);
        F += p.F;
        rz[j] = (float)p.dF;
    }
    F = block_sum(F, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = F;
}

vmat_status launch_update(const vmat_ctx* h, hipStream_t st) {
    k_update<<<h->n_part, BLOCK, 0, st>>>(h->nv, h->z, h->dz, h->abT, h->rz, h->ms, h->part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

}  // namespace vmat
