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
#include "vmat_ctrl.h"
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
                                                   double* __restrict__ x, Gate gate) {
    if (gate.closed()) return;
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
                           const uint8_t* occ, const float* scale, double* x, Gate gate,
                           hipStream_t st) {
    const unsigned grid = (unsigned)((h->nb + BLOCK - 1) / BLOCK);
    k_fluence<<<grid, BLOCK, 0, st>>>(h->nb, h->R, h->C, v, l, r, occ, scale, x, gate);
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
                                                Gate gate) {
    if (gate.closed()) return;
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
static vmat_status spmv_fmt(const QuadCsr& A, const XT* x, double* out, Gate gate, hipStream_t st) {
    const int G = A.lanes_per_row;
    const unsigned grid = (unsigned)((A.n_rows * G + BLOCK - 1) / BLOCK);
    if (grid == 0) return VMAT_OK;
    switch (G) {
        case 4: k_spmv<FMT, 4, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, gate); break;
        case 8: k_spmv<FMT, 8, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, gate); break;
        case 16: k_spmv<FMT, 16, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, gate); break;
        case 32: k_spmv<FMT, 32, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, gate); break;
        default: k_spmv<FMT, 64, XT><<<grid, BLOCK, 0, st>>>(A.qptr, A.col, A.val, A.scale, A.n_rows, x, out, gate); break;
    }
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

template <typename XT>
static vmat_status spmv_any(const vmat_ctx* h, const QuadCsr& A, const XT* x, double* out, Gate gate,
                            hipStream_t st) {
    switch (h->d_store) {
        case VMAT_F32: return spmv_fmt<FMT_F32>(A, x, out, gate, st);
        case VMAT_F16: return spmv_fmt<FMT_F16>(A, x, out, gate, st);
        case VMAT_BF16: return spmv_fmt<FMT_BF16>(A, x, out, gate, st);
        default: return spmv_fmt<FMT_FP8>(A, x, out, gate, st);
    }
}

vmat_status launch_spmv(const vmat_ctx* h, const QuadCsr& A, const double* x, double* out, Gate gate,
                        hipStream_t st) {
    return spmv_any(h, A, x, out, gate, st);
}

vmat_status launch_spmv(const vmat_ctx* h, const QuadCsr& A, const float* x, double* out, Gate gate,
                        hipStream_t st) {
    return spmv_any(h, A, x, out, gate, st);
}

// ---------------------------------------------------------------- eq. 1 penalty

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
                                                     Gate gate) {
    __shared__ double sh[4];
    if (gate.closed()) return;
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
                             const uint8_t* occ, double* out, Gate gate, hipStream_t st) {
    k_beam_sums<<<h->N, BLOCK, 0, st>>>(h->R, h->C, g, l, r, occ, out, gate);
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

__global__ __launch_bounds__(CTRL) void k_dfdy(int N, const double* __restrict__ y, const double* __restrict__ th,
                                               int circ, double gamma, const double* __restrict__ gF,
                                               double* __restrict__ dfdy) {
    for (int k = threadIdx.x; k < N; k += CTRL) dfdy[k] = gF[k] + gamma * dG_at(k, y, th, N, circ);
}

vmat_status launch_dfdy(const vmat_ctx* h, const double* y, const double* gF, double* dfdy, hipStream_t st) {
    k_dfdy<<<1, CTRL, 0, st>>>(h->N, y, h->d_theta, h->circular, h->gamma, gF, dfdy);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

vmat_status launch_cost_only(const vmat_ctx* h, double* cost, hipStream_t st) {
    k_grad_finish<<<1, CTRL, 0, st>>>(h->N, h->part, h->n_part, nullptr, h->d_theta, h->circular, h->gamma,
                                     nullptr, cost, nullptr, 1);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// Largest intensity change per degree over the eq. 2 pairs, and G.
__global__ __launch_bounds__(CTRL) void k_max_rate(int N, int circ, const double* __restrict__ y,
                                                   const double* __restrict__ th, double* __restrict__ out) {
    __shared__ double sh[4];
    double m = 0.0;
    for (int p = threadIdx.x; p < n_pairs(N, circ); p += CTRL) {
        int a, b;
        double w;
        smoothing_pair(p, N, circ, th, a, b, w);
        m = fmax(m, fabs(y[b] - y[a]) / w);
    }
    m = bmax(m, sh);
    const double G = smoothing_G(y, th, N, circ, sh);
    if (threadIdx.x == 0) {
        out[0] = m;
        out[1] = G;
    }
}

vmat_status launch_max_rate(const vmat_ctx* h, const double* y, double* out, hipStream_t st) {
    k_max_rate<<<1, CTRL, 0, st>>>(h->N, h->circular, y, h->d_theta, out);
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
__global__ __launch_bounds__(CTRL) void k_master_grad(MasterPtrs m, const double* __restrict__ part, int n_part,
                                                      int first) {
    __shared__ double sh[4];
    if (!first && m.ms->done) return;
    const double F = reduce_part(part, n_part, sh);
    ctrl_grad(m, F, first, sh);
}

vmat_status launch_master_grad(const vmat_ctx* h, const double* y, const uint8_t* occ, int first, hipStream_t st) {
    k_master_grad<<<1, CTRL, 0, st>>>(master_ptrs(h, const_cast<double*>(y), occ, nullptr, nullptr), h->part,
                                     h->n_part, first);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// KKT test, then the search direction on the free face and the line-search set-up.
__global__ __launch_bounds__(CTRL) void k_master_dir(MasterPtrs m) {
    __shared__ double sh[4];
    __shared__ int shi[4];
    ctrl_dir(m, sh, shi);
}

vmat_status launch_master_dir(const vmat_ctx* h, const double* y, const uint8_t* occ, hipStream_t st) {
    k_master_dir<<<1, CTRL, 0, st>>>(master_ptrs(h, const_cast<double*>(y), occ, nullptr, nullptr));
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// phi'(t) and phi''(t) partial sums over voxels at t = t_eval.
__global__ __launch_bounds__(BLOCK) void k_ls_eval(int64_t nv, const double* __restrict__ z,
                                                   const double* __restrict__ dz, const float4* __restrict__ abT,
                                                   const MasterState* __restrict__ ms, double* __restrict__ part,
                                                   int n_part) {
    __shared__ double sh[4];
    if (ms->done == 1 || ms->ls_done) return;
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

// A chain of line-search evaluations in which each evaluation first completes
// the previous one: every block reduces the previous partial sums in the same
// fixed order and applies the safeguarded-Newton step to its own copy of the
// state read from src (identical in all blocks); block 0 writes that state to
// dst, the other buffer of the pair, so no block reads what another writes.
// The same arithmetic as alternating evaluation and control launches.
__global__ __launch_bounds__(BLOCK) void k_ls_fused(int64_t nv, const double* __restrict__ z,
                                                    const double* __restrict__ dz, const float4* __restrict__ abT,
                                                    const MasterState* __restrict__ src, MasterState* __restrict__ dst,
                                                    int consume, const double* __restrict__ part_in,
                                                    double* __restrict__ part_out, int n_part) {
    __shared__ double sh[4];
    __shared__ MasterState s;
    __shared__ int run;
    const double pF = consume ? reduce_part(part_in, n_part, sh) : 0.0;
    const double hF = consume ? reduce_part(part_in + n_part, n_part, sh) : 0.0;
    if (threadIdx.x == 0) {
        s = *src;
        if (consume && !(s.done == 1 || s.ls_done)) ctrl_ls_step(s, pF, hF);
        if (blockIdx.x == 0) *dst = s;
        run = !(s.done == 1 || s.ls_done);
    }
    __syncthreads();
    if (!run) return;
    const double t = s.t_eval;
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
        part_out[blockIdx.x] = p;
        part_out[n_part + blockIdx.x] = q;
    }
}

// Completes the last evaluation of a chain: state src -> dst (may alias).
__global__ __launch_bounds__(BLOCK) void k_ls_finish(const MasterState* src, MasterState* dst,
                                                     const double* __restrict__ part, int n_part) {
    __shared__ double sh[4];
    const double pF = reduce_part(part, n_part, sh);
    const double hF = reduce_part(part + n_part, n_part, sh);
    if (threadIdx.x == 0) {
        MasterState s = *src;
        if (!(s.done == 1 || s.ls_done)) ctrl_ls_step(s, pF, hF);
        *dst = s;
    }
}

vmat_status launch_ls_chain(const vmat_ctx* h, int n, hipStream_t st) {
    MasterState* bufs[2] = {h->ms, h->ms2};
    double* parts[2] = {h->part, h->part + 2 * (int64_t)h->n_part};
    for (int i = 1; i <= n; ++i) {
        k_ls_fused<<<h->n_part, BLOCK, 0, st>>>(h->nv, h->z, h->dz, h->abT, bufs[(i - 1) % 2], bufs[i % 2], i > 1,
                                               parts[(i - 1) % 2], parts[i % 2], h->n_part);
        VMAT_LAUNCH_CHECK();
    }
    k_ls_finish<<<1, BLOCK, 0, st>>>(bufs[n % 2], bufs[0], parts[n % 2], h->n_part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// Safeguarded Newton on the piecewise-linear, non-decreasing phi' inside a bracket.
__global__ __launch_bounds__(BLOCK) void k_ls_ctrl(MasterState* ms, const double* __restrict__ part, int n_part) {
    __shared__ double sh[4];
    if (ms->done == 1 || ms->ls_done) return;
    const double pF = reduce_part(part, n_part, sh);
    const double hF = reduce_part(part + n_part, n_part, sh);
    if (threadIdx.x == 0) ctrl_ls_step(*ms, pF, hF);
}

vmat_status launch_ls_ctrl(const vmat_ctx* h, hipStream_t st) {
    k_ls_ctrl<<<1, BLOCK, 0, st>>>(h->ms, h->part, h->n_part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// y <- max(0, y + t* d); bounds that block at t* = t_max become exactly 0.
__global__ __launch_bounds__(CTRL) void k_master_step(MasterPtrs m) {
    if (m.ms->done) return;
    ctrl_step(m);
}

vmat_status launch_master_step(const vmat_ctx* h, double* y, hipStream_t st) {
    k_master_step<<<1, CTRL, 0, st>>>(master_ptrs(h, y, nullptr, nullptr, nullptr));
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

// The step and the dose update in one launch: block 0 also moves y (and the
// previous direction, gradient and face) as k_master_step does; the update
// reads only t* and the dose vectors, which the step does not touch.  An
// unfinished line search stalls the iteration (done = 2: the kernels after
// this one skip, the line-search evaluations continue); a finished one
// releases it.  Every block takes the same decision: done == 1 and ls_done
// are not written here, and the value block 0 writes is never 1.
__global__ __launch_bounds__(BLOCK) void k_update_step(MasterPtrs m, int64_t nv, double* __restrict__ z,
                                                       const double* __restrict__ dz,
                                                       const float4* __restrict__ abT, float* __restrict__ rz,
                                                       double* __restrict__ part) {
    __shared__ double sh[4];
    MasterState* ms = m.ms;
    if (ms->done == 1) return;
    if (!ms->ls_done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) ms->done = 2;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ms->done = 0;
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
    if (blockIdx.x == 0) ctrl_step(m);
}

vmat_status launch_step_update(const vmat_ctx* h, double* y, hipStream_t st) {
    k_update_step<<<h->n_part, BLOCK, 0, st>>>(master_ptrs(h, y, nullptr, nullptr, nullptr), h->nv, h->z, h->dz,
                                               h->abT, h->rz, h->part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// Gradient after a step, then the KKT test and the next direction, in one
// single-block launch (k_master_grad followed by k_master_dir).
__global__ __launch_bounds__(CTRL) void k_grad_dir(MasterPtrs m, const double* __restrict__ part, int n_part) {
    __shared__ double sh[4];
    __shared__ int shi[4];
    if (m.ms->done) return;
    const double F = reduce_part(part, n_part, sh);
    ctrl_grad(m, F, 0, sh);
    __syncthreads();
    ctrl_dir(m, sh, shi);
}

vmat_status launch_grad_dir(const vmat_ctx* h, const double* y, const uint8_t* occ, hipStream_t st) {
    k_grad_dir<<<1, CTRL, 0, st>>>(master_ptrs(h, const_cast<double*>(y), occ, nullptr, nullptr), h->part,
                                   h->n_part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

}  // namespace vmat
