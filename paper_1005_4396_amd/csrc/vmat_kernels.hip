// Hot-path kernels: fluence expansion, the sparse dose product and its adjoint,
// the eq. 1 penalty with its derivative, the exact line search reductions, and
// the single-workgroup control steps of the gradient-projection master.
//
// Determinism: no floating-point atomics anywhere.  Every reduction runs in a
// fixed order (per-lane sequential, fixed shuffle tree, fixed number of blocks
// with a fixed-order final sum), so repeated runs are bitwise identical.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>

#include "vmat_block.h"
#include "vmat_ctrl.h"
#include "vmat_formats.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"

namespace vmat {

constexpr int BLOCK = 256;
// Line-search passes per master iteration (captured with the iteration): 3,
// or VMAT_LS_PASSES (1, 3, 5 or 7) as read when an iteration is captured or
// launched.  The grouping of passes into replays changes no result: a search
// that needs more passes than a replay holds stalls that replay and goes on in
// the next.  The count must be odd: pass i writes state buffer i % 2 and
// partial-sum buffer i % 2, so after an odd chain the step kernel reads ms2
// and the second partial-sum half while it writes ms and the first half; an
// even chain would have it read what its own blocks write.  Other values
// take the default.
static int ls_passes() {
    const char* e = getenv("VMAT_LS_PASSES");
    const int n = e ? atoi(e) : 3;
    return n >= 1 && n <= 7 && (n & 1) ? n : 3;
}

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

// Four block sums at once: each value takes block_sum's tree (wave tree,
// then (w0 + w1) + (w2 + w3)), so the results are those of four block_sum
// calls, with one barrier round instead of four.  Valid on thread 0.
__device__ __forceinline__ void block_sum4(double v[4], double* sh16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) sh16[q * 4 + (threadIdx.x >> 6)] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (sh16[q * 4 + 0] + sh16[q * 4 + 1]) + (sh16[q * 4 + 2] + sh16[q * 4 + 3]);
    __syncthreads();
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
                                                       int fresh, uint32_t seq) {
    for (int k = threadIdx.x; k < N; k += CTRL)
        if (!occ[k]) y[k] = 0.0;
    if (threadIdx.x == 0) {
        MasterState s = {};
        s.seq = seq;
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
    k_master_begin<<<1, CTRL, 0, st>>>(h->N, y, occ, h->ms, max_iter, ls_max, tol, kkt_ref, fresh, h->chains);
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

// Sums of a[i] over n entries for NA arrays a = part + q n, q < NA, each in
// the fixed order of reduce_part; valid on thread 0.
template <int NA>
__device__ __forceinline__ void reduce_parts(const double* part, int n, double* out, double* sh) {
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    for (int i = threadIdx.x; i < n; i += BLOCK)
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[q] += part[(int64_t)q * n + i];
    if constexpr (NA == 4) {
        __shared__ double sh16[16];
        block_sum4(acc, sh16);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = acc[q];
    } else {
#pragma unroll
        for (int q = 0; q < NA; ++q) out[q] = block_sum(acc[q], sh);
    }
}

// Penalty weights of the voxels: abT per voxel, or (LAB) a one-byte label per
// voxel into a table staged in LDS.  Both give the same float4.  The table is
// staged at its full capacity (WTAB_CAP entries, unused ones zero), so a
// captured kernel stays valid when vmat_set_weights changes the number of
// distinct triples.
struct VoxW {
    const float4* abT;
    const uint8_t* lab;
    const float4* tab;
    int n_tab;  // > 0: labels in use
};

inline VoxW voxw(const vmat_ctx* h) { return VoxW{h->abT, h->wlab, h->wtab, h->n_wtab}; }

template <bool LAB>
__device__ __forceinline__ void stage_tab(const VoxW& vw, float4* stab) {
    if (LAB)
        for (int i = threadIdx.x; i < WTAB_CAP; i += BLOCK) stab[i] = vw.tab[i];
}

// U voxels a grid stride apart, loaded before any arithmetic so that a grid
// of a few hundred blocks keeps enough loads in flight.  Voxels past nv read
// as z = dz = 0 with finite weights and add exact zeros.
template <int U, bool LAB>
struct VoxLoad {
    double z[U], dz[U];
    float4 w[U];
    __device__ __forceinline__ void load(int64_t j0, int64_t stride, int64_t nv, const double* __restrict__ zp,
                                         const double* __restrict__ dzp, const VoxW& vw, const float4* stab) {
        uint32_t lv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + u * stride;
            const bool in = j < nv;
            z[u] = in ? zp[j] : 0.0;
            dz[u] = in ? dzp[j] : 0.0;
            if (LAB) lv[u] = in ? vw.lab[j] : 0u;
            else w[u] = in ? vw.abT[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (LAB)
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = stab[lv[u]];
    }
};

// phi'(t), phi''(t) voxel sums at one or two points.
template <int U, bool LAB>
__device__ __forceinline__ void ls_sums(int64_t nv, const double* __restrict__ z, const double* __restrict__ dz,
                                        const VoxW& vw, const float4* stab, double ta, double tb, bool two,
                                        double acc[4]) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j0 < nv; j0 += U * stride) {
        VoxLoad<U, LAB> v;
        v.load(j0, stride, nv, z, dz, vw, stab);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const Pen a = penalty_at(v.z[u] + ta * v.dz[u], v.w[u]);
            acc[0] += v.dz[u] * a.dF;
            acc[1] += v.dz[u] * v.dz[u] * a.curv;
            if (two) {
                const Pen b = penalty_at(v.z[u] + tb * v.dz[u], v.w[u]);
                acc[2] += v.dz[u] * b.dF;
                acc[3] += v.dz[u] * v.dz[u] * b.curv;
            }
        }
    }
}

// A chain of line-search passes in which each pass first completes the
// previous one: every block reduces the previous partial sums in the same
// fixed order and takes the control step on its own copy of the state read
// from src (identical in all blocks); block 0 writes that state to dst, the
// other buffer of the pair, so no block reads what another writes.  Padding
// voxels (zero dz, zero weights) add exact zeros.
template <bool LAB>
__global__ __launch_bounds__(BLOCK) void k_ls_fused(int64_t nv, const double* __restrict__ z,
                                                    const double* __restrict__ dz, VoxW vw,
                                                    const MasterState* __restrict__ src, MasterState* __restrict__ dst,
                                                    int consume, const double* __restrict__ part_in,
                                                    double* __restrict__ part_out, int n_part,
                                                    MasterMirror* mirror) {
    __shared__ double sh[4];
    __shared__ MasterState s;
    __shared__ int run;
    __shared__ float4 stab[LAB ? 256 : 1];
    if (threadIdx.x == 0) s = *src;
    stage_tab<LAB>(vw, stab);
    __syncthreads();
    const bool active = !(s.done == 1 || s.ls_done);
    if (consume && active) {
        double r[4];
        reduce_parts<4>(part_in, n_part, r, sh);
        if (threadIdx.x == 0) ctrl_ls_pass(s, r[0], r[1], r[2], r[3]);
    }
    if (threadIdx.x == 0) {
        // the last pass of a chain (mirror set) counts the chain and shows the
        // state to the host
        if (mirror) s.seq += 1;
        if (blockIdx.x == 0) {
            *dst = s;
            if (mirror) {
                mirror->s[s.seq & 1u] = s;
                __hip_atomic_store(&mirror->seq, s.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        run = !(s.done == 1 || s.ls_done);
    }
    __syncthreads();
    if (!run) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    ls_sums<8, LAB>(nv, z, dz, vw, stab, s.t_eval, s.t_eval2, s.n_eval == 2, acc);
    __shared__ double sh16[16];
    block_sum4(acc, sh16);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) part_out[(int64_t)q * n_part + blockIdx.x] = acc[q];
}

// The buffers of pass i of a chain: it reads the state from bufs[(i-1) % 2]
// and the previous partials from parts[(i-1) % 2], writes bufs[i % 2] and
// parts[i % 2].  The last pass's sums are consumed by the next step.
static void ls_buffers(const vmat_ctx* h, MasterState* bufs[2], double* parts[2]) {
    bufs[0] = h->ms;
    bufs[1] = h->ms2;
    parts[0] = h->part;
    parts[1] = h->part + 4 * (int64_t)h->n_part;
}

vmat_status launch_ls_passes(const vmat_ctx* h, hipStream_t st) {
    MasterState* bufs[2];
    double* parts[2];
    ls_buffers(h, bufs, parts);
    const VoxW vw = voxw(h);
    const int np = ls_passes();
    for (int i = 1; i <= np; ++i) {
        MasterMirror* mir = i == np ? h->mirror_dev : nullptr;
        if (vw.n_tab > 0)
            k_ls_fused<true><<<h->n_part, BLOCK, 0, st>>>(h->nv, h->z, h->dz, vw, bufs[(i - 1) % 2], bufs[i % 2],
                                                         i > 1, parts[(i - 1) % 2], parts[i % 2], h->n_part, mir);
        else
            k_ls_fused<false><<<h->n_part, BLOCK, 0, st>>>(h->nv, h->z, h->dz, vw, bufs[(i - 1) % 2], bufs[i % 2],
                                                          i > 1, parts[(i - 1) % 2], parts[i % 2], h->n_part, mir);
        VMAT_LAUNCH_CHECK();
    }
    return VMAT_OK;
}

// The step and the dose update in one launch, after a chain of line-search
// passes.  Every block first completes the chain's last pass on its own copy
// of the state (the same fixed-order reduction and control step in all
// blocks); block 0 writes the result to the master state.  If the line search
// is still unfinished the iteration stalls (done = 2: the kernels after this
// one skip, the next chain continues the search); otherwise the stall is
// released, block 0 moves y (and the previous direction, gradient and face),
// and all blocks update the dose, F'(z) and the partial sums of F, U voxels
// a grid stride apart per thread and sweep (each thread adds its voxels' F in
// increasing index order for any U).
template <bool LAB, int U>
__global__ __launch_bounds__(BLOCK) void k_update_step(MasterPtrs m, const MasterState* __restrict__ src,
                                                       const double* __restrict__ part_ls, int64_t nv,
                                                       double* __restrict__ z, const double* __restrict__ dz,
                                                       VoxW vw, float* __restrict__ rz, double* __restrict__ part,
                                                       int n_part) {
    __shared__ double sh[4];
    __shared__ MasterState s;
    __shared__ float4 stab[LAB ? 256 : 1];
    if (threadIdx.x == 0) s = *src;
    stage_tab<LAB>(vw, stab);
    __syncthreads();
    if (s.done != 1 && !s.ls_done) {
        double r[4];
        reduce_parts<4>(part_ls, n_part, r, sh);
        if (threadIdx.x == 0) {
            ctrl_ls_pass(s, r[0], r[1], r[2], r[3]);
            if (!s.ls_done) s.done = 2;
        }
    }
    if (threadIdx.x == 0 && s.done == 2 && s.ls_done) s.done = 0;
    if (threadIdx.x == 0 && s.done == 0) s.have_prev = 1;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *m.ms = s;
    if (s.done != 0) return;
    const double t = s.t_star;
    if (blockIdx.x == 0) ctrl_step_vec(m, t, s.t_max);
    double F = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j0 < nv; j0 += U * stride) {
        VoxLoad<U, LAB> v;
        v.load(j0, stride, nv, z, dz, vw, stab);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + u * stride;
            const double zj = v.z[u] + t * v.dz[u];
            const Pen p = penalty_at(zj, v.w[u]);
            if (j < nv) {
                z[j] = zj;
                rz[j] = (float)p.dF;
                F += p.F;
            }
        }
    }
    F = block_sum(F, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = F;
}

vmat_status launch_step_update(const vmat_ctx* h, double* y, hipStream_t st) {
    MasterState* bufs[2];
    double* parts[2];
    ls_buffers(h, bufs, parts);
    const int np = ls_passes();  // the last pass of the chain wrote bufs[np % 2], parts[np % 2]
    const VoxW vw = voxw(h);
    const MasterPtrs m = master_ptrs(h, y, nullptr, nullptr, nullptr);
    // eight voxels per thread where the grid covers the dose in one sweep
    // (prostate plans 0.4-0.9% faster than four, same bits), four otherwise
    // (head-and-neck plan 0.4% faster than eight)
    const bool one_sweep = h->nv <= (int64_t)h->n_part * BLOCK * 8;
    auto go = [&](auto kern) {
        kern<<<h->n_part, BLOCK, 0, st>>>(m, bufs[np % 2], parts[np % 2], h->nv, h->z, h->dz, vw, h->rz, h->part,
                                          h->n_part);
    };
    if (vw.n_tab > 0)
        one_sweep ? go(k_update_step<true, 8>) : go(k_update_step<true, 4>);
    else
        one_sweep ? go(k_update_step<false, 8>) : go(k_update_step<false, 4>);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// Gradient after a step, then the KKT test and the next direction, in one
// single-block launch (k_master_grad followed by k_master_dir).  bpart
// (nullable): the beam gradient in Q parts per beam (gF_k = sum of
// bpart[k*Q .. k*Q+Q-1] in order), written to gF first.  With lds, the
// per-beam vectors and the state are copied to LDS with one round of loads,
// the same control code runs on the copies, and the outputs (gradient, face,
// direction, gF, state) are written back once: the same arithmetic without a
// global round trip between its phases.
__global__ __launch_bounds__(CTRL) void k_grad_dir(MasterPtrs m, const double* __restrict__ part, int n_part,
                                                   const double* __restrict__ bpart, int Q, int lds) {
    __shared__ double sh[4];
    __shared__ int shi[4];
    __shared__ MasterState s_ms;
    extern __shared__ double dyn[];
    if (m.ms->done) return;
    const int N = m.N;
    if (lds) {
        double* y = dyn;
        double* gF = y + N;
        double* grad = gF + N;
        double* grad_prev = grad + N;
        double* d = grad_prev + N;
        double* d_prev = d + N;
        double* th = d_prev + N;
        uint8_t* occ = reinterpret_cast<uint8_t*>(th + N);
        uint8_t* W = occ + N;
        uint8_t* W_prev = W + N;
        for (int k = threadIdx.x; k < N; k += CTRL) {
            double g = 0.0;
            if (bpart)
                for (int q = 0; q < Q; ++q) g += bpart[(int64_t)k * Q + q];
            else
                g = m.gF[k];
            gF[k] = g;
            y[k] = m.y[k];
            grad_prev[k] = m.grad_prev[k];
            d_prev[k] = m.d_prev[k];
            th[k] = m.th[k];
            occ[k] = m.occ[k];
            W_prev[k] = m.W_prev[k];
        }
        if (threadIdx.x == 0) s_ms = *m.ms;
        __syncthreads();
        MasterPtrs L = m;
        L.y = y; L.gF = gF; L.grad = grad; L.grad_prev = grad_prev; L.d = d; L.d_prev = d_prev; L.th = th;
        L.occ = occ; L.W = W; L.W_prev = W_prev; L.ms = &s_ms;
        const double F = reduce_part(part, n_part, sh);
        ctrl_grad(L, F, 0, sh);
        __syncthreads();
        ctrl_dir(L, sh, shi);
        __syncthreads();
        for (int k = threadIdx.x; k < N; k += CTRL) {
            m.grad[k] = grad[k];
            m.d[k] = d[k];
            m.W[k] = W[k];
            if (bpart) m.gF[k] = gF[k];
        }
        if (threadIdx.x == 0) *m.ms = s_ms;
        return;
    }
    if (bpart) {
        for (int k = threadIdx.x; k < N; k += CTRL) {
            double g = 0.0;
            for (int q = 0; q < Q; ++q) g += bpart[(int64_t)k * Q + q];
            m.gF[k] = g;
        }
        __syncthreads();
    }
    const double F = reduce_part(part, n_part, sh);
    ctrl_grad(m, F, 0, sh);
    __syncthreads();
    ctrl_dir(m, sh, shi);
}

vmat_status launch_grad_dir(const vmat_ctx* h, const double* y, const uint8_t* occ, const double* bpart, int Q,
                            hipStream_t st) {
    // VMAT_GRAD_DIR_GLOBAL: the global-memory form (read when an iteration is
    // captured or launched directly)
    const size_t dyn = (size_t)h->N * (7 * sizeof(double) + 3);
    const int lds = dyn <= 48 * 1024 && !getenv("VMAT_GRAD_DIR_GLOBAL") ? 1 : 0;
    k_grad_dir<<<1, CTRL, lds ? dyn : 0, st>>>(master_ptrs(h, const_cast<double*>(y), occ, nullptr, nullptr), h->part,
                                               h->n_part, Q > 0 ? bpart : nullptr, Q, lds);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

}  // namespace vmat
