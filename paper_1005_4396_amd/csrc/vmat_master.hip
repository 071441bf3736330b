// Master iteration (Sec. 2.2, gradient projection) as a gated kernel pipeline.
//
// Every kernel of an iteration carries a gate on the device-resident phase
// and returns at once outside it; only single-workgroup control kernels move
// the phase on, so kernel boundaries give all the ordering needed:
//   READY      fluence(d) staged inside the forward; dz = D^T x
//   READY|LS   line-search evaluation phi'(t), phi''(t); control -> LS | LS_DONE
//   LS_DONE    z += t* dz, F'(z), partial sums of F, y step; adjoint;
//              beamlet prices and aperture sums; control: gradient, KKT
//              test, next direction -> READY | DONE
// The host enqueues the fixed pattern for several iterations and reads the
// state once per chunk; a line search that needs more evaluations than its
// slots goes on in the next iteration's slots.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "vmat_block.h"
#include "vmat_ctrl.h"
#include "vmat_formats.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"
#include "vmat_rows.h"

namespace vmat {

constexpr int MAX_WAVES = TILE_THREADS / 64;
constexpr uint32_t M_READY = 1u << PH_READY, M_LS = 1u << PH_LS, M_LS_DONE = 1u << PH_LS_DONE;

// Sum over the block (any multiple of 64 threads up to TILE_THREADS); valid on thread 0.
__device__ __forceinline__ double block_total(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    __syncthreads();
    return r;
}

// Fixed-order sum of n partials by the whole block; valid on thread 0.
__device__ __forceinline__ double sum_partials(const double* p, int n, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
    return block_total(s, sh);
}

__device__ __forceinline__ bool phase_in(const MasterState* ms, uint32_t mask) { return (1u << ms->phase) & mask; }

// Forward with the fluence of the direction built while the block's beamlets
// are staged: x_i = d_k on the aperture of beam k (times the FP8 scale).
template <int FMT, int G, int U>
__global__ __launch_bounds__(TILE_THREADS) void k_mfwd(const int4* __restrict__ work, const uint32_t* __restrict__ loff,
                                                     const uint32_t* __restrict__ list,
                                                     const uint32_t* __restrict__ lpack,
                                                     const uint32_t* __restrict__ qptr,
                                                     const uint16_t* __restrict__ col16, const void* __restrict__ val,
                                                     const float* __restrict__ scale, MasterPtrs m,
                                                     double* __restrict__ dz) {
    __shared__ double xs[TILE_LIST];
    __shared__ uint32_t rq[TILE_ROWS + 1];
    if (!phase_in(m.ms, M_READY)) return;
    const int4 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    const uint32_t l0 = loff[wk.x], ln = loff[wk.x + 1] - l0;
    const int nrows = wk.z - wk.y;
    stage_rows(rq, qptr + wk.y, nrows);
    constexpr int K = TILE_LIST / TILE_THREADS;
    uint32_t pk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t u = threadIdx.x + k * TILE_THREADS;
        pk[k] = u < ln ? lpack[l0 + u] : 0u;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t u = threadIdx.x + k * TILE_THREADS;
        if (u < ln) {
            const uint32_t kb = pk[k] >> 20, rho = (pk[k] >> 8) & 0xFFFu, c = pk[k] & 0xFFu;
            const int64_t kr = (int64_t)kb * m.R + rho;
            double v = (m.occ[kb] && (int)c >= m.l[kr] && (int)c < m.r[kr]) ? m.d[kb] : 0.0;
            if (scale) v *= (double)scale[list[l0 + u]];
            xs[u] = v;
        }
    }
    __syncthreads();
    StoreRow epi{dz};
    rows_of_item<FMT, G, U, double>(rq, nrows, wk.y, val, reinterpret_cast<const u16x4*>(col16), xs, epi);
}

// phi'(t_eval), phi''(t_eval) partial sums over voxels.
__global__ __launch_bounds__(CTRL) void k_mls(int64_t nv, const double* __restrict__ z, const double* __restrict__ dz,
                                              const float4* __restrict__ abT, const MasterState* __restrict__ ms,
                                              double* __restrict__ part, int n_part) {
    __shared__ double sh[MAX_WAVES];
    if (!phase_in(ms, M_READY | M_LS)) return;
    const double t = ms->t_eval;
    double p = 0.0, q = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * CTRL + threadIdx.x; j < nv; j += (int64_t)gridDim.x * CTRL) {
        const double dzj = dz[j];
        const Pen pn = penalty_at(z[j] + t * dzj, abT[j]);
        p += dzj * pn.dF;
        q += dzj * dzj * pn.curv;
    }
    p = block_total(p, sh);
    q = block_total(q, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = p;
        part[n_part + blockIdx.x] = q;
    }
}

__global__ __launch_bounds__(CTRL) void k_mls_ctrl(MasterState* ms, const double* __restrict__ part, int n_part) {
    __shared__ double sh[MAX_WAVES];
    if (!phase_in(ms, M_READY | M_LS)) return;
    const double pF = sum_partials(part, n_part, sh);
    const double hF = sum_partials(part + n_part, n_part, sh);
    if (threadIdx.x == 0) ctrl_ls_step(*ms, pF, hF);
}

// z += t* dz, F'(z) for the adjoint, partial sums of F; workgroup 0 steps y.
__global__ __launch_bounds__(CTRL) void k_mupdate(int64_t nv, double* __restrict__ z, const double* __restrict__ dz,
                                                  const float4* __restrict__ abT, float* __restrict__ rz, MasterPtrs m,
                                                  double* __restrict__ partF) {
    __shared__ double sh[MAX_WAVES];
    if (!phase_in(m.ms, M_LS_DONE)) return;
    const double t = m.ms->t_star;
    double F = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * CTRL + threadIdx.x; j < nv; j += (int64_t)gridDim.x * CTRL) {
        const double zj = z[j] + t * dz[j];
        z[j] = zj;
        const Pen pn = penalty_at(zj, abT[j]);
        F += pn.F;
        rz[j] = (float)pn.dF;
    }
    F = block_total(F, sh);
    if (threadIdx.x == 0) partF[blockIdx.x] = F;
    if (blockIdx.x == 0) ctrl_step(m);
}

// One workgroup per beam: the beam's beamlet prices (from the slot sums of
// the tiled adjoint, or as written by the plain one) and their sum over the
// aperture.
__global__ __launch_bounds__(CTRL) void k_mfinish(MasterPtrs m, const uint32_t* __restrict__ red_ptr,
                                                  const uint32_t* __restrict__ red_slot,
                                                  const double* __restrict__ slot_sum,
                                                  const float* __restrict__ scale, double* __restrict__ g) {
    __shared__ double sh[MAX_WAVES];
    if (!phase_in(m.ms, M_LS_DONE)) return;
    const int k = blockIdx.x;
    const int RC = m.R * m.C;
    const int64_t base = (int64_t)k * RC;
    const bool occk = m.occ[k] != 0;
    double acc = 0.0;
    for (int e = threadIdx.x; e < RC; e += CTRL) {
        const int64_t i = base + e;
        double s;
        if (red_ptr) {
            s = 0.0;
            for (uint32_t q = red_ptr[i]; q < red_ptr[i + 1]; ++q) s += slot_sum[red_slot[q]];
            if (scale) s *= (double)scale[i];
            g[i] = s;
        } else {
            s = g[i];
        }
        const int rho = e / m.C, c = e - rho * m.C;
        const int64_t kr = (int64_t)k * m.R + rho;
        if (occk && c >= m.l[kr] && c < m.r[kr]) acc += s;
    }
    acc = block_total(acc, sh);
    if (threadIdx.x == 0) m.gF[k] = acc;
}

// Gradient, cost, KKT test and the next direction.
__global__ __launch_bounds__(CTRL) void k_mgrad_dir(MasterPtrs m, const double* __restrict__ partF, int n_part) {
    __shared__ double sh[MAX_WAVES];
    __shared__ int shi[4];
    __shared__ double Fs;
    if (!phase_in(m.ms, M_LS_DONE)) return;
    const double F = sum_partials(partF, n_part, sh);
    if (threadIdx.x == 0) Fs = F;
    __syncthreads();
    ctrl_grad(m, Fs, 0, sh);
    __syncthreads();
    ctrl_dir(m, sh, shi);
}

__global__ __launch_bounds__(CTRL) void k_mdir(MasterPtrs m) {
    __shared__ double sh[4];
    __shared__ int shi[4];
    ctrl_dir(m, sh, shi);
}

template <int FMT>
static void launch_mfwd(const vmat_ctx* h, const MasterPtrs& m, hipStream_t st) {
    const Tiled& t = h->tl;
#define MF(GG) k_mfwd<FMT, GG, FWD_U><<<(unsigned)t.n_fwork, TILE_THREADS, 0, st>>>( \
        t.fwork, t.loff, t.list, t.lpack, h->vm.qptr, t.fcol, h->vm.val, h->bm.scale, m, h->dz)
    switch (t.fG) {
        case 2: MF(2); break;
        case 4: MF(4); break;
        case 8: MF(8); break;
        case 16: MF(16); break;
        default: MF(32); break;
    }
#undef MF
}

static vmat_status enqueue_iteration(vmat_ctx* h, const MasterPtrs& m, int n_ls, hipStream_t st) {
    Gate ready, ls_done;
    ready.p = ls_done.p = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(h->ms) +
                                                           offsetof(MasterState, phase));
    ready.mask = M_READY;
    ls_done.mask = M_LS_DONE;
    if (h->tl.on && h->tl.lpack) {
        switch (h->d_store) {
            case VMAT_F32: launch_mfwd<FMT_F32>(h, m, st); break;
            case VMAT_F16: launch_mfwd<FMT_F16>(h, m, st); break;
            case VMAT_BF16: launch_mfwd<FMT_BF16>(h, m, st); break;
            default: launch_mfwd<FMT_FP8>(h, m, st); break;
        }
        VMAT_LAUNCH_CHECK();
    } else {
        vmat_status rc = launch_fluence(h, m.d, m.l, m.r, m.occ, h->bm.scale, h->x, ready, st);
        if (rc == VMAT_OK) rc = launch_fwd(h, h->x, h->dz, ready, st);
        if (rc != VMAT_OK) return rc;
    }
    for (int i = 0; i < n_ls; ++i) {
        k_mls<<<h->n_part, CTRL, 0, st>>>(h->nv, h->z, h->dz, h->abT, h->ms, h->part, h->n_part);
        VMAT_LAUNCH_CHECK();
        k_mls_ctrl<<<1, CTRL, 0, st>>>(h->ms, h->part, h->n_part);
        VMAT_LAUNCH_CHECK();
    }
    double* partF = h->part + 2 * h->n_part;
    k_mupdate<<<h->n_part, CTRL, 0, st>>>(h->nv, h->z, h->dz, h->abT, h->rz, m, partF);
    VMAT_LAUNCH_CHECK();
    vmat_status rc = h->tl.on ? launch_adj_slots(h, h->rz, ls_done, st) : launch_adj(h, h->rz, h->g, ls_done, st);
    if (rc != VMAT_OK) return rc;
    k_mfinish<<<h->N, CTRL, 0, st>>>(m, h->tl.on ? h->tl.red_ptr : nullptr, h->tl.red_slot, h->tl.part, h->bm.scale,
                                     h->g);
    VMAT_LAUNCH_CHECK();
    k_mgrad_dir<<<1, CTRL, 0, st>>>(m, partF, h->n_part);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// Iterations enqueued between two reads of the state, and line-search
// evaluations enqueued per iteration.
constexpr int CHUNK_ITERS = 4;
constexpr int LS_SLOTS = 3;

vmat_status run_master_fused(vmat_ctx* h, const int32_t* l, const int32_t* r, const uint8_t* occ, double* y,
                             const vmat_master_opts& o, int fresh, hipStream_t st) {
    MasterPtrs m = master_ptrs(h, y, occ, l, r);
    vmat_status rc = launch_master_begin(h, y, occ, o.max_iter, o.ls_max_steps, o.tol_rel, o.kkt_ref, fresh, st);
    if (rc != VMAT_OK) return rc;
    if (fresh) {
        if ((rc = launch_fluence(h, y, l, r, occ, h->bm.scale, h->x, Gate{}, st)) != VMAT_OK) return rc;
        if ((rc = launch_fwd(h, h->x, h->z, Gate{}, st)) != VMAT_OK) return rc;
    }
    if ((rc = launch_penalty(h, h->z, nullptr, nullptr, st)) != VMAT_OK) return rc;
    if (fresh && (rc = launch_adj(h, h->rz, h->g, Gate{}, st)) != VMAT_OK) return rc;
    if ((rc = launch_beam_sums(h, h->g, l, r, occ, h->mgF, Gate{}, st)) != VMAT_OK) return rc;
    if ((rc = launch_master_grad(h, y, occ, fresh ? 1 : 2, st)) != VMAT_OK) return rc;
    k_mdir<<<1, CTRL, 0, st>>>(m);
    VMAT_LAUNCH_CHECK();
    // an iteration needs at most 2 + ls_max line-search evaluations
    const int64_t max_chunks =
        ((int64_t)o.max_iter + 1) * (((int64_t)o.ls_max_steps + 2 + LS_SLOTS - 1) / LS_SLOTS) / CHUNK_ITERS + 4;
    for (int64_t chunk = 0;; ++chunk) {
        for (int i = 0; i < CHUNK_ITERS; ++i)
            if ((rc = enqueue_iteration(h, m, LS_SLOTS, st)) != VMAT_OK) return rc;
        VMAT_HIP(hipMemcpyAsync(h->ms_host, h->ms, sizeof(MasterState), hipMemcpyDeviceToHost, st));
        VMAT_HIP(hipStreamSynchronize(st));
        if (h->ms_host->phase == PH_DONE) break;
        if (chunk > max_chunks) return fail(VMAT_ERR_DEVICE, "master pipeline made no progress");
    }
    return VMAT_OK;
}

}  // namespace vmat
