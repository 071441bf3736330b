// Plan variants sharing one D: products with many right-hand sides (SpMM)
// and the batched cost and gradient.
//
// Layout: RHS-contiguous, X[i*B + b] (beamlets) and Z[j*B + b] (voxels).  A
// row of D is read once per tile of TB right-hand sides; TB lanes of a wave
// share the row (its index and value loads are broadcasts) and gather TB
// consecutive values per non-zero, so each gather is one contiguous span.
// 64/TB rows go through a wave at once.  The tile width trades re-reading D
// (B/TB passes) against the footprint of the gathered RHS tile in the caches;
// vmat_tune_batched measures the choices on the actual problem.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "vmat_block.h"
#include "vmat_ctrl.h"
#include "vmat_formats.h"
#include "vmat_graph.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"

namespace vmat {

constexpr int SPMM_THREADS = 256;

// X[i][b] as the product needs it; FP8 storage keeps a scale per beamlet i,
// folded in here on the forward (column) side.
template <int FMT>
__device__ __forceinline__ double xval(const float* __restrict__ X, const float* __restrict__ cscale, uint32_t i,
                                       int B, int b) {
    const double v = (double)X[(int64_t)i * B + b];
    if constexpr (FMT == FMT_FP8) return v * (double)cscale[i];
    else return v;
}

// Forward, tiled layout: rows are voxels of the block, the block's beamlet
// list is staged in LDS and maps the 16-bit indices to beamlets.
template <int FMT, int TB>
__global__ __launch_bounds__(SPMM_THREADS) void k_spmm_fwd_tiled(const int4* __restrict__ work,
                                                                const uint32_t* __restrict__ loff,
                                                                const uint32_t* __restrict__ list,
                                                                const uint32_t* __restrict__ qptr,
                                                                const uint16_t* __restrict__ col16,
                                                                const void* __restrict__ val,
                                                                const float* __restrict__ cscale, int B,
                                                                const float* __restrict__ X, double* __restrict__ Z) {
    __shared__ uint32_t ls[TILE_LIST];
    const int4 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    const uint32_t l0 = loff[wk.x], ln = loff[wk.x + 1] - l0;
    for (uint32_t u = threadIdx.x; u < ln; u += SPMM_THREADS) ls[u] = list[l0 + u];
    __syncthreads();
    constexpr int RPW = 64 / TB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * TB + (lane % TB);
    const bool col_ok = b < B;
    const u16x4* c4 = reinterpret_cast<const u16x4*>(col16);
    for (int row = wk.y + wave * RPW + lane / TB; row < wk.z; row += (SPMM_THREADS / 64) * RPW) {
        double acc = 0.0;
        const uint32_t q1 = qptr[row + 1];
        for (uint32_t q = qptr[row]; q < q1; ++q) {
            const float4 v = Quad<FMT>::load(val, q);
            const u16x4 c = c4[q];
            if (col_ok) {
                const uint32_t i0 = ls[c.x], i1 = ls[c.y], i2 = ls[c.z], i3 = ls[c.w];
                acc = fma((double)v.x, xval<FMT>(X, cscale, i0, B, b), acc);
                acc = fma((double)v.y, xval<FMT>(X, cscale, i1, B, b), acc);
                acc = fma((double)v.z, xval<FMT>(X, cscale, i2, B, b), acc);
                acc = fma((double)v.w, xval<FMT>(X, cscale, i3, B, b), acc);
            }
        }
        if (col_ok) Z[(int64_t)row * B + b] = acc;
    }
}

// Quad-CSR rows with 32-bit column indices: the plain voxel-major copy
// (forward) or the beamlet-major copy (adjoint, with the FP8 row scale).
template <int FMT, int TB>
__global__ __launch_bounds__(SPMM_THREADS) void k_spmm_rows(const uint32_t* __restrict__ qptr,
                                                           const int32_t* __restrict__ col,
                                                           const void* __restrict__ val,
                                                           const float* __restrict__ cscale,
                                                           const float* __restrict__ rscale, int64_t nrows, int B,
                                                           const float* __restrict__ X, double* __restrict__ Z) {
    constexpr int RPW = 64 / TB;
    const int lane = threadIdx.x & 63;
    const int64_t row = ((int64_t)blockIdx.x * SPMM_THREADS + threadIdx.x) / 64 * RPW + lane / TB;
    const int b = blockIdx.y * TB + (lane % TB);
    if (row >= nrows || b >= B) return;
    const i32x4* c4 = reinterpret_cast<const i32x4*>(col);
    double acc = 0.0;
    const uint32_t q1 = qptr[row + 1];
    for (uint32_t q = qptr[row]; q < q1; ++q) {
        const float4 v = Quad<FMT>::load(val, q);
        const i32x4 c = c4[q];
        if (cscale) {
            acc = fma((double)v.x, xval<FMT>(X, cscale, (uint32_t)c.x, B, b), acc);
            acc = fma((double)v.y, xval<FMT>(X, cscale, (uint32_t)c.y, B, b), acc);
            acc = fma((double)v.z, xval<FMT>(X, cscale, (uint32_t)c.z, B, b), acc);
            acc = fma((double)v.w, xval<FMT>(X, cscale, (uint32_t)c.w, B, b), acc);
        } else {
            acc = fma((double)v.x, (double)X[(int64_t)c.x * B + b], acc);
            acc = fma((double)v.y, (double)X[(int64_t)c.y * B + b], acc);
            acc = fma((double)v.z, (double)X[(int64_t)c.z * B + b], acc);
            acc = fma((double)v.w, (double)X[(int64_t)c.w * B + b], acc);
        }
    }
    Z[row * B + b] = rscale ? acc * (double)rscale[row] : acc;
}

// Full-wave tile (64 right-hand sides): one row per wave at a time.  The
// wave loads up to 64 quads of the row at once, one per lane (coalesced),
// then walks them with the quad's indices and values broadcast from the
// owning lane, so the gathers of several quads are in flight together.
__device__ __forceinline__ uint32_t bcast(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ float bcastf(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// ROWS: 0 = tiled forward (16-bit local indices through the LDS list),
// 1 = 32-bit indices.  CS: the FP8 column scale applies (forward side).
template <int FMT, int ROWS, bool CS>
__device__ __forceinline__ double row_w64(uint32_t q0, uint32_t q1, const void* __restrict__ val,
                                          const void* __restrict__ colp, const uint32_t* __restrict__ ls,
                                          const float* __restrict__ cscale, int B, int b,
                                          const float* __restrict__ X) {
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    for (uint32_t base = q0; base < q1; base += 64) {
        const uint32_t n = min(64u, q1 - base);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        if ((uint32_t)lane < n) {
            v = Quad<FMT>::load(val, base + lane);
            if constexpr (ROWS == 0) {
                const u16x4 c = reinterpret_cast<const u16x4*>(colp)[base + lane];
                c0 = ls[c.x];
                c1 = ls[c.y];
                c2 = ls[c.z];
                c3 = ls[c.w];
            } else {
                const i32x4 c = reinterpret_cast<const i32x4*>(colp)[base + lane];
                c0 = (uint32_t)c.x;
                c1 = (uint32_t)c.y;
                c2 = (uint32_t)c.z;
                c3 = (uint32_t)c.w;
            }
        }
        // lanes past the last right-hand side gather a valid column and store
        // nothing; quads past the row's end (lanes >= n) hold zeros and index 0
        const int bb = b < B ? b : B - 1;
        constexpr int XF = CS ? FMT : FMT_F32;
        for (uint32_t k = 0; k < n; k += 4) {
            double xs[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xs[u][0] = xval<XF>(X, cscale, bcast(c0, k + u), B, bb);
                xs[u][1] = xval<XF>(X, cscale, bcast(c1, k + u), B, bb);
                xs[u][2] = xval<XF>(X, cscale, bcast(c2, k + u), B, bb);
                xs[u][3] = xval<XF>(X, cscale, bcast(c3, k + u), B, bb);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc = fma((double)bcastf(v.x, k + u), xs[u][0], acc);
                acc = fma((double)bcastf(v.y, k + u), xs[u][1], acc);
                acc = fma((double)bcastf(v.z, k + u), xs[u][2], acc);
                acc = fma((double)bcastf(v.w, k + u), xs[u][3], acc);
            }
        }
    }
    return acc;
}

template <int FMT>
__global__ __launch_bounds__(SPMM_THREADS) void k_spmm_fwd_tiled_w64(const int4* __restrict__ work, int n_items,
                                                                    const uint32_t* __restrict__ loff,
                                                                    const uint32_t* __restrict__ list,
                                                                    const uint32_t* __restrict__ qptr,
                                                                    const uint16_t* __restrict__ col16,
                                                                    const void* __restrict__ val,
                                                                    const float* __restrict__ cscale, int B,
                                                                    const float* __restrict__ X,
                                                                    double* __restrict__ Z) {
    __shared__ uint32_t ls[TILE_LIST];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    // persistent: a fixed grid (a multiple of 8 workgroups, so item i keeps
    // running on XCD i mod 8) walks the work items
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 wk = work[it];
        if (wk.x < 0) continue;
        const uint32_t l0 = loff[wk.x], ln = loff[wk.x + 1] - l0;
        for (uint32_t u = threadIdx.x; u < ln; u += SPMM_THREADS) ls[u] = list[l0 + u];
        __syncthreads();
        for (int row = wk.y + wave; row < wk.z; row += SPMM_THREADS / 64) {
            const double acc =
                row_w64<FMT, 0, FMT == FMT_FP8>(qptr[row], qptr[row + 1], val, col16, ls, cscale, B, b, X);
            if (b < B) Z[(int64_t)row * B + b] = acc;
        }
        __syncthreads();
    }
}

template <int FMT, bool CS>
__global__ __launch_bounds__(SPMM_THREADS) void k_spmm_rows_w64(const uint32_t* __restrict__ qptr,
                                                               const int32_t* __restrict__ col,
                                                               const void* __restrict__ val,
                                                               const float* __restrict__ cscale,
                                                               const float* __restrict__ rscale, int64_t nrows,
                                                               int B, const float* __restrict__ X,
                                                               double* __restrict__ Z) {
    const int lane = threadIdx.x & 63;
    // the grid is a multiple of 8 blocks; workgroup w runs on XCD w mod 8, so
    // XCD x takes the x-th eighth of the rows (neighbouring rows gather
    // neighbouring right-hand-side rows through the same L2)
    const int64_t per = gridDim.x / 8;
    const int64_t blk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    const int64_t row = (blk * SPMM_THREADS + threadIdx.x) / 64;
    const int b = blockIdx.y * 64 + lane;
    if (row >= nrows) return;
    const double acc = row_w64<FMT, 1, CS>(qptr[row], qptr[row + 1], val, col, nullptr, cscale, B, b, X);
    if (b < B) Z[row * B + b] = rscale ? acc * (double)rscale[row] : acc;
}

// Adjoint over the tiled slot rows (one beamlet's entries within one voxel
// block, 16-bit voxel offsets): the W rows a block gathers belong to its
// voxel range and stay in the L2 of the XCD its work items run on.  One slot
// row per wave at a time; sums go to part[slot][b].
template <int FMT>
__global__ __launch_bounds__(SPMM_THREADS) void k_spmm_adj_slots_w64(const int4* __restrict__ work, int n_items,
                                                                    const int32_t* __restrict__ bounds,
                                                                    const uint32_t* __restrict__ aqptr,
                                                                    const uint16_t* __restrict__ acol,
                                                                    const void* __restrict__ aval, int B,
                                                                    const float* __restrict__ W,
                                                                    double* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = lane;
    const int bb = b < B ? b : B - 1;
    const u16x4* __restrict__ c4 = reinterpret_cast<const u16x4*>(acol);
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {  // persistent, as the forward
        const int4 wk = work[it];
        if (wk.x < 0) continue;
        const float* __restrict__ Wb = W + (int64_t)bounds[wk.x] * B;
        for (int row = wk.y + wave; row < wk.z; row += SPMM_THREADS / 64) {
            const uint32_t q0 = aqptr[row], q1 = aqptr[row + 1];
            double acc = 0.0;
            for (uint32_t base = q0; base < q1; base += 64) {
                const uint32_t n = min(64u, q1 - base);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
                if ((uint32_t)lane < n) {
                    v = Quad<FMT>::load(aval, base + lane);
                    const u16x4 c = c4[base + lane];
                    c0 = c.x;
                    c1 = c.y;
                    c2 = c.z;
                    c3 = c.w;
                }
                for (uint32_t k = 0; k < n; k += 8) {
                    double xs[8][4];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        xs[u][0] = (double)Wb[(int64_t)bcast(c0, k + u) * B + bb];
                        xs[u][1] = (double)Wb[(int64_t)bcast(c1, k + u) * B + bb];
                        xs[u][2] = (double)Wb[(int64_t)bcast(c2, k + u) * B + bb];
                        xs[u][3] = (double)Wb[(int64_t)bcast(c3, k + u) * B + bb];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        acc = fma((double)bcastf(v.x, k + u), xs[u][0], acc);
                        acc = fma((double)bcastf(v.y, k + u), xs[u][1], acc);
                        acc = fma((double)bcastf(v.z, k + u), xs[u][2], acc);
                        acc = fma((double)bcastf(v.w, k + u), xs[u][3], acc);
                    }
                }
            }
            if (b < B) part[(int64_t)row * B + b] = acc;
        }
    }
}

// G[i][b] = scale_i * sum of beamlet i's slot sums (block order).
__global__ __launch_bounds__(256) void k_spmm_adj_reduce(int64_t nb, int B, const uint32_t* __restrict__ red_ptr,
                                                         const uint32_t* __restrict__ red_slot,
                                                         const double* __restrict__ part,
                                                         const float* __restrict__ scale, double* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nb * B) return;
    const int64_t i = e / B;
    const int b = (int)(e - i * B);
    double s = 0.0;
    for (uint32_t k = red_ptr[i]; k < red_ptr[i + 1]; ++k) s += part[(int64_t)red_slot[k] * B + b];
    G[e] = scale ? s * (double)scale[i] : s;
}

// Workgroups of the persistent 64-wide kernels: at most per_cu per compute
// unit (256 CUs), a multiple of 8 (work items are placed round-robin on the
// XCDs).  Measured on the prostate case: the adjoint is fastest with 2 per
// CU, the forward (whose LDS list limits residency) with 4.
static unsigned persistent_grid(int n_items, int per_cu) {
    const int g = std::min(n_items, per_cu * 256);
    return (unsigned)std::max(8, (g + 7) / 8 * 8);
}

// Blocks for nrows rows at rpb rows per block, rounded up to a multiple of 8.
static unsigned xcd_grid(int64_t nrows, int64_t rpb) {
    const int64_t n = (nrows + rpb - 1) / rpb;
    return (unsigned)((n + 7) / 8 * 8);
}

template <int FMT, int TB>
static void spmm_fwd_t(const vmat_ctx* h, int B, const float* X, double* Z, hipStream_t st) {
    const unsigned tiles = (unsigned)((B + TB - 1) / TB);
    if constexpr (TB == 64) {
        if (h->tl.on) {
            const Tiled& t = h->tl;
            k_spmm_fwd_tiled_w64<FMT><<<dim3(persistent_grid(t.n_fwork_half, 8), tiles), SPMM_THREADS, 0, st>>>(
                t.fwork_half, t.n_fwork_half, t.loff, t.list, h->vm.qptr, t.fcol, h->vm.val, h->bm.scale, B, X, Z);
        } else {
            const int64_t rpb = SPMM_THREADS / 64;
            k_spmm_rows_w64<FMT, FMT == FMT_FP8><<<dim3(xcd_grid(h->nv, rpb), tiles), SPMM_THREADS, 0, st>>>(
                h->vm.qptr, h->vm.col, h->vm.val, h->bm.scale, nullptr, h->nv, B, X, Z);
        }
        return;
    }
    if (h->tl.on) {
        const Tiled& t = h->tl;
        k_spmm_fwd_tiled<FMT, TB><<<dim3((unsigned)t.n_fwork, tiles), SPMM_THREADS, 0, st>>>(
            t.fwork, t.loff, t.list, h->vm.qptr, t.fcol, h->vm.val, h->bm.scale, B, X, Z);
    } else {
        const int64_t rows_per_block = (SPMM_THREADS / 64) * (64 / TB);
        k_spmm_rows<FMT, TB><<<dim3((unsigned)((h->nv + rows_per_block - 1) / rows_per_block), tiles),
                               SPMM_THREADS, 0, st>>>(h->vm.qptr, h->vm.col, h->vm.val, h->bm.scale, nullptr, h->nv, B, X, Z);
    }
}

template <int FMT, int TB>
static void spmm_adj_t(const vmat_ctx* h, int B, const float* W, double* G, hipStream_t st) {
    const unsigned tiles = (unsigned)((B + TB - 1) / TB);
    if constexpr (TB == 64) {
        const BatchState* bs = h->bs;
        if (h->tl.on && bs && bs->spart && B <= bs->cap && h->tl.n_awork > 0) {
            const Tiled& t = h->tl;
            k_spmm_adj_slots_w64<FMT><<<persistent_grid(t.n_awork, 2), SPMM_THREADS, 0, st>>>(
                t.awork, t.n_awork, t.bounds, t.aqptr, t.acol, t.aval, B, W, bs->spart);
            k_spmm_adj_reduce<<<(unsigned)((h->nb * B + 255) / 256), 256, 0, st>>>(h->nb, B, t.red_ptr, t.red_slot,
                                                                                   bs->spart, h->bm.scale, G);
            return;
        }
        const int64_t rpb = SPMM_THREADS / 64;
        k_spmm_rows_w64<FMT, false><<<dim3(xcd_grid(h->nb, rpb), tiles), SPMM_THREADS, 0, st>>>(
            h->bm.qptr, h->bm.col, h->bm.val, nullptr, h->bm.scale, h->nb, B, W, G);
        return;
    }
    const int64_t rows_per_block = (SPMM_THREADS / 64) * (64 / TB);
    k_spmm_rows<FMT, TB><<<dim3((unsigned)((h->nb + rows_per_block - 1) / rows_per_block), tiles), SPMM_THREADS, 0,
                           st>>>(h->bm.qptr, h->bm.col, h->bm.val, nullptr, h->bm.scale, h->nb, B, W, G);
}

template <int FMT>
static void spmm_dispatch(const vmat_ctx* h, bool fwd, int TB, int B, const float* X, double* Z, hipStream_t st) {
#define CASE(T)                                          \
    case T:                                              \
        if (fwd) spmm_fwd_t<FMT, T>(h, B, X, Z, st);     \
        else spmm_adj_t<FMT, T>(h, B, X, Z, st);         \
        break;
    switch (TB) {
        CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) default : CASE(64)
    }
#undef CASE
}

static const int kTiles[] = {1, 2, 4, 8, 16, 32, 64};

// Untuned: one tile over all right-hand sides (the smallest width >= B).
static int default_tile(int B) {
    int t = 1;
    while (t < B && t < 64) t <<= 1;
    return t;
}

static vmat_status launch_spmm(const vmat_ctx* h, bool fwd, int B, const float* X, double* Z, hipStream_t st, int TB) {
    if (TB <= 0) {
        TB = (fwd ? h->tune_fwd : h->tune_adj)[B];
        if (TB <= 0) TB = default_tile(B);
    }
    switch (h->d_store) {
        case VMAT_F32: spmm_dispatch<FMT_F32>(h, fwd, TB, B, X, Z, st); break;
        case VMAT_F16: spmm_dispatch<FMT_F16>(h, fwd, TB, B, X, Z, st); break;
        case VMAT_BF16: spmm_dispatch<FMT_BF16>(h, fwd, TB, B, X, Z, st); break;
        default: spmm_dispatch<FMT_FP8>(h, fwd, TB, B, X, Z, st); break;
    }
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// ---------------------------------------------------------------- batched cost

// F of every variant and F'(z) (FP32) for the adjoint, eq. 1 with the
// weights and threshold of voxel j's structure in variant b.  A block covers
// 256/B voxels per step and thread t keeps variant t mod B, so every
// per-variant sum is taken in a fixed order.
__global__ __launch_bounds__(256) void k_pen_batched(int64_t nv, int B, int S, const uint8_t* __restrict__ label,
                                                     const float* __restrict__ table, const double* __restrict__ Z,
                                                     float* __restrict__ dF, double* __restrict__ part) {
    __shared__ double sh[256];
    __shared__ float tb[64 * 16 * 3];
    for (int u = threadIdx.x; u < B * S * 3; u += 256) tb[u] = table[u];
    __syncthreads();
    const int per = 256 / B, t = threadIdx.x;
    double F = 0.0;
    if (t < per * B) {
        const int b = t % B;
        for (int64_t j = (int64_t)blockIdx.x * per + t / B; j < nv; j += (int64_t)gridDim.x * per) {
            const float* w = tb + (b * S + min((int)label[j], S - 1)) * 3;
            const Pen pn = penalty_at(Z[j * B + b], make_float4(w[0], w[1], w[2], 0.f));
            F += pn.F;
            dF[j * B + b] = (float)pn.dF;
        }
    }
    sh[t] = F;
    __syncthreads();
    if (t < B) {
        double s = 0.0;
        for (int u = t; u < per * B; u += B) s += sh[u];
        part[(int64_t)t * gridDim.x + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(64) void k_pen_batched_sum(int B, int n_part, const double* __restrict__ part,
                                                        double* __restrict__ cost) {
    const int b = threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int k = 0; k < n_part; ++k) s += part[(int64_t)b * n_part + k];
    cost[b] = s;
}


// ---------------------------------------------------------------- batched solve
// Column generation for B plan variants in lockstep: every product is one
// SpMM over all variants; the master's control logic runs one workgroup per
// variant on that variant's state; a variant whose master has stopped keeps
// its dose and prices and contributes a zero direction.

constexpr int BT = 256;

// X[i][b] = d_b[k] on the aperture of variant b (FP32), 0 elsewhere and for
// variants whose master is done.
__global__ __launch_bounds__(BT) void k_bfluence(int64_t nb, int N, int R, int C, int B,
                                                 const double* __restrict__ v, const int32_t* __restrict__ l,
                                                 const int32_t* __restrict__ r, const uint8_t* __restrict__ occ,
                                                 const MasterState* __restrict__ ms, float* __restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= nb * B) return;
    const int64_t i = e / B;
    const int b = (int)(e - i * B);
    const int64_t kr = i / C;
    const int c = (int)(i - kr * C);
    const int64_t k = kr / R;
    const int64_t NR = (int64_t)N * R;
    float xi = 0.f;
    if (!ms[b].done && occ[(int64_t)b * N + k] && c >= l[b * NR + kr] && c < r[b * NR + kr])
        xi = (float)v[(int64_t)b * N + k];
    X[e] = xi;
}

// Shared layout of the per-voxel batched kernels: a block covers 256/B voxels
// per step; thread t keeps variant t mod B; sums are per variant in fixed order.
struct VarTables {
    float tb[64 * 16 * 3];
    double t[64];
    double t2[64];
    int on[64];
    int two[64];
    double sh[BT];
    double sh2[BT];
};

__device__ __forceinline__ void stage_table(VarTables& S_, const float* table, int B, int S) {
    for (int u = threadIdx.x; u < B * S * 3; u += BT) S_.tb[u] = table[u];
}

__device__ __forceinline__ void variant_sums(VarTables& S_, int B, double a, double b2, double* pa, double* pb2) {
    const int per = BT / B, t = threadIdx.x;
    S_.sh[t] = a;
    S_.sh2[t] = b2;
    __syncthreads();
    // variants that took no part keep their partial sums (they still belong
    // to their current dose)
    if (t < B && S_.on[t]) {
        double s = 0.0, s2 = 0.0;
        for (int u = t; u < per * B; u += B) {
            s += S_.sh[u];
            s2 += S_.sh2[u];
        }
        pa[(int64_t)t * gridDim.x + blockIdx.x] = s;
        if (pb2) pb2[(int64_t)t * gridDim.x + blockIdx.x] = s2;
    }
}

// phi' and phi'' voxel sums along dZ at each searching variant's one or two
// line-search points (t_eval, and t_eval2 when n_eval == 2): one pass over
// the variants' doses serves both points.
__global__ __launch_bounds__(BT) void k_bls_eval(int64_t nv, int B, int S, const uint8_t* __restrict__ label,
                                                 const float* __restrict__ table, const double* __restrict__ Z,
                                                 const double* __restrict__ dZ, const MasterState* __restrict__ ms,
                                                 double* __restrict__ pp, double* __restrict__ qq,
                                                 double* __restrict__ pp2, double* __restrict__ qq2) {
    __shared__ VarTables S_;
    stage_table(S_, table, B, S);
    for (int u = threadIdx.x; u < B; u += BT) {
        S_.on[u] = !(ms[u].done || ms[u].ls_done);
        S_.t[u] = ms[u].t_eval;
        S_.t2[u] = ms[u].t_eval2;
        S_.two[u] = ms[u].n_eval == 2;
    }
    __syncthreads();
    const int per = BT / B, t = threadIdx.x;
    double p = 0.0, q = 0.0, p2 = 0.0, q2 = 0.0;
    if (t < per * B && S_.on[t % B]) {
        const int b = t % B;
        const double tb = S_.t[b], tb2 = S_.t2[b];
        const bool two = S_.two[b];
        for (int64_t j = (int64_t)blockIdx.x * per + t / B; j < nv; j += (int64_t)gridDim.x * per) {
            const float* w = S_.tb + (b * S + min((int)label[j], S - 1)) * 3;
            const float4 wv = make_float4(w[0], w[1], w[2], 0.f);
            const double dz = dZ[j * B + b], z = Z[j * B + b];
            const Pen pn = penalty_at(z + tb * dz, wv);
            p += dz * pn.dF;
            q += dz * dz * pn.curv;
            if (two) {
                const Pen pm = penalty_at(z + tb2 * dz, wv);
                p2 += dz * pm.dF;
                q2 += dz * dz * pm.curv;
            }
        }
    }
    variant_sums(S_, B, p, q, pp, qq);
    __syncthreads();
    variant_sums(S_, B, p2, q2, pp2, qq2);
}

// z <- z + t*_b dz for every variant still iterating; F'(z) and F partial sums.
__global__ __launch_bounds__(BT) void k_bupdate(int64_t nv, int B, int S, const uint8_t* __restrict__ label,
                                                const float* __restrict__ table, double* __restrict__ Z,
                                                const double* __restrict__ dZ, const MasterState* __restrict__ ms,
                                                float* __restrict__ RZ, double* __restrict__ pf) {
    __shared__ VarTables S_;
    stage_table(S_, table, B, S);
    for (int u = threadIdx.x; u < B; u += BT) {
        S_.on[u] = !ms[u].done;
        S_.t[u] = ms[u].t_star;
    }
    __syncthreads();
    const int per = BT / B, t = threadIdx.x;
    double F = 0.0;
    if (t < per * B && S_.on[t % B]) {
        const int b = t % B;
        const double tb = S_.t[b];
        for (int64_t j = (int64_t)blockIdx.x * per + t / B; j < nv; j += (int64_t)gridDim.x * per) {
            const float* w = S_.tb + (b * S + min((int)label[j], S - 1)) * 3;
            const double zj = Z[j * B + b] + tb * dZ[j * B + b];
            Z[j * B + b] = zj;
            const Pen pn = penalty_at(zj, make_float4(w[0], w[1], w[2], 0.f));
            F += pn.F;
            RZ[j * B + b] = (float)pn.dF;
        }
    }
    variant_sums(S_, B, F, 0.0, pf, nullptr);
}

// dF/dy_k per variant: the sum of G over variant b's aperture of beam k.
__global__ __launch_bounds__(BT) void k_bbeam_sums(int N, int R, int C, int B, const double* __restrict__ G,
                                                   const int32_t* __restrict__ l, const int32_t* __restrict__ r,
                                                   const uint8_t* __restrict__ occ, double* __restrict__ gF) {
    __shared__ double sh[BT];
    const int k = blockIdx.x, per = BT / B, t = threadIdx.x;
    const int RC = R * C;
    const int64_t NR = (int64_t)N * R;
    double s = 0.0;
    if (t < per * B) {
        const int b = t % B;
        if (occ[(int64_t)b * N + k]) {
            const double* gk = G + (int64_t)k * RC * B;
            for (int e = t / B; e < RC; e += per) {
                const int rho = e / C, c = e - rho * C;
                const int64_t kr = b * NR + (int64_t)k * R + rho;
                if (c >= l[kr] && c < r[kr]) s += gk[(int64_t)e * B + b];
            }
        }
    }
    sh[t] = s;
    __syncthreads();
    if (t < B) {
        double a = 0.0;
        for (int u = t; u < per * B; u += B) a += sh[u];
        gF[(int64_t)t * N + k] = a;
    }
}

__device__ inline MasterPtrs variant_ptrs(MasterPtrs m, int b) {
    const int64_t N = m.N, NR = (int64_t)m.N * m.R;
    m.y += b * N;
    if (m.occ) m.occ += b * N;
    if (m.l) m.l += b * NR;
    if (m.r) m.r += b * NR;
    m.grad += b * N;
    m.grad_prev += b * N;
    m.d += b * N;
    m.d_prev += b * N;
    m.W += b * N;
    m.W_prev += b * N;
    m.gF += b * N;
    m.ms += b;
    return m;
}

__device__ __forceinline__ double reduce_row(const double* part, int n, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += CTRL) s += part[i];
    return bsum(s, sh);
}

// vmask (nullable): only the variants that start a master solve now.
__global__ __launch_bounds__(CTRL) void k_bmaster_begin(int N, double* __restrict__ y, const uint8_t* __restrict__ occ,
                                                        MasterState* ms, int max_iter, int ls_max, double tol,
                                                        double kkt_ref, const double* __restrict__ kref,
                                                        const uint8_t* __restrict__ vmask) {
    const int b = blockIdx.x;
    if (vmask && !vmask[b]) return;
    for (int k = threadIdx.x; k < N; k += CTRL)
        if (!occ[(int64_t)b * N + k]) y[(int64_t)b * N + k] = 0.0;
    if (threadIdx.x == 0) {
        MasterState s = {};
        s.max_iter = max_iter;
        s.ls_max = ls_max;
        s.tol = tol;
        s.kkt_ref = kkt_ref > 0.0 ? kkt_ref : kref[b];
        s.ls_done = 1;
        ms[b] = s;
    }
}

__global__ __launch_bounds__(CTRL) void k_bmaster_grad(MasterPtrs m0, const double* __restrict__ pf, int n_part,
                                                       int first, const uint8_t* __restrict__ vmask) {
    __shared__ double sh[4];
    if (vmask && !vmask[blockIdx.x]) return;
    const MasterPtrs m = variant_ptrs(m0, blockIdx.x);
    if (!first && m.ms->done) return;
    const double F = reduce_row(pf + (int64_t)blockIdx.x * n_part, n_part, sh);
    ctrl_grad(m, F, first, sh);
}

__global__ __launch_bounds__(CTRL) void k_bmaster_dir(MasterPtrs m0) {
    __shared__ double sh[4];
    __shared__ int shi[4];
    ctrl_dir(variant_ptrs(m0, blockIdx.x), sh, shi, true);
}

__global__ __launch_bounds__(CTRL) void k_bls_ctrl(MasterState* ms, const double* __restrict__ pp,
                                                   const double* __restrict__ qq, const double* __restrict__ pp2,
                                                   const double* __restrict__ qq2, int n_part) {
    __shared__ double sh[4];
    MasterState& s = ms[blockIdx.x];
    if (s.done || s.ls_done) return;
    const double pF = reduce_row(pp + (int64_t)blockIdx.x * n_part, n_part, sh);
    const double hF = reduce_row(qq + (int64_t)blockIdx.x * n_part, n_part, sh);
    const bool two = s.n_eval == 2;
    const double pF2 = two ? reduce_row(pp2 + (int64_t)blockIdx.x * n_part, n_part, sh) : 0.0;
    const double hF2 = two ? reduce_row(qq2 + (int64_t)blockIdx.x * n_part, n_part, sh) : 0.0;
    if (threadIdx.x == 0) ctrl_ls_pass(s, pF, hF, pF2, hF2);
}

__global__ __launch_bounds__(CTRL) void k_bmaster_step(MasterPtrs m0) {
    const MasterPtrs m = variant_ptrs(m0, blockIdx.x);
    if (m.ms->done) return;
    ctrl_step(m);
}

// kkt reference of each variant from its first pricing: |p_k*|, 1 if zero.
__global__ void k_bkref(int B, const double* __restrict__ pscore, double* __restrict__ kref) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double p = pscore[b * 3];
    kref[b] = p != 0.0 && isfinite(p) ? fabs(p) : 1.0;
}
}  // namespace vmat

using namespace vmat;

namespace {

vmat_status check_batch(vmat_handle h, int B) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    if (B < 1 || B > 64) return fail(VMAT_ERR_INVALID_ARG, "the number of right-hand sides must be in [1, 64]");
    if (!h->bm.col || !h->bm.val) return fail(VMAT_ERR_INVALID_ARG, "handle without the beamlet-major copy of D");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return fail(VMAT_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    return VMAT_OK;
}

}  // namespace

extern "C" vmat_status vmat_forward_batched(vmat_handle h, int32_t B, const float* X, double* Z, hipStream_t st) {
    vmat_status rc = check_batch(h, B);
    if (rc != VMAT_OK) return rc;
    if (!X || !Z) return fail(VMAT_ERR_INVALID_ARG, "null X or Z");
    return launch_spmm(h, true, B, X, Z, st, 0);
}

extern "C" vmat_status vmat_adjoint_batched(vmat_handle h, int32_t B, const float* W, double* G, hipStream_t st) {
    vmat_status rc = check_batch(h, B);
    if (rc != VMAT_OK) return rc;
    if (!W || !G) return fail(VMAT_ERR_INVALID_ARG, "null W or G");
    return launch_spmm(h, false, B, W, G, st, 0);
}

extern "C" vmat_status vmat_grad_batched(vmat_handle h, int32_t B, int32_t n_struct, const uint8_t* label,
                                         const float* table, const float* X, double* Z, double* cost, float* dF,
                                         double* G, hipStream_t st) {
    vmat_status rc = check_batch(h, B);
    if (rc != VMAT_OK) return rc;
    if (n_struct < 1 || n_struct > 16) return fail(VMAT_ERR_INVALID_ARG, "n_struct must be in [1, 16]");
    if (!label || !table || !X || !Z || !cost || !dF)
        return fail(VMAT_ERR_INVALID_ARG, "null argument");
    if ((rc = launch_spmm(h, true, B, X, Z, st, 0)) != VMAT_OK) return rc;
    k_pen_batched<<<h->n_part, 256, 0, st>>>(h->nv, B, n_struct, label, table, Z, dF, h->part_b);
    VMAT_LAUNCH_CHECK();
    k_pen_batched_sum<<<1, 64, 0, st>>>(B, h->n_part, h->part_b, cost);
    VMAT_LAUNCH_CHECK();
    if (G) return launch_spmm(h, false, B, dF, G, st, 0);
    return VMAT_OK;
}

// Times each tile width for both products at B right-hand sides on the
// caller's buffers and keeps the fastest for later batched calls.
extern "C" vmat_status vmat_tune_batched(vmat_handle h, int32_t B, const float* X, double* Z, const float* W,
                                         double* G, int32_t reps, int32_t* best, float* times_ms,
                                         hipStream_t st) {
    vmat_status rc = check_batch(h, B);
    if (rc != VMAT_OK) return rc;
    if (!X || !Z || !W || !G || reps < 1) return fail(VMAT_ERR_INVALID_ARG, "null buffer or reps < 1");
    // the timing events are released on every path out
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    VMAT_HIP(hipEventCreate(&ev.e[0]));
    VMAT_HIP(hipEventCreate(&ev.e[1]));
    int bt[2] = {0, 0};
    float bm[2] = {INFINITY, INFINITY};
    int idx = 0;
    for (int dir = 0; dir < 2; ++dir) {
        for (int TB : kTiles) {
            float ms = INFINITY;
            if (TB < 2 * B) {
                const bool fwd = dir == 0;
                const float* in = fwd ? X : W;
                double* out = fwd ? Z : G;
                if ((rc = launch_spmm(h, fwd, B, in, out, st, TB)) != VMAT_OK) return rc;
                VMAT_HIP(hipEventRecord(ev.e[0], st));
                for (int k = 0; k < reps; ++k)
                    if ((rc = launch_spmm(h, fwd, B, in, out, st, TB)) != VMAT_OK) return rc;
                VMAT_HIP(hipEventRecord(ev.e[1], st));
                VMAT_HIP(hipEventSynchronize(ev.e[1]));
                VMAT_HIP(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
                ms /= (float)reps;
                if (ms < bm[dir]) {
                    bm[dir] = ms;
                    bt[dir] = TB;
                }
            }
            if (times_ms) times_ms[idx] = ms;
            ++idx;
        }
    }
    if (rc != VMAT_OK) return rc;
    h->tune_fwd[B] = bt[0];
    h->tune_adj[B] = bt[1];
    if (best) {
        best[0] = bt[0];
        best[1] = bt[1];
    }
    return VMAT_OK;
}

extern "C" vmat_status vmat_set_batched_tile(vmat_handle h, int32_t B, int32_t fwd_tile, int32_t adj_tile) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    if (B < 1 || B > 64) return fail(VMAT_ERR_INVALID_ARG, "the number of right-hand sides must be in [1, 64]");
    auto ok = [](int t) { return t == 0 || (t <= 64 && (t & (t - 1)) == 0 && t > 0); };
    if (!ok(fwd_tile) || !ok(adj_tile)) return fail(VMAT_ERR_INVALID_ARG, "tile widths must be 0 or 1, 2, 4, ..., 64");
    h->tune_fwd[B] = fwd_tile;
    h->tune_adj[B] = adj_tile;
    return VMAT_OK;
}

// ---------------------------------------------------------------- batched solve (host)

namespace vmat {

void free_batch(vmat_ctx* h) {
    BatchState* b = h->bs;
    if (!b) return;
    auto F = [](void* p) { if (p) (void)hipFree(p); };
    F(b->X); F(b->Z); F(b->dZ); F(b->RZ); F(b->G);
    F(b->grad); F(b->grad_prev); F(b->d); F(b->d_prev); F(b->gF); F(b->W); F(b->W_prev);
    F(b->ms); F(b->pp); F(b->qq); F(b->pp2); F(b->qq2); F(b->pf);
    F(b->rowS); F(b->rowm); F(b->rowl); F(b->rowr); F(b->bprice); F(b->pbeam); F(b->pscore); F(b->kref);
    F(b->cost); F(b->tr.beam); F(b->tr.price); F(b->tr.margin); F(b->tr.row_margin); F(b->tr.y); F(b->vmask); F(b->viter);
    F(b->spart);
    if (b->ms_host) (void)hipHostFree(b->ms_host);
    if (b->mask_host) (void)hipHostFree(b->mask_host);
    if (b->iter_host) (void)hipHostFree(b->iter_host);
    h->bytes -= b->bytes;
    delete b;
    h->bs = nullptr;
}

}  // namespace vmat

namespace {

template <typename T>
vmat_status balloc(BatchState* b, T** p, size_t count) {
    const size_t n = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc((void**)p, n) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(VMAT_ERR_ALLOC, "device allocation failed (batched solve state)");
    }
    b->bytes += (int64_t)n;
    return VMAT_OK;
}

#define BTRY(x)                                  \
    do {                                         \
        vmat_status rc_ = (x);                   \
        if (rc_ != VMAT_OK) return rc_;          \
    } while (0)

vmat_status sync_batch(vmat_ctx* h, int B, hipStream_t st) {
    VMAT_HIP(hipMemcpyAsync(h->bs->ms_host, h->bs->ms, sizeof(MasterState) * B, hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipStreamSynchronize(st));
    return VMAT_OK;
}

MasterPtrs batch_ptrs(const vmat_ctx* h, double* y, const uint8_t* occ, const int32_t* l, const int32_t* r) {
    const BatchState& b = *h->bs;
    MasterPtrs m;
    m.N = h->N; m.R = h->R; m.C = h->C; m.circ = h->circular; m.gamma = h->d_gamma;
    m.th = h->d_theta; m.y = y; m.occ = occ; m.l = l; m.r = r;
    m.grad = b.grad; m.grad_prev = b.grad_prev; m.d = b.d; m.d_prev = b.d_prev;
    m.W = b.W; m.W_prev = b.W_prev; m.gF = b.gF; m.ms = b.ms;
    return m;
}

struct BatchArgs {
    int B, S;
    const uint8_t* label;
    const float* table;
};

// One lockstep master iteration over the variants whose master is running
// (the others keep their state: zero direction, no step), as two captured
// sequences: [direction, its fluence and dose SpMM, three line-search passes
// (one or two points each)] and, after the state read and any further
// line-search rounds,
// [step, dose update, adjoint SpMM, beam gradients].  Returns with the states
// read back; *any_active = false when no master was running (the second
// sequence is then skipped).
vmat_status batch_iteration(vmat_ctx* h, const BatchArgs& a, const int32_t* l, const int32_t* r,
                            const uint8_t* occ, double* y, int64_t* n_spmm, bool* any_active, hipStream_t st) {
    BatchState& bs = *h->bs;
    const int B = a.B, np = h->n_part;
    const MasterPtrs m = batch_ptrs(h, y, occ, l, r);
    const int64_t nbB = h->nb * B;
    const GraphKey key = {(uint64_t)(uintptr_t)y, (uint64_t)(uintptr_t)l, (uint64_t)(uintptr_t)r,
                          (uint64_t)(uintptr_t)occ, (uint64_t)(uintptr_t)a.label, (uint64_t)(uintptr_t)a.table,
                          (uint64_t)B | ((uint64_t)a.S << 8) | ((uint64_t)(uint32_t)h->tune_fwd[B] << 16) |
                              ((uint64_t)(uint32_t)h->tune_adj[B] << 32),
                          (uint64_t)(uintptr_t)bs.X};
    auto ls_round = [&](hipStream_t s) -> vmat_status {
        for (int i = 0; i < 3; ++i) {
            k_bls_eval<<<np, BT, 0, s>>>(h->nv, B, a.S, a.label, a.table, bs.Z, bs.dZ, bs.ms, bs.pp, bs.qq,
                                         bs.pp2, bs.qq2);
            VMAT_LAUNCH_CHECK();
            k_bls_ctrl<<<B, CTRL, 0, s>>>(bs.ms, bs.pp, bs.qq, bs.pp2, bs.qq2, np);
            VMAT_LAUNCH_CHECK();
        }
        return VMAT_OK;
    };
    auto direction = [&](hipStream_t s) -> vmat_status {
        k_bmaster_dir<<<B, CTRL, 0, s>>>(m);
        VMAT_LAUNCH_CHECK();
        k_bfluence<<<(unsigned)((nbB + BT - 1) / BT), BT, 0, s>>>(h->nb, h->N, h->R, h->C, B, bs.d, l, r, occ,
                                                                  bs.ms, bs.X);
        VMAT_LAUNCH_CHECK();
        BTRY(launch_spmm(h, true, B, bs.X, bs.dZ, s, 0));
        return ls_round(s);
    };
    auto step = [&](hipStream_t s) -> vmat_status {
        k_bmaster_step<<<B, CTRL, 0, s>>>(m);
        VMAT_LAUNCH_CHECK();
        k_bupdate<<<np, BT, 0, s>>>(h->nv, B, a.S, a.label, a.table, bs.Z, bs.dZ, bs.ms, bs.RZ, bs.pf);
        VMAT_LAUNCH_CHECK();
        BTRY(launch_spmm(h, false, B, bs.RZ, bs.G, s, 0));
        k_bbeam_sums<<<h->N, BT, 0, s>>>(h->N, h->R, h->C, B, bs.G, l, r, occ, bs.gF);
        VMAT_LAUNCH_CHECK();
        k_bmaster_grad<<<B, CTRL, 0, s>>>(m, bs.pf, np, 0, nullptr);
        VMAT_LAUNCH_CHECK();
        return VMAT_OK;
    };
    BTRY(run_iteration(h, G_BATCH_DIR, key, direction, st));
    n_spmm[0] += 1;
    BTRY(sync_batch(h, B, st));
    bool active = false;
    for (int b = 0; b < B; ++b) active = active || !bs.ms_host[b].done;
    *any_active = active;
    if (!active) return VMAT_OK;
    for (;;) {
        bool searching = false;
        for (int b = 0; b < B; ++b) searching = searching || (!bs.ms_host[b].done && !bs.ms_host[b].ls_done);
        if (!searching) break;
        BTRY(ls_round(st));
        BTRY(sync_batch(h, B, st));
    }
    BTRY(run_iteration(h, G_BATCH_STEP, key, step, st));
    n_spmm[1] += 1;
    return VMAT_OK;
}

}  // namespace

extern "C" vmat_status vmat_reserve_batched(vmat_handle h, int32_t max_variants) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    if (max_variants < 1 || max_variants > 64) return fail(VMAT_ERR_INVALID_ARG, "max_variants must be in [1, 64]");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return fail(VMAT_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    VMAT_HIP(hipDeviceSynchronize());
    free_batch(h);
    BatchState* b = new BatchState();
    h->bs = b;
    const size_t B = (size_t)max_variants, N = (size_t)h->N, NR = N * (size_t)h->R;
    const size_t nb = (size_t)h->nb, nv = (size_t)h->nv, np = (size_t)h->n_part;
    b->cap = max_variants;
    vmat_status rc = VMAT_OK;
    auto A = [&](auto** p, size_t n) { if (rc == VMAT_OK) rc = balloc(b, p, n); };
    A(&b->X, nb * B); A(&b->Z, nv * B); A(&b->dZ, nv * B); A(&b->RZ, nv * B); A(&b->G, nb * B);
    A(&b->grad, B * N); A(&b->grad_prev, B * N); A(&b->d, B * N); A(&b->d_prev, B * N); A(&b->gF, B * N);
    A(&b->W, B * N); A(&b->W_prev, B * N); A(&b->ms, B);
    A(&b->pp, B * np); A(&b->qq, B * np); A(&b->pp2, B * np); A(&b->qq2, B * np); A(&b->pf, B * np);
    A(&b->rowS, B * NR); A(&b->rowm, B * NR); A(&b->rowl, B * NR); A(&b->rowr, B * NR);
    A(&b->bprice, B * N); A(&b->pbeam, B * (1 + 2 * (size_t)h->R)); A(&b->pscore, B * 3); A(&b->kref, B);
    A(&b->cost, B);
    A(&b->tr.beam, B * N); A(&b->tr.price, B * N); A(&b->tr.margin, B * N); A(&b->tr.row_margin, B * N);
    A(&b->tr.y, B * N * N);
    A(&b->vmask, B); A(&b->viter, B);
    if (h->tl.on) A(&b->spart, (size_t)h->tl.S * B);
    if (rc == VMAT_OK && (hipHostMalloc((void**)&b->ms_host, sizeof(MasterState) * B) != hipSuccess ||
                          hipHostMalloc((void**)&b->mask_host, B) != hipSuccess ||
                          hipHostMalloc((void**)&b->iter_host, sizeof(int32_t) * B) != hipSuccess))
        rc = fail(VMAT_ERR_ALLOC, "pinned host allocation failed");
    h->bytes += b->bytes;
    if (rc != VMAT_OK) {
        free_batch(h);
        return rc;
    }
    return VMAT_OK;
}

extern "C" vmat_status vmat_solve_batched(vmat_handle h, const vmat_solve_opts* opts, int32_t B, int32_t n_struct,
                                          const uint8_t* label, const float* table, int32_t* l, int32_t* r,
                                          uint8_t* occ, double* y, vmat_solve_report* rep,
                                          vmat_solve_trace* trace, int64_t* n_spmm, hipStream_t st) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    if (!h->bs) return fail(VMAT_ERR_INVALID_ARG, "call vmat_reserve_batched first");
    if (B < 1 || B > h->bs->cap) return fail(VMAT_ERR_INVALID_ARG, "B must be in [1, reserved variants]");
    if (n_struct < 1 || n_struct > 16) return fail(VMAT_ERR_INVALID_ARG, "n_struct must be in [1, 16]");
    if (!label || !table || !l || !r || !occ || !y || !rep) return fail(VMAT_ERR_INVALID_ARG, "null argument");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return fail(VMAT_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    vmat_solve_opts so;
    so.max_cg_iter = 0;
    so.master_mode = 0;
    so.master.max_iter = 200;
    so.master.ls_max_steps = 50;
    so.master.tol_rel = 1e-5;
    so.master.kkt_ref = 0.0;
    if (opts) so = *opts;
    if (so.master.max_iter < 1 || so.master.ls_max_steps < 1 || !(so.master.tol_rel > 0.0) ||
        !std::isfinite(so.master.kkt_ref) || so.master.kkt_ref < 0.0)
        return fail(VMAT_ERR_INVALID_ARG, "invalid master options");
    const int N = h->N;
    const int64_t NR = (int64_t)N * h->R;
    std::vector<uint8_t> occ_h((size_t)B * N);
    VMAT_HIP(hipMemcpyAsync(occ_h.data(), occ, occ_h.size(), hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipStreamSynchronize(st));
    for (uint8_t o : occ_h)
        if (o) return fail(VMAT_ERR_UNSUPPORTED, "batched solves start from empty plans (occ all 0)");
    int iters = N;
    if (so.max_cg_iter > 0) iters = std::min(iters, so.max_cg_iter);
    BatchState& bs = *h->bs;
    BatchArgs a{B, n_struct, label, table};
    int64_t cnt[2] = {0, 0};

    // empty plans: z = 0, prices g = D F'(0), cost_0
    VMAT_HIP(hipMemsetAsync(y, 0, sizeof(double) * B * N, st));
    VMAT_HIP(hipMemsetAsync(bs.Z, 0, sizeof(double) * h->nv * B, st));
    k_pen_batched<<<h->n_part, 256, 0, st>>>(h->nv, B, n_struct, label, table, bs.Z, bs.RZ, bs.pf);
    VMAT_LAUNCH_CHECK();
    k_pen_batched_sum<<<1, 64, 0, st>>>(B, h->n_part, bs.pf, bs.cost);
    VMAT_LAUNCH_CHECK();
    BTRY(launch_spmm(h, false, B, bs.RZ, bs.G, st, 0));
    cnt[1] += 1;
    std::vector<double> cost0(B);
    VMAT_HIP(hipMemcpyAsync(cost0.data(), bs.cost, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipStreamSynchronize(st));
    std::vector<vmat_solve_report> R(B);
    std::vector<std::vector<double>> costs(B, std::vector<double>(iters + 1, 0.0));
    std::vector<std::vector<int32_t>> miters(B, std::vector<int32_t>(iters, 0));
    for (int b = 0; b < B; ++b) {
        R[b] = vmat_solve_report{};
        R[b].n_adjoint = 1;
        costs[b][0] = cost0[b];
    }
    // Each variant opens its next aperture as soon as its own master has
    // stopped; the masters that are running advance together, one SpMM per
    // product.  cg_t[b]: apertures opened by variant b.
    std::vector<int> cg_t(B, 0);
    std::vector<uint8_t> recorded(B, 1);
    const MasterPtrs m = batch_ptrs(h, y, occ, l, r);
    bool first = true;
    for (;;) {
        int n_restart = 0;
        bool finished = true;
        for (int b = 0; b < B; ++b) {
            const MasterState& s = bs.ms_host[b];
            const bool ready = first || s.done;
            if (ready && !recorded[b]) {
                const int t = cg_t[b] - 1;
                R[b].master_iters += s.it;
                R[b].n_forward += s.n_fwd;
                R[b].n_adjoint += s.n_adj;
                R[b].n_ls_evals += s.n_ls;
                if (!s.converged) R[b].not_converged++;
                R[b].cg_iters = t + 1;
                R[b].F = s.F;
                R[b].gG = s.gG;
                R[b].kkt_ref = s.kkt_ref;
                costs[b][t + 1] = s.F + s.gG;
                miters[b][t] = s.it;
                recorded[b] = 1;
            }
            const bool go = ready && cg_t[b] < iters;
            bs.mask_host[b] = go ? 1 : 0;
            bs.iter_host[b] = cg_t[b];
            n_restart += go ? 1 : 0;
            finished = finished && ready && cg_t[b] >= iters;
        }
        if (finished) break;
        if (n_restart > 0) {
            VMAT_HIP(hipMemcpyAsync(bs.vmask, bs.mask_host, B, hipMemcpyHostToDevice, st));
            VMAT_HIP(hipMemcpyAsync(bs.viter, bs.iter_host, sizeof(int32_t) * B, hipMemcpyHostToDevice, st));
            BTRY(launch_price_variants(h, B, bs.G, y, l, r, occ, bs.rowS, bs.rowl, bs.rowr, bs.rowm, bs.bprice,
                                       bs.pbeam, bs.pscore, nullptr, 1, 0, l, r, occ, y, bs.tr, st, bs.vmask,
                                       bs.viter));
            if (first) {
                k_bkref<<<1, 64, 0, st>>>(B, bs.pscore, bs.kref);
                VMAT_LAUNCH_CHECK();
            }
            k_bmaster_begin<<<B, CTRL, 0, st>>>(h->N, y, occ, bs.ms, so.master.max_iter, so.master.ls_max_steps,
                                                so.master.tol_rel, so.master.kkt_ref, bs.kref, bs.vmask);
            VMAT_LAUNCH_CHECK();
            k_bbeam_sums<<<h->N, BT, 0, st>>>(h->N, h->R, h->C, B, bs.G, l, r, occ, bs.gF);
            VMAT_LAUNCH_CHECK();
            k_bmaster_grad<<<B, CTRL, 0, st>>>(m, bs.pf, h->n_part, 2, bs.vmask);
            VMAT_LAUNCH_CHECK();
            for (int b = 0; b < B; ++b)
                if (bs.mask_host[b]) {
                    cg_t[b] += 1;
                    recorded[b] = 0;
                }
        }
        first = false;
        bool active = false;
        BTRY(batch_iteration(h, a, l, r, occ, y, cnt, &active, st));
    }
    for (int b = 0; b < B; ++b) rep[b] = R[b];
    if (n_spmm) {
        n_spmm[0] = cnt[0];
        n_spmm[1] = cnt[1];
    }
    if (trace) {
        const int n = iters;
        for (int b = 0; b < B; ++b) {
            vmat_solve_trace& T = trace[b];
            if (T.beam && n) VMAT_HIP(hipMemcpyAsync(T.beam, bs.tr.beam + (int64_t)b * N, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            if (T.price && n) VMAT_HIP(hipMemcpyAsync(T.price, bs.tr.price + (int64_t)b * N, n * sizeof(double), hipMemcpyDeviceToHost, st));
            if (T.margin && n) VMAT_HIP(hipMemcpyAsync(T.margin, bs.tr.margin + (int64_t)b * N, n * sizeof(double), hipMemcpyDeviceToHost, st));
            if (T.row_margin && n) VMAT_HIP(hipMemcpyAsync(T.row_margin, bs.tr.row_margin + (int64_t)b * N, n * sizeof(double), hipMemcpyDeviceToHost, st));
            if (T.y && n)
                VMAT_HIP(hipMemcpyAsync(T.y, bs.tr.y + (int64_t)b * N * N, (size_t)n * N * sizeof(double),
                                        hipMemcpyDeviceToHost, st));
        }
        VMAT_HIP(hipStreamSynchronize(st));
        for (int b = 0; b < B; ++b) {
            vmat_solve_trace& T = trace[b];
            if (T.cost) std::copy(costs[b].begin(), costs[b].end(), T.cost);
            if (T.master_iters) std::copy(miters[b].begin(), miters[b].end(), T.master_iters);
        }
    }
    (void)NR;
    return VMAT_OK;
}
