// Tiled dose product and adjoint with LDS-staged gathers (layout described
// with `Tiled` in vmat_internal.h), and the builder of that layout.
//
// Why: in the plain quad-CSR kernels each non-zero gathers one x (or w) value
// from global memory at a scattered address; the texture path serves such a
// gather at about one cache line per lane, which bounds the product well below
// the HBM rate.  Here a block's gathered values sit in LDS, the column indices
// shrink to 16 bits (6 B per FP32 non-zero instead of 8), and the global
// traffic is the coalesced stream of D plus small per-block staging.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "vmat_formats.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"

namespace vmat {


// ---------------------------------------------------------------- kernels
//
// A work item is (block, rows [r0, r1)) with at most TILE_ROWS rows, cut into
// 64-row slices (rows sorted longest first).  One workgroup takes one item:
// it stages the block's gathered values in LDS, then its waves sum the
// item's slices, one lane per row.


// The slices of one work item.  Wave w starts with slice w; a wave that
// finishes a slice takes the next one nobody has taken (counter *qnext in
// LDS, starting at the number of waves), so a long slice does not hold the
// workgroup while the other waves idle.  Lane i owns row i of the slice and
// walks its quads in order, U quads in flight; the last len mod U quads are
// loaded together too.  The order of the sums within a row does not depend
// on which wave takes the slice.  Row sums go to os[row - first row of the
// item] in LDS: the rows of a slice are scattered over the item (sorted by
// length), and 64 scattered 8-byte global stores cost the memory pipeline
// about as much as several of the slice's streaming loads.
template <int FMT, int U, typename ST>
__device__ __forceinline__ void sell_rows(const int4 wk, const uint32_t* __restrict__ s_off,
                                          const uint32_t* __restrict__ s_len, const uint32_t* __restrict__ s_row,
                                          const uint16_t* __restrict__ s_col, const void* __restrict__ s_val,
                                          const ST* __restrict__ xs, double* __restrict__ os,
                                          uint32_t* qnext) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nsl = (wk.z - wk.y + 63) / 64;
    const u16x4* __restrict__ c4 = reinterpret_cast<const u16x4*>(s_col);
    for (int j = wave; j < nsl;) {
        const int64_t sl = (int64_t)wk.w + j;
        const uint32_t base = s_off[sl] + lane, len = s_len[sl];
        const uint32_t row = s_row[sl * 64 + lane];
        double acc = 0.0;
        uint32_t k = 0;
        for (; k + U <= len; k += U) {
            // the stored words first, decoded only when summed: decoding at
            // the load let the compiler reuse one register for every FP8
            // load and wait for each in turn
            typename Quad<FMT>::raw_t rv[U];
            u16x4 c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                rv[u] = Quad<FMT>::raw(s_val, base + (k + u) * 64);
                c[u] = __builtin_nontemporal_load(c4 + base + (k + u) * 64);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float4 vu = Quad<FMT>::dec(rv[u]);
                acc = fma((double)vu.x, (double)xs[c[u].x], acc);
                acc = fma((double)vu.y, (double)xs[c[u].y], acc);
                acc = fma((double)vu.z, (double)xs[c[u].z], acc);
                acc = fma((double)vu.w, (double)xs[c[u].w], acc);
            }
        }
        if (k < len) {
            // the last rem < U quads; addresses past the row's end re-read
            // its last quad and are not summed
            const uint32_t rem = len - k;
            typename Quad<FMT>::raw_t rv[U - 1];
            u16x4 c[U - 1];
#pragma unroll
            for (int u = 0; u < U - 1; ++u) {
                const uint32_t kk = k + min((uint32_t)u, rem - 1);
                rv[u] = Quad<FMT>::raw(s_val, base + kk * 64);
                c[u] = __builtin_nontemporal_load(c4 + base + kk * 64);
            }
#pragma unroll
            for (int u = 0; u < U - 1; ++u) {
                if ((uint32_t)u < rem) {
                    const float4 vu = Quad<FMT>::dec(rv[u]);
                    acc = fma((double)vu.x, (double)xs[c[u].x], acc);
                    acc = fma((double)vu.y, (double)xs[c[u].y], acc);
                    acc = fma((double)vu.z, (double)xs[c[u].z], acc);
                    acc = fma((double)vu.w, (double)xs[c[u].w], acc);
                }
            }
        }
        if (row != 0xFFFFFFFFu) os[row - (uint32_t)wk.y] = acc;
        uint32_t nj = 0;
        if (lane == 0) nj = atomicAdd(qnext, 1u);
        j = (int)__builtin_amdgcn_readlane(nj, 0);
    }
}

// Writes the item's row sums (rows wk.y .. wk.z - 1, staged in os) to
// out[wk.y ...] with coalesced stores, once every wave has finished.  NT:
// non-temporal stores (the forward's dose: 2-3% faster forwards on MI355X;
// the adjoint's slot sums, read at once by the reduction, keep plain stores).
template <bool NT>
__device__ __forceinline__ void flush_rows(const int4 wk, const double* os, double* __restrict__ out) {
    __syncthreads();
    const int n = wk.z - wk.y;
    for (int i = threadIdx.x; i < n; i += TILE_THREADS) {
        if (NT)
            __builtin_nontemporal_store(os[i], out + (int64_t)wk.y + i);
        else
            out[(int64_t)wk.y + i] = os[i];
    }
}

// Forward over the sliced layout: after the block's x values are staged in
// LDS, the waves take the item's slices as sell_rows describes; lane i owns
// row i of the slice and walks its quads in order (quad k of the 64 rows is
// one contiguous 1-KB load for FP32 values), no cross-lane sums.  XL: x is
// given in block-list order (xl[e] = x[list[e]], as k_fluence_list writes
// it), so staging is one contiguous read instead of the list and a gather.
template <int FMT, int U, bool XL>
__global__ __launch_bounds__(TILE_THREADS) void k_fwd_sell(const int4* __restrict__ work,
                                                         const uint32_t* __restrict__ loff,
                                                         const uint32_t* __restrict__ list,
                                                         const uint32_t* __restrict__ s_off,
                                                         const uint32_t* __restrict__ s_len,
                                                         const uint32_t* __restrict__ s_row,
                                                         const uint16_t* __restrict__ s_col,
                                                         const void* __restrict__ s_val,
                                                         const double* __restrict__ x, double* __restrict__ out,
                                                         Gate gate) {
    __shared__ double xs[TILE_LIST];
    __shared__ double os[TILE_ROWS];
    __shared__ uint32_t qn;
    if (gate.closed()) return;
    if (threadIdx.x == 0) qn = TILE_THREADS / 64;
    const int4 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    const uint32_t l0 = loff[wk.x], ln = loff[wk.x + 1] - l0;
    {
        constexpr int K = TILE_LIST / TILE_THREADS;
        double v[K];
        if constexpr (XL) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t u = threadIdx.x + k * TILE_THREADS;
                v[k] = u < ln ? x[l0 + u] : 0.0;
            }
        } else {
            uint32_t id[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t u = threadIdx.x + k * TILE_THREADS;
                id[k] = u < ln ? list[l0 + u] : 0u;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t u = threadIdx.x + k * TILE_THREADS;
                v[k] = u < ln ? x[id[k]] : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t u = threadIdx.x + k * TILE_THREADS;
            if (u < ln) xs[u] = v[k];
        }
    }
    __syncthreads();
    sell_rows<FMT, U>(wk, s_off, s_len, s_row, s_col, s_val, xs, os, &qn);
    flush_rows<true>(wk, os, out);
}

// Builder of the sliced layout: one wave per slice copies each row's quads
// (values and local columns) to their column-major places, zero quads with
// column 0 after a row's end.  QT: the bytes of one quad of values.
template <typename QT>
__global__ __launch_bounds__(64) void k_sell_fill(const uint32_t* __restrict__ s_off,
                                                  const uint32_t* __restrict__ s_len,
                                                  const uint32_t* __restrict__ s_row,
                                                  const uint32_t* __restrict__ qptr,
                                                  const uint16_t* __restrict__ fcol, const QT* __restrict__ val,
                                                  uint16_t* __restrict__ scol, QT* __restrict__ sval) {
    const int64_t sl = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t row = s_row[sl * 64 + lane];
    const uint32_t q0 = row != 0xFFFFFFFFu ? qptr[row] : 0u;
    const uint32_t rl = row != 0xFFFFFFFFu ? qptr[row + 1] - q0 : 0u;
    const uint32_t base = s_off[sl] + lane, len = s_len[sl];
    const u16x4* __restrict__ c4 = reinterpret_cast<const u16x4*>(fcol);
    u16x4* __restrict__ o4 = reinterpret_cast<u16x4*>(scol);
    for (uint32_t k = 0; k < len; ++k) {
        const uint32_t d = base + k * 64;
        if (k < rl) {
            sval[d] = val[q0 + k];
            o4[d] = c4[q0 + k];
        } else {
            sval[d] = QT{};
            o4[d] = u16x4{0, 0, 0, 0};
        }
    }
}


// Adjoint over the sliced layout: rows are the block's slots, the block's
// slice of w is staged in LDS; each slot row's sum goes to part[slot].
template <int FMT, int U>
__global__ __launch_bounds__(TILE_THREADS) void k_adj_sell(const int4* __restrict__ work,
                                                         const int32_t* __restrict__ bounds,
                                                         const uint32_t* __restrict__ s_off,
                                                         const uint32_t* __restrict__ s_len,
                                                         const uint32_t* __restrict__ s_row,
                                                         const uint16_t* __restrict__ s_col,
                                                         const void* __restrict__ s_val,
                                                         const float* __restrict__ w, double* __restrict__ part,
                                                         Gate gate) {
    __shared__ float ws[TILE_VOXELS];
    __shared__ double os[TILE_ROWS];
    __shared__ uint32_t qn;
    if (gate.closed()) return;
    if (threadIdx.x == 0) qn = TILE_THREADS / 64;
    const int4 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    const int32_t j0 = bounds[wk.x], jn = bounds[wk.x + 1] - j0;
    {
        constexpr int K = TILE_VOXELS / TILE_THREADS;
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int u = threadIdx.x + k * TILE_THREADS;
            v[k] = u < jn ? w[j0 + u] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int u = threadIdx.x + k * TILE_THREADS;
            if (u < jn) ws[u] = v[k];
        }
    }
    __syncthreads();
    sell_rows<FMT, U>(wk, s_off, s_len, s_row, s_col, s_val, ws, os, &qn);
    flush_rows<false>(wk, os, part);
}

// g_i = scale_i * sum of beamlet i's slot sums, in block order.
__global__ __launch_bounds__(256) void k_adj_reduce(int64_t nb, const uint32_t* __restrict__ red_ptr,
                                                    const uint32_t* __restrict__ red_slot,
                                                    const double* __restrict__ part,
                                                    const float* __restrict__ scale, double* __restrict__ g,
                                                    Gate gate) {
    if (gate.closed()) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nb) return;
    const double s = slot_sum(red_ptr[i], red_ptr[i + 1], red_slot, part, 1, 0);
    g[i] = scale ? s * (double)scale[i] : s;
}

// g as k_adj_reduce, and the sum of g over the exposed beamlets of each
// occupied beam in parts: block (k, q) takes the beamlets q*256 .. q*256+255
// of beam k and writes its block sum (fixed tree) to bpart[k*Q + q].
__global__ __launch_bounds__(256) void k_adj_reduce_beams(int R, int C, int Q, const uint32_t* __restrict__ red_ptr,
                                                          const uint32_t* __restrict__ red_slot,
                                                          const double* __restrict__ part,
                                                          const float* __restrict__ scale, double* __restrict__ g,
                                                          const int32_t* __restrict__ l, const int32_t* __restrict__ r,
                                                          const uint8_t* __restrict__ occ, double* __restrict__ bpart,
                                                          Gate gate) {
    __shared__ double sh[4];
    if (gate.closed()) return;
    const int k = blockIdx.x / Q, q = blockIdx.x - k * Q;
    const int RC = R * C;
    const int e = q * 256 + threadIdx.x;
    double ex = 0.0;
    if (e < RC) {
        const int64_t i = (int64_t)k * RC + e;
        const double s = slot_sum(red_ptr[i], red_ptr[i + 1], red_slot, part, 1, 0);
        const double gi = scale ? s * (double)scale[i] : s;
        g[i] = gi;
        const int rho = e / C, c = e - rho * C;
        const int64_t kr = (int64_t)k * R + rho;
        if (occ[k] && c >= l[kr] && c < r[kr]) ex = gi;
    }
    double v = ex;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) bpart[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// The fluence of a plan (as k_fluence) at each entry of the blocks' beamlet
// lists: xl[e] = x_i for i = list[e], the forward's staging order.
__global__ __launch_bounds__(256) void k_fluence_list(int64_t S, const uint32_t* __restrict__ list, int R, int C,
                                                      const double* __restrict__ v, const int32_t* __restrict__ l,
                                                      const int32_t* __restrict__ r, const uint8_t* __restrict__ occ,
                                                      const float* __restrict__ scale, double* __restrict__ xl,
                                                      Gate gate) {
    if (gate.closed()) return;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= S) return;
    const int64_t i = list[e];
    const int64_t kr = i / C;
    const int c = (int)(i - kr * C);
    const int64_t k = kr / R;
    double xi = 0.0;
    if (occ[k] && c >= l[kr] && c < r[kr]) xi = v[k];
    if (scale) xi *= (double)scale[i];
    xl[e] = xi;
}

// ---------------------------------------------------------------- launchers

// Quads in flight per lane of the sliced products: VMAT_SELL_U (2, 4 or 8)
// when set, else the handle's choice.
static int sell_u(const vmat_ctx* h, bool fwd) {
    const char* e = getenv("VMAT_SELL_U");
    const int env = e ? atoi(e) : 0;
    if (env == 2 || env == 4 || env == 8) return env;
    return fwd ? h->sell_u_fwd : h->sell_u_adj;
}

template <int FMT, bool XL>
static vmat_status fwd_fmt(const vmat_ctx* h, const double* x, double* out, Gate gate, hipStream_t st) {
    const Tiled& t = h->tl;
    const unsigned grid = (unsigned)t.n_fwork;
    if (grid == 0) return VMAT_OK;
    const int su = sell_u(h, true);
#define SELL(UU) k_fwd_sell<FMT, UU, XL><<<grid, TILE_THREADS, 0, st>>>(t.fwork, t.loff, t.list, t.s_off, t.s_len, \
                                                                  t.s_row, t.s_col, t.s_val, x, out, gate)
    switch (su) {
        case 2: SELL(2); break;
        case 8: SELL(8); break;
        default: SELL(4); break;
    }
#undef SELL
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

template <int FMT>
static vmat_status adj_fmt(const vmat_ctx* h, const float* w, double* g, Gate gate, hipStream_t st,
                           bool slots_only = false) {
    const Tiled& t = h->tl;
    if (t.n_awork > 0) {
        const int su = sell_u(h, false);
#define ASELL(UU) k_adj_sell<FMT, UU><<<(unsigned)t.n_awork, TILE_THREADS, 0, st>>>( \
    t.awork, t.bounds, t.as_off, t.as_len, t.as_row, t.as_col, t.as_val, w, t.part, gate)
        switch (su) {
            case 2: ASELL(2); break;
            case 8: ASELL(8); break;
            default: ASELL(4); break;
        }
#undef ASELL
        VMAT_LAUNCH_CHECK();
    }
    if (slots_only) return VMAT_OK;
    k_adj_reduce<<<(unsigned)((h->nb + 255) / 256), 256, 0, st>>>(h->nb, t.red_ptr, t.red_slot, t.part, h->bm.scale,
                                                                  g, gate);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

vmat_status launch_fwd(const vmat_ctx* h, const double* x, double* out, Gate gate, hipStream_t st) {
    if (!h->tl.on) return launch_spmv(h, h->vm, x, out, gate, st);
    switch (h->d_store) {
        case VMAT_F32: return fwd_fmt<FMT_F32, false>(h, x, out, gate, st);
        case VMAT_F16: return fwd_fmt<FMT_F16, false>(h, x, out, gate, st);
        case VMAT_BF16: return fwd_fmt<FMT_BF16, false>(h, x, out, gate, st);
        default: return fwd_fmt<FMT_FP8, false>(h, x, out, gate, st);
    }
}

// The dose of a plan's fluence: with the tiled layout the fluence is formed
// in block-list order (h->xl) and staged from there; otherwise in beamlet
// order (h->x) for the plain product.  Same bits either way.
vmat_status launch_fwd_plan(const vmat_ctx* h, const double* v, const int32_t* l, const int32_t* r,
                            const uint8_t* occ, double* out, Gate gate, hipStream_t st) {
    if (!h->tl.on || !h->xl) {
        vmat_status rc = launch_fluence(h, v, l, r, occ, h->bm.scale, h->x, gate, st);
        if (rc != VMAT_OK) return rc;
        return launch_fwd(h, h->x, out, gate, st);
    }
    const Tiled& t = h->tl;
    k_fluence_list<<<(unsigned)((t.S + 255) / 256), 256, 0, st>>>(t.S, t.list, h->R, h->C, v, l, r, occ,
                                                                    h->bm.scale, h->xl, gate);
    VMAT_LAUNCH_CHECK();
    switch (h->d_store) {
        case VMAT_F32: return fwd_fmt<FMT_F32, true>(h, h->xl, out, gate, st);
        case VMAT_F16: return fwd_fmt<FMT_F16, true>(h, h->xl, out, gate, st);
        case VMAT_BF16: return fwd_fmt<FMT_BF16, true>(h, h->xl, out, gate, st);
        default: return fwd_fmt<FMT_FP8, true>(h, h->xl, out, gate, st);
    }
}

vmat_status launch_adj_slots(const vmat_ctx* h, const float* w, Gate gate, hipStream_t st) {
    switch (h->d_store) {
        case VMAT_F32: return adj_fmt<FMT_F32>(h, w, nullptr, gate, st, true);
        case VMAT_F16: return adj_fmt<FMT_F16>(h, w, nullptr, gate, st, true);
        case VMAT_BF16: return adj_fmt<FMT_BF16>(h, w, nullptr, gate, st, true);
        default: return adj_fmt<FMT_FP8>(h, w, nullptr, gate, st, true);
    }
}

// Times the sliced forward and adjoint with 4 and 8 quads in flight on the
// handle's own layout (zero operands; the time does not depend on the values)
// and keeps the faster of each.  Either choice gives the same bits: every
// lane sums its quads in order.
vmat_status tune_sell(vmat_ctx* h, hipStream_t st) {
    const Tiled& t = h->tl;
    if (!t.on || !t.s_val || !t.as_val) return VMAT_OK;
    VMAT_HIP(hipMemsetAsync(h->x, 0, (size_t)h->nb * sizeof(double), st));
    VMAT_HIP(hipMemsetAsync(h->rz, 0, (size_t)h->nv * sizeof(float), st));
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    VMAT_HIP(hipEventCreate(&ev.e[0]));
    VMAT_HIP(hipEventCreate(&ev.e[1]));
    // three rounds, the two variants in alternating order, the best round of
    // each kept: the two often differ by 2-3%, less than one timing's spread
    constexpr int reps = 3, rounds = 3;
    float best[2][2] = {{1e30f, 1e30f}, {1e30f, 1e30f}};
    for (int fwd = 0; fwd < 2; ++fwd)
        for (int round = 0; round < rounds; ++round)
            for (int k = 0; k < 2; ++k) {
                const int ui = (round & 1) ? 1 - k : k;
                (fwd ? h->sell_u_fwd : h->sell_u_adj) = ui ? 8 : 4;
                for (int r = -1; r < reps; ++r) {
                    if (r == 0) VMAT_HIP(hipEventRecord(ev.e[0], st));
                    const vmat_status rc = fwd ? launch_fwd(h, h->x, h->dz, Gate{}, st)
                                               : launch_adj(h, h->rz, h->g, Gate{}, st);
                    if (rc != VMAT_OK) return rc;
                }
                VMAT_HIP(hipEventRecord(ev.e[1], st));
                VMAT_HIP(hipEventSynchronize(ev.e[1]));
                float ms = 0.f;
                VMAT_HIP(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
                best[fwd][ui] = std::min(best[fwd][ui], ms);
            }
    h->sell_u_adj = best[0][1] < best[0][0] ? 8 : 4;
    h->sell_u_fwd = best[1][1] < best[1][0] ? 8 : 4;
    return VMAT_OK;
}

int beam_parts(const vmat_ctx* h) { return h->tl.on ? (h->R * h->C + 255) / 256 : 0; }

vmat_status launch_adj_beams(const vmat_ctx* h, const float* w, double* g, const int32_t* l, const int32_t* r,
                             const uint8_t* occ, double* bpart, Gate gate, hipStream_t st) {
    const int Q = beam_parts(h);
    vmat_status rc;
    if (Q == 0) {
        if ((rc = launch_adj(h, w, g, gate, st)) != VMAT_OK) return rc;
        return launch_beam_sums(h, g, l, r, occ, bpart, gate, st);
    }
    if ((rc = launch_adj_slots(h, w, gate, st)) != VMAT_OK) return rc;
    const Tiled& t = h->tl;
    k_adj_reduce_beams<<<(unsigned)(h->N * Q), 256, 0, st>>>(h->R, h->C, Q, t.red_ptr, t.red_slot, t.part,
                                                              h->bm.scale, g, l, r, occ, bpart, gate);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

vmat_status launch_adj(const vmat_ctx* h, const float* w, double* g, Gate gate, hipStream_t st) {
    if (!h->tl.on) return launch_spmv(h, h->bm, w, g, gate, st);
    switch (h->d_store) {
        case VMAT_F32: return adj_fmt<FMT_F32>(h, w, g, gate, st);
        case VMAT_F16: return adj_fmt<FMT_F16>(h, w, g, gate, st);
        case VMAT_BF16: return adj_fmt<FMT_BF16>(h, w, g, gate, st);
        default: return adj_fmt<FMT_FP8>(h, w, g, gate, st);
    }
}

// ---------------------------------------------------------------- builder kernels

// Mark the beamlets of every block in a bitmap (one bitmap of W words per block).
__global__ void k_blk_mark(int nblk, const int32_t* __restrict__ bounds, const uint32_t* __restrict__ vqptr,
                           const int32_t* __restrict__ vcol, int64_t W, uint32_t* __restrict__ bits) {
    const int b = blockIdx.y;
    if (b >= nblk) return;
    const int64_t e0 = (int64_t)vqptr[bounds[b]] * 4, e1 = (int64_t)vqptr[bounds[b + 1]] * 4;
    uint32_t* bm = bits + (int64_t)b * W;
    for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)vcol[e];
        atomicOr(&bm[i >> 5], 1u << (i & 31));
    }
}

__global__ void k_blk_popc(int nblk, int64_t W, const uint32_t* __restrict__ bits, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t sh[256];
    const int b = blockIdx.x;
    uint32_t c = 0;
    for (int64_t w = threadIdx.x; w < W; w += 256) c += __popc(bits[(int64_t)b * W + w]);
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[b] = sh[0];
}

// List of each block (ascending beamlet ids) and per-word rank prefixes.
__global__ void k_blk_list(int64_t W, const uint32_t* __restrict__ bits, const uint32_t* __restrict__ loff,
                           uint32_t* __restrict__ wpref, uint32_t* __restrict__ list) {
    __shared__ uint32_t sh[256];
    const int b = blockIdx.x;
    const int64_t per = (W + 255) / 256;
    const int64_t w0 = min(W, (int64_t)threadIdx.x * per), w1 = min(W, w0 + per);
    const uint32_t* bm = bits + (int64_t)b * W;
    uint32_t c = 0;
    for (int64_t w = w0; w < w1; ++w) c += __popc(bm[w]);
    sh[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int t = 0; t < 256; ++t) {
            const uint32_t v = sh[t];
            sh[t] = acc;
            acc += v;
        }
    }
    __syncthreads();
    uint32_t pos = sh[threadIdx.x];
    for (int64_t w = w0; w < w1; ++w) {
        wpref[(int64_t)b * W + w] = pos;
        uint32_t word = bm[w];
        while (word) {
            const int bit = __ffs(word) - 1;
            list[loff[b] + pos] = (uint32_t)(w * 32 + bit);
            ++pos;
            word &= word - 1;
        }
    }
}

// 16-bit list index of every voxel-major entry.
__global__ void k_fw_col16(int nblk, const int32_t* __restrict__ bounds, const uint32_t* __restrict__ vqptr,
                           const int32_t* __restrict__ vcol, int64_t W, const uint32_t* __restrict__ bits,
                           const uint32_t* __restrict__ wpref, uint16_t* __restrict__ fcol) {
    const int b = blockIdx.y;
    if (b >= nblk) return;
    const int64_t e0 = (int64_t)vqptr[bounds[b]] * 4, e1 = (int64_t)vqptr[bounds[b + 1]] * 4;
    const uint32_t* bm = bits + (int64_t)b * W;
    const uint32_t* wp = wpref + (int64_t)b * W;
    for (int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e1; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)vcol[e];
        const uint32_t below = bm[i >> 5] & ((1u << (i & 31)) - 1u);
        fcol[e] = (uint16_t)(wp[i >> 5] + __popc(below));
    }
}

__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* a, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Segment of every slot's beamlet row inside its block (from the caller's CSR).
__global__ void k_adj_len(int64_t S, int nblk, const uint32_t* __restrict__ loff, const int32_t* __restrict__ bounds,
                          const uint32_t* __restrict__ list, const int64_t* __restrict__ rp,
                          const int32_t* __restrict__ col, int64_t* __restrict__ seg_lo,
                          uint32_t* __restrict__ quads) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    int lo = 0, hi = nblk;  // block of slot s: loff[b] <= s < loff[b+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)loff[mid] <= s) lo = mid; else hi = mid;
    }
    const int b = lo;
    const uint32_t i = list[s];
    const int64_t a = lower_bound_i32(col, rp[i], rp[i + 1], bounds[b]);
    const int64_t e = lower_bound_i32(col, a, rp[i + 1], bounds[b + 1]);
    seg_lo[s] = a;
    quads[s] = (uint32_t)((e - a + 3) >> 2);
}

// Copy every slot's segment (encoded values from the beamlet-major copy) with
// 16-bit offsets from the block start; pad to whole quads.  One wave per slot.
template <typename VT>
__global__ void k_adj_fill(int64_t S, int nblk, const uint32_t* __restrict__ loff,
                           const int32_t* __restrict__ bounds, const uint32_t* __restrict__ list,
                           const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const uint32_t* __restrict__ bm_qptr, const VT* __restrict__ bm_val,
                           const int64_t* __restrict__ seg_lo, const uint32_t* __restrict__ aqptr,
                           uint16_t* __restrict__ acol, VT* __restrict__ aval) {
    const int64_t s = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (s >= S) return;
    int lo = 0, hi = nblk;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)loff[mid] <= s) lo = mid; else hi = mid;
    }
    const int32_t j0 = bounds[lo], j1 = bounds[lo + 1];
    const uint32_t i = list[s];
    const int64_t a = seg_lo[s];
    const int64_t n = lower_bound_i32(col, a, rp[i + 1], j1) - a;   // entries of row i inside the block
    const int64_t dst = (int64_t)aqptr[s] * 4, npad = (int64_t)(aqptr[s + 1] - aqptr[s]) * 4;
    const int64_t src = (int64_t)bm_qptr[i] * 4 + (a - rp[i]);
    for (int64_t e = lane; e < npad; e += 64) {
        const bool real = e < n;
        acol[dst + e] = real ? (uint16_t)(col[a + e] - j0) : (uint16_t)0;
        aval[dst + e] = real ? bm_val[src + e] : (VT)0;
    }
}

__global__ void k_red_count(int64_t S, const uint32_t* __restrict__ list, uint32_t* __restrict__ cnt) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s < S) atomicAdd(&cnt[list[s]], 1u);
}

__global__ void k_red_fill(int64_t S, const uint32_t* __restrict__ list, const uint32_t* __restrict__ red_ptr,
                           uint32_t* __restrict__ fill, uint32_t* __restrict__ slot) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    const uint32_t i = list[s];
    slot[red_ptr[i] + atomicAdd(&fill[i], 1u)] = (uint32_t)s;
}

__global__ void k_red_sort(int64_t nb, const uint32_t* __restrict__ red_ptr, uint32_t* __restrict__ slot) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nb) return;
    const uint32_t a = red_ptr[i], b = red_ptr[i + 1];
    for (uint32_t k = a + 1; k < b; ++k) {
        const uint32_t v = slot[k];
        uint32_t m = k;
        while (m > a && slot[m - 1] > v) {
            slot[m] = slot[m - 1];
            --m;
        }
        slot[m] = v;
    }
}

// ---------------------------------------------------------------- builder (host)

vmat_status scan_u32_dev(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t st);  // vmat_build.hip

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    template <typename T>
    T* as() { return reinterpret_cast<T*>(p); }
};

hipError_t dmalloc(DevBuf& b, size_t bytes) {
    return hipMalloc(&b.p, std::max<size_t>(bytes, 16));
}

// Work items of about `qpw` quads each (at most max_rows rows), never
// crossing a block, placed for the XCDs.  Workgroups are dealt to the eight
// XCDs in turn (w and w + 8 on the same XCD; measured on MI355X: XCD
// (w + 7) mod 8), so slot x of each group of eight is one XCD's sequence.
// The items, in block order, are cut into eight runs of about equal quads;
// run x becomes sequence x, so an XCD's items share their blocks' staged
// values in its L2.  Each sequence is ordered by quads, largest first: a
// compute unit that frees a slot late in the launch takes a small item, so
// the launch ends with short items (longest-processing-time order).
std::vector<int4> make_work(const std::vector<int64_t>& row_begin_of_block, const std::vector<uint32_t>& rowq,
                            int nblk, int64_t qpw, int64_t max_rows) {
    std::vector<int4> items;
    for (int b = 0; b < nblk; ++b) {
        const int64_t r0 = row_begin_of_block[b], r1 = row_begin_of_block[b + 1];
        int64_t start = r0;
        uint64_t acc = 0;
        for (int64_t r = r0; r < r1; ++r) {
            acc += rowq[r + 1] - rowq[r];
            if ((int64_t)acc >= qpw || r + 1 - start >= max_rows) {
                items.push_back(make_int4(b, (int)start, (int)(r + 1), 0));
                start = r + 1;
                acc = 0;
            }
        }
        if (start < r1) items.push_back(make_int4(b, (int)start, (int)r1, 0));
    }
    auto quads = [&](const int4& it) { return (uint64_t)(rowq[it.z] - rowq[it.y]); };
    uint64_t total = 0;
    for (const int4& it : items) total += quads(it);
    std::vector<std::vector<int4>> seq(8);
    uint64_t before = 0;
    for (const int4& it : items) {
        // the run holding the item's midpoint
        const uint64_t mid = before + quads(it) / 2;
        seq[(size_t)std::min<uint64_t>(7, mid * 8 / std::max<uint64_t>(1, total))].push_back(it);
        before += quads(it);
    }
    size_t per = 0;
    for (std::vector<int4>& q : seq) {
        std::stable_sort(q.begin(), q.end(), [&](const int4& a, const int4& b) { return quads(a) > quads(b); });
        per = std::max(per, q.size());
    }
    std::vector<int4> out(per * 8, make_int4(-1, 0, 0, 0));
    for (int x = 0; x < 8; ++x)
        for (size_t k = 0; k < seq[(size_t)x].size(); ++k) out[k * 8 + (size_t)x] = seq[(size_t)x][k];
    return out;
}

// Sliced layout of the rows of every work item (item.w becomes its first
// slice): rows sorted by quad count, longest first (ties by row), 64 per
// slice, each slice padded to its first row's length.  False if the quads
// exceed 32-bit offsets.
bool make_slices(std::vector<int4>& items, const std::vector<uint32_t>& qp, std::vector<uint32_t>& s_off,
                 std::vector<uint32_t>& s_len, std::vector<uint32_t>& s_row, uint64_t& quads) {
    uint64_t off = 0;
    std::vector<std::pair<uint32_t, uint32_t>> rows;
    for (int4& it : items) {
        it.w = (int)s_len.size();
        if (it.x < 0) continue;
        rows.clear();
        for (int r = it.y; r < it.z; ++r) rows.push_back({qp[r + 1] - qp[r], (uint32_t)r});
        std::stable_sort(rows.begin(), rows.end(),
                         [](const std::pair<uint32_t, uint32_t>& a, const std::pair<uint32_t, uint32_t>& b) {
                             return a.first > b.first;
                         });
        for (size_t j = 0; j < rows.size(); j += 64) {
            s_off.push_back((uint32_t)off);
            s_len.push_back(rows[j].first);
            off += (uint64_t)rows[j].first * 64;
            for (size_t i = j; i < j + 64; ++i) s_row.push_back(i < rows.size() ? rows[i].second : 0xFFFFFFFFu);
        }
    }
    quads = off;
    return off < ((uint64_t)1 << 32);
}

}  // namespace

// Builds h->tl from the voxel-major and beamlet-major copies and the caller's
// CSR.  Returns VMAT_ERR_UNSUPPORTED when some block cannot be made to fit.
vmat_status build_tiled(vmat_ctx* h, const vmat_problem* p, hipStream_t st) {
    Tiled& t = h->tl;
    const int64_t nv = h->nv, nb = h->nb;
    const int64_t W = (nb + 31) / 32;
    if (h->R > 4095 || h->N > 4095) return fail(VMAT_ERR_UNSUPPORTED, "tiled layout needs N, R < 4096");
    std::vector<int64_t> bounds;
    for (int64_t j = 0; j < nv; j += TILE_VOXELS) bounds.push_back(j);
    bounds.push_back(nv);

    DevBuf d_bounds, d_bits, d_cnt;
    std::vector<uint32_t> cnt;
    for (int round = 0;; ++round) {
        const int nblk = (int)bounds.size() - 1;
        if ((double)nblk * (double)W * 4.0 > 2e9 || nblk > 60000)
            return fail(VMAT_ERR_UNSUPPORTED, "voxel blocking needs too many blocks");
        std::vector<int32_t> b32(bounds.begin(), bounds.end());
        d_bounds = DevBuf();
        d_bits = DevBuf();
        d_cnt = DevBuf();
        VMAT_HIP(dmalloc(d_bounds, b32.size() * 4));
        VMAT_HIP(dmalloc(d_bits, (size_t)nblk * W * 4));
        VMAT_HIP(dmalloc(d_cnt, (size_t)nblk * 4));
        VMAT_HIP(hipMemcpyAsync(d_bounds.p, b32.data(), b32.size() * 4, hipMemcpyHostToDevice, st));
        VMAT_HIP(hipMemsetAsync(d_bits.p, 0, (size_t)nblk * W * 4, st));
        k_blk_mark<<<dim3(64, nblk), 256, 0, st>>>(nblk, d_bounds.as<int32_t>(), h->vm.qptr, h->vm.col, W,
                                                  d_bits.as<uint32_t>());
        VMAT_LAUNCH_CHECK();
        k_blk_popc<<<nblk, 256, 0, st>>>(nblk, W, d_bits.as<uint32_t>(), d_cnt.as<uint32_t>());
        VMAT_LAUNCH_CHECK();
        cnt.assign(nblk, 0);
        VMAT_HIP(hipMemcpyAsync(cnt.data(), d_cnt.p, (size_t)nblk * 4, hipMemcpyDeviceToHost, st));
        VMAT_HIP(hipStreamSynchronize(st));
        std::vector<int64_t> nb2;
        bool split = false, stuck = false;
        for (int b = 0; b < nblk; ++b) {
            nb2.push_back(bounds[b]);
            if (cnt[b] > (uint32_t)TILE_LIST) {
                const int64_t len = bounds[b + 1] - bounds[b];
                if (len <= 64) {
                    stuck = true;
                } else {
                    nb2.push_back(bounds[b] + len / 2);
                    split = true;
                }
            }
        }
        nb2.push_back(nv);
        if (stuck) return fail(VMAT_ERR_UNSUPPORTED, "a 64-voxel block reaches more than 8192 beamlets");
        if (!split) break;
        bounds.swap(nb2);
        if (round > 20) return fail(VMAT_ERR_UNSUPPORTED, "voxel blocking did not converge");
    }
    const int nblk = (int)bounds.size() - 1;
    t.nblk = nblk;
    std::vector<uint32_t> loff(nblk + 1, 0);
    for (int b = 0; b < nblk; ++b) loff[b + 1] = loff[b] + cnt[b];
    t.S = loff[nblk];

    auto alloc = [&](void** ptr, size_t bytes) -> vmat_status {
        hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) return fail(VMAT_ERR_ALLOC, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        h->bytes += (int64_t)bytes;
        return VMAT_OK;
    };
#define A(ptr, bytes) do { vmat_status r_ = alloc((void**)&(ptr), (bytes)); if (r_ != VMAT_OK) return r_; } while (0)
    A(t.bounds, (nblk + 1) * 4);
    VMAT_HIP(hipMemcpyAsync(t.bounds, d_bounds.p, (nblk + 1) * 4, hipMemcpyDeviceToDevice, st));
    A(t.loff, (nblk + 1) * 4);
    VMAT_HIP(hipMemcpyAsync(t.loff, loff.data(), (nblk + 1) * 4, hipMemcpyHostToDevice, st));
    A(t.list, t.S * 4);
    DevBuf d_wpref;
    VMAT_HIP(dmalloc(d_wpref, (size_t)nblk * W * 4));
    k_blk_list<<<nblk, 256, 0, st>>>(W, d_bits.as<uint32_t>(), t.loff, d_wpref.as<uint32_t>(), t.list);
    VMAT_LAUNCH_CHECK();

    // forward indices
    A(t.fcol, (size_t)h->vm.n_quads * 4 * 2);
    k_fw_col16<<<dim3(64, nblk), 256, 0, st>>>(nblk, t.bounds, h->vm.qptr, h->vm.col, W, d_bits.as<uint32_t>(),
                                              d_wpref.as<uint32_t>(), t.fcol);
    VMAT_LAUNCH_CHECK();

    // adjoint slot rows
    DevBuf d_seglo, d_aq;
    VMAT_HIP(dmalloc(d_seglo, (size_t)t.S * 8));
    VMAT_HIP(dmalloc(d_aq, (size_t)(t.S + 1) * 4));
    if (t.S > 0) {
        k_adj_len<<<(unsigned)((t.S + 255) / 256), 256, 0, st>>>(t.S, nblk, t.loff, t.bounds, t.list, p->row_ptr,
                                                                 p->col, d_seglo.as<int64_t>(), d_aq.as<uint32_t>());
        VMAT_LAUNCH_CHECK();
    }
    A(t.aqptr, (t.S + 1) * 4);
    {
        vmat_status rc = scan_u32_dev(d_aq.as<uint32_t>(), t.S, t.aqptr, st);
        if (rc != VMAT_OK) return rc;
    }
    uint32_t aq_tot = 0;
    VMAT_HIP(hipMemcpyAsync(&aq_tot, t.aqptr + t.S, 4, hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipStreamSynchronize(st));
    t.a_quads = aq_tot;
    const int vb = fmt_bytes(h->d_store);  // vmat_dtype values equal the Fmt values
    A(t.acol, (size_t)t.a_quads * 4 * 2);
    A(t.aval, (size_t)t.a_quads * 4 * vb);
    if (t.S > 0) {
        const unsigned g4 = (unsigned)((t.S + 3) / 4);
        if (vb == 4)
            k_adj_fill<float><<<g4, 256, 0, st>>>(t.S, nblk, t.loff, t.bounds, t.list, p->row_ptr, p->col,
                                                  h->bm.qptr, (const float*)h->bm.val, d_seglo.as<int64_t>(),
                                                  t.aqptr, t.acol, (float*)t.aval);
        else if (vb == 2)
            k_adj_fill<uint16_t><<<g4, 256, 0, st>>>(t.S, nblk, t.loff, t.bounds, t.list, p->row_ptr, p->col,
                                                     h->bm.qptr, (const uint16_t*)h->bm.val, d_seglo.as<int64_t>(),
                                                     t.aqptr, t.acol, (uint16_t*)t.aval);
        else
            k_adj_fill<uint8_t><<<g4, 256, 0, st>>>(t.S, nblk, t.loff, t.bounds, t.list, p->row_ptr, p->col,
                                                    h->bm.qptr, (const uint8_t*)h->bm.val, d_seglo.as<int64_t>(),
                                                    t.aqptr, t.acol, (uint8_t*)t.aval);
        VMAT_LAUNCH_CHECK();
    }

    // per-beamlet slot lists, in block order
    A(t.part, t.S * 8);
    A(t.red_ptr, (nb + 1) * 4);
    A(t.red_slot, t.S * 4);
    DevBuf d_rc, d_rf;
    VMAT_HIP(dmalloc(d_rc, (size_t)(nb + 1) * 4));
    VMAT_HIP(dmalloc(d_rf, (size_t)(nb + 1) * 4));
    VMAT_HIP(hipMemsetAsync(d_rc.p, 0, (size_t)(nb + 1) * 4, st));
    VMAT_HIP(hipMemsetAsync(d_rf.p, 0, (size_t)(nb + 1) * 4, st));
    if (t.S > 0) {
        k_red_count<<<(unsigned)((t.S + 255) / 256), 256, 0, st>>>(t.S, t.list, d_rc.as<uint32_t>());
        VMAT_LAUNCH_CHECK();
    }
    {
        vmat_status rc = scan_u32_dev(d_rc.as<uint32_t>(), nb, t.red_ptr, st);
        if (rc != VMAT_OK) return rc;
    }
    if (t.S > 0) {
        k_red_fill<<<(unsigned)((t.S + 255) / 256), 256, 0, st>>>(t.S, t.list, t.red_ptr, d_rf.as<uint32_t>(),
                                                                  t.red_slot);
        VMAT_LAUNCH_CHECK();
    }
    k_red_sort<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nb, t.red_ptr, t.red_slot);
    VMAT_LAUNCH_CHECK();

    // work lists
    std::vector<uint32_t> vq(nv + 1), aq(t.S + 1);
    VMAT_HIP(hipMemcpyAsync(vq.data(), h->vm.qptr, (nv + 1) * 4, hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipMemcpyAsync(aq.data(), t.aqptr, (t.S + 1) * 4, hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipStreamSynchronize(st));
    const int64_t target_items = 1024;
    const int64_t fq = std::max<int64_t>(1, (int64_t)vq[nv]);
    const int64_t aqn = std::max<int64_t>(1, (int64_t)aq[t.S]);
    std::vector<int64_t> rb(bounds.begin(), bounds.end());
    std::vector<int64_t> sb(nblk + 1);
    for (int b = 0; b <= nblk; ++b) sb[b] = loff[b];
    const int64_t mrows = TILE_ROWS;
    std::vector<int4> fw = make_work(rb, vq, nblk, std::max<int64_t>(256, fq / target_items), mrows);
    // the adjoint's slot rows are long and few (460,800 on prostate: 7.5
    // slices per item at 1,024 items, fewer than a workgroup's 8 waves);
    // 512 items, one per resident workgroup, measured best on prostate
    // (3.4% faster than 1,024) and 1.6-1.9% faster on head-and-neck FP32 and
    // BF16; FP8 keeps 1,024 (1.6% faster than 512 on head-and-neck)
    const int64_t adj_items = h->d_store == VMAT_FP8_E4M3 ? 1024 : 512;
    std::vector<int4> aw = make_work(sb, aq, nblk, std::max<int64_t>(256, aqn / adj_items), mrows);
    // the products stage an item's row sums in LDS (TILE_ROWS of them)
    for (const std::vector<int4>* items : {&fw, &aw})
        for (const int4& it : *items)
            if (it.x >= 0 && (it.z < it.y || it.z - it.y > TILE_ROWS))
                return fail(VMAT_ERR_UNSUPPORTED, "work item longer than TILE_ROWS rows");
    // sliced layouts: rows of each work item sorted by length, 64 per slice
    std::vector<uint32_t> s_off, s_len, s_row, as_off, as_len, as_row;
    {
        uint64_t fq_s = 0, aq_s = 0;
        if (!make_slices(fw, vq, s_off, s_len, s_row, fq_s) || !make_slices(aw, aq, as_off, as_len, as_row, aq_s))
            return fail(VMAT_ERR_UNSUPPORTED, "sliced layout exceeds 2^32 quads");
        t.n_slices = (int64_t)s_len.size();
        t.s_quads = (int64_t)fq_s;
        t.an_slices = (int64_t)as_len.size();
        t.as_quads = (int64_t)aq_s;
    }
    {
        // slices grouped by block, and XCD block ranges, for the batched products
        auto group = [&](const std::vector<int4>& items, int64_t n_sl, const std::vector<uint32_t>& slen,
                         uint32_t*& d_ptr, uint32_t*& d_sl, int32_t* xr) -> vmat_status {
            std::vector<std::vector<uint32_t>> per(nblk);
            for (const int4& it : items) {
                if (it.x < 0) continue;
                const int ns = (it.z - it.y + 63) / 64;
                for (int k = 0; k < ns; ++k) per[it.x].push_back((uint32_t)(it.w + k));
            }
            std::vector<uint32_t> ptr(nblk + 1, 0), sl;
            sl.reserve((size_t)n_sl);
            std::vector<double> load(nblk, 0.0);
            for (int b = 0; b < nblk; ++b) {
                for (uint32_t x : per[b]) {
                    sl.push_back(x);
                    load[b] += 64.0 * slen[x];
                }
                ptr[b + 1] = (uint32_t)sl.size();
            }
            double tot = 0.0;
            for (double v : load) tot += v;
            // XCD i takes the blocks whose cumulative load starts in its eighth
            xr[0] = 0;
            double acc = 0.0;
            int b = 0;
            for (int i = 1; i < 8; ++i) {
                while (b < nblk && acc + 0.5 * load[b] < tot * i / 8.0) acc += load[b++];
                xr[i] = b;
            }
            xr[8] = nblk;
            A(d_ptr, ptr.size() * 4);
            A(d_sl, std::max<size_t>(sl.size(), 1) * 4);
            VMAT_HIP(hipMemcpyAsync(d_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, st));
            if (!sl.empty()) VMAT_HIP(hipMemcpyAsync(d_sl, sl.data(), sl.size() * 4, hipMemcpyHostToDevice, st));
            VMAT_HIP(hipStreamSynchronize(st));
            return VMAT_OK;
        };
        vmat_status rg = group(fw, t.n_slices, s_len, t.fb_ptr, t.fb_sl, t.fx);
        if (rg != VMAT_OK) return rg;
        rg = group(aw, t.an_slices, as_len, t.ab_ptr, t.ab_sl, t.ax);
        if (rg != VMAT_OK) return rg;
    }
    A(t.fwork, fw.size() * sizeof(int4));
    A(t.awork, aw.size() * sizeof(int4));
    VMAT_HIP(hipMemcpyAsync(t.fwork, fw.data(), fw.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    VMAT_HIP(hipMemcpyAsync(t.awork, aw.data(), aw.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    t.n_fwork = (int)fw.size();
    t.n_awork = (int)aw.size();
    {
        const int vb = h->d_store == VMAT_F32 ? 4 : (h->d_store == VMAT_FP8_E4M3 ? 1 : 2);
        auto sliced = [&](int64_t n_sl, int64_t quads, const std::vector<uint32_t>& so,
                          const std::vector<uint32_t>& sn, const std::vector<uint32_t>& sr, const uint32_t* qp,
                          const uint16_t* col, const void* val, uint32_t*& d_off, uint32_t*& d_len,
                          uint32_t*& d_row, uint16_t*& d_col, void*& d_val) -> vmat_status {
            const size_t ns = (size_t)std::max<int64_t>(n_sl, 1);
            A(d_off, ns * 4);
            A(d_len, ns * 4);
            A(d_row, ns * 64 * 4);
            A(d_col, (size_t)std::max<int64_t>(quads, 1) * 8);
            A(d_val, (size_t)std::max<int64_t>(quads, 1) * 4 * vb);
            if (n_sl == 0) return VMAT_OK;
            VMAT_HIP(hipMemcpyAsync(d_off, so.data(), so.size() * 4, hipMemcpyHostToDevice, st));
            VMAT_HIP(hipMemcpyAsync(d_len, sn.data(), sn.size() * 4, hipMemcpyHostToDevice, st));
            VMAT_HIP(hipMemcpyAsync(d_row, sr.data(), sr.size() * 4, hipMemcpyHostToDevice, st));
            const unsigned g = (unsigned)n_sl;
            if (vb == 4)
                k_sell_fill<f32x4><<<g, 64, 0, st>>>(d_off, d_len, d_row, qp, col,
                                                    reinterpret_cast<const f32x4*>(val), d_col,
                                                    reinterpret_cast<f32x4*>(d_val));
            else if (vb == 2)
                k_sell_fill<u32x2><<<g, 64, 0, st>>>(d_off, d_len, d_row, qp, col,
                                                    reinterpret_cast<const u32x2*>(val), d_col,
                                                    reinterpret_cast<u32x2*>(d_val));
            else
                k_sell_fill<uint32_t><<<g, 64, 0, st>>>(d_off, d_len, d_row, qp, col,
                                                       reinterpret_cast<const uint32_t*>(val), d_col,
                                                       reinterpret_cast<uint32_t*>(d_val));
            VMAT_HIP(hipGetLastError());
            return VMAT_OK;
        };
        vmat_status rs = sliced(t.n_slices, t.s_quads, s_off, s_len, s_row, h->vm.qptr, t.fcol, h->vm.val, t.s_off,
                                t.s_len, t.s_row, t.s_col, t.s_val);
        if (rs != VMAT_OK) return rs;
        rs = sliced(t.an_slices, t.as_quads, as_off, as_len, as_row, t.aqptr, t.acol, t.aval, t.as_off, t.as_len,
                    t.as_row, t.as_col, t.as_val);
        if (rs != VMAT_OK) return rs;
    }
    VMAT_HIP(hipStreamSynchronize(st));
#undef A
    // the CSR-shaped forms were the sources of the sliced ones; every product
    // runs on the sliced forms
    auto release = [&](void*& p, int64_t bytes) {
        if (!p) return;
        (void)hipFree(p);
        h->bytes -= bytes;
        p = nullptr;
    };
    release(reinterpret_cast<void*&>(t.fcol), h->vm.n_quads * 4 * 2);
    release(reinterpret_cast<void*&>(t.aqptr), (t.S + 1) * 4);
    release(reinterpret_cast<void*&>(t.acol), t.a_quads * 4 * 2);
    release(t.aval, t.a_quads * 4 * (int64_t)vb);
    t.on = true;
    return VMAT_OK;
}

void free_tiled(vmat_ctx* h) {
    Tiled& t = h->tl;
    void* ps[] = {t.bounds, t.loff, t.list, t.fcol, t.fwork, t.aqptr, t.acol, t.aval, t.awork, t.part, t.red_ptr,
                  t.red_slot, t.s_off, t.s_len, t.s_row, t.s_col, t.s_val, t.as_off, t.as_len, t.as_row, t.as_col,
                  t.as_val, t.fb_ptr, t.fb_sl, t.ab_ptr, t.ab_sl};
    for (void* q : ps)
        if (q) (void)hipFree(q);
    t = Tiled();
}

}  // namespace vmat
