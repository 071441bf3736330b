// Plan variants sharing one D: products with many right-hand sides (SpMM)
// and the batched cost and gradient.
//
// Layout: RHS-contiguous, X[i*B + b] (beamlets) and Z[j*B + b] (voxels).  A
// row of D is read once per tile of TB right-hand sides; the lanes of a wave
// that share the row gather TB consecutive values per non-zero, so each
// gather is one contiguous span.  The row's index and value quads reach those
// lanes as broadcast loads (every lane loads the same quad), or, in the tiled
// forward, loaded once per row and spread across its lanes by DPP.
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

// ---- tiled layout: XCD-owned voxel blocks over the sliced layouts
//
// A row of D (a voxel of the forward, a slot row of the adjoint) is walked by
// LPR lanes, each holding V consecutive right-hand sides (TB = LPR * V per
// pass over the row; RPW = 64 / LPR rows per wave).  Every (row, RHS) sum
// runs over the row's quads in order, entries in order: the bits do not
// depend on LPR, V or the schedule.
//
// Schedule: workgroups are dealt to the XCDs in turn, so those with the
// same w % 8 share an XCD (measured on MI355X: XCD (w + 7) mod 8); group i of
// them (one XCD) walks its own contiguous
// range of voxel blocks in order, and within a block the right-hand sides in
// tiles of TB, all its workgroups on one (block, tile) at a time, so the rows
// a block gathers (at most TILE_LIST beamlets, or the block's voxels, times
// TB values) stay in that XCD's L2 while its workgroups read them.  Within a
// (block, tile) the units of work are (slice, group of RPW rows), dealt to
// the XCD's waves in order.  Gathered rows are addressed by 32-bit element
// offsets from a uniform base.

// V consecutive floats at p (V-aligned: V | B and the column is a multiple of V).
template <int V>
__device__ __forceinline__ void ld_vec(const float* __restrict__ p, float (&o)[V]) {
    if constexpr (V == 1) {
        o[0] = *p;
    } else if constexpr (V == 2) {
        const f32x2 a = *reinterpret_cast<const f32x2*>(p);
        o[0] = a.x;
        o[1] = a.y;
    } else {
#pragma unroll
        for (int h = 0; h < V / 4; ++h) {
            const f32x4 a = reinterpret_cast<const f32x4*>(p)[h];
            o[4 * h + 0] = a.x;
            o[4 * h + 1] = a.y;
            o[4 * h + 2] = a.z;
            o[4 * h + 3] = a.w;
        }
    }
}

// Blocks of XCD xcd: [xr.b[xcd], xr.b[xcd + 1]).
struct XcdRanges {
    int32_t b[9];
};

// One row's sums over its quads [q, q + 64 len) (column-major slice: the
// row's next quad is 64 quads on), V right-hand sides.  ROW(c16) gives the
// element offset of the gathered row's first right-hand side of this lane
// (from the uniform base Y); SC(c16) its column scale (CS only).  Two quads
// per step keep eight gathers in flight.
template <int FMT, int V, bool CS, class ROW, class SCL>
__device__ __forceinline__ void row_sums(uint32_t q, uint32_t len, const u16x4* __restrict__ col,
                                         const void* __restrict__ val, const float* __restrict__ Y, ROW rowoff,
                                         SCL scl, double (&acc)[V]) {
    uint32_t k = 0;
    for (; k + 2 <= len; k += 2) {
        float4 v[2];
        u16x4 cc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            v[h] = Quad<FMT>::ld(val, q + (k + h) * 64);
            cc[h] = col[q + (k + h) * 64];
        }
        float y[2][4][V];
        float sc[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint16_t ce[4] = {cc[h].x, cc[h].y, cc[h].z, cc[h].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ld_vec<V>(Y + rowoff(ce[e]), y[h][e]);
                if constexpr (CS) sc[h][e] = scl(ce[e]);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float ve[4] = {v[h].x, v[h].y, v[h].z, v[h].w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    double xv = (double)y[h][e][j];
                    if constexpr (CS) xv *= (double)sc[h][e];
                    acc[j] = fma((double)ve[e], xv, acc[j]);
                }
        }
    }
    if (k < len) {
        const float4 v1 = Quad<FMT>::ld(val, q + k * 64);
        const u16x4 c1 = col[q + k * 64];
        const uint16_t ce[4] = {c1.x, c1.y, c1.z, c1.w};
        const float ve[4] = {v1.x, v1.y, v1.z, v1.w};
        float y[4][V];
#pragma unroll
        for (int e = 0; e < 4; ++e) ld_vec<V>(Y + rowoff(ce[e]), y[e]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double s = CS ? (double)scl(ce[e]) : 1.0;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                double xv = (double)y[e][j];
                if constexpr (CS) xv *= s;
                acc[j] = fma((double)ve[e], xv, acc[j]);
            }
        }
    }
}

// The same sums with the row's quads loaded once per row instead of once per
// lane: lane `sub` of the row's LPR lanes loads quad k0 + sub (chunks of LPR
// quads), and quad k0 + K reaches every lane of the row by a DPP broadcast
// inside the 16-lane DPP rows (LPR 16: row_newbcast; LPR 8: two half-row
// broadcasts under bank masks; LPR 4: quad_perm).  The raw value bits travel
// (4, 2 or 1 dwords per quad) and are decoded after the broadcast.  Every
// lane of a wave runs the same number of quads (rows of one slice share its
// length), so no source lane is ever inactive.  Same sums, same order, same
// bits as row_sums.
template <int FMT>
struct QuadBits {
    static constexpr int ND = FMT == FMT_F32 ? 4 : (FMT == FMT_FP8 ? 1 : 2);
    uint32_t d[ND];
    __device__ __forceinline__ void load(const void* base, int64_t q) {
        if constexpr (ND == 4) {
            const uint4 u = reinterpret_cast<const uint4*>(base)[q];
            d[0] = u.x; d[1] = u.y; d[2] = u.z; d[3] = u.w;
        } else if constexpr (ND == 2) {
            const u32x2 u = reinterpret_cast<const u32x2*>(base)[q];
            d[0] = u.x; d[1] = u.y;
        } else {
            d[0] = reinterpret_cast<const uint32_t*>(base)[q];
        }
    }
    __device__ __forceinline__ float4 dec() const {
        if constexpr (ND == 4) {
            return make_float4(__uint_as_float(d[0]), __uint_as_float(d[1]), __uint_as_float(d[2]),
                               __uint_as_float(d[3]));
        } else if constexpr (ND == 2) {
            u32x2 u;
            u.x = d[0];
            u.y = d[1];
            return Quad<FMT>::dec(u);
        } else {
            return Quad<FMT>::dec(d[0]);
        }
    }
};

template <int LPR, int K>
__device__ __forceinline__ uint32_t row_bcast(uint32_t v) {
    static_assert(K < LPR, "source lane outside the row");
    if constexpr (LPR == 16) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + K, 0xF, 0xF, false);
    } else if constexpr (LPR == 8) {
        const int a = __builtin_amdgcn_update_dpp(0, (int)v, 0x150 + K, 0xF, 0x3, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(a, (int)v, 0x158 + K, 0xF, 0xC, false);
    } else {
        static_assert(LPR == 4, "broadcast widths 4, 8 and 16");
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, K * 0x55, 0xF, 0xF, false);
    }
}

// Quad K of the chunk: decoded values and the four column indices.
template <int FMT, int LPR, int K>
__device__ __forceinline__ void quad_from(const QuadBits<FMT>& vb, const uint32_t (&cb)[2], float (&ve)[4],
                                          uint16_t (&ce)[4]) {
    QuadBits<FMT> t;
#pragma unroll
    for (int w = 0; w < QuadBits<FMT>::ND; ++w) t.d[w] = row_bcast<LPR, K>(vb.d[w]);
    const float4 v = t.dec();
    ve[0] = v.x; ve[1] = v.y; ve[2] = v.z; ve[3] = v.w;
    const uint32_t c0 = row_bcast<LPR, K>(cb[0]), c1 = row_bcast<LPR, K>(cb[1]);
    ce[0] = (uint16_t)(c0 & 0xFFFFu); ce[1] = (uint16_t)(c0 >> 16);
    ce[2] = (uint16_t)(c1 & 0xFFFFu); ce[3] = (uint16_t)(c1 >> 16);
}

template <int FMT, int V, int LPR, bool CS, int K, class ROW, class SCL>
__device__ __forceinline__ void chunk_sums(uint32_t n, const QuadBits<FMT>& vb, const uint32_t (&cb)[2],
                                           const float* __restrict__ Y, ROW rowoff, SCL scl, double (&acc)[V]) {
    if constexpr (K < LPR) {
        if (K + 1 < n) {
            float ve[2][4];
            uint16_t ce[2][4];
            quad_from<FMT, LPR, K>(vb, cb, ve[0], ce[0]);
            quad_from<FMT, LPR, K + 1>(vb, cb, ve[1], ce[1]);
            float y[2][4][V];
            float sc[2][4];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ld_vec<V>(Y + rowoff(ce[h][e]), y[h][e]);
                    if constexpr (CS) sc[h][e] = scl(ce[h][e]);
                }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        double xv = (double)y[h][e][j];
                        if constexpr (CS) xv *= (double)sc[h][e];
                        acc[j] = fma((double)ve[h][e], xv, acc[j]);
                    }
            chunk_sums<FMT, V, LPR, CS, K + 2>(n, vb, cb, Y, rowoff, scl, acc);
        } else if (K < n) {
            float ve[4];
            uint16_t ce[4];
            quad_from<FMT, LPR, K>(vb, cb, ve, ce);
            float y[4][V];
#pragma unroll
            for (int e = 0; e < 4; ++e) ld_vec<V>(Y + rowoff(ce[e]), y[e]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double s = CS ? (double)scl(ce[e]) : 1.0;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    double xv = (double)y[e][j];
                    if constexpr (CS) xv *= s;
                    acc[j] = fma((double)ve[e], xv, acc[j]);
                }
            }
        }
    }
}

template <int FMT, int V, int LPR, bool CS, class ROW, class SCL>
__device__ __forceinline__ void row_sums_bc(uint32_t q, uint32_t len, int sub, const u16x4* __restrict__ col,
                                            const void* __restrict__ val, const float* __restrict__ Y,
                                            ROW rowoff, SCL scl, double (&acc)[V]) {
    if (len == 0) return;
    // the next chunk's quads are loaded while this chunk is summed (past the
    // row's end the lanes load its last quad again)
    QuadBits<FMT> vb;
    u32x2 cw;
    {
        const int64_t kq = (int64_t)q + (int64_t)min((uint32_t)sub, len - 1) * 64;
        vb.load(val, kq);
        cw = reinterpret_cast<const u32x2*>(col)[kq];
    }
    for (uint32_t k0 = 0; k0 < len; k0 += LPR) {
        const int64_t kn = (int64_t)q + (int64_t)min(k0 + LPR + (uint32_t)sub, len - 1) * 64;
        QuadBits<FMT> vn;
        vn.load(val, kn);
        const u32x2 cn = reinterpret_cast<const u32x2*>(col)[kn];
        const uint32_t cb[2] = {cw.x, cw.y};
        chunk_sums<FMT, V, LPR, CS, 0>(min(len - k0, (uint32_t)LPR), vb, cb, Y, rowoff, scl, acc);
        vb = vn;
        cw = cn;
    }
}

// The forward takes its quads through the broadcasts (11-19% faster at 64
// right-hand sides on the prostate and head-and-neck cases, every format;
// loading the next chunk during the sums took another 8% on the prostate and
// 16% on the head-and-neck FP32 forward).
// The adjoint keeps the per-lane loads: its tuned variants hold eight
// right-hand sides per lane, and the broadcast chunk's registers cost it a
// wave per SIMD (slower in every format measured).
template <int LPR>
constexpr bool use_bcast() {
    return LPR == 4 || LPR == 8 || LPR == 16;
}

constexpr int BFWD_THREADS = 256;

// Forward Z = D^T X on the sliced voxel rows.  The block's beamlet list is
// staged in LDS as element offsets of the beamlets' rows of X (beamlet * B),
// with the FP8 column scales beside them; entries past the list's end read as
// beamlet 0 (padding quads).
template <int FMT, int LPR, int V>
__global__ __launch_bounds__(BFWD_THREADS) void k_bfwd(XcdRanges xr, const uint32_t* __restrict__ bptr,
                                                      const uint32_t* __restrict__ bsl,
                                                      const uint32_t* __restrict__ loff,
                                                      const uint32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ s_off,
                                                      const uint32_t* __restrict__ s_len,
                                                      const uint32_t* __restrict__ s_row,
                                                      const u16x4* __restrict__ s_col, const void* __restrict__ s_val,
                                                      const float* __restrict__ cscale, int B,
                                                      const float* __restrict__ X, double* __restrict__ Z) {
    constexpr int RPW = 64 / LPR, TB = LPR * V, UPS = LPR;  // units (row groups) per slice
    constexpr int WAVES = BFWD_THREADS / 64;
    constexpr bool CS = FMT == FMT_FP8;
    __shared__ uint32_t ls[TILE_LIST];
    __shared__ float lsc[CS ? TILE_LIST : 1];
    const int xcd = blockIdx.x & 7, wl = blockIdx.x >> 3, G = gridDim.x >> 3;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rg = lane / LPR, sub = lane % LPR;
    for (int b = xr.b[xcd]; b < xr.b[xcd + 1]; ++b) {
        const uint32_t l0 = loff[b], ln = loff[b + 1] - l0;
        __syncthreads();
        for (uint32_t u = threadIdx.x; u < TILE_LIST; u += BFWD_THREADS) {
            const uint32_t i = u < ln ? list[l0 + u] : 0u;
            ls[u] = i * (uint32_t)B;
            if constexpr (CS) lsc[u] = cscale[i];
        }
        __syncthreads();
        const uint32_t s0 = bptr[b], nunits = (bptr[b + 1] - s0) * UPS;
        for (int b0 = 0; b0 < B; b0 += TB) {
            const int c = min(b0 + sub * V, B - V);
            auto rowoff = [&](uint32_t c16) { return ls[c16] + (uint32_t)c; };
            auto scl = [&](uint32_t c16) { return CS ? lsc[c16] : 1.0f; };
            for (uint32_t unit = (uint32_t)wl * WAVES + wave; unit < nunits; unit += (uint32_t)G * WAVES) {
                const uint32_t sl = bsl[s0 + unit / UPS];
                const uint32_t r = (unit % UPS) * RPW + rg;
                const uint32_t row = s_row[(int64_t)sl * 64 + r];
                double acc[V];
#pragma unroll
                for (int j = 0; j < V; ++j) acc[j] = 0.0;
                if constexpr (use_bcast<LPR>())
                    row_sums_bc<FMT, V, LPR, CS>(s_off[sl] + r, s_len[sl], sub, s_col, s_val, X, rowoff, scl, acc);
                else
                    row_sums<FMT, V, CS>(s_off[sl] + r, s_len[sl], s_col, s_val, X, rowoff, scl, acc);
                if (row != 0xFFFFFFFFu && b0 + sub * V < B)
#pragma unroll
                    for (int j = 0; j < V; ++j) Z[(int64_t)row * B + c + j] = acc[j];
            }
        }
    }
}

// One row per wave, one right-hand side per lane (TB = 64, RPW = 1): the row
// is the same for every lane, so its quads of D (and, in the forward, the
// beamlets they name) come through scalar loads, and each gather is one
// coalesced 256-byte row of the right-hand sides: a uniform row pointer
// indexed by the lane.  The FP8 column scale folds into the uniform value:
// fma(d * s, x, acc) rounds the same exact product d * s * x as
// fma(d, x * s, acc).  ROWP(c16): the uniform pointer to the gathered row.
template <int FMT, bool CS, class ROWP, class SCL>
__device__ __forceinline__ double row_sum_w(uint32_t q, uint32_t len, const u16x4* __restrict__ col,
                                            const void* __restrict__ val, int lane, ROWP rowp, SCL scl) {
    double acc = 0.0;
    uint32_t k = 0;
    for (; k + 2 <= len; k += 2) {
        float4 v[2];
        u16x4 cc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            v[h] = Quad<FMT>::ld(val, q + (k + h) * 64);
            cc[h] = col[q + (k + h) * 64];
        }
        float y[8];
        double d[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint16_t ce[4] = {cc[h].x, cc[h].y, cc[h].z, cc[h].w};
            const float ve[4] = {v[h].x, v[h].y, v[h].z, v[h].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                y[4 * h + e] = rowp(ce[e])[lane];
                d[4 * h + e] = CS ? (double)ve[e] * (double)scl(ce[e]) : (double)ve[e];
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) acc = fma(d[e], (double)y[e], acc);
    }
    if (k < len) {
        const float4 v1 = Quad<FMT>::ld(val, q + k * 64);
        const u16x4 c1 = col[q + k * 64];
        const uint16_t ce[4] = {c1.x, c1.y, c1.z, c1.w};
        const float ve[4] = {v1.x, v1.y, v1.z, v1.w};
        float y[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) y[e] = rowp(ce[e])[lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double dv = CS ? (double)ve[e] * (double)scl(ce[e]) : (double)ve[e];
            acc = fma(dv, (double)y[e], acc);
        }
    }
    return acc;
}

// The uniform wave index (every value derived from it stays scalar).
__device__ __forceinline__ uint32_t wave_id() {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

template <int FMT>
__global__ __launch_bounds__(SPMM_THREADS) void k_bfwd_w(XcdRanges xr, const uint32_t* __restrict__ bptr,
                                                        const uint32_t* __restrict__ bsl,
                                                        const uint32_t* __restrict__ loff,
                                                        const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ s_off,
                                                        const uint32_t* __restrict__ s_len,
                                                        const uint32_t* __restrict__ s_row,
                                                        const u16x4* __restrict__ s_col,
                                                        const void* __restrict__ s_val,
                                                        const float* __restrict__ cscale, int B,
                                                        const float* __restrict__ X, double* __restrict__ Z) {
    constexpr int WAVES = SPMM_THREADS / 64;
    constexpr bool CS = FMT == FMT_FP8;
    const int xcd = blockIdx.x & 7, wl = blockIdx.x >> 3, G = gridDim.x >> 3;
    const uint32_t wave = wave_id();
    const int lane = (int)(threadIdx.x & 63);
    const int cl = min(lane, B - 1);
    for (int b = xr.b[xcd]; b < xr.b[xcd + 1]; ++b) {
        const uint32_t* __restrict__ lb = list + loff[b];
        auto rowp = [&](uint32_t c16) { return X + (size_t)(lb[c16] * (uint32_t)B); };
        auto scl = [&](uint32_t c16) { return CS ? cscale[lb[c16]] : 1.0f; };
        const uint32_t s0 = bptr[b], nunits = (bptr[b + 1] - s0) * 64;
        for (uint32_t unit = (uint32_t)wl * WAVES + wave; unit < nunits; unit += (uint32_t)G * WAVES) {
            const uint32_t sl = bsl[s0 + unit / 64];
            const uint32_t r = unit % 64;
            const uint32_t row = s_row[(int64_t)sl * 64 + r];
            const double acc = row_sum_w<FMT, CS>(s_off[sl] + r, s_len[sl], s_col, s_val, cl, rowp, scl);
            if (row != 0xFFFFFFFFu && lane < B) Z[(int64_t)row * B + lane] = acc;
        }
    }
}

template <int FMT>
__global__ __launch_bounds__(SPMM_THREADS) void k_badj_w(XcdRanges xr, const uint32_t* __restrict__ bptr,
                                                        const uint32_t* __restrict__ bsl,
                                                        const int32_t* __restrict__ bounds,
                                                        const uint32_t* __restrict__ s_off,
                                                        const uint32_t* __restrict__ s_len,
                                                        const uint32_t* __restrict__ s_row,
                                                        const u16x4* __restrict__ s_col,
                                                        const void* __restrict__ s_val, int B,
                                                        const float* __restrict__ W, double* __restrict__ part) {
    constexpr int WAVES = SPMM_THREADS / 64;
    const int xcd = blockIdx.x & 7, wl = blockIdx.x >> 3, G = gridDim.x >> 3;
    const uint32_t wave = wave_id();
    const int lane = (int)(threadIdx.x & 63);
    const int cl = min(lane, B - 1);
    for (int b = xr.b[xcd]; b < xr.b[xcd + 1]; ++b) {
        const float* __restrict__ Wb = W + (int64_t)bounds[b] * B;
        auto rowp = [&](uint32_t c16) { return Wb + (size_t)(c16 * (uint32_t)B); };
        auto scl = [](uint32_t) { return 1.0f; };
        const uint32_t s0 = bptr[b], nunits = (bptr[b + 1] - s0) * 64;
        for (uint32_t unit = (uint32_t)wl * WAVES + wave; unit < nunits; unit += (uint32_t)G * WAVES) {
            const uint32_t sl = bsl[s0 + unit / 64];
            const uint32_t r = unit % 64;
            const uint32_t row = s_row[(int64_t)sl * 64 + r];
            const double acc = row_sum_w<FMT, false>(s_off[sl] + r, s_len[sl], s_col, s_val, cl, rowp, scl);
            if (row != 0xFFFFFFFFu && lane < B) part[(int64_t)row * B + lane] = acc;
        }
    }
}

// Adjoint slot sums part[slot][b] = sum over the slot row's entries of
// D * W[voxel][b], on the sliced slot rows (16-bit voxel offsets from the
// block's first voxel); k_spmm_adj_reduce then sums each beamlet's slots.
template <int FMT, int LPR, int V>
__global__ __launch_bounds__(SPMM_THREADS) void k_badj(XcdRanges xr, const uint32_t* __restrict__ bptr,
                                                      const uint32_t* __restrict__ bsl,
                                                      const int32_t* __restrict__ bounds,
                                                      const uint32_t* __restrict__ s_off,
                                                      const uint32_t* __restrict__ s_len,
                                                      const uint32_t* __restrict__ s_row,
                                                      const u16x4* __restrict__ s_col, const void* __restrict__ s_val,
                                                      int B, const float* __restrict__ W, double* __restrict__ part) {
    constexpr int RPW = 64 / LPR, TB = LPR * V, UPS = LPR;
    constexpr int WAVES = SPMM_THREADS / 64;
    const int xcd = blockIdx.x & 7, wl = blockIdx.x >> 3, G = gridDim.x >> 3;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rg = lane / LPR, sub = lane % LPR;
    for (int b = xr.b[xcd]; b < xr.b[xcd + 1]; ++b) {
        const float* __restrict__ Wb = W + (int64_t)bounds[b] * B;
        const uint32_t s0 = bptr[b], nunits = (bptr[b + 1] - s0) * UPS;
        for (int b0 = 0; b0 < B; b0 += TB) {
            const int c = min(b0 + sub * V, B - V);
            auto rowoff = [&](uint32_t c16) { return c16 * (uint32_t)B + (uint32_t)c; };
            auto scl = [](uint32_t) { return 1.0f; };
            for (uint32_t unit = (uint32_t)wl * WAVES + wave; unit < nunits; unit += (uint32_t)G * WAVES) {
                const uint32_t sl = bsl[s0 + unit / UPS];
                const uint32_t r = (unit % UPS) * RPW + rg;
                const uint32_t row = s_row[(int64_t)sl * 64 + r];
                double acc[V];
#pragma unroll
                for (int j = 0; j < V; ++j) acc[j] = 0.0;
                row_sums<FMT, V, false>(s_off[sl] + r, s_len[sl], s_col, s_val, Wb, rowoff, scl, acc);
                if (row != 0xFFFFFFFFu && b0 + sub * V < B)
#pragma unroll
                    for (int j = 0; j < V; ++j) part[(int64_t)row * B + c + j] = acc[j];
            }
        }
    }
}

// ---- plain layout (quad CSR with 32-bit indices): the untileable fallback,
// and the adjoint of a handle without the batched state's slot sums

// TB lanes of a wave share a row (its index and value loads are broadcasts)
// and gather TB consecutive right-hand sides per non-zero; 64/TB rows go
// through a wave at once.
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

// G[i][b] = scale_i * sum of beamlet i's slot sums (block order).
__global__ __launch_bounds__(256) void k_spmm_adj_reduce(int64_t nb, int B, const uint32_t* __restrict__ red_ptr,
                                                         const uint32_t* __restrict__ red_slot,
                                                         const double* __restrict__ part,
                                                         const float* __restrict__ scale, double* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nb * B) return;
    const int64_t i = e / B;
    const int b = (int)(e - i * B);
    const double s = slot_sum(red_ptr[i], red_ptr[i + 1], red_slot, part, B, b);
    G[e] = scale ? s * (double)scale[i] : s;
}

// The product variants: TB right-hand sides per pass over a row and RPW rows
// per wave (LPR = 64 / RPW lanes per row, V = TB / LPR per lane).  The tiled
// layout runs every listed pair; the plain layout runs k_spmm_rows<TB>
// (RPW = 64 / TB) whatever RPW is asked.
struct SpmmCfg {
    int tb, rpw;
};
static const SpmmCfg kCfgs[] = {{1, 64}, {2, 32}, {4, 16}, {8, 8},  {16, 4}, {16, 8}, {32, 2},
                                {32, 4}, {32, 8}, {64, 1}, {64, 2}, {64, 4}, {64, 8}};
constexpr int N_CFGS = sizeof(kCfgs) / sizeof(kCfgs[0]);

static bool cfg_known(int tb, int rpw) {
    for (const SpmmCfg& c : kCfgs)
        if (c.tb == tb && c.rpw == rpw) return true;
    return false;
}

// Untuned: one pass over all right-hand sides (the smallest width >= B),
// four rows per wave where the width allows.
static SpmmCfg default_cfg(int B) {
    int t = 1;
    while (t < B && t < 64) t <<= 1;
    return SpmmCfg{t, std::max(4, 64 / t)};
}

// Persistent grids: as many workgroups as can be resident at once (the
// occupancy of the kernel, on the 32 compute units of each XCD), a multiple
// of 8 so that the workgroups with one value of w % 8 are one XCD's.
template <class K>
static unsigned resident_grid(K kernel, int threads) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount >= 8)
            cus = prop.multiProcessorCount;
    }
    return (unsigned)(cus / 8 * 8 * per_cu);
}

template <int FMT, int LPR, int V>
static void tiled_fwd(const vmat_ctx* h, int B, const float* X, double* Z, hipStream_t st) {
    const Tiled& t = h->tl;
    XcdRanges xr;
    for (int i = 0; i < 9; ++i) xr.b[i] = t.fx[i];
    static const unsigned grid = resident_grid(k_bfwd<FMT, LPR, V>, BFWD_THREADS);
    k_bfwd<FMT, LPR, V><<<grid, BFWD_THREADS, 0, st>>>(
        xr, t.fb_ptr, t.fb_sl, t.loff, t.list, t.s_off, t.s_len, t.s_row, reinterpret_cast<const u16x4*>(t.s_col),
        t.s_val, h->bm.scale, B, X, Z);
}

template <int FMT, int LPR, int V>
static void tiled_adj(const vmat_ctx* h, int B, const float* W, double* part, hipStream_t st) {
    const Tiled& t = h->tl;
    XcdRanges xr;
    for (int i = 0; i < 9; ++i) xr.b[i] = t.ax[i];
    static const unsigned grid = resident_grid(k_badj<FMT, LPR, V>, SPMM_THREADS);
    k_badj<FMT, LPR, V><<<grid, SPMM_THREADS, 0, st>>>(
        xr, t.ab_ptr, t.ab_sl, t.bounds, t.as_off, t.as_len, t.as_row, reinterpret_cast<const u16x4*>(t.as_col),
        t.as_val, B, W, part);
}

template <int FMT>
static void tiled_dispatch(const vmat_ctx* h, bool fwd, SpmmCfg c, int B, const float* in, double* out,
                           hipStream_t st) {
    const int lpr = 64 / c.rpw, v = c.tb / lpr;
    if (c.tb == 64 && c.rpw == 1) {
        const Tiled& t = h->tl;
        XcdRanges xr;
        if (fwd) {
            for (int i = 0; i < 9; ++i) xr.b[i] = t.fx[i];
            static const unsigned grid = resident_grid(k_bfwd_w<FMT>, SPMM_THREADS);
            k_bfwd_w<FMT><<<grid, SPMM_THREADS, 0, st>>>(xr, t.fb_ptr, t.fb_sl, t.loff, t.list, t.s_off, t.s_len,
                                                       t.s_row, reinterpret_cast<const u16x4*>(t.s_col), t.s_val,
                                                       h->bm.scale, B, in, out);
        } else {
            for (int i = 0; i < 9; ++i) xr.b[i] = t.ax[i];
            static const unsigned grid = resident_grid(k_badj_w<FMT>, SPMM_THREADS);
            k_badj_w<FMT><<<grid, SPMM_THREADS, 0, st>>>(xr, t.ab_ptr, t.ab_sl, t.bounds, t.as_off, t.as_len,
                                                       t.as_row, reinterpret_cast<const u16x4*>(t.as_col), t.as_val,
                                                       B, in, out);
        }
        return;
    }
#define CASE(L, VV)                                                     \
    if (lpr == L && v == VV) {                                          \
        if (fwd) tiled_fwd<FMT, L, VV>(h, B, in, out, st);              \
        else tiled_adj<FMT, L, VV>(h, B, in, out, st);                  \
        return;                                                         \
    }
    CASE(1, 1) CASE(2, 1) CASE(4, 1) CASE(8, 1) CASE(16, 1) CASE(8, 2) CASE(32, 1) CASE(16, 2) CASE(8, 4)
    CASE(32, 2) CASE(16, 4) CASE(8, 8)
#undef CASE
}

template <int FMT>
static void plain_dispatch(const vmat_ctx* h, bool fwd, int TB, int B, const float* in, double* out,
                           hipStream_t st) {
    const unsigned tiles = (unsigned)((B + TB - 1) / TB);
    const int64_t nrows = fwd ? h->nv : h->nb;
    const QuadCsr& A = fwd ? h->vm : h->bm;
    const float* cs = fwd && FMT == FMT_FP8 ? h->bm.scale : nullptr;
    const float* rs = fwd ? nullptr : h->bm.scale;
    const int64_t rows_per_block = (SPMM_THREADS / 64) * (64 / TB);
    const dim3 grid((unsigned)((nrows + rows_per_block - 1) / rows_per_block), tiles);
#define CASE(T) \
    case T: k_spmm_rows<FMT, T><<<grid, SPMM_THREADS, 0, st>>>(A.qptr, A.col, A.val, cs, rs, nrows, B, in, out); break;
    switch (TB) { CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) default : CASE(64) }
#undef CASE
}

// Whether the adjoint runs on the tiled slot rows (their sums need the
// batched state's buffer of S x B doubles, sized by vmat_reserve_batched).
static bool tiled_adj_ready(const vmat_ctx* h, int B) {
    const BatchState* bs = h->bs;
    return h->tl.on && bs && bs->spart && B <= bs->cap;
}

static vmat_status launch_spmm(const vmat_ctx* h, bool fwd, int B, const float* X, double* Z, hipStream_t st,
                               SpmmCfg c = SpmmCfg{0, 0}) {
    if (c.tb <= 0) {
        const int32_t packed = (fwd ? h->tune_fwd : h->tune_adj)[B];
        c = packed > 0 ? SpmmCfg{packed & 0xFF, packed >> 8} : default_cfg(B);
    }
    // V must divide B, and the gathered rows must be aligned for V-wide loads
    // (vector gathers stay inside each row of the RHS block): else V = 1
    const int v = c.tb / (64 / c.rpw);
    if (B % v != 0 || ((uintptr_t)X & (uintptr_t)(4 * v - 1)) != 0) c.rpw = 64 / c.tb;
    const bool tiled = h->tl.on && (fwd || tiled_adj_ready(h, B));
    if (tiled) {
        if (h->nb * B >= ((int64_t)1 << 32))
            return fail(VMAT_ERR_UNSUPPORTED, "beamlets x right-hand sides exceed 2^32 elements");
        double* out = fwd ? Z : h->bs->spart;
        switch (h->d_store) {
            case VMAT_F32: tiled_dispatch<FMT_F32>(h, fwd, c, B, X, out, st); break;
            case VMAT_F16: tiled_dispatch<FMT_F16>(h, fwd, c, B, X, out, st); break;
            case VMAT_BF16: tiled_dispatch<FMT_BF16>(h, fwd, c, B, X, out, st); break;
            default: tiled_dispatch<FMT_FP8>(h, fwd, c, B, X, out, st); break;
        }
        VMAT_LAUNCH_CHECK();
        if (!fwd) {
            const Tiled& t = h->tl;
            k_spmm_adj_reduce<<<(unsigned)((h->nb * B + 255) / 256), 256, 0, st>>>(h->nb, B, t.red_ptr, t.red_slot,
                                                                                   h->bs->spart, h->bm.scale, Z);
            VMAT_LAUNCH_CHECK();
        }
        return VMAT_OK;
    }
    if (fwd && !h->vm.col) return fail(VMAT_ERR_DEVICE, "no voxel-major copy for the plain batched forward");
    switch (h->d_store) {
        case VMAT_F32: plain_dispatch<FMT_F32>(h, fwd, c.tb, B, X, Z, st); break;
        case VMAT_F16: plain_dispatch<FMT_F16>(h, fwd, c.tb, B, X, Z, st); break;
        case VMAT_BF16: plain_dispatch<FMT_BF16>(h, fwd, c.tb, B, X, Z, st); break;
        default: plain_dispatch<FMT_FP8>(h, fwd, c.tb, B, X, Z, st); break;
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
    return launch_spmm(h, true, B, X, Z, st);
}

extern "C" vmat_status vmat_adjoint_batched(vmat_handle h, int32_t B, const float* W, double* G, hipStream_t st) {
    vmat_status rc = check_batch(h, B);
    if (rc != VMAT_OK) return rc;
    if (!W || !G) return fail(VMAT_ERR_INVALID_ARG, "null W or G");
    return launch_spmm(h, false, B, W, G, st);
}

extern "C" vmat_status vmat_grad_batched(vmat_handle h, int32_t B, int32_t n_struct, const uint8_t* label,
                                         const float* table, const float* X, double* Z, double* cost, float* dF,
                                         double* G, hipStream_t st) {
    vmat_status rc = check_batch(h, B);
    if (rc != VMAT_OK) return rc;
    if (n_struct < 1 || n_struct > 16) return fail(VMAT_ERR_INVALID_ARG, "n_struct must be in [1, 16]");
    if (!label || !table || !X || !Z || !cost || !dF)
        return fail(VMAT_ERR_INVALID_ARG, "null argument");
    if ((rc = launch_spmm(h, true, B, X, Z, st)) != VMAT_OK) return rc;
    k_pen_batched<<<h->n_part, 256, 0, st>>>(h->nv, B, n_struct, label, table, Z, dF, h->part_b);
    VMAT_LAUNCH_CHECK();
    k_pen_batched_sum<<<1, 64, 0, st>>>(B, h->n_part, h->part_b, cost);
    VMAT_LAUNCH_CHECK();
    if (G) return launch_spmm(h, false, B, dF, G, st);
    return VMAT_OK;
}

// Times each product variant (tile width x rows per wave) for both products
// at B right-hand sides on the caller's buffers and keeps the fastest for
// later batched calls.
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
    SpmmCfg bc[2] = {default_cfg(B), default_cfg(B)};
    float bms[2] = {INFINITY, INFINITY};
    int idx = 0;
    for (int dir = 0; dir < 2; ++dir) {
        for (const SpmmCfg& c : kCfgs) {
            float ms = INFINITY;
            const int v = c.tb / (64 / c.rpw);
            const bool plain_dup = !h->tl.on && c.rpw != 64 / c.tb;  // the plain layout ignores rpw
            if (c.tb < 2 * B && B % v == 0 && !plain_dup) {
                const bool fwd = dir == 0;
                const float* in = fwd ? X : W;
                double* out = fwd ? Z : G;
                if ((rc = launch_spmm(h, fwd, B, in, out, st, c)) != VMAT_OK) return rc;
                VMAT_HIP(hipEventRecord(ev.e[0], st));
                for (int k = 0; k < reps; ++k)
                    if ((rc = launch_spmm(h, fwd, B, in, out, st, c)) != VMAT_OK) return rc;
                VMAT_HIP(hipEventRecord(ev.e[1], st));
                VMAT_HIP(hipEventSynchronize(ev.e[1]));
                VMAT_HIP(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
                ms /= (float)reps;
                if (ms < bms[dir]) {
                    bms[dir] = ms;
                    bc[dir] = c;
                }
            }
            if (times_ms) times_ms[idx] = ms;
            ++idx;
        }
    }
    h->tune_fwd[B] = bc[0].tb | (bc[0].rpw << 8);
    h->tune_adj[B] = bc[1].tb | (bc[1].rpw << 8);
    if (best) {
        best[0] = bc[0].tb;
        best[1] = bc[0].rpw;
        best[2] = bc[1].tb;
        best[3] = bc[1].rpw;
    }
    return VMAT_OK;
}

extern "C" vmat_status vmat_set_batched_tile(vmat_handle h, int32_t B, int32_t fwd_tile, int32_t fwd_rpw,
                                             int32_t adj_tile, int32_t adj_rpw) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    if (B < 1 || B > 64) return fail(VMAT_ERR_INVALID_ARG, "the number of right-hand sides must be in [1, 64]");
    auto ok = [](int t, int r) { return (t == 0 && r == 0) || cfg_known(t, r); };
    if (!ok(fwd_tile, fwd_rpw) || !ok(adj_tile, adj_rpw))
        return fail(VMAT_ERR_INVALID_ARG, "unknown (tile width, rows per wave) pair");
    h->tune_fwd[B] = fwd_tile | (fwd_rpw << 8);
    h->tune_adj[B] = adj_tile | (adj_rpw << 8);
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
        BTRY(launch_spmm(h, true, B, bs.X, bs.dZ, s));
        return ls_round(s);
    };
    auto step = [&](hipStream_t s) -> vmat_status {
        k_bmaster_step<<<B, CTRL, 0, s>>>(m);
        VMAT_LAUNCH_CHECK();
        k_bupdate<<<np, BT, 0, s>>>(h->nv, B, a.S, a.label, a.table, bs.Z, bs.dZ, bs.ms, bs.RZ, bs.pf);
        VMAT_LAUNCH_CHECK();
        BTRY(launch_spmm(h, false, B, bs.RZ, bs.G, s));
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
    BTRY(launch_spmm(h, false, B, bs.RZ, bs.G, st));
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
