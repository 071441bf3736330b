// Row loops shared by the tiled kernels (header-only device templates).
//
// A work item is (block, rows [r0, r1)) with at most TILE_ROWS rows.  Its row
// starts are staged in LDS with the gathered values, so no global load sits
// between one row and the next.  G lanes share a row; each lane issues the
// loads of up to U quads of a row at once, and the loads of the group's next
// row are issued before the current row is summed (two rows in flight per
// lane group).  Longer rows finish in extra passes.
#pragma once

#include <hip/hip_runtime.h>

#include "vmat_formats.h"
#include "vmat_internal.h"

namespace vmat {

typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

struct StoreRow {
    double* out;
    __device__ __forceinline__ void operator()(int row, double acc) const { out[row] = acc; }
};

template <int FMT, int U>
struct RowBuf {
    float4 v[U];
    u16x4 c[U];
};

template <int FMT, int G, int U>
__device__ __forceinline__ void load_pass(RowBuf<FMT, U>& b, const void* __restrict__ val, const u16x4* __restrict__ c4,
                                          uint32_t q, uint32_t q1) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t qq = q + (uint32_t)(u * G);
        if (qq < q1) {
            b.v[u] = Quad<FMT>::load(val, qq);
            b.c[u] = __builtin_nontemporal_load(c4 + qq);
        } else {
            b.v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            b.c[u] = u16x4{0, 0, 0, 0};
        }
    }
}

template <int FMT, int U, typename ST>
__device__ __forceinline__ double use_pass(const RowBuf<FMT, U>& b, const ST* __restrict__ xs, double acc) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        acc = fma((double)b.v[u].x, (double)xs[b.c[u].x], acc);
        acc = fma((double)b.v[u].y, (double)xs[b.c[u].y], acc);
        acc = fma((double)b.v[u].z, (double)xs[b.c[u].z], acc);
        acc = fma((double)b.v[u].w, (double)xs[b.c[u].w], acc);
    }
    return acc;
}

// Rows of one work item: rq[k] = start quad of row r0 + k (k <= nrows).
template <int FMT, int G, int U, typename ST, typename EPI>
__device__ __forceinline__ void rows_of_item(const uint32_t* __restrict__ rq, int nrows, int row_base,
                                             const void* __restrict__ val, const u16x4* __restrict__ c4,
                                             const ST* __restrict__ xs, EPI& epi) {
    const int grp = threadIdx.x / G, lane = threadIdx.x & (G - 1);
    constexpr int NGRP = TILE_THREADS / G;
    int row = grp;
    RowBuf<FMT, U> cur, nxt;
    if (row < nrows) load_pass<FMT, G, U>(cur, val, c4, rq[row] + lane, rq[row + 1]);
    while (row < nrows) {
        const int next = row + NGRP;
        if (next < nrows) load_pass<FMT, G, U>(nxt, val, c4, rq[next] + lane, rq[next + 1]);
        double acc = use_pass<FMT, U>(cur, xs, 0.0);
        const uint32_t q1 = rq[row + 1];
        for (uint32_t q = rq[row] + lane + U * G; q < q1; q += U * G) {
            RowBuf<FMT, U> more;
            load_pass<FMT, G, U>(more, val, c4, q, q1);
            acc = use_pass<FMT, U>(more, xs, acc);
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (lane == 0) epi(row_base + row, acc);
        cur = nxt;
        row = next;
    }
}

// Row starts of a work item into LDS, all loads issued before the stores.
__device__ __forceinline__ void stage_rows(uint32_t* __restrict__ rq, const uint32_t* __restrict__ src, int nrows) {
    constexpr int K = (TILE_ROWS + TILE_THREADS) / TILE_THREADS;
    uint32_t v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int u = threadIdx.x + k * TILE_THREADS;
        v[k] = u <= nrows ? src[u] : 0u;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int u = threadIdx.x + k * TILE_THREADS;
        if (u <= nrows) rq[u] = v[k];
    }
}

}  // namespace vmat
