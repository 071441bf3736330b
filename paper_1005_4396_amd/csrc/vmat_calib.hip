// Measurement aids: a plain streaming read of a device buffer, the practical
// HBM read ceiling of the part against which the product kernels' rates are
// read, and the same read with a given share of writes mixed in (the
// products write their outputs while they stream D).  Not steps of the
// method.
#include <hip/hip_runtime.h>

#include "vmat.h"
#include "vmat_internal.h"

namespace vmat {

typedef float f32x4r __attribute__((ext_vector_type(4)));

// Each lane reads 8 non-temporal 16-byte words a grid stride apart per step;
// one partial sum per block keeps the loads live.
__global__ __launch_bounds__(256) void k_read_stream(const f32x4r* __restrict__ a, int64_t n4,
                                                     float* __restrict__ out) {
    constexpr int U = 8;
    __shared__ float sh[4];
    float s = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += U * stride) {
        f32x4r v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = i + u * stride;
            v[u] = j < n4 ? __builtin_nontemporal_load(a + j) : f32x4r{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// As k_read_stream, and each wave also writes its share of nch chunks of
// wbuf (512 bytes: 64 lanes x 8), spread evenly over its read steps: wave w
// of W owns chunks w, w + W, ...; its k-th chunk is due once
// step >= k * steps / (its chunk count).  Chunks still due after the last
// step are written then, so exactly nch chunks are written.
__global__ __launch_bounds__(256) void k_read_write_stream(const f32x4r* __restrict__ a, int64_t n4,
                                                           double* __restrict__ wbuf, int64_t nch,
                                                           float* __restrict__ out) {
    constexpr int U = 8;
    __shared__ float sh[4];
    float s = 0.0f;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * 256, step = U * stride;
    const int64_t W = (int64_t)gridDim.x * 4, w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t n_w = w < nch ? (nch - w + W - 1) / W : 0;
    const int64_t i0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63);  // the wave's first lane
    const int64_t steps = i0 < n4 ? (n4 - i0 + step - 1) / step : 0;
    int64_t k = 0;
    for (int64_t t = 0; t < steps; ++t) {
        const int64_t i = i0 + lane + t * step;
        f32x4r v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = i + u * stride;
            v[u] = j < n4 ? __builtin_nontemporal_load(a + j) : f32x4r{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
        for (; k < n_w && k * steps <= t * n_w; ++k) wbuf[(w + k * W) * 64 + lane] = (double)s;
    }
    for (; k < n_w; ++k) wbuf[(w + k * W) * 64 + lane] = (double)s;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

}  // namespace vmat

extern "C" vmat_status vmat_read_write_stream(const void* buf, int64_t bytes, double* wbuf, int64_t wbytes,
                                              float* partials, int32_t grid, hipStream_t st) {
    if (!buf || !partials) return vmat::fail(VMAT_ERR_INVALID_ARG, "null buffer");
    if (bytes <= 0 || bytes % 16 != 0) return vmat::fail(VMAT_ERR_INVALID_ARG, "bytes must be a positive multiple of 16");
    if (wbytes < 0 || wbytes % 512 != 0) return vmat::fail(VMAT_ERR_INVALID_ARG, "wbytes must be a multiple of 512");
    if (wbytes > 0 && !wbuf) return vmat::fail(VMAT_ERR_INVALID_ARG, "null write buffer");
    if (grid < 1 || grid > 65536) return vmat::fail(VMAT_ERR_INVALID_ARG, "grid must be in [1, 65536]");
    vmat::k_read_write_stream<<<(unsigned)grid, 256, 0, st>>>(reinterpret_cast<const vmat::f32x4r*>(buf), bytes / 16,
                                                               wbuf, wbytes / 512, partials);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return vmat::fail(VMAT_ERR_DEVICE, hipGetErrorString(e));
    return VMAT_OK;
}

extern "C" vmat_status vmat_read_stream(const void* buf, int64_t bytes, float* partials, int32_t grid,
                                        hipStream_t st) {
    if (!buf || !partials) return vmat::fail(VMAT_ERR_INVALID_ARG, "null buffer");
    if (bytes <= 0 || bytes % 16 != 0) return vmat::fail(VMAT_ERR_INVALID_ARG, "bytes must be a positive multiple of 16");
    if (grid < 1 || grid > 65536) return vmat::fail(VMAT_ERR_INVALID_ARG, "grid must be in [1, 65536]");
    vmat::k_read_stream<<<(unsigned)grid, 256, 0, st>>>(reinterpret_cast<const vmat::f32x4r*>(buf), bytes / 16,
                                                         partials);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return vmat::fail(VMAT_ERR_DEVICE, hipGetErrorString(e));
    return VMAT_OK;
}
