// Handle construction: argument and data validation, the beamlet-major and
// voxel-major quad-CSR layouts of D (optionally in a reduced storage format),
// and the work buffers.  Runs once per problem; nothing here is on the
// optimisation path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "vmat_formats.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"

namespace vmat {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

vmat_status fail(vmat_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------------- validation

enum : int {
    BAD_ROWPTR = 1, BAD_COL = 2, BAD_ORDER = 4, BAD_VAL = 8, BAD_ALPHA = 16, BAD_BETA = 32, BAD_T = 64
};

__global__ void k_validate_rows(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const float* __restrict__ val, int64_t nb, int64_t nv, int64_t nnz,
                                int* __restrict__ flag) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= nb) return;
    const int64_t a = rp[row], b = rp[row + 1];
    int bad = 0;
    if (row == 0 && a != 0) bad |= BAD_ROWPTR;
    if (row == nb - 1 && b != nnz) bad |= BAD_ROWPTR;
    if (b < a || a < 0 || b > nnz) {
        if (lane == 0) atomicOr(flag, bad | BAD_ROWPTR);
        return;
    }
    for (int64_t p = a + lane; p < b; p += 64) {
        const int32_t c = col[p];
        const float v = val[p];
        if (c < 0 || (int64_t)c >= nv) bad |= BAD_COL;
        if (p + 1 < b && col[p + 1] <= c) bad |= BAD_ORDER;
        if (!(v >= 0.0f) || !isfinite(v)) bad |= BAD_VAL;
    }
    if (bad) atomicOr(flag, bad);
}

__global__ void k_validate_voxels(const float* __restrict__ alpha, const float* __restrict__ beta,
                                  const float* __restrict__ T, int64_t nv, float4* __restrict__ abT,
                                  int* __restrict__ flag) {
    int bad = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nv;
         j += (int64_t)gridDim.x * blockDim.x) {
        const float a = alpha[j], b = beta[j], t = T[j];
        if (!(a >= 0.0f) || !isfinite(a)) bad |= BAD_ALPHA;
        if (!(b >= 0.0f) || !isfinite(b)) bad |= BAD_BETA;
        if (!isfinite(t)) bad |= BAD_T;
        abT[j] = make_float4(a, b, t, 0.0f);
    }
    if (bad) atomicOr(flag, bad);
}

// ---------------------------------------------------------------- scan (exclusive, uint64)

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// in: n counts (uint32).  out[i] = sum_{k<i} in[k], out[n] = total.  Three passes.
__global__ void k_scan_tiles(const uint32_t* __restrict__ in, int64_t n, uint64_t* __restrict__ tile_sum) {
    __shared__ uint64_t sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        if (i < n) s += in[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = SCAN_BLOCK / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = sh[0];
}

__global__ void k_scan_tile_sums(uint64_t* __restrict__ tile_sum, int64_t ntiles) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t acc = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        const uint64_t v = tile_sum[t];
        tile_sum[t] = acc;
        acc += v;
    }
    tile_sum[ntiles] = acc;
}

__global__ void k_scan_apply(const uint32_t* __restrict__ in, int64_t n, const uint64_t* __restrict__ tile_off,
                             int64_t ntiles, uint32_t* __restrict__ out, int* __restrict__ overflow) {
    __shared__ uint64_t sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint64_t loc[SCAN_ITEMS];
    uint64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        loc[k] = s;
        if (i < n) s += in[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread sums
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        uint64_t v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    const uint64_t excl = sh[threadIdx.x] - s + tile_off[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        if (i < n) {
            const uint64_t v = excl + loc[k];
            if (v > 0xFFFFFFFFull) atomicOr(overflow, 1);
            out[i] = (uint32_t)v;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t tot = tile_off[ntiles];
        if (tot > 0xFFFFFFFFull) atomicOr(overflow, 1);
        out[n] = (uint32_t)tot;
    }
}

// ---------------------------------------------------------------- beamlet-major layout

__global__ void k_row_quads(const int64_t* __restrict__ rp, int64_t nb, uint32_t* __restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) q[i] = (uint32_t)((rp[i + 1] - rp[i] + 3) >> 2);
}

// One wave per beamlet row: row maximum (FP8 scale), then copy + encode.
template <int FMT>
__global__ void k_fill_bm(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const float* __restrict__ val, int64_t nb, const uint32_t* __restrict__ qptr,
                          int32_t* __restrict__ ocol, void* __restrict__ oval, float* __restrict__ oscale) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= nb) return;
    const int64_t a = rp[row], n = rp[row + 1] - a;
    const int64_t o = (int64_t)qptr[row] * 4, npad = (int64_t)(qptr[row + 1] - qptr[row]) * 4;
    float s = 1.0f;
    if (FMT == FMT_FP8) {
        float m = 0.0f;
        for (int64_t p = lane; p < n; p += 64) m = fmaxf(m, val[a + p]);
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        s = m > 0.0f ? m / 448.0f : 1.0f;
        if (lane == 0) oscale[row] = s;
    }
    const int32_t pad_col = n > 0 ? col[a] : 0;
    for (int64_t p = lane; p < npad; p += 64) {
        const bool real = p < n;
        const float v = real ? val[a + p] : 0.0f;
        ocol[o + p] = real ? col[a + p] : pad_col;
        if (FMT == FMT_F32) reinterpret_cast<float*>(oval)[o + p] = v;
        if (FMT == FMT_BF16) reinterpret_cast<uint16_t*>(oval)[o + p] = f32_to_bf16_rne(v);
        if (FMT == FMT_F16) reinterpret_cast<uint16_t*>(oval)[o + p] = f32_to_f16_rne(v);
        if (FMT == FMT_FP8) reinterpret_cast<uint8_t*>(oval)[o + p] = f64_to_e4m3_rne((double)v / (double)s);
    }
}

// ---------------------------------------------------------------- voxel-major layout

__global__ void k_count_cols(const int32_t* __restrict__ col, int64_t nnz, uint32_t* __restrict__ cnt) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[p]], 1u);
}

__global__ void k_quads_of(const uint32_t* __restrict__ cnt, int64_t n, uint32_t* __restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = (cnt[i] + 3u) >> 2;
}

// One wave per beamlet row: scatter (beamlet index, encoded value) into the
// voxel rows; the slot within a voxel row comes from an atomic counter, and the
// rows are put in beamlet order afterwards by k_sort_vm.
template <int FMT>
__global__ void k_scatter_vm(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const void* __restrict__ bm_val, const uint32_t* __restrict__ bm_qptr,
                             int64_t nb, const uint32_t* __restrict__ vqptr, uint32_t* __restrict__ fill,
                             int32_t* __restrict__ vcol, void* __restrict__ vval) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= nb) return;
    const int64_t a = rp[row], n = rp[row + 1] - a;
    const int64_t o = (int64_t)bm_qptr[row] * 4;
    for (int64_t p = lane; p < n; p += 64) {
        const int32_t j = col[a + p];
        const int64_t dst = (int64_t)vqptr[j] * 4 + atomicAdd(&fill[j], 1u);
        vcol[dst] = (int32_t)row;
        if (FMT == FMT_F32) reinterpret_cast<float*>(vval)[dst] = reinterpret_cast<const float*>(bm_val)[o + p];
        if (FMT == FMT_BF16 || FMT == FMT_F16)
            reinterpret_cast<uint16_t*>(vval)[dst] = reinterpret_cast<const uint16_t*>(bm_val)[o + p];
        if (FMT == FMT_FP8) reinterpret_cast<uint8_t*>(vval)[dst] = reinterpret_cast<const uint8_t*>(bm_val)[o + p];
    }
}

// One wave per voxel row: rank sort by beamlet index (keys are unique within a
// row), staged through LDS when the row fits, into a temporary copy.
constexpr int SORT_LDS = 2048;

template <typename VT>
__global__ void k_rank_vm(const uint32_t* __restrict__ vqptr, const uint32_t* __restrict__ cnt, int64_t nv,
                          const int32_t* __restrict__ vcol, const VT* __restrict__ val,
                          int32_t* __restrict__ tmp_col, VT* __restrict__ tval) {
    __shared__ int32_t skey[4][SORT_LDS];
    const int w = threadIdx.x / 64;
    const int64_t row = (int64_t)blockIdx.x * 4 + w;
    const int lane = threadIdx.x & 63;
    const bool valid = row < nv;
    const int64_t o = valid ? (int64_t)vqptr[row] * 4 : 0;
    const int64_t n = valid ? cnt[row] : 0;
    const bool lds = n <= SORT_LDS;
    if (lds)
        for (int64_t p = lane; p < n; p += 64) skey[w][p] = vcol[o + p];
    __syncthreads();
    for (int64_t p = lane; p < n; p += 64) {
        const int32_t key = lds ? skey[w][p] : vcol[o + p];
        int64_t rank = 0;
        for (int64_t q = 0; q < n; ++q) rank += (lds ? skey[w][q] : vcol[o + q]) < key;
        tmp_col[o + rank] = key;
        tval[o + rank] = val[o + p];
    }
}

// Copy the sorted rows back and fill the padding.
template <typename VT>
__global__ void k_pad_vm(const uint32_t* __restrict__ vqptr, const uint32_t* __restrict__ cnt, int64_t nv,
                         const int32_t* __restrict__ tmp_col, const VT* __restrict__ tval,
                         int32_t* __restrict__ vcol, VT* __restrict__ val) {
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= nv) return;
    const int64_t o = (int64_t)vqptr[row] * 4;
    const int64_t npad = (int64_t)(vqptr[row + 1] - vqptr[row]) * 4;
    const int64_t n = cnt[row];
    for (int64_t p = lane; p < npad; p += 64) {
        const bool real = p < n;
        vcol[o + p] = real ? tmp_col[o + p] : (n > 0 ? tmp_col[o] : 0);
        val[o + p] = real ? tval[o + p] : (VT)0;
    }
}

// ---------------------------------------------------------------- helpers

static int pick_lanes(double mean_len) {
    // about three quads per lane per row
    int g = 1;
    while (g < 64 && g * 12 < mean_len) g <<= 1;
    return std::max(g, 4);
}

template <typename T>
static vmat_status dalloc(vmat_ctx* h, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(VMAT_ERR_ALLOC, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    h->bytes += (int64_t)(count * sizeof(T));
    return VMAT_OK;
}

#define VMAT_TRY(x)                          \
    do {                                     \
        vmat_status s_ = (x);                \
        if (s_ != VMAT_OK) return s_;        \
    } while (0)

static vmat_status scan_u32(const uint32_t* in, int64_t n, uint32_t* out, uint64_t* tiles, int* overflow,
                            hipStream_t st) {
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles > 0) {
        k_scan_tiles<<<(unsigned)ntiles, SCAN_BLOCK, 0, st>>>(in, n, tiles);
        VMAT_LAUNCH_CHECK();
    }
    k_scan_tile_sums<<<1, 1, 0, st>>>(tiles, ntiles);
    VMAT_LAUNCH_CHECK();
    k_scan_apply<<<(unsigned)std::max<int64_t>(ntiles, 1), SCAN_BLOCK, 0, st>>>(in, n, tiles, ntiles, out, overflow);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

vmat_status scan_u32_dev(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t st) {
    uint64_t* tiles = nullptr;
    int* ovf = nullptr;
    const int64_t ntiles = n / SCAN_TILE + 2;
    if (hipMalloc((void**)&tiles, (ntiles + 1) * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void**)&ovf, sizeof(int)) != hipSuccess) {
        if (tiles) (void)hipFree(tiles);
        return fail(VMAT_ERR_ALLOC, "hipMalloc failed in scan");
    }
    int flag = 0;
    vmat_status rc = VMAT_OK;
    if (hipMemsetAsync(ovf, 0, sizeof(int), st) != hipSuccess) rc = fail(VMAT_ERR_DEVICE, "hipMemsetAsync failed");
    if (rc == VMAT_OK) rc = scan_u32(in, n, out, tiles, ovf, st);
    if (rc == VMAT_OK && (hipMemcpyAsync(&flag, ovf, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
                          hipStreamSynchronize(st) != hipSuccess))
        rc = fail(VMAT_ERR_DEVICE, "scan readback failed");
    (void)hipFree(tiles);
    (void)hipFree(ovf);
    if (rc == VMAT_OK && flag) rc = fail(VMAT_ERR_UNSUPPORTED, "index range exceeds 32 bits");
    return rc;
}

template <int FMT>
static vmat_status build_layouts(vmat_ctx* h, const vmat_problem* p, hipStream_t st, int* dflag) {
    const int64_t nb = h->nb, nv = h->nv;
    const int vb = fmt_bytes(FMT);
    uint32_t *qcount = nullptr, *cnt = nullptr, *fill = nullptr;
    uint64_t* tiles = nullptr;
    int32_t* tmp_col = nullptr;
    void* tmp_val = nullptr;
    vmat_status rc = VMAT_OK;
    const int64_t ntiles = std::max<int64_t>(nb, nv) / SCAN_TILE + 2;
    auto cleanup = [&]() {
        (void)hipFree(qcount); (void)hipFree(cnt); (void)hipFree(fill); (void)hipFree(tiles); (void)hipFree(tmp_col); (void)hipFree(tmp_val);
    };
#define TRY_C(x) do { rc = (x); if (rc != VMAT_OK) { cleanup(); return rc; } } while (0)
#define HIP_C(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { cleanup(); return fail(VMAT_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); } } while (0)
    HIP_C(hipMalloc((void**)&qcount, (std::max(nb, nv) + 1) * sizeof(uint32_t)));
    HIP_C(hipMalloc((void**)&cnt, (nv + 1) * sizeof(uint32_t)));
    HIP_C(hipMalloc((void**)&fill, (nv + 1) * sizeof(uint32_t)));
    HIP_C(hipMalloc((void**)&tiles, (ntiles + 1) * sizeof(uint64_t)));

    // beamlet-major
    h->bm.n_rows = nb;
    TRY_C(dalloc(h, &h->bm.qptr, nb + 1));
    k_row_quads<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(p->row_ptr, nb, qcount);
    HIP_C(hipGetLastError());
    TRY_C(scan_u32(qcount, nb, h->bm.qptr, tiles, dflag, st));
    uint32_t tot = 0;
    HIP_C(hipMemcpyAsync(&tot, h->bm.qptr + nb, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    int ovf = 0;
    HIP_C(hipMemcpyAsync(&ovf, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_C(hipStreamSynchronize(st));
    if (ovf) { cleanup(); return fail(VMAT_ERR_UNSUPPORTED, "padded nnz exceeds 2^34"); }
    h->bm.n_quads = tot;
    TRY_C(dalloc(h, &h->bm.col, (size_t)tot * 4));
    {
        uint8_t* v = nullptr;
        TRY_C(dalloc(h, &v, (size_t)tot * 4 * vb));
        h->bm.val = v;
    }
    if (FMT == FMT_FP8) TRY_C(dalloc(h, &h->bm.scale, nb));
    k_fill_bm<FMT><<<(unsigned)((nb + 3) / 4), 256, 0, st>>>(p->row_ptr, p->col, p->val, nb, h->bm.qptr,
                                                              h->bm.col, h->bm.val, h->bm.scale);
    HIP_C(hipGetLastError());

    // voxel-major
    h->vm.n_rows = nv;
    TRY_C(dalloc(h, &h->vm.qptr, nv + 1));
    HIP_C(hipMemsetAsync(cnt, 0, (nv + 1) * sizeof(uint32_t), st));
    HIP_C(hipMemsetAsync(fill, 0, (nv + 1) * sizeof(uint32_t), st));
    if (h->nnz > 0) {
        k_count_cols<<<2048, 256, 0, st>>>(p->col, h->nnz, cnt);
        HIP_C(hipGetLastError());
    }
    k_quads_of<<<(unsigned)((nv + 255) / 256), 256, 0, st>>>(cnt, nv, qcount);
    HIP_C(hipGetLastError());
    TRY_C(scan_u32(qcount, nv, h->vm.qptr, tiles, dflag, st));
    HIP_C(hipMemcpyAsync(&tot, h->vm.qptr + nv, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_C(hipMemcpyAsync(&ovf, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_C(hipStreamSynchronize(st));
    if (ovf) { cleanup(); return fail(VMAT_ERR_UNSUPPORTED, "padded nnz exceeds 2^34"); }
    h->vm.n_quads = tot;
    TRY_C(dalloc(h, &h->vm.col, (size_t)tot * 4));
    {
        uint8_t* v = nullptr;
        TRY_C(dalloc(h, &v, (size_t)tot * 4 * vb));
        h->vm.val = v;
    }
    HIP_C(hipMalloc((void**)&tmp_col, (size_t)std::max<uint32_t>(tot, 1) * 4 * sizeof(int32_t)));
    HIP_C(hipMalloc((void**)&tmp_val, (size_t)std::max<uint32_t>(tot, 1) * 4 * vb));
    k_scatter_vm<FMT><<<(unsigned)((nb + 3) / 4), 256, 0, st>>>(p->row_ptr, p->col, h->bm.val, h->bm.qptr, nb,
                                                                 h->vm.qptr, fill, h->vm.col, h->vm.val);
    HIP_C(hipGetLastError());
    {
        using VT = typename std::conditional<FMT == FMT_F32, float,
                   typename std::conditional<FMT == FMT_FP8, uint8_t, uint16_t>::type>::type;
        k_rank_vm<VT><<<(unsigned)((nv + 3) / 4), 256, 0, st>>>(h->vm.qptr, cnt, nv, h->vm.col,
                                                               reinterpret_cast<const VT*>(h->vm.val), tmp_col,
                                                               reinterpret_cast<VT*>(tmp_val));
        HIP_C(hipGetLastError());
        k_pad_vm<VT><<<(unsigned)((nv + 3) / 4), 256, 0, st>>>(h->vm.qptr, cnt, nv, tmp_col,
                                                              reinterpret_cast<const VT*>(tmp_val), h->vm.col,
                                                              reinterpret_cast<VT*>(h->vm.val));
        HIP_C(hipGetLastError());
    }
    HIP_C(hipStreamSynchronize(st));
    h->bm.lanes_per_row = pick_lanes(nb > 0 ? 4.0 * (double)h->bm.n_quads / (double)nb : 0.0);
    h->vm.lanes_per_row = pick_lanes(nv > 0 ? 4.0 * (double)h->vm.n_quads / (double)nv : 0.0);
    h->vm.scale = nullptr;
    cleanup();
    if (h->layout_req != 1) {
        rc = build_tiled(h, p, st);
        if (rc != VMAT_OK) {
            free_tiled(h);
            if (h->layout_req == 2 || rc != VMAT_ERR_UNSUPPORTED) return rc;
            set_error("");
        } else {
            // the tiled copy replaces the voxel-major quad CSR; the
            // beamlet-major copy stays for the aperture-dose bound and the
            // adjoint with many right-hand sides before its slot sums are
            // reserved
            const int64_t vbytes = h->d_store == VMAT_F32 ? 4 : (h->d_store == VMAT_FP8_E4M3 ? 1 : 2);
            (void)hipFree(h->vm.col);
            (void)hipFree(h->vm.val);
            (void)hipFree(h->vm.qptr);
            h->bytes -= (int64_t)h->vm.n_quads * 4 * (4 + vbytes) + (nv + 1) * 4;
            h->vm.col = nullptr;
            h->vm.val = nullptr;
            h->vm.qptr = nullptr;
        }
    }
    return VMAT_OK;
#undef TRY_C
#undef HIP_C
}

static void free_all(vmat_ctx* h) {
    auto F = [](void* p) { if (p) (void)hipFree(p); };
    F(h->d_theta);
    if (h->d_owner) {
        // the layouts of D belong to the owner; only the slot sums are ours
        F(h->tl.part);
    } else {
        F(h->bm.qptr); F(h->bm.col); F(h->bm.val); F(h->bm.scale);
        F(h->vm.qptr); F(h->vm.col); F(h->vm.val); F(h->vm.scale);
        free_tiled(h);
    }
    F(h->abT); F(h->wlab); F(h->wtab); F(h->x); F(h->xl); F(h->z); F(h->dz); F(h->rz); F(h->g); F(h->bpart); F(h->part); F(h->part_b);
    F(h->pl); F(h->pr); F(h->pocc); F(h->d_gamma); F(h->vflag);
    F(h->my); F(h->mgrad); F(h->mgrad_prev); F(h->md); F(h->md_prev); F(h->mgF); F(h->mW); F(h->mW_prev);
    F(h->ms);
    F(h->ms2);
    if (h->ms_host) (void)hipHostFree(h->ms_host);
    if (h->mirror) (void)hipHostFree(h->mirror);
    free_batch(h);
    free_apdose(h);
    for (auto& g : h->iter_graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    F(h->row_S); F(h->row_l); F(h->row_r); F(h->row_m); F(h->bprice); F(h->pbeam); F(h->pscore); F(h->cost2);
    F(h->tr.beam); F(h->tr.price); F(h->tr.margin); F(h->tr.row_margin); F(h->tr.cost); F(h->tr.miters); F(h->tr.y);
}

// Labels of the voxel weights: the distinct (alpha, beta, T) triples, compared
// bit for bit, in order of first appearance.  Returns false when there are
// more than WTAB_CAP of them.
static bool label_weights(const float* a, const float* b, const float* t, int64_t nv, std::vector<float4>& tab,
                          std::vector<uint8_t>& lab) {
    auto same = [](const float4& u, const float4& v) { return std::memcmp(&u, &v, 3 * sizeof(float)) == 0; };
    tab.clear();
    lab.assign((size_t)nv, 0);
    int last = -1;
    for (int64_t j = 0; j < nv; ++j) {
        const float4 w = make_float4(a[j], b[j], t[j], 0.0f);
        if (last < 0 || !same(w, tab[last])) {
            last = -1;
            for (int q = 0; q < (int)tab.size(); ++q)
                if (same(w, tab[q])) {
                    last = q;
                    break;
                }
            if (last < 0) {
                if ((int)tab.size() == WTAB_CAP) return false;
                tab.push_back(w);
                last = (int)tab.size() - 1;
            }
        }
        lab[j] = (uint8_t)last;
    }
    return true;
}

// Uploads labels and table (the table padded with zeros to WTAB_CAP).
static vmat_status upload_labels(vmat_ctx* h, const std::vector<float4>& tab, const std::vector<uint8_t>& lab,
                                 hipStream_t st) {
    std::vector<float4> full(WTAB_CAP, make_float4(0.f, 0.f, 0.f, 0.f));
    std::copy(tab.begin(), tab.end(), full.begin());
    if (hipMemcpyAsync(h->wlab, lab.data(), (size_t)h->nv, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h->wtab, full.data(), WTAB_CAP * sizeof(float4), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VMAT_ERR_DEVICE, "upload of the weight labels failed");
    h->n_wtab = (int)tab.size();
    return VMAT_OK;
}

// Host copies of the caller's device weights.
static vmat_status weights_to_host(const float* a, const float* b, const float* t, int64_t nv,
                                   std::vector<float>& ha, std::vector<float>& hb, std::vector<float>& ht,
                                   hipStream_t st) {
    ha.resize((size_t)nv);
    hb.resize((size_t)nv);
    ht.resize((size_t)nv);
    if (hipMemcpyAsync(ha.data(), a, (size_t)nv * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hb.data(), b, (size_t)nv * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(ht.data(), t, (size_t)nv * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VMAT_ERR_DEVICE, "copy of the voxel weights failed");
    return VMAT_OK;
}

// The voxel weights as one-byte labels when there are at most WTAB_CAP
// distinct triples (one per structure in the usual case); else the kernels
// read abT.  VMAT_NO_WEIGHT_LABELS in the environment at creation also keeps
// abT only.  The label mode chosen here stays with the handle.
static vmat_status build_weight_labels(vmat_ctx* h, const vmat_problem* p, hipStream_t st) {
    if (getenv("VMAT_NO_WEIGHT_LABELS")) return VMAT_OK;
    std::vector<float> a, b, t;
    vmat_status rc = weights_to_host(p->alpha, p->beta, p->T, h->nv, a, b, t, st);
    if (rc != VMAT_OK) return rc;
    std::vector<float4> tab;
    std::vector<uint8_t> lab;
    if (!label_weights(a.data(), b.data(), t.data(), h->nv, tab, lab)) return VMAT_OK;
    if ((rc = dalloc(h, &h->wlab, h->nv)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->wtab, (int64_t)WTAB_CAP)) != VMAT_OK) return rc;
    return upload_labels(h, tab, lab, st);
}

}  // namespace vmat

using namespace vmat;

extern "C" const char* vmat_last_error(void) { return vmat::last_error(); }

// The state of one plan on a handle: work buffers, the plan copy, the master
// state and its pinned mirror, pricing results and the trace; theta and gamma
// on the device.  Everything that is not a layout of D.
static vmat_status alloc_plan_state(vmat_ctx* h, hipStream_t st) {
    vmat_status rc = VMAT_OK;
    const int64_t N = h->N, NR = (int64_t)h->N * h->R;
    // partial-sum workgroups of the voxel passes: one per 2048 voxels, at
    // least 256 (a small grid leaves CUs idle on these latency-bound passes)
    // and at most 1024 (every pass reduces all partials of the previous one)
    h->n_part = (int)std::min<int64_t>(1024, std::max<int64_t>(256, (h->nv + 2047) / 2048));
    if ((rc = dalloc(h, &h->d_theta, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->x, h->nb)) != VMAT_OK) return rc;
    if (h->tl.on && h->tl.S > 0 && (rc = dalloc(h, &h->xl, h->tl.S)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->z, h->nv)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->dz, h->nv)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->rz, h->nv)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->g, h->nb)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->bpart, (size_t)N * std::max(AP_GRAD_PARTS, (h->R * h->C + 255) / 256))) != VMAT_OK)
        return rc;
    if ((rc = dalloc(h, &h->part, (size_t)h->n_part * 8)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->part_b, (size_t)h->n_part * 64)) != VMAT_OK) return rc;
    double** vecs[] = {&h->my, &h->mgrad, &h->mgrad_prev, &h->md, &h->md_prev, &h->mgF};
    for (double** v : vecs)
        if ((rc = dalloc(h, v, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->pl, NR)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->pr, NR)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->pocc, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->d_gamma, 1)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->vflag, 1)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->mW, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->mW_prev, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->ms, 1)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->ms2, 1)) != VMAT_OK) return rc;
    if (hipHostMalloc((void**)&h->ms_host, sizeof(MasterState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->mirror, sizeof(MasterMirror), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess)
        return fail(VMAT_ERR_ALLOC, "hipHostMalloc failed");
    std::memset((void*)h->mirror, 0, sizeof(MasterMirror));
    if (hipHostGetDevicePointer((void**)&h->mirror_dev, h->mirror, 0) != hipSuccess)
        return fail(VMAT_ERR_DEVICE, "hipHostGetDevicePointer failed");
    if ((rc = dalloc(h, &h->row_S, NR)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->row_l, NR)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->row_r, NR)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->row_m, NR)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->bprice, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->pbeam, 1 + 2 * (int64_t)h->R)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->pscore, 3)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->cost2, 2)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->tr.beam, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->tr.price, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->tr.margin, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->tr.row_margin, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->tr.cost, N + 1)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->tr.miters, N)) != VMAT_OK) return rc;
    if ((rc = dalloc(h, &h->tr.y, N * N)) != VMAT_OK) return rc;
    if (hipMemcpyAsync(h->d_theta, h->theta.data(), N * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VMAT_ERR_DEVICE, "copy of theta failed");
    return set_gamma(h, h->gamma, st);
}

extern "C" vmat_status vmat_create(const vmat_problem* p, hipStream_t st, vmat_handle* out) {
    set_error("");
    if (!p || !out) return fail(VMAT_ERR_INVALID_ARG, "null problem or output pointer");
    *out = nullptr;
    if (p->n_beams < 1 || p->n_rows < 1 || p->n_cols < 1)
        return fail(VMAT_ERR_INVALID_ARG, "n_beams, n_rows and n_cols must be >= 1");
    if (p->n_cols > 64) return fail(VMAT_ERR_UNSUPPORTED, "n_cols > 64 is not supported");
    if (p->n_voxels < 1 || p->n_voxels >= (int64_t)1 << 31) return fail(VMAT_ERR_INVALID_ARG, "n_voxels out of range");
    const int64_t nb = (int64_t)p->n_beams * p->n_rows * p->n_cols;
    if (nb >= (int64_t)1 << 31) return fail(VMAT_ERR_INVALID_ARG, "too many beamlets");
    if (p->nnz < 0 || p->nnz >= (int64_t)1 << 33) return fail(VMAT_ERR_INVALID_ARG, "nnz out of range");
    if (!p->theta_deg || !p->row_ptr || (p->nnz > 0 && (!p->col || !p->val)) || !p->alpha || !p->beta || !p->T)
        return fail(VMAT_ERR_INVALID_ARG, "null array in problem");
    if (p->d_store < VMAT_F32 || p->d_store > VMAT_FP8_E4M3) return fail(VMAT_ERR_INVALID_ARG, "unknown d_store");
    if (p->layout < 0 || p->layout > 2) return fail(VMAT_ERR_INVALID_ARG, "unknown layout");
    if (p->n_beams > 4096) return fail(VMAT_ERR_UNSUPPORTED, "more than 4096 beams");
    if (!std::isfinite(p->gamma) || p->gamma < 0.0) return fail(VMAT_ERR_INVALID_ARG, "gamma must be finite and >= 0");
    for (int k = 0; k < p->n_beams; ++k) {
        const double t = p->theta_deg[k];
        if (!std::isfinite(t) || t < 0.0 || t >= 360.0)
            return fail(VMAT_ERR_INVALID_ARG, "theta_deg must lie in [0, 360)");
        if (k > 0 && !(t > p->theta_deg[k - 1]))
            return fail(VMAT_ERR_INVALID_ARG, "theta_deg must be strictly increasing");
    }
    vmat_ctx* h = new (std::nothrow) vmat_ctx();
    if (!h) return fail(VMAT_ERR_ALLOC, "host allocation failed");
    h->N = p->n_beams; h->R = p->n_rows; h->C = p->n_cols;
    h->nb = nb; h->nv = p->n_voxels; h->nnz = p->nnz;
    h->d_store = p->d_store; h->gamma = p->gamma;
    h->circular = p->circular ? 1 : 0; h->delta = p->max_leaf_step;
    h->layout_req = p->layout;
    h->theta.assign(p->theta_deg, p->theta_deg + p->n_beams);
    (void)hipGetDevice(&h->device);

    vmat_status rc = VMAT_OK;
    int* dflag = nullptr;
    auto bail = [&](vmat_status code) {
        if (dflag) (void)hipFree(dflag);
        free_all(h);
        delete h;
        return code;
    };
    if (hipMalloc((void**)&dflag, sizeof(int)) != hipSuccess) return bail(fail(VMAT_ERR_ALLOC, "hipMalloc failed"));
    if (hipMemsetAsync(dflag, 0, sizeof(int), st) != hipSuccess) return bail(fail(VMAT_ERR_DEVICE, "hipMemsetAsync failed"));
    if ((rc = dalloc(h, &h->abT, h->nv)) != VMAT_OK) return bail(rc);
    k_validate_rows<<<(unsigned)((nb + 3) / 4), 256, 0, st>>>(p->row_ptr, p->col, p->val, nb, h->nv, h->nnz, dflag);
    k_validate_voxels<<<1024, 256, 0, st>>>(p->alpha, p->beta, p->T, h->nv, h->abT, dflag);
    int flag = 0;
    if (hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return bail(fail(VMAT_ERR_DEVICE, std::string("validation failed: ") + hipGetErrorString(hipGetLastError())));
    if (flag) {
        std::string m = "invalid problem data:";
        if (flag & BAD_ROWPTR) m += " row_ptr";
        if (flag & BAD_COL) m += " col out of range";
        if (flag & BAD_ORDER) m += " col not ascending within a row";
        if (flag & BAD_VAL) m += " D value negative or not finite";
        if (flag & BAD_ALPHA) m += " alpha";
        if (flag & BAD_BETA) m += " beta";
        if (flag & BAD_T) m += " T";
        return bail(fail(VMAT_ERR_INVALID_ARG, m));
    }
    if ((rc = build_weight_labels(h, p, st)) != VMAT_OK) return bail(rc);
    switch (h->d_store) {
        case VMAT_F32: rc = build_layouts<FMT_F32>(h, p, st, dflag); break;
        case VMAT_F16: rc = build_layouts<FMT_F16>(h, p, st, dflag); break;
        case VMAT_BF16: rc = build_layouts<FMT_BF16>(h, p, st, dflag); break;
        default: rc = build_layouts<FMT_FP8>(h, p, st, dflag); break;
    }
    if (rc != VMAT_OK) return bail(rc);
    (void)hipFree(dflag);
    dflag = nullptr;

    // work buffers and the plan state
    if ((rc = alloc_plan_state(h, st)) != VMAT_OK) return bail(rc);
    if ((rc = tune_sell(h, st)) != VMAT_OK) return bail(rc);
    // the streaming master's iteration, captured once on the handle's plan
    if ((rc = capture_master(h, 0)) != VMAT_OK) return bail(rc);
    *out = h;
    return VMAT_OK;
}

extern "C" vmat_status vmat_create_plan(vmat_handle src, hipStream_t st, vmat_handle* out) {
    set_error("");
    if (out) *out = nullptr;
    if (!src || !out) return fail(VMAT_ERR_INVALID_ARG, "null handle or output pointer");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != src->device)
        return fail(VMAT_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    vmat_ctx* o = src->d_owner ? src->d_owner : src;
    vmat_ctx* h = new (std::nothrow) vmat_ctx();
    if (!h) return fail(VMAT_ERR_ALLOC, "host allocation failed");
    h->N = src->N; h->R = src->R; h->C = src->C;
    h->nb = src->nb; h->nv = src->nv; h->nnz = src->nnz;
    h->d_store = src->d_store; h->gamma = src->gamma;
    h->circular = src->circular; h->delta = src->delta;
    h->device = src->device;
    h->theta = src->theta;
    h->layout_req = src->layout_req;
    h->sell_u_fwd = o->sell_u_fwd; h->sell_u_adj = o->sell_u_adj;
    std::copy(std::begin(src->tune_fwd), std::end(src->tune_fwd), std::begin(h->tune_fwd));
    std::copy(std::begin(src->tune_adj), std::end(src->tune_adj), std::begin(h->tune_adj));
    // the layouts of D, read-only from here on; the slot sums the tiled
    // adjoint writes are this context's own
    h->bm = o->bm;
    h->vm = o->vm;
    h->tl = o->tl;
    h->tl.part = nullptr;
    h->d_owner = o;
    auto bail = [&](vmat_status code) {
        free_all(h);
        delete h;
        return code;
    };
    vmat_status rc = VMAT_OK;
    if (h->tl.on && (rc = dalloc(h, &h->tl.part, (size_t)h->tl.S)) != VMAT_OK) return bail(rc);
    // the source's current weights, in its form (labels or per-voxel)
    if ((rc = dalloc(h, &h->abT, h->nv)) != VMAT_OK) return bail(rc);
    if (hipMemcpyAsync(h->abT, src->abT, (size_t)h->nv * sizeof(float4), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return bail(fail(VMAT_ERR_DEVICE, "copy of the voxel weights failed"));
    if (src->n_wtab > 0) {
        if ((rc = dalloc(h, &h->wlab, h->nv)) != VMAT_OK) return bail(rc);
        if ((rc = dalloc(h, &h->wtab, (int64_t)WTAB_CAP)) != VMAT_OK) return bail(rc);
        if (hipMemcpyAsync(h->wlab, src->wlab, (size_t)h->nv, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(h->wtab, src->wtab, WTAB_CAP * sizeof(float4), hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
            return bail(fail(VMAT_ERR_DEVICE, "copy of the weight labels failed"));
        h->n_wtab = src->n_wtab;
    }
    if ((rc = alloc_plan_state(h, st)) != VMAT_OK) return bail(rc);
    if ((rc = capture_master(h, 0)) != VMAT_OK) return bail(rc);
    o->n_plans.fetch_add(1);
    *out = h;
    return VMAT_OK;
}

// Checks the voxel weights without writing anything.
__global__ void k_check_voxels(const float* __restrict__ alpha, const float* __restrict__ beta,
                               const float* __restrict__ T, int64_t nv, int* __restrict__ flag) {
    int bad = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nv; j += (int64_t)gridDim.x * blockDim.x) {
        const float a = alpha[j], b = beta[j], t = T[j];
        if (!(a >= 0.0f) || !isfinite(a)) bad |= BAD_ALPHA;
        if (!(b >= 0.0f) || !isfinite(b)) bad |= BAD_BETA;
        if (!isfinite(t)) bad |= BAD_T;
    }
    if (bad) atomicOr(flag, bad);
}

extern "C" vmat_status vmat_set_weights(vmat_handle h, const float* alpha, const float* beta, const float* T,
                                        hipStream_t st) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return fail(VMAT_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    if (!alpha || !beta || !T) return fail(VMAT_ERR_INVALID_ARG, "null alpha, beta or T");
    VMAT_HIP(hipMemsetAsync(h->vflag, 0, sizeof(int), st));
    k_check_voxels<<<1024, 256, 0, st>>>(alpha, beta, T, h->nv, h->vflag);
    VMAT_LAUNCH_CHECK();
    int flag = 0;
    VMAT_HIP(hipMemcpyAsync(&flag, h->vflag, sizeof(int), hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipStreamSynchronize(st));
    if (flag) {
        std::string m = "invalid voxel weights:";
        if (flag & BAD_ALPHA) m += " alpha";
        if (flag & BAD_BETA) m += " beta";
        if (flag & BAD_T) m += " T";
        return fail(VMAT_ERR_INVALID_ARG, m);
    }
    std::vector<float4> tab;
    std::vector<uint8_t> lab;
    if (h->n_wtab > 0) {
        std::vector<float> a, b, t;
        vmat_status rc = weights_to_host(alpha, beta, T, h->nv, a, b, t, st);
        if (rc != VMAT_OK) return rc;
        if (!label_weights(a.data(), b.data(), t.data(), h->nv, tab, lab))
            return fail(VMAT_ERR_UNSUPPORTED, "more than 256 distinct (alpha, beta, T) on a handle created with "
                                              "labelled weights");
    }
    k_validate_voxels<<<1024, 256, 0, st>>>(alpha, beta, T, h->nv, h->abT, h->vflag);
    VMAT_LAUNCH_CHECK();
    if (h->n_wtab > 0) return upload_labels(h, tab, lab, st);
    VMAT_HIP(hipStreamSynchronize(st));
    return VMAT_OK;
}

extern "C" vmat_status vmat_destroy(vmat_handle h) {
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    if (h->n_plans.load() > 0)
        return fail(VMAT_ERR_INVALID_ARG, "plan contexts made from this handle still read its layouts of D");
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    free_all(h);
    (void)hipSetDevice(cur);
    if (h->d_owner) h->d_owner->n_plans.fetch_sub(1);
    delete h;
    return VMAT_OK;
}

extern "C" vmat_status vmat_device_bytes(vmat_handle h, int64_t* bytes) {
    if (!h || !bytes) return fail(VMAT_ERR_INVALID_ARG, "null argument");
    *bytes = h->bytes;
    return VMAT_OK;
}
