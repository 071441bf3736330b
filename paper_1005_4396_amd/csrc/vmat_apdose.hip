// Aperture doses for the master over the generated apertures (Sec. 2.2).
//
// The master problem keeps the apertures fixed and optimises one intensity
// per aperture, so the dose is z = sum_k y_k d_k with d_k = D^T 1_{A_k}.  Each
// d_k is computed once, when its aperture is opened (one dose product), and
// stored sparsely; the master's dose products and its beam gradients
// dF/dy_k = <d_k, F'(z)> then touch only these vectors, which hold far fewer
// entries than D (an aperture exposes a small part of its beam).
//
// Storage (ApDose in vmat_internal.h): an aperture-major copy, appended per
// aperture with voxels ascending, for the per-aperture sums; a voxel-major
// copy, rebuilt by merging each new aperture into the previous one, for the
// dose.  Values are stored in FP32: each d_k entry (a sum of FP32 D values
// formed in FP64) is rounded once, to 2^-24 relative, and every product with
// them accumulates in FP64.  Every sum runs in a fixed order: deterministic
// results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "vmat_block.h"
#include "vmat_formats.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"

namespace vmat {

constexpr int AP_CHUNK = 1024;  // voxels per chunk of the compaction
constexpr int AP_T = 256;       // threads per block

// Unit intensity on the aperture being stored: beam = *src if src, else beam_h.
__global__ __launch_bounds__(AP_T) void k_ap_unit(int N, const int32_t* __restrict__ src, int beam_h,
                                                  double* __restrict__ unit, int32_t* __restrict__ beam_out) {
    const int kb = src ? src[0] : beam_h;
    for (int k = threadIdx.x; k < N; k += AP_T) unit[k] = k == kb ? 1.0 : 0.0;
    if (threadIdx.x == 0) beam_out[0] = kb;
}

__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* sh, uint32_t* total) {
    // sh: at least AP_T / 64 entries.  Inclusive scan within each wave
    // (shuffles), then the wave totals in order; exact integer sums.
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int w = 0; w < AP_T / 64; ++w) {
        const uint32_t t = sh[w];
        if (w < wid) base += t;
        tot += t;
    }
    *total = tot;
    __syncthreads();
    return base + x - v;
}

// Non-zeros of d per chunk of AP_CHUNK voxels.
__global__ __launch_bounds__(AP_T) void k_ap_count(int64_t nv, const double* __restrict__ d,
                                                   uint32_t* __restrict__ chunk) {
    __shared__ uint32_t sh[AP_T + 1];
    const int64_t j0 = (int64_t)blockIdx.x * AP_CHUNK + threadIdx.x * 4;
    uint32_t c = 0;
    for (int u = 0; u < 4; ++u)
        if (j0 + u < nv && d[j0 + u] != 0.0) ++c;
    uint32_t tot;
    (void)block_excl_scan_u32(c, sh, &tot);
    if (threadIdx.x == 0) chunk[blockIdx.x] = tot;
}

// Exclusive scan of the chunk counts (one block, tiles of AP_T in order);
// chunk[n] = total.
__global__ __launch_bounds__(AP_T) void k_ap_scan(int n, uint32_t* __restrict__ chunk) {
    __shared__ uint32_t sh[AP_T + 1];
    uint32_t carry = 0;
    for (int base = 0; base < n; base += AP_T) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < n ? chunk[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u32(v, sh, &tot);
        if (i < n) chunk[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) chunk[n] = carry;
}

// Appends the non-zeros of d (voxels ascending) to the aperture-major copy at
// offset col_ptr[slot] (the entries of the apertures stored before) and
// places them in the voxel-major copy (old -> new): new_ptr[j] = old_ptr[j] +
// (non-zeros before voxel j) = old_ptr[j] + shift[j]; voxel j's new entry
// follows its old entries, which k_ap_copy moves.  Each block takes AP_CHUNK
// voxels, four per thread.
__global__ __launch_bounds__(AP_T) void k_ap_emit(int64_t nv, int n_chunks, const double* __restrict__ d,
                                                  const uint32_t* __restrict__ chunk,
                                                  const int32_t* __restrict__ beam,
                                                  const uint32_t* __restrict__ col_ptr, int slot,
                                                  ApEntry* __restrict__ col,
                                                  const uint32_t* __restrict__ optr,
                                                  uint32_t* __restrict__ nptr, uint32_t* __restrict__ shift,
                                                  uint16_t* __restrict__ nbeam, float* __restrict__ nval,
                                                  uint32_t* __restrict__ nvox) {
    __shared__ uint32_t sh[AP_T + 1];
    const int64_t j0 = (int64_t)blockIdx.x * AP_CHUNK + threadIdx.x * 4;
    double v[4];
    uint32_t c = 0;
    for (int u = 0; u < 4; ++u) {
        v[u] = j0 + u < nv ? d[j0 + u] : 0.0;
        if (v[u] != 0.0) ++c;
    }
    uint32_t tot;
    uint32_t p = chunk[blockIdx.x] + block_excl_scan_u32(c, sh, &tot);
    const uint16_t kb = (uint16_t)beam[0];
    const uint32_t top = col_ptr[slot];  // entries of the apertures stored before
    for (int u = 0; u < 4; ++u) {
        const int64_t j = j0 + u;
        if (j >= nv) break;
        const uint32_t o0 = optr[j], o1 = optr[j + 1];
        shift[j] = p;
        const uint32_t n0 = o0 + p;
        nptr[j] = n0;
        if (v[u] != 0.0) {
            nbeam[n0 + (o1 - o0)] = kb;
            const float vf = (float)v[u];
            nval[n0 + (o1 - o0)] = vf;
            nvox[n0 + (o1 - o0)] = (uint32_t)j;
            col[top + p] = ApEntry{(uint32_t)j, vf};
            ++p;
        }
        if (j == nv - 1) nptr[nv] = optr[nv] + chunk[n_chunks];
    }
}

// Moves every old entry of the voxel-major copy to its new place: entry e
// of voxel j = vox[e] goes to e + shift[j].  One entry per thread, so the
// work does not depend on how the entries are spread over the voxels; reads
// and writes stream (consecutive entries move to consecutive places, shift is
// gathered through the cache).
__global__ __launch_bounds__(AP_T) void k_ap_copy(uint32_t n_old, const uint32_t* __restrict__ shift,
                                                  const uint16_t* __restrict__ obeam,
                                                  const float* __restrict__ oval, const uint32_t* __restrict__ ovox,
                                                  uint16_t* __restrict__ nbeam, float* __restrict__ nval,
                                                  uint32_t* __restrict__ nvox) {
    const uint32_t e = blockIdx.x * AP_T + threadIdx.x;
    if (e >= n_old) return;
    const uint32_t j = ovox[e];
    const uint32_t dst = e + shift[j];
    nbeam[dst] = obeam[e];
    nval[dst] = oval[e];
    nvox[dst] = j;
}

// Closes an append: the new aperture's slot, then the device view of the
// store's current pointers.
__global__ void k_ap_slot(int slot, const int32_t* __restrict__ beam, const uint32_t* __restrict__ chunk,
                          int n_chunks, uint32_t* __restrict__ col_ptr, int32_t* __restrict__ beam_slot,
                          ApView* view, ApView v) {
    col_ptr[slot + 1] = col_ptr[slot] + chunk[n_chunks];
    beam_slot[beam[0]] = slot;
    *view = v;
}

// out_j = sum over voxel j's entries of val * vec[beam]; the per-beam vector
// is staged in LDS.  G lanes share a voxel: lane t of the group takes the
// voxel's entries t, t + G, ... in order, two at a time, and the group sums
// with a fixed shuffle tree, so a voxel with an entry from every aperture
// (the target's) costs its group 1/G of the serial walk.  G = 2 measured
// fastest on the prostate plan (1, 4 and 8 slower: a lone lane walks the
// target voxels serially, wider groups idle on the many voxels with few
// entries); a grid with fewer voxels than it takes to fill the chip's wave
// slots at G = 2 uses G = 4 (more loads in flight).
template <int AP_DG>
__global__ __launch_bounds__(AP_T) void k_ap_dose(int64_t nv, int N, const ApView* __restrict__ view,
                                                  const double* __restrict__ vec, double* __restrict__ out,
                                                  Gate gate) {
    extern __shared__ double vs[];  // [N]
    if (gate.closed()) return;
    for (int k = threadIdx.x; k < N; k += AP_T) vs[k] = vec[k];
    __syncthreads();
    const int64_t j = ((int64_t)blockIdx.x * AP_T + threadIdx.x) / AP_DG;
    const int t = threadIdx.x % AP_DG;
    const uint32_t* __restrict__ ptr = view->vx_ptr;
    const uint16_t* __restrict__ beam = view->vx_beam;
    const float* __restrict__ val = view->vx_val;
    double s = 0.0;
    if (j < nv) {
        const uint32_t e1 = ptr[j + 1];
        uint32_t e = ptr[j] + t;
        for (; e + AP_DG < e1; e += 2 * AP_DG) {
            const float v0 = val[e], v1 = val[e + AP_DG];
            const uint16_t b0 = beam[e], b1 = beam[e + AP_DG];
            s = fma((double)v0, vs[b0], s);
            s = fma((double)v1, vs[b1], s);
        }
        if (e < e1) s = fma((double)val[e], vs[beam[e]], s);
    }
    for (int off = AP_DG / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, AP_DG);
    if (j < nv && t == 0) out[j] = s;
}

// gF_k = <d_k, w> (0 without a stored aperture) in Q parts: block (k, q)
// takes the q-th of Q equal contiguous shares of aperture k's entries; thread
// t takes entries t, t + AP_GT, ... of the share with four loads in flight,
// then a fixed reduction tree; out[k*Q + q] = the share's sum.  AP_GT = 512
// on grids that fill the chip at two lanes per voxel (their apertures hold
// more entries per share: 1% faster on the prostate plan), else 256 (512 is
// 1.5% slower on the mixed-resolution plan's coarse grid).
template <int AP_GT>
__global__ __launch_bounds__(AP_GT) void k_ap_grad(const ApView* __restrict__ view, const float* __restrict__ w,
                                                   int Q, double* __restrict__ out, Gate gate) {
    __shared__ double sh[AP_GT / 64];
    if (gate.closed()) return;
    const int k = blockIdx.x / Q, q = blockIdx.x - k * Q;
    const int s = view->beam_slot[k];
    double acc = 0.0;
    if (s >= 0) {
        const ApEntry* __restrict__ col = view->col;
        const uint32_t a0 = view->col_ptr[s], a1 = view->col_ptr[s + 1];
        const uint32_t share = (a1 - a0 + Q - 1) / Q;
        const uint32_t e0 = a0 + min(a1 - a0, (uint32_t)q * share);
        const uint32_t e1 = a0 + min(a1 - a0, (uint32_t)(q + 1) * share);
        uint32_t e = e0 + threadIdx.x;
        for (; e + 3 * AP_GT < e1; e += 4 * AP_GT) {
            const ApEntry c0 = col[e], c1 = col[e + AP_GT], c2 = col[e + 2 * AP_GT], c3 = col[e + 3 * AP_GT];
            const float w0 = w[c0.vox], w1 = w[c1.vox], w2 = w[c2.vox], w3 = w[c3.vox];
            acc = fma((double)c0.val, (double)w0, acc);
            acc = fma((double)c1.val, (double)w1, acc);
            acc = fma((double)c2.val, (double)w2, acc);
            acc = fma((double)c3.val, (double)w3, acc);
        }
        for (; e < e1; e += AP_GT) {
            const ApEntry c = col[e];
            acc = fma((double)c.val, (double)w[c.vox], acc);
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < AP_GT / 64; ++i) t += sh[i];
        out[blockIdx.x] = t;
    }
}

__global__ void k_ap_view(ApView* view, ApView v) { *view = v; }

static int n_chunks_of(int64_t nv) { return (int)((nv + AP_CHUNK - 1) / AP_CHUNK); }


template <typename T>
static vmat_status ap_alloc(ApDose* a, T** p, size_t count) {
    const size_t n = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc((void**)p, n) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(VMAT_ERR_ALLOC, "device allocation failed (aperture doses)");
    }
    a->bytes += (int64_t)n;
    return VMAT_OK;
}

// Frees the entry arrays (those allocated: after a failed allocation some are
// null) and takes exactly their bytes off the count.
static void ap_free_entries(ApDose* a) {
    const int64_t cap = std::max<int64_t>(a->cap, 1);
    auto F = [&](auto*& p) {
        if (!p) return;
        (void)hipFree(p);
        a->bytes -= cap * (int64_t)sizeof(*p);
        p = nullptr;
    };
    F(a->col);
    F(a->vx_beam[0]); F(a->vx_beam[1]); F(a->vx_val[0]); F(a->vx_val[1]); F(a->vx_vox[0]); F(a->vx_vox[1]);
    a->cap = 0;
}

// The entry arrays at capacity cap; on failure the ones allocated stay for
// ap_free_entries.
static vmat_status ap_alloc_entries(ApDose* a, int64_t cap) {
    vmat_status rc = VMAT_OK;
    a->cap = cap;
    auto A = [&](auto** p) { if (rc == VMAT_OK) rc = ap_alloc(a, p, (size_t)cap); };
    A(&a->col);
    A(&a->vx_beam[0]); A(&a->vx_beam[1]); A(&a->vx_val[0]); A(&a->vx_val[1]); A(&a->vx_vox[0]); A(&a->vx_vox[1]);
    return rc;
}

void free_apdose(vmat_ctx* h) {
    ApDose* a = h->ap;
    if (!a) return;
    auto F = [](void* p) { if (p) (void)hipFree(p); };
    ap_free_entries(a);
    F(a->col_ptr); F(a->beam_slot); F(a->vx_ptr[0]); F(a->vx_ptr[1]); F(a->chunk); F(a->shift); F(a->unit);
    F(a->view);
    if (a->total_host) (void)hipHostFree(a->total_host);
    if (a->counted) (void)hipEventDestroy(a->counted);
    h->bytes -= a->bytes;
    delete a;
    h->ap = nullptr;
}

// The store's pointers with voxel-major copy c.
static ApView view_of(const ApDose* a, int c) {
    return ApView{a->vx_ptr[c], a->vx_beam[c], a->vx_val[c], a->col_ptr, a->col, a->beam_slot};
}

// Writes the current pointers to the device view.
static vmat_status ap_publish(vmat_ctx* h, hipStream_t st) {
    k_ap_view<<<1, 1, 0, st>>>(h->ap->view, view_of(h->ap, h->ap->cur));
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// Voxels each beam reaches: bit j % 32 of bits[k * words + j / 32] is set when
// a stored entry of a beamlet row of beam k at voxel j is non-zero.  One wave
// per beamlet row, lanes over its quads (padding entries hold zeros).
// Integer atomics only; the result does not depend on their order.
template <int FMT>
__global__ __launch_bounds__(256) void k_beam_voxel_bits(int64_t nb, int RC, const uint32_t* __restrict__ qptr,
                                                         const int32_t* __restrict__ col,
                                                         const void* __restrict__ val, int64_t words,
                                                         uint32_t* __restrict__ bits) {
    const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= nb) return;
    uint32_t* b = bits + (row / RC) * words;
    const i32x4* c4 = reinterpret_cast<const i32x4*>(col);
    const uint32_t q1 = qptr[row + 1];
    for (uint32_t q = qptr[row] + lane; q < q1; q += 64) {
        const float4 v = Quad<FMT>::load(val, q);
        const i32x4 c = c4[q];
        if (v.x != 0.f) atomicOr(b + (c.x >> 5), 1u << (c.x & 31));
        if (v.y != 0.f) atomicOr(b + (c.y >> 5), 1u << (c.y & 31));
        if (v.z != 0.f) atomicOr(b + (c.z >> 5), 1u << (c.z & 31));
        if (v.w != 0.f) atomicOr(b + (c.w >> 5), 1u << (c.w & 31));
    }
}

// Set bits of n words, as one partial count per block.
__global__ __launch_bounds__(AP_T) void k_popcount(int64_t n, const uint32_t* __restrict__ bits,
                                                   unsigned long long* __restrict__ part) {
    __shared__ unsigned long long sh[AP_T / 64];
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * AP_T + threadIdx.x; i < n; i += (int64_t)gridDim.x * AP_T)
        c += (unsigned long long)__popc(bits[i]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < AP_T / 64; ++w) t += sh[w];
        part[blockIdx.x] = t;
    }
}

// U = sum over beams of the voxels the beam reaches: no set of apertures (one
// per beam) has more aperture-dose entries than U.
static vmat_status beam_voxel_bound(vmat_ctx* h, int64_t* U) {
    const int64_t words = (h->nv + 31) / 32, n = words * h->N;
    constexpr int NPART = 1024;
    uint32_t* bits = nullptr;
    unsigned long long* part = nullptr;
    if (hipMalloc((void**)&bits, (size_t)n * 4) != hipSuccess) return fail(VMAT_ERR_ALLOC, "device allocation failed (aperture-dose bound)");
    if (hipMalloc((void**)&part, NPART * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipFree(bits);
        return fail(VMAT_ERR_ALLOC, "device allocation failed (aperture-dose bound)");
    }
    std::vector<unsigned long long> ph(NPART);
    hipError_t e = hipMemset(bits, 0, (size_t)n * 4);
    const unsigned grid = (unsigned)((h->nb * 64 + 255) / 256);
    const int RC = h->R * h->C;
    if (e == hipSuccess && grid > 0) {
        switch (h->d_store) {
            case VMAT_F32: k_beam_voxel_bits<FMT_F32><<<grid, 256>>>(h->nb, RC, h->bm.qptr, h->bm.col, h->bm.val, words, bits); break;
            case VMAT_F16: k_beam_voxel_bits<FMT_F16><<<grid, 256>>>(h->nb, RC, h->bm.qptr, h->bm.col, h->bm.val, words, bits); break;
            case VMAT_BF16: k_beam_voxel_bits<FMT_BF16><<<grid, 256>>>(h->nb, RC, h->bm.qptr, h->bm.col, h->bm.val, words, bits); break;
            default: k_beam_voxel_bits<FMT_FP8><<<grid, 256>>>(h->nb, RC, h->bm.qptr, h->bm.col, h->bm.val, words, bits); break;
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        k_popcount<<<NPART, AP_T>>>(n, bits, part);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(ph.data(), part, NPART * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    (void)hipFree(bits);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(VMAT_ERR_DEVICE, std::string("aperture-dose bound: ") + hipGetErrorString(e));
    unsigned long long t = 0;
    for (unsigned long long v : ph) t += v;
    *U = (int64_t)t;
    return VMAT_OK;
}

// The store at its final size: U + nv entries, where U bounds the entries of
// any aperture set (beam_voxel_bound) and the extra dose vector is the room an
// append needs before the previous aperture's count reaches the host.  So no
// plan ever grows the store.
vmat_status ap_reserve(vmat_ctx* h) {
    if (h->ap) return VMAT_OK;
    int64_t U = 0;
    vmat_status rc = beam_voxel_bound(h, &U);
    if (rc != VMAT_OK) return rc;
    const int64_t cap = std::max<int64_t>(1, U + h->nv);
    if (cap >= ((int64_t)1 << 32)) return fail(VMAT_ERR_UNSUPPORTED, "aperture doses would exceed 2^32 entries");
    ApDose* a = new ApDose();
    h->ap = a;
    const int64_t nch = n_chunks_of(h->nv);
    auto A = [&](auto** p, size_t n) { if (rc == VMAT_OK) rc = ap_alloc(a, p, n); };
    A(&a->col_ptr, (size_t)h->N + 1);
    A(&a->beam_slot, (size_t)h->N);
    A(&a->vx_ptr[0], (size_t)h->nv + 1);
    A(&a->vx_ptr[1], (size_t)h->nv + 1);
    A(&a->chunk, (size_t)nch + 2);
    A(&a->shift, (size_t)h->nv);
    A(&a->unit, (size_t)h->N + 1);  // unit[N] keeps the beam index being stored
    A(&a->view, 1);
    if (rc == VMAT_OK) rc = ap_alloc_entries(a, cap);
    if (rc == VMAT_OK && hipHostMalloc((void**)&a->total_host, sizeof(uint32_t)) != hipSuccess) {
        a->total_host = nullptr;
        rc = fail(VMAT_ERR_ALLOC, "pinned host allocation failed");
    }
    if (rc == VMAT_OK && hipEventCreateWithFlags(&a->counted, hipEventDisableTiming) != hipSuccess) {
        a->counted = nullptr;
        rc = fail(VMAT_ERR_DEVICE, "event creation failed");
    }
    h->bytes += a->bytes;
    if (rc != VMAT_OK) {
        free_apdose(h);
        return rc;
    }
    // publish the (empty) store so the view holds valid pointers from the start
    return ap_reset(h, nullptr);
}

// Empty store (reserved by ap_reserve).
vmat_status ap_reset(vmat_ctx* h, hipStream_t st) {
    ApDose* a = h->ap;
    if (!a) return fail(VMAT_ERR_UNSUPPORTED, "aperture-dose store not reserved");
    if (a->pending) VMAT_HIP(hipEventSynchronize(a->counted));
    a->top = 0;
    a->pending = 0;
    a->n_slots = 0;
    a->cur = 0;
    VMAT_HIP(hipMemsetAsync(a->col_ptr, 0, sizeof(uint32_t) * (h->N + 1), st));
    VMAT_HIP(hipMemsetAsync(a->beam_slot, 0xFF, sizeof(int32_t) * h->N, st));
    VMAT_HIP(hipMemsetAsync(a->vx_ptr[0], 0, sizeof(uint32_t) * (h->nv + 1), st));
    return ap_publish(h, st);
}

// Stores the dose of the aperture of one beam: beam_dev (device, e.g. the
// pricing result) or, if null, beam_h.  One dose product plus compaction.
// Nothing waits for the device: the aperture's place in the store comes from
// the device-side aperture pointers, its non-zero count reaches the host one
// append later (through pinned memory and an event that, between two
// column-generation iterations, has long completed), and the store is kept
// at least one dose vector (nv entries) ahead of the counted entries, so no
// aperture can overflow it before its count is known.
vmat_status ap_append(vmat_ctx* h, const int32_t* l, const int32_t* r, const uint8_t* occ,
                      const int32_t* beam_dev, int beam_h, hipStream_t st) {
    ApDose* a = h->ap;
    if (!a) return fail(VMAT_ERR_INVALID_ARG, "aperture doses not initialised");
    if (a->n_slots >= h->N) return fail(VMAT_ERR_INVALID_ARG, "more apertures than beams");
    if (a->pending) {
        VMAT_HIP(hipEventSynchronize(a->counted));
        a->top += *a->total_host;
        a->pending = 0;
    }
    vmat_status rc;
    // cannot happen: the reserved capacity bounds every plan
    if (a->top + h->nv > a->cap) return fail(VMAT_ERR_DEVICE, "aperture-dose store full");
    int32_t* kb = reinterpret_cast<int32_t*>(a->unit + h->N);
    k_ap_unit<<<1, AP_T, 0, st>>>(h->N, beam_dev, beam_h, a->unit, kb);
    VMAT_LAUNCH_CHECK();
    if ((rc = launch_fwd_plan(h, a->unit, l, r, occ, h->dz, Gate{}, st)) != VMAT_OK) return rc;
    const int nch = n_chunks_of(h->nv);
    k_ap_count<<<nch, AP_T, 0, st>>>(h->nv, h->dz, a->chunk);
    VMAT_LAUNCH_CHECK();
    k_ap_scan<<<1, AP_T, 0, st>>>(nch, a->chunk);
    VMAT_LAUNCH_CHECK();
    VMAT_HIP(hipMemcpyAsync(a->total_host, a->chunk + nch, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipEventRecord(a->counted, st));
    a->pending = 1;
    const int c = a->cur, n = 1 - c;
    k_ap_emit<<<nch, AP_T, 0, st>>>(h->nv, nch, h->dz, a->chunk, kb, a->col_ptr, a->n_slots, a->col,
                                    a->vx_ptr[c], a->vx_ptr[n], a->shift, a->vx_beam[n],
                                    a->vx_val[n], a->vx_vox[n]);
    VMAT_LAUNCH_CHECK();
    if (a->top > 0) {
        k_ap_copy<<<(unsigned)((a->top + AP_T - 1) / AP_T), AP_T, 0, st>>>((uint32_t)a->top, a->shift,
                                                                          a->vx_beam[c], a->vx_val[c],
                                                                          a->vx_vox[c], a->vx_beam[n],
                                                                          a->vx_val[n], a->vx_vox[n]);
        VMAT_LAUNCH_CHECK();
    }
    k_ap_slot<<<1, 1, 0, st>>>(a->n_slots, kb, a->chunk, nch, a->col_ptr, a->beam_slot, a->view, view_of(a, n));
    VMAT_LAUNCH_CHECK();
    a->n_slots += 1;
    a->cur = n;
    return VMAT_OK;
}

// A voxel grid that fills the chip's wave slots (256 CUs x 4 SIMDs x 8 waves
// x 64 lanes) at two lanes per voxel.
static bool ap_large_grid(const vmat_ctx* h) {
    constexpr int64_t LANE_SLOTS = 256 * 4 * 8 * 64;
    return 2 * h->nv >= LANE_SLOTS;
}

vmat_status ap_dose(const vmat_ctx* h, const double* vec, double* out, Gate gate, hipStream_t st) {
    const size_t lds = sizeof(double) * h->N;
    if (ap_large_grid(h))
        k_ap_dose<2><<<(unsigned)((2 * h->nv + AP_T - 1) / AP_T), AP_T, lds, st>>>(h->nv, h->N, h->ap->view, vec,
                                                                                 out, gate);
    else
        k_ap_dose<4><<<(unsigned)((4 * h->nv + AP_T - 1) / AP_T), AP_T, lds, st>>>(h->nv, h->N, h->ap->view, vec,
                                                                                 out, gate);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

vmat_status ap_grad(const vmat_ctx* h, const float* w, double* out, int Q, Gate gate, hipStream_t st) {
    if (ap_large_grid(h))
        k_ap_grad<512><<<(unsigned)(h->N * Q), 512, 0, st>>>(h->ap->view, w, Q, out, gate);
    else
        k_ap_grad<256><<<(unsigned)(h->N * Q), 256, 0, st>>>(h->ap->view, w, Q, out, gate);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

}  // namespace vmat
