// Plan variants sharing one D, K at a time: each variant is a full
// column-generation plan (vmat_solve) on one of K plan contexts that read the
// caller's handle's layouts of D, each context on its own host thread and
// stream.  A plan with the master over stored aperture doses is bound by
// launch latency (a chain of small kernels per master iteration), so plans on
// separate streams overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "vmat_internal.h"
#include "vmat_kernels.h"

namespace {

// The weights of variant b: (alpha, beta, T)[j] = table[b][min(label[j], S-1)].
__global__ void k_expand_weights(int64_t nv, int S, const uint8_t* __restrict__ label,
                                 const float* __restrict__ tb, float* __restrict__ alpha,
                                 float* __restrict__ beta, float* __restrict__ T) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nv; j += (int64_t)gridDim.x * blockDim.x) {
        const float* w = tb + min((int)label[j], S - 1) * 3;
        alpha[j] = w[0];
        beta[j] = w[1];
        T[j] = w[2];
    }
}

struct Worker {
    vmat_handle ctx = nullptr;
    hipStream_t stream = nullptr;
    float* w = nullptr;  // [3 nv]: alpha, beta, T of the current variant
    vmat_status rc = VMAT_OK;
    std::string msg;
};

}  // namespace

using namespace vmat;

extern "C" vmat_status vmat_solve_variants(vmat_handle h, const vmat_solve_opts* opts, int32_t B, int32_t n_struct,
                                           const uint8_t* label, const float* table, int32_t K, int32_t* l,
                                           int32_t* r, uint8_t* occ, double* y, vmat_solve_report* rep,
                                           hipStream_t st) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    if (B < 1) return fail(VMAT_ERR_INVALID_ARG, "B must be >= 1");
    if (K < 1 || K > 16) return fail(VMAT_ERR_INVALID_ARG, "K must be in [1, 16]");
    if (n_struct < 1 || n_struct > 256) return fail(VMAT_ERR_INVALID_ARG, "n_struct must be in [1, 256]");
    if (!label || !table || !l || !r || !occ || !y || !rep) return fail(VMAT_ERR_INVALID_ARG, "null argument");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return fail(VMAT_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    vmat_solve_opts so{};
    so.master.max_iter = 200;
    so.master.ls_max_steps = 50;
    so.master.tol_rel = 1e-5;
    if (opts) so = *opts;
    if (so.master_mode != 0 && so.master_mode != 1) return fail(VMAT_ERR_INVALID_ARG, "unknown master mode");
    const int workers = std::min(K, B);
    const int64_t nv = h->nv, N = h->N, NR = (int64_t)h->N * h->R;
    VMAT_HIP(hipStreamSynchronize(st));

    std::vector<Worker> wk((size_t)workers);
    // releases everything the call made, on every path out
    struct Cleanup {
        std::vector<Worker>& w;
        ~Cleanup() {
            for (Worker& x : w) {
                if (x.stream) (void)hipStreamSynchronize(x.stream);
                if (x.ctx) (void)vmat_destroy(x.ctx);
                if (x.w) (void)hipFree(x.w);
                if (x.stream) (void)hipStreamDestroy(x.stream);
            }
        }
    } cleanup{wk};
    for (Worker& x : wk) {
        if (hipMalloc((void**)&x.w, (size_t)3 * nv * sizeof(float)) != hipSuccess) {
            x.w = nullptr;
            return fail(VMAT_ERR_ALLOC, "device allocation failed (variant weights)");
        }
        vmat_status rc = vmat_create_plan(h, st, &x.ctx);
        if (rc != VMAT_OK) return rc;
        if (so.master_mode == 1 && (rc = vmat_reserve_solve(x.ctx)) != VMAT_OK) return rc;
    }
    // The workers' streams are made after the contexts (and the streams the
    // contexts capture their iterations on), one after another, default
    // priority.  Measured on 64 prostate plans at K = 4: 6.35 s this way;
    // 9.4 s with each worker's stream made just before its context, 7.8 s
    // with all of them made before the contexts.
    for (Worker& x : wk) VMAT_HIP(hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking));

    auto run = [&](int t) {
        Worker& x = wk[(size_t)t];
        if (hipSetDevice(h->device) != hipSuccess) {
            x.rc = VMAT_ERR_DEVICE;
            x.msg = "hipSetDevice failed in a worker thread";
            return;
        }
        for (int b = t; b < B; b += workers) {
            float *a = x.w, *be = x.w + nv, *T = x.w + 2 * nv;
            k_expand_weights<<<1024, 256, 0, x.stream>>>(nv, n_struct, label, table + (int64_t)b * n_struct * 3, a,
                                                         be, T);
            int32_t* lb = l + (int64_t)b * NR;
            int32_t* rb = r + (int64_t)b * NR;
            uint8_t* ob = occ + (int64_t)b * N;
            double* yb = y + (int64_t)b * N;
            if (hipGetLastError() != hipSuccess || hipMemsetAsync(lb, 0, NR * 4, x.stream) != hipSuccess ||
                hipMemsetAsync(rb, 0, NR * 4, x.stream) != hipSuccess ||
                hipMemsetAsync(ob, 0, N, x.stream) != hipSuccess ||
                hipMemsetAsync(yb, 0, N * 8, x.stream) != hipSuccess) {
                x.rc = VMAT_ERR_DEVICE;
                x.msg = "launch failed in a worker thread";
                return;
            }
            vmat_status rc = vmat_set_weights(x.ctx, a, be, T, x.stream);
            if (rc == VMAT_OK) rc = vmat_solve(x.ctx, &so, lb, rb, ob, yb, nullptr, &rep[b], nullptr, x.stream);
            if (rc != VMAT_OK && rc != VMAT_ERR_NOT_CONVERGED) {
                x.rc = rc;
                x.msg = vmat_last_error();
                return;
            }
        }
    };
    std::vector<std::thread> threads;
    threads.reserve((size_t)workers);
    for (int t = 0; t < workers; ++t) threads.emplace_back(run, t);
    for (std::thread& th : threads) th.join();
    for (const Worker& x : wk)
        if (x.rc != VMAT_OK) return fail(x.rc, x.msg);
    return VMAT_OK;
}
