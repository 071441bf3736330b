// C-ABI entry points: argument checks, then the kernel sequences of the dose,
// gradient, pricing, master and column-generation calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "vmat_internal.h"
#include "vmat_graph.h"
#include "vmat_kernels.h"

using namespace vmat;

namespace {

#define TRY(x)                          \
    do {                                \
        vmat_status s_ = (x);           \
        if (s_ != VMAT_OK) return s_;   \
    } while (0)

vmat_status check_handle(vmat_handle h) {
    set_error("");
    if (!h) return fail(VMAT_ERR_INVALID_ARG, "null handle");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return fail(VMAT_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    return VMAT_OK;
}

vmat_status check_plan(const double* y, const int32_t* l, const int32_t* r, const uint8_t* occ) {
    if (!y || !l || !r || !occ) return fail(VMAT_ERR_INVALID_ARG, "null plan array (y, l, r or occ)");
    return VMAT_OK;
}

__global__ void k_to_float(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ void k_set_f64(double* p, double v) { *p = v; }

__global__ void k_scale_copy(int64_t n, const double* __restrict__ x, const float* __restrict__ s,
                             double* __restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) o[i] = x[i] * (double)s[i];
}

vmat_status to_float(const double* a, float* b, int64_t n, hipStream_t st) {
    if (n <= 0) return VMAT_OK;
    k_to_float<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, b);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// x as the forward product needs it: the FP8 per-beamlet scale folded in.
vmat_status forward_from_fluence(vmat_ctx* h, const double* x, hipStream_t st) {
    const double* xs = x;
    if (h->bm.scale) {
        k_scale_copy<<<(unsigned)((h->nb + 255) / 256), 256, 0, st>>>(h->nb, x, h->bm.scale, h->x);
        VMAT_LAUNCH_CHECK();
        xs = h->x;
    }
    return launch_fwd(h, xs, h->z, Gate{}, st);
}

vmat_status forward_from_plan(vmat_ctx* h, const double* y, const int32_t* l, const int32_t* r,
                              const uint8_t* occ, double* zout, Gate gate, hipStream_t st) {
    return launch_fwd_plan(h, y, l, r, occ, zout, gate, st);
}

vmat_master_opts defaults(const vmat_master_opts* o) {
    vmat_master_opts d;
    d.max_iter = 200;
    d.ls_max_steps = 50;
    d.tol_rel = 1e-5;
    d.kkt_ref = 0.0;
    if (o) d = *o;
    return d;
}

vmat_status check_opts(const vmat_master_opts& o) {
    if (o.max_iter < 0 || o.ls_max_steps < 1 || !(o.tol_rel >= 0.0) || !std::isfinite(o.tol_rel) ||
        !std::isfinite(o.kkt_ref))
        return fail(VMAT_ERR_INVALID_ARG, "invalid master options");
    return VMAT_OK;
}

// Waits until the device has completed line-search chain `want` of this
// handle (the mirror's count), spinning on the pinned mirror; after about two
// seconds without progress it drains the stream and looks once more.  Then
// copies chain `want`'s state (its mirror slot, which no chain enqueued so far
// writes again) to ms_host.
vmat_status wait_chain(vmat_ctx* h, uint32_t want, hipStream_t st) {
    const MasterMirror* mir = h->mirror;
    auto reached = [&]() {
        return (int32_t)(__atomic_load_n(&mir->seq, __ATOMIC_ACQUIRE) - want) >= 0;
    };
    if (!reached()) {
        const auto t0 = std::chrono::steady_clock::now();
        for (uint32_t spin = 0; !reached(); ++spin) {
            if ((spin & 1023u) == 1023u) {
                if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
                    VMAT_HIP(hipStreamSynchronize(st));
                    if (!reached()) return fail(VMAT_ERR_DEVICE, "master state not signalled by the device");
                    break;
                }
                std::this_thread::yield();
            }
        }
    }
    std::memcpy((void*)h->ms_host, (const void*)&mir->s[want & 1u], sizeof(MasterState));
    return VMAT_OK;
}

// The master state's done flag as a launch gate: open while the solve runs.
Gate master_gate(const vmat_ctx* h) {
    Gate done;
    done.p = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(h->ms) + offsetof(MasterState, done));
    done.mask = 1u;
    return done;
}

// The master (Sec. 2.2) works on the handle's plan: leaf pairs pl/pr,
// occupancy pocc and intensities my, copied in from the caller's arrays by
// the entry points and copied back at the end.
//
// Line search of a direction: its dose (fluence expansion and forward product
// for the master that streams D, the stored aperture doses otherwise), then a
// chain of line-search passes.
vmat_status search(vmat_ctx* h, int mode, hipStream_t s) {
    const Gate done = master_gate(h);
    if (mode == 1) {
        TRY(ap_dose(h, h->md, h->dz, done, s));
    } else {
        TRY(launch_fwd_plan(h, h->md, h->pl, h->pr, h->pocc, h->dz, done, s));
    }
    return launch_ls_passes(h, s);
}

// One master iteration: completion of the line search with the step and the
// dose update, the beam gradient (adjoint with the exposed-beamlet sums, or
// the aperture doses against F'(z)), the gradient with the next direction,
// and the next line search.
vmat_status iteration(vmat_ctx* h, int mode, hipStream_t s) {
    TRY(launch_step_update(h, h->my, s));
    if (mode == 1) {
        TRY(ap_grad(h, h->rz, h->bpart, AP_GRAD_PARTS, master_gate(h), s));
        TRY(launch_grad_dir(h, h->my, h->pocc, h->bpart, AP_GRAD_PARTS, s));
    } else {
        const int Q = beam_parts(h);
        TRY(launch_adj_beams(h, h->rz, h->g, h->pl, h->pr, h->pocc, Q > 0 ? h->bpart : h->mgF, master_gate(h), s));
        TRY(launch_grad_dir(h, h->my, h->pocc, h->bpart, Q, s));
    }
    return search(h, mode, s);
}

int master_kind(int mode) { return mode == 1 ? G_MASTER_AP : G_MASTER_D; }

// Enqueues one master iteration: a replay of the captured graph, or the
// kernels one by one when graphs are off.
vmat_status enqueue_iteration(vmat_ctx* h, int mode, hipStream_t st) {
    if (graphs_off()) return iteration(h, mode, st);
    const hipGraphExec_t g = h->iter_graph[master_kind(mode)];
    if (!g) return fail(VMAT_ERR_DEVICE, "master iteration graph not captured");
    VMAT_HIP(hipGraphLaunch(g, st));
    return VMAT_OK;
}

// The master iterations after the first direction and its line search: each
// replay of the captured iteration is enqueued before the host has read the
// state the previous one left, so the device never waits for the host.  The
// last line-search pass of every chain writes the state and a sequence
// number to pinned host memory, so no copy is enqueued for the host.  A
// replay enqueued after the solve has ended, or while a line search is
// unfinished, does no work beyond the line search (the done flag gates every
// kernel), so the arithmetic is that of one read per iteration.  The pending
// replay at exit finds done == 1 and leaves the state as it is.  h->chains
// counts the chains enqueued; the device's count starts from it at every
// master start, so a value left in the mirror by an earlier master is
// always behind the one waited for.
vmat_status master_loop(vmat_ctx* h, int mode, hipStream_t st) {
    uint32_t want = h->chains;  // the first search's chain
    for (;;) {
        TRY(enqueue_iteration(h, mode, st));
        h->chains += 1;
        TRY(wait_chain(h, want, st));
        if (h->ms_host->done == 1) break;
        want += 1;
    }
    return VMAT_OK;
}

// One master solve on the handle's plan.  fresh == 0: the handle's z, F'(z)
// and g already belong to my (column generation adds apertures at y = 0), so
// no product is needed to start.  mode 1: the iterations run on the stored
// aperture doses (the dose of a direction is sum_k d_k dir_k, the beam
// gradient <d_k, F'(z)>), so no product with D runs inside the master and the
// beamlet prices g are not maintained.
vmat_status run_master(vmat_ctx* h, const vmat_master_opts& o, vmat_master_report* rep, hipStream_t st,
                       int fresh = 1, int mode = 0) {
    TRY(launch_master_begin(h, h->my, h->pocc, o.max_iter, o.ls_max_steps, o.tol_rel, o.kkt_ref, fresh, st));
    if (mode == 1) {
        if (fresh) TRY(ap_dose(h, h->my, h->z, Gate{}, st));
        TRY(launch_penalty(h, h->z, nullptr, nullptr, st));
        TRY(ap_grad(h, h->rz, h->mgF, 1, Gate{}, st));
    } else {
        if (fresh) TRY(forward_from_plan(h, h->my, h->pl, h->pr, h->pocc, h->z, Gate{}, st));
        TRY(launch_penalty(h, h->z, nullptr, nullptr, st));
        if (fresh) TRY(launch_adj(h, h->rz, h->g, Gate{}, st));
        TRY(launch_beam_sums(h, h->g, h->pl, h->pr, h->pocc, h->mgF, Gate{}, st));
    }
    TRY(launch_master_grad(h, h->my, h->pocc, fresh ? 1 : 2, st));
    TRY(launch_master_dir(h, h->my, h->pocc, st));
    TRY(search(h, mode, st));
    h->chains += 1;
    TRY(master_loop(h, mode, st));
    const MasterState& s = *h->ms_host;
    if (rep) {
        rep->iters = s.it;
        rep->converged = s.converged;
        rep->n_forward = s.n_fwd;
        rep->n_adjoint = s.n_adj;
        rep->n_ls_evals = s.n_ls;
        rep->reserved = 0;
        rep->F = s.F;
        rep->gG = s.gG;
        rep->kkt = s.kkt;
        rep->kkt_ref = s.kkt_ref;
    }
    return s.converged ? VMAT_OK : VMAT_ERR_NOT_CONVERGED;
}

// The caller's plan into the handle's plan buffers (y may be null: not copied).
vmat_status plan_in(vmat_ctx* h, const double* y, const int32_t* l, const int32_t* r, const uint8_t* occ,
                    hipStream_t st) {
    const size_t NR = (size_t)h->N * h->R;
    VMAT_HIP(hipMemcpyAsync(h->pl, l, NR * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    VMAT_HIP(hipMemcpyAsync(h->pr, r, NR * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    VMAT_HIP(hipMemcpyAsync(h->pocc, occ, (size_t)h->N, hipMemcpyDeviceToDevice, st));
    if (y) VMAT_HIP(hipMemcpyAsync(h->my, y, (size_t)h->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    return VMAT_OK;
}

// A plan the column-generation loop may resume from (Sec. 2.2): every
// occupied beam has 0 <= l <= r <= C in each row and a finite y >= 0, and,
// with a leaf-speed limit delta >= 0, each leaf of an occupied beam lies
// within delta * (index distance) of the same leaf of the next occupied beam
// (around the circle when circular), as column generation leaves it.
vmat_status check_resume(const vmat_ctx* h, const std::vector<int32_t>& l, const std::vector<int32_t>& r,
                         const std::vector<uint8_t>& occ, const std::vector<double>& y) {
    const int N = h->N, R = h->R, C = h->C;
    for (int k = 0; k < N; ++k) {
        if (!occ[k]) continue;
        if (!std::isfinite(y[k]) || y[k] < 0.0)
            return fail(VMAT_ERR_INVALID_ARG, "resumed plan: y of occupied beam " + std::to_string(k) +
                                                  " is negative or not finite");
        for (int rho = 0; rho < R; ++rho) {
            const int64_t a = (int64_t)k * R + rho;
            if (l[a] < 0 || l[a] > r[a] || r[a] > C)
                return fail(VMAT_ERR_INVALID_ARG, "resumed plan: beam " + std::to_string(k) + " row " +
                                                      std::to_string(rho) + " violates 0 <= l <= r <= C");
        }
    }
    if (h->delta < 0) return VMAT_OK;
    for (int k = 0; k < N; ++k) {
        if (!occ[k]) continue;
        int k2 = -1, dist = 0;
        for (int d = 1; d < N; ++d) {
            int kk = k + d;
            if (kk >= N) {
                if (!h->circular) break;
                kk -= N;
            }
            if (occ[kk]) {
                k2 = kk;
                dist = d;
                break;
            }
        }
        if (k2 < 0) continue;
        const int64_t reach = (int64_t)h->delta * dist;
        for (int rho = 0; rho < R; ++rho) {
            const int64_t a = (int64_t)k * R + rho, b = (int64_t)k2 * R + rho;
            if (std::llabs((int64_t)l[a] - l[b]) > reach || std::llabs((int64_t)r[a] - r[b]) > reach)
                return fail(VMAT_ERR_INVALID_ARG, "resumed plan: beams " + std::to_string(k) + " and " +
                                                      std::to_string(k2) + " row " + std::to_string(rho) +
                                                      " exceed the leaf-speed limit");
        }
    }
    return VMAT_OK;
}

}  // namespace

namespace vmat {

vmat_status set_gamma(vmat_ctx* h, double gamma, hipStream_t st) {
    h->gamma = gamma;
    k_set_f64<<<1, 1, 0, st>>>(h->d_gamma, gamma);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

vmat_status capture_master(vmat_ctx* h, int mode) {
    const GraphKey key = {(uint64_t)mode + 1};
    return capture_graph(h, master_kind(mode), key, [&](hipStream_t s) { return iteration(h, mode, s); });
}

}  // namespace vmat


extern "C" vmat_status vmat_dose(vmat_handle h, const double* y, const int32_t* l, const int32_t* r,
                                 const uint8_t* occ, float* z, hipStream_t st) {
    TRY(check_handle(h));
    TRY(check_plan(y, l, r, occ));
    if (!z) return fail(VMAT_ERR_INVALID_ARG, "null z");
    TRY(forward_from_plan(h, y, l, r, occ, h->z, Gate{}, st));
    return to_float(h->z, z, h->nv, st);
}

extern "C" vmat_status vmat_dose_fluence(vmat_handle h, const double* x, float* z, hipStream_t st) {
    TRY(check_handle(h));
    if (!x || !z) return fail(VMAT_ERR_INVALID_ARG, "null x or z");
    TRY(forward_from_fluence(h, x, st));
    return to_float(h->z, z, h->nv, st);
}

extern "C" vmat_status vmat_forward(vmat_handle h, const double* x, double* z, hipStream_t st) {
    TRY(check_handle(h));
    if (!x || !z) return fail(VMAT_ERR_INVALID_ARG, "null x or z");
    const double* xs = x;
    if (h->bm.scale) {
        k_scale_copy<<<(unsigned)((h->nb + 255) / 256), 256, 0, st>>>(h->nb, x, h->bm.scale, h->x);
        VMAT_LAUNCH_CHECK();
        xs = h->x;
    }
    return launch_fwd(h, xs, z, Gate{}, st);
}

extern "C" vmat_status vmat_adjoint(vmat_handle h, const float* w, double* g, hipStream_t st) {
    TRY(check_handle(h));
    if (!w || !g) return fail(VMAT_ERR_INVALID_ARG, "null w or g");
    return launch_adj(h, w, g, Gate{}, st);
}

extern "C" vmat_status vmat_grad(vmat_handle h, const double* y, const int32_t* l, const int32_t* r,
                                 const uint8_t* occ, double* cost, float* z, float* dFdz, double* g,
                                 double* dfdy, hipStream_t st) {
    TRY(check_handle(h));
    TRY(check_plan(y, l, r, occ));
    if (!cost) return fail(VMAT_ERR_INVALID_ARG, "null cost");
    double* gout = g ? g : h->g;
    TRY(forward_from_plan(h, y, l, r, occ, h->z, Gate{}, st));
    TRY(launch_penalty(h, h->z, z, dFdz, st));
    if (!g && !dfdy) return launch_grad_finish(h, y, h->mgF, cost, nullptr, st);
    TRY(launch_adj(h, h->rz, gout, Gate{}, st));
    TRY(launch_beam_sums(h, gout, l, r, occ, h->mgF, Gate{}, st));
    return launch_grad_finish(h, y, h->mgF, cost, dfdy, st);
}

extern "C" vmat_status vmat_grad_apertures(vmat_handle h, const double* y, const int32_t* l, const int32_t* r,
                                           const uint8_t* occ, const float* w, double* g, double* dfdy,
                                           hipStream_t st) {
    TRY(check_handle(h));
    TRY(check_plan(y, l, r, occ));
    if (!w || !dfdy) return fail(VMAT_ERR_INVALID_ARG, "null w or dfdy");
    double* gout = g ? g : h->g;
    TRY(launch_adj(h, w, gout, Gate{}, st));
    TRY(launch_beam_sums(h, gout, l, r, occ, h->mgF, Gate{}, st));
    return launch_dfdy(h, y, h->mgF, dfdy, st);
}

extern "C" vmat_status vmat_grad_fluence(vmat_handle h, const double* x, double* cost, float* z, float* dFdz,
                                         double* g, hipStream_t st) {
    TRY(check_handle(h));
    if (!x || !cost) return fail(VMAT_ERR_INVALID_ARG, "null x or cost");
    TRY(forward_from_fluence(h, x, st));
    TRY(launch_penalty(h, h->z, z, dFdz, st));
    if (g) TRY(launch_adj(h, h->rz, g, Gate{}, st));
    return launch_cost_only(h, cost, st);
}

extern "C" vmat_status vmat_price(vmat_handle h, const double* g, const double* y, const int32_t* l,
                                  const int32_t* r, const uint8_t* occ, int32_t* out_beam, double* out_price,
                                  double* beam_prices, hipStream_t st) {
    TRY(check_handle(h));
    TRY(check_plan(y, l, r, occ));
    if (!g || !out_beam || !out_price) return fail(VMAT_ERR_INVALID_ARG, "null g or output");
    return launch_price(h, g, y, l, r, occ, out_beam, out_price, beam_prices, 0, 0, nullptr, nullptr, nullptr,
                        nullptr, st);
}

extern "C" vmat_status vmat_layout(vmat_handle h, vmat_layout_info* out) {
    TRY(check_handle(h));
    if (!out) return fail(VMAT_ERR_INVALID_ARG, "null output");
    const int64_t vb = h->d_store == VMAT_F32 ? 4 : (h->d_store == VMAT_FP8_E4M3 ? 1 : 2);
    const int64_t nb = h->nb, nv = h->nv, sc = h->d_store == VMAT_FP8_E4M3 ? 4 * nb : 0;
    vmat_layout_info L = {};
    L.tiled = h->tl.on ? 1 : 0;
    L.weight_labels = h->n_wtab;
    L.fwd_entries = h->vm.n_quads * 4;
    if (h->tl.on) {
        const Tiled& t = h->tl;
        L.n_blocks = t.nblk;
        L.fwd_lanes = 1;  // the sliced products give every row one lane
        L.adj_lanes = 1;
        L.adj_entries = t.a_quads * 4;
        L.slots = t.S;
        L.fwd_bytes = L.fwd_entries * (vb + 2) + 4 * (nv + 1) + 4 * t.S + 8 * nb + 8 * nv;
        L.adj_bytes = L.adj_entries * (vb + 2) + 4 * (t.S + 1) + 4 * nv + 16 * t.S + 4 * (nb + 1) + 4 * t.S +
                      8 * nb + sc;
    } else {
        L.fwd_lanes = h->vm.lanes_per_row;
        L.adj_lanes = h->bm.lanes_per_row;
        L.adj_entries = h->bm.n_quads * 4;
        L.fwd_bytes = L.fwd_entries * (vb + 4) + 4 * (nv + 1) + 8 * nb + 8 * nv;
        L.adj_bytes = L.adj_entries * (vb + 4) + 4 * (nb + 1) + 4 * nv + 8 * nb + sc;
    }
    *out = L;
    return VMAT_OK;
}

extern "C" vmat_status vmat_master(vmat_handle h, const int32_t* l, const int32_t* r, const uint8_t* occ, double* y,
                                   const vmat_master_opts* opts, vmat_master_report* rep, hipStream_t st) {
    TRY(check_handle(h));
    TRY(check_plan(y, l, r, occ));
    const vmat_master_opts o = defaults(opts);
    TRY(check_opts(o));
    TRY(plan_in(h, y, l, r, occ, st));
    const vmat_status rc = run_master(h, o, rep, st);
    if (rc != VMAT_OK && rc != VMAT_ERR_NOT_CONVERGED) return rc;
    VMAT_HIP(hipMemcpyAsync(y, h->my, (size_t)h->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    // the replay enqueued after the last iteration does nothing, but the call
    // returns with the stream drained
    VMAT_HIP(hipStreamSynchronize(st));
    return rc;
}

extern "C" vmat_status vmat_reserve_solve(vmat_handle h) {
    TRY(check_handle(h));
    if (h->ap) return VMAT_OK;
    VMAT_HIP(hipDeviceSynchronize());
    TRY(ap_reserve(h));
    vmat_status rc = capture_master(h, 1);
    if (rc == VMAT_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(VMAT_ERR_DEVICE, "vmat_reserve_solve: device synchronisation failed");
    if (rc != VMAT_OK) {
        free_apdose(h);
        return rc;
    }
    return VMAT_OK;
}

extern "C" vmat_status vmat_solve(vmat_handle h, const vmat_solve_opts* opts, int32_t* l, int32_t* r, uint8_t* occ,
                                  double* y, float* z, vmat_solve_report* rep, vmat_solve_trace* trace,
                                  hipStream_t st) {
    TRY(check_handle(h));
    TRY(check_plan(y, l, r, occ));
    vmat_solve_opts so;
    so.max_cg_iter = 0;
    so.master_mode = 0;
    so.master = defaults(nullptr);
    if (opts) so = *opts;
    TRY(check_opts(so.master));
    if (so.master_mode != 0 && so.master_mode != 1) return fail(VMAT_ERR_INVALID_ARG, "master_mode must be 0 or 1");
    const int mode = so.master_mode;
    if (mode == 1 && !h->ap)
        return fail(VMAT_ERR_UNSUPPORTED, "master_mode 1 needs the aperture-dose store: call vmat_reserve_solve first");
    const int N = h->N;
    const size_t NR = (size_t)N * h->R;
    std::vector<uint8_t> occ_h(N);
    std::vector<int32_t> l_h(NR), r_h(NR);
    std::vector<double> y_h(N);
    VMAT_HIP(hipMemcpyAsync(occ_h.data(), occ, N, hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipMemcpyAsync(l_h.data(), l, NR * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipMemcpyAsync(r_h.data(), r, NR * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipMemcpyAsync(y_h.data(), y, N * sizeof(double), hipMemcpyDeviceToHost, st));
    VMAT_HIP(hipStreamSynchronize(st));
    TRY(check_resume(h, l_h, r_h, occ_h, y_h));
    int n_occ = 0;
    for (uint8_t o : occ_h) n_occ += o ? 1 : 0;
    int iters = N - n_occ;
    if (so.max_cg_iter > 0) iters = std::min(iters, so.max_cg_iter);
    TRY(plan_in(h, y, l, r, occ, st));

    vmat_solve_report R = {};
    std::vector<double> costs(iters + 1, 0.0);
    std::vector<int32_t> miters(iters, 0);
    double ref = so.master.kkt_ref;
    vmat_master_report mr{};
    // D products of one master solve: in mode 0 each direction takes a
    // forward and each step an adjoint; in mode 1 the master runs on the
    // aperture doses and the column-generation loop adds the products
    auto count = [&](const vmat_master_report& m) {
        R.master_iters += m.iters;
        R.n_ls_evals += m.n_ls_evals;
        if (mode == 0) {
            R.n_forward += m.n_forward;
            R.n_adjoint += m.n_adjoint;
        }
    };
    if (mode == 1) TRY(ap_reset(h, st));
    if (n_occ > 0) {
        if (mode == 1) {
            for (int k = 0; k < N; ++k)
                if (occ_h[k]) {
                    TRY(ap_append(h, h->pl, h->pr, h->pocc, nullptr, k, st));
                    R.n_forward += 1;
                }
        }
        vmat_status rc = run_master(h, so.master, &mr, st, 1, mode);
        if (rc != VMAT_OK && rc != VMAT_ERR_NOT_CONVERGED) return rc;
        if (rc == VMAT_ERR_NOT_CONVERGED) R.not_converged++;
        count(mr);
        if (mode == 1 && iters > 0) {
            TRY(launch_adj(h, h->rz, h->g, Gate{}, st));
            R.n_adjoint += 1;
        }
        if (!(ref > 0.0)) ref = mr.kkt_ref;
        costs[0] = mr.F + mr.gG;
    } else {
        VMAT_HIP(hipMemsetAsync(h->z, 0, h->nv * sizeof(double), st));
        TRY(launch_penalty(h, h->z, nullptr, nullptr, st));
        TRY(launch_adj(h, h->rz, h->g, Gate{}, st));
        TRY(launch_cost_only(h, h->cost2, st));
        R.n_adjoint += 1;
        double c0 = 0.0;
        VMAT_HIP(hipMemcpyAsync(&c0, h->cost2, sizeof(double), hipMemcpyDeviceToHost, st));
        VMAT_HIP(hipStreamSynchronize(st));
        costs[0] = c0;
    }
    for (int t = 0; t < iters; ++t) {
        TRY(launch_price(h, h->g, h->my, h->pl, h->pr, h->pocc, h->pbeam, h->pscore, nullptr, 1, t, h->pl, h->pr,
                         h->pocc, h->my, st));
        if (!(ref > 0.0)) {
            double ps[3];
            VMAT_HIP(hipMemcpyAsync(ps, h->pscore, sizeof(ps), hipMemcpyDeviceToHost, st));
            VMAT_HIP(hipStreamSynchronize(st));
            ref = ps[0] != 0.0 && std::isfinite(ps[0]) ? std::fabs(ps[0]) : 1.0;
        }
        if (mode == 1) {
            TRY(ap_append(h, h->pl, h->pr, h->pocc, h->pbeam, -1, st));
            R.n_forward += 1;
        }
        vmat_master_opts mo = so.master;
        mo.kkt_ref = ref;
        vmat_status rc = run_master(h, mo, &mr, st, /*fresh=*/0, mode);
        if (rc != VMAT_OK && rc != VMAT_ERR_NOT_CONVERGED) return rc;
        if (rc == VMAT_ERR_NOT_CONVERGED) R.not_converged++;
        count(mr);
        if (mode == 1 && t + 1 < iters) {
            // beamlet prices for the next pricing
            TRY(launch_adj(h, h->rz, h->g, Gate{}, st));
            R.n_adjoint += 1;
        }
        costs[t + 1] = mr.F + mr.gG;
        miters[t] = mr.iters;
        R.cg_iters = t + 1;
        R.F = mr.F;
        R.gG = mr.gG;
    }
    if (iters == 0 && n_occ > 0) {
        R.F = mr.F;
        R.gG = mr.gG;
    }
    R.kkt_ref = ref;
    VMAT_HIP(hipMemcpyAsync(l, h->pl, NR * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    VMAT_HIP(hipMemcpyAsync(r, h->pr, NR * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    VMAT_HIP(hipMemcpyAsync(occ, h->pocc, (size_t)N, hipMemcpyDeviceToDevice, st));
    VMAT_HIP(hipMemcpyAsync(y, h->my, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (z) TRY(to_float(h->z, z, h->nv, st));
    if (trace) {
        const int n = R.cg_iters;
        if (trace->beam && n) VMAT_HIP(hipMemcpyAsync(trace->beam, h->tr.beam, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        if (trace->price && n) VMAT_HIP(hipMemcpyAsync(trace->price, h->tr.price, n * sizeof(double), hipMemcpyDeviceToHost, st));
        if (trace->margin && n) VMAT_HIP(hipMemcpyAsync(trace->margin, h->tr.margin, n * sizeof(double), hipMemcpyDeviceToHost, st));
        if (trace->row_margin && n)
            VMAT_HIP(hipMemcpyAsync(trace->row_margin, h->tr.row_margin, n * sizeof(double), hipMemcpyDeviceToHost, st));
        if (trace->y && n)
            VMAT_HIP(hipMemcpyAsync(trace->y, h->tr.y, (size_t)n * N * sizeof(double), hipMemcpyDeviceToHost, st));
        VMAT_HIP(hipStreamSynchronize(st));
        if (trace->cost) std::copy(costs.begin(), costs.begin() + n + 1, trace->cost);
        if (trace->master_iters) std::copy(miters.begin(), miters.begin() + n, trace->master_iters);
    }
    VMAT_HIP(hipStreamSynchronize(st));
    if (rep) *rep = R;
    return VMAT_OK;
}

extern "C" vmat_status vmat_enforce_rate(vmat_handle h, const vmat_rate_opts* opts, const int32_t* l,
                                         const int32_t* r, const uint8_t* occ, double* y, vmat_rate_report* rep,
                                         hipStream_t st) {
    TRY(check_handle(h));
    TRY(check_plan(y, l, r, occ));
    if (!opts || !rep) return fail(VMAT_ERR_INVALID_ARG, "null options or report");
    if (!(opts->rate_max >= 0.0) || !std::isfinite(opts->rate_max))
        return fail(VMAT_ERR_INVALID_ARG, "rate_max must be finite and >= 0");
    if (!(opts->factor > 1.0) || !std::isfinite(opts->factor)) return fail(VMAT_ERR_INVALID_ARG, "factor must be > 1");
    if (opts->max_rounds < 0) return fail(VMAT_ERR_INVALID_ARG, "max_rounds must be >= 0");
    vmat_master_opts mo = opts->master;
    if (mo.max_iter <= 0) mo.max_iter = 200;
    if (mo.ls_max_steps <= 0) mo.ls_max_steps = 50;
    if (!(mo.tol_rel > 0.0)) mo.tol_rel = 1e-5;
    TRY(check_opts(mo));
    TRY(plan_in(h, y, l, r, occ, st));
    vmat_rate_report R = {};
    const double gamma0 = h->gamma;
    double g_now = gamma0;
    double rate_G[2];
    auto read_rate = [&]() -> vmat_status {
        TRY(launch_max_rate(h, h->my, h->cost2, st));
        VMAT_HIP(hipMemcpyAsync(rate_G, h->cost2, sizeof(rate_G), hipMemcpyDeviceToHost, st));
        VMAT_HIP(hipStreamSynchronize(st));
        return VMAT_OK;
    };
    // unoccupied beams carry y = 0 (as in the master) before the first check
    TRY(launch_master_begin(h, h->my, h->pocc, 1, 1, 1.0, 0.0, 1, st));
    TRY(read_rate());
    vmat_status rc = VMAT_OK;
    while (rate_G[0] > opts->rate_max && R.rounds < opts->max_rounds) {
        g_now *= opts->factor;
        if ((rc = set_gamma(h, g_now, st)) != VMAT_OK) break;
        vmat_master_report mr{};
        rc = run_master(h, mo, &mr, st, R.rounds == 0 ? 1 : 0);
        if (rc != VMAT_OK && rc != VMAT_ERR_NOT_CONVERGED) break;
        if (rc == VMAT_ERR_NOT_CONVERGED) R.not_converged++;
        rc = VMAT_OK;
        R.rounds++;
        R.master_iters += mr.iters;
        R.F = mr.F;
        R.gG = mr.gG;
        if ((rc = read_rate()) != VMAT_OK) break;
    }
    const vmat_status rg = set_gamma(h, gamma0, st);
    if (rc != VMAT_OK) return rc;
    if (rg != VMAT_OK) return rg;
    VMAT_HIP(hipMemcpyAsync(y, h->my, (size_t)h->N * sizeof(double), hipMemcpyDeviceToDevice, st));
    VMAT_HIP(hipStreamSynchronize(st));
    R.gamma = g_now;
    R.rate = rate_G[0];
    R.feasible = rate_G[0] <= opts->rate_max ? 1 : 0;
    if (R.rounds == 0) R.gG = g_now * rate_G[1];
    *rep = R;
    return VMAT_OK;
}
