// Launch wrappers of the hot-path kernels (all asynchronous on `st`).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vmat_internal.h"

namespace vmat {

// x_i = v_k if beamlet i of beam k is exposed (occ_k, l <= c < r), else 0;
// times the per-beamlet FP8 scale when `scale` is given.  Runs only when the gate is open.
vmat_status launch_fluence(const vmat_ctx* h, const double* v, const int32_t* l, const int32_t* r,
                           const uint8_t* occ, const float* scale, double* x, Gate gate,
                           hipStream_t st);

// out_row = sum_e val_e x[col_e] (FP64 accumulation) for every row of A; the
// per-row scale of A multiplies the result when present.  Runs only when the gate is open.
vmat_status launch_spmv(const vmat_ctx* h, const QuadCsr& A, const double* x, double* out,
                        Gate gate, hipStream_t st);
vmat_status launch_spmv(const vmat_ctx* h, const QuadCsr& A, const float* x, double* out,
                        Gate gate, hipStream_t st);

// Dispatch to the tiled or the plain layout.
// forward: out = D^T x (x: fluence, FP8 scale already folded in); adjoint: g = D w.
vmat_status launch_fwd(const vmat_ctx* h, const double* x, double* out, Gate gate, hipStream_t st);
// fluence of the plan (v, l, r, occ) and its dose into out, in two launches
vmat_status launch_fwd_plan(const vmat_ctx* h, const double* v, const int32_t* l, const int32_t* r,
                            const uint8_t* occ, double* out, Gate gate, hipStream_t st);
// picks the quads in flight of the sliced products by timing (at creation)
vmat_status tune_sell(vmat_ctx* h, hipStream_t st);
vmat_status launch_adj(const vmat_ctx* h, const float* w, double* g, Gate gate, hipStream_t st);
// Tiled adjoint up to the slot sums (h->tl.part).
vmat_status launch_adj_slots(const vmat_ctx* h, const float* w, Gate gate, hipStream_t st);
// Partial beam sums per beam in the tiled layout (0: the plain layout, where
// the beam sums are whole).
int beam_parts(const vmat_ctx* h);
// launch_adj followed by the sums of g over the exposed beamlets of each
// occupied beam: bpart[N * max(1, beam_parts(h))], beam k's parts at
// k * beam_parts(h) (the whole sums at k when beam_parts(h) == 0)
vmat_status launch_adj_beams(const vmat_ctx* h, const float* w, double* g, const int32_t* l, const int32_t* r,
                             const uint8_t* occ, double* bpart, Gate gate, hipStream_t st);
vmat_status build_tiled(vmat_ctx* h, const vmat_problem* p, hipStream_t st);
void free_tiled(vmat_ctx* h);
void free_batch(vmat_ctx* h);  // batched-solve state (vmat_batch.hip)

// ---- aperture doses (vmat_apdose.hip)
void free_apdose(vmat_ctx* h);
// allocates the store at the size no plan can exceed (kept until destroy)
vmat_status ap_reserve(vmat_ctx* h);
// empties the reserved store
vmat_status ap_reset(vmat_ctx* h, hipStream_t st);
// stores d_k = D^T 1_{A_k} for beam *beam_dev (device) or beam_h (beam_dev null)
vmat_status ap_append(vmat_ctx* h, const int32_t* l, const int32_t* r, const uint8_t* occ,
                      const int32_t* beam_dev, int beam_h, hipStream_t st);
// out = sum_k vec_k d_k over the stored apertures
vmat_status ap_dose(const vmat_ctx* h, const double* vec, double* out, Gate gate, hipStream_t st);
// gF_k = <d_k, w> (0 for beams without a stored aperture)
// the beam gradient from the stored aperture doses in Q parts per beam:
// out[k*Q + q] (Q = 1: out = gF); Q <= AP_GRAD_PARTS
constexpr int AP_GRAD_PARTS = 8;
vmat_status ap_grad(const vmat_ctx* h, const float* w, double* out, int Q, Gate gate, hipStream_t st);
vmat_status scan_u32_dev(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t st);

// F'(z) into rz (FP32, for the adjoint gather), optional FP32 copies of z and
// F'(z), and block partial sums of F(z) into part slot 0.
vmat_status launch_penalty(const vmat_ctx* h, const double* z, float* z_out, float* dF_out, hipStream_t st);

// sum_k-per-beam sums over apertures: out[k] = sum_{i in A_k} g_i.  Runs only when the gate is open.
vmat_status launch_beam_sums(const vmat_ctx* h, const double* g, const int32_t* l, const int32_t* r,
                             const uint8_t* occ, double* out, Gate gate, hipStream_t st);

// cost[0] = F (from partial slot 0), cost[1] = gamma G(y); dfdy = gF + gamma dG/dy.
vmat_status launch_grad_finish(const vmat_ctx* h, const double* y, const double* gF, double* cost,
                               double* dfdy, hipStream_t st);
// dfdy = gF + gamma dG/dy.
vmat_status launch_dfdy(const vmat_ctx* h, const double* y, const double* gF, double* dfdy, hipStream_t st);
// cost[0] = F only (fluence form).
vmat_status launch_cost_only(const vmat_ctx* h, double* cost, hipStream_t st);

// ---- master iteration pieces (device-resident state in h->ms)
vmat_status launch_master_begin(const vmat_ctx* h, double* y, const uint8_t* occ, int max_iter, int ls_max,
                                double tol, double kkt_ref, int fresh, hipStream_t st);
// first: 0 after a master step, 1 at a fresh start, 2 at a carried-over start.
vmat_status launch_master_grad(const vmat_ctx* h, const double* y, const uint8_t* occ, int first,
                               hipStream_t st);
vmat_status launch_master_dir(const vmat_ctx* h, const double* y, const uint8_t* occ, hipStream_t st);
// a chain of line-search passes, each completing the previous one; the last
// is completed by launch_step_update
vmat_status launch_ls_passes(const vmat_ctx* h, hipStream_t st);
// completes the line search, then the master step (y, previous direction,
// gradient and face) and the dose update with F'(z) and the partial sums of
// F, in one launch; stalls the iteration while the line search is unfinished
vmat_status launch_step_update(const vmat_ctx* h, double* y, hipStream_t st);
// launch_master_grad(first = 0) + launch_master_dir in one launch
// bpart, Q: the beam gradient in parts (launch_adj_beams); Q == 0: gF is whole
vmat_status launch_grad_dir(const vmat_ctx* h, const double* y, const uint8_t* occ, const double* bpart, int Q,
                            hipStream_t st);

// max over eq. 2 pairs of |y_b - y_a| / (theta_b - theta_a) -> out[0]; G(y) -> out[1]
vmat_status launch_max_rate(const vmat_ctx* h, const double* y, double* out, hipStream_t st);

// the handle's gamma (host copy and the device scalar the control kernels read)
vmat_status set_gamma(vmat_ctx* h, double gamma, hipStream_t st);
// captures one master iteration on the handle's plan (mode 0: the master that
// streams D; mode 1: the aperture-dose master, after ap_reserve)
vmat_status capture_master(vmat_ctx* h, int mode);

// ---- pricing
// apply != 0: also occupy the chosen beam in (l, r, occ, y), record the trace
// entry `iter` and set the master's reference scale on the first call.
vmat_status launch_price(const vmat_ctx* h, const double* g, const double* y, const int32_t* l,
                         const int32_t* r, const uint8_t* occ, int32_t* out_beam, double* out_price,
                         double* beam_prices, int apply, int iter, int32_t* lw, int32_t* rw, uint8_t* occw,
                         double* yw, hipStream_t st);
// B plan variants at once: g RHS-contiguous [nb][B]; plan, row, price and
// trace arrays variant-major.  vmask (nullable, device [B]): variants to
// price; iter_v (nullable, device [B]): trace index per variant.
vmat_status launch_price_variants(const vmat_ctx* h, int B, const double* g, const double* y, const int32_t* l,
                                  const int32_t* r, const uint8_t* occ, double* rowS, int32_t* rowl, int32_t* rowr,
                                  double* rowm, double* bprice, int32_t* out_beam, double* out_price,
                                  double* beam_prices, int apply, int iter, int32_t* lw, int32_t* rw, uint8_t* occw,
                                  double* yw, SolveTraceDev tr, hipStream_t st, const uint8_t* vmask = nullptr,
                                  const int32_t* iter_v = nullptr);

}  // namespace vmat
