/*
 * vmat.h - C ABI of the MI355X (gfx950) column-generation VMAT hot path.
 *
 * The problem is the paper's model (Sec. 2.1, eq. 1-3):
 *   N beams sorted by angle theta_k in [0, 360) degrees; beam k has R leaf rows
 *   of C beamlets; beamlet i = (k*R + rho)*C + c, nb = N*R*C.
 *   D (nb x nv, row = beamlet, column = voxel) holds the dose-deposition
 *   coefficients D_ij >= 0.  An aperture A_k is one open interval
 *   [l_{k,rho}, r_{k,rho}) of columns per leaf row (l == r: closed row) and
 *   exists only when occ[k] != 0; y_k >= 0 is its intensity.
 *   Dose:      z_j = sum_k y_k sum_{i in A_k} D_ij                    (eq. 3)
 *   Penalty:   F(z) = sum_j a_j max(0,T_j-z_j)^2 + b_j max(0,z_j-T_j)^2 (eq. 1)
 *   Smoothing: G(y) = sum_k (y_{k+1}-y_k)^2 / (theta_{k+1}-theta_k)    (eq. 2)
 *              plus the pair (N,1) with gap theta_1+360-theta_N when circular.
 *   Model:     min F(z) + gamma G(y), y >= 0                           (eq. 3)
 *
 * Conventions for every call
 *   - "DEVICE" pointers are HIP device memory of the current device; "HOST"
 *     pointers are ordinary host memory.  The caller owns every pointer it
 *     passes; the library keeps none of them after the call returns.
 *   - Work is ordered on the given stream.  vmat_dose, vmat_grad, vmat_price
 *     and the *_fluence calls are asynchronous; vmat_create, vmat_master and
 *     vmat_solve synchronise the stream before they return.
 *   - Every call returns a vmat_status and never aborts.  Arguments are
 *     checked before any launch, so VMAT_ERR_INVALID_ARG leaves outputs
 *     untouched.  vmat_last_error() gives a text for the last failure on the
 *     calling thread.
 *   - A handle is not thread-safe; distinct handles are independent.  Device
 *     memory is allocated by vmat_create (D's layouts, work buffers and the
 *     captured iteration of the master that streams D), by vmat_create_plan
 *     (the same without D, which it reads from its source), by
 *     vmat_solve_variants (its worker contexts, for the call), by vmat_reserve_solve
 *     (the aperture-dose store at the size no plan exceeds, and the captured
 *     iteration of the aperture-dose master) and by vmat_reserve_batched
 *     (batched state); vmat_destroy releases all of it.  The dose, gradient,
 *     pricing, product, master and column-generation calls allocate no device
 *     memory: they work on the handle's own copy of the plan (copied in from
 *     the caller's arrays and back out at the end).
 */
#ifndef VMAT_H
#define VMAT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vmat_status;
enum {
    VMAT_OK = 0,
    VMAT_ERR_INVALID_ARG = 1,   /* bad pointer, size or value; nothing was launched   */
    VMAT_ERR_DEVICE = 2,        /* a HIP call failed; text in vmat_last_error()       */
    VMAT_ERR_ALLOC = 3,         /* device allocation in vmat_create failed            */
    VMAT_ERR_NOT_CONVERGED = 4, /* master hit its iteration cap; outputs are valid    */
    VMAT_ERR_UNSUPPORTED = 5    /* option not available (e.g. n_cols > 64)            */
};

/* Storage of the library's device copies of D.  Accumulation is FP64 for every
 * format; the reduced formats are the only approximation.                      */
typedef enum {
    VMAT_F32 = 0,       /* D as given                                            */
    VMAT_F16 = 1,       /* IEEE half, round to nearest even                      */
    VMAT_BF16 = 2,      /* bfloat16, round to nearest even                       */
    VMAT_FP8_E4M3 = 3   /* OCP FP8 E4M3 with a per-beamlet FP32 scale            */
                        /* s_i = max_j D_ij / 448, code = RNE(D_ij / s_i)          */
} vmat_dtype;

typedef struct vmat_ctx* vmat_handle;

typedef struct vmat_problem {
    int32_t n_beams;          /* N >= 1                                                  */
    int32_t n_rows;           /* R >= 1 leaf rows per beam                               */
    int32_t n_cols;           /* C, 1 <= C <= 64 beamlets per row                        */
    int32_t d_store;          /* vmat_dtype                                              */
    int64_t n_voxels;         /* nv >= 1, < 2^31                                          */
    int64_t nnz;              /* non-zeros of D, < 2^33                                   */
    const double* theta_deg;  /* HOST [N] strictly increasing, in [0, 360)                */
    const int64_t* row_ptr;   /* DEVICE [nb+1] beamlet-major CSR; row_ptr[0]=0, [nb]=nnz */
    const int32_t* col;       /* DEVICE [nnz] voxel index in [0,nv), ascending per row   */
    const float* val;         /* DEVICE [nnz] D_ij, finite, >= 0                          */
    const float* alpha;       /* DEVICE [nv] underdose weight, finite, >= 0  (eq. 1)       */
    const float* beta;        /* DEVICE [nv] overdose weight, finite, >= 0   (eq. 1)       */
    const float* T;           /* DEVICE [nv] threshold dose, finite          (eq. 1)       */
    double gamma;             /* smoothing weight, finite, >= 0 (eq. 3; the paper: > 0)   */
    int32_t circular;         /* 0: open chain of eq. 2; 1: add the wrap pair (N,1)       */
    int32_t max_leaf_step;    /* delta: columns a leaf may move per beam index step when  */
                              /* a new aperture is priced; < 0 means unconstrained        */
    int32_t layout;           /* device layout of D: 0 auto (tiled when every voxel block */
                              /* fits, else plain), 1 plain quad CSR, 2 tiled (fails with */
                              /* VMAT_ERR_UNSUPPORTED when a block does not fit)          */
    int32_t reserved;
} vmat_problem;

/* Copies D, alpha, beta, T into the library's own device layouts (beamlet-major
 * and voxel-major quad CSR, and the tiled and sliced forms of both products,
 * in d_store precision) and validates them (one pass; invalid data gives
 * VMAT_ERR_INVALID_ARG).  With the sliced forms it also times each product
 * with 4 and 8 quads in flight per lane (a few launches on zero operands) and
 * keeps the faster; the choice changes no result.  The caller may free its
 * arrays afterwards.                                                          */
vmat_status vmat_create(const vmat_problem* prob, hipStream_t stream, vmat_handle* out);
vmat_status vmat_destroy(vmat_handle h);
const char* vmat_last_error(void);
/* Device bytes held by the handle (all layouts and work buffers). */
vmat_status vmat_device_bytes(vmat_handle h, int64_t* bytes);

/* Plan variants on one handle: replaces the voxel weights and thresholds of
 * eq. 1 (alpha, beta, T: DEVICE float [nv], the same rules as in
 * vmat_problem).  D, the beams and gamma stay.  The weights are checked before
 * anything changes (VMAT_ERR_INVALID_ARG leaves the handle as it was).  A
 * handle whose weights were held as one-byte labels (at most 256 distinct
 * (alpha, beta, T), see vmat_layout_info.weight_labels) keeps that form and
 * returns VMAT_ERR_UNSUPPORTED, unchanged, for weights with more distinct
 * triples.  Allocates nothing; the captured master iterations stay valid.
 * Synchronises the stream.                                                    */
vmat_status vmat_set_weights(vmat_handle h, const float* alpha, const float* beta, const float* T,
                             hipStream_t stream);

/* Plan variants sharing one D: a second handle (a plan context) that reads
 * src's device layouts of D and owns everything else a plan needs: a copy of
 * src's current voxel weights (vmat_set_weights changes only this context's),
 * gamma, the work buffers, the plan, the master state and its captured
 * iteration, and what vmat_reserve_solve / vmat_reserve_batched add to it.
 * Every call that takes a handle takes a context, with the same results as on
 * src; contexts on different streams run concurrently (each is, like any
 * handle, used from one thread at a time).  Allocates the context's state
 * (about 37 bytes per voxel, 16 per beamlet and 8 per slot of the tiled
 * adjoint), not D; vmat_device_bytes counts that state only.  A context made
 * from a context reads the same owner's D.  The owner outlives its contexts:
 * vmat_destroy on a handle whose layouts a live context reads returns
 * VMAT_ERR_INVALID_ARG and frees nothing.  Synchronises the stream.         */
vmat_status vmat_create_plan(vmat_handle src, hipStream_t stream, vmat_handle* out);

/* The device layout of D chosen by vmat_create and the bytes one product has to
 * move through HBM with it (the figure the achieved bandwidth is quoted on):
 * stored entries x (value + index bytes), row pointers, the gathered vector
 * read once, the output written once, and for the tiled layout the per-block
 * beamlet lists, the slot sums (written and read) and their index map.        */
typedef struct vmat_layout_info {
    int32_t tiled;          /* 1: tiled layout (LDS-staged gathers), 0: plain quad CSR   */
    int32_t n_blocks;       /* voxel blocks of the tiled layout                          */
    int32_t fwd_lanes;      /* lanes per row of the forward: 1 in the tiled layout (its   */
                            /* sliced kernels give every row one lane), else the plain    */
                            /* layout's lane group                                        */
    int32_t adj_lanes;      /* lanes per row of the adjoint, likewise                     */
    int64_t fwd_entries;    /* stored entries of the forward layout, padding included     */
    int64_t adj_entries;    /* stored entries of the adjoint layout, padding included     */
    int64_t slots;          /* (block, beamlet) pairs of the tiled layout                 */
    int64_t fwd_bytes;      /* HBM bytes one vmat_forward moves with this layout          */
    int64_t adj_bytes;      /* HBM bytes one vmat_adjoint moves with this layout          */
    int32_t weight_labels;  /* distinct (alpha, beta, T) held as one-byte voxel labels    */
                            /* for the master's voxel passes (at most 256); 0: per-voxel  */
                            /* weights (more than 256 distinct, or VMAT_NO_WEIGHT_LABELS  */
                            /* set in the environment at vmat_create)                     */
    int32_t reserved;
} vmat_layout_info;
vmat_status vmat_layout(vmat_handle h, vmat_layout_info* out);

/* Dose of a plan (Sec. 2.1; the constraint of eq. 3):
 *   z_j = sum_k y_k sum_{i in A_k} D_ij, accumulated in FP64, stored as FP32.
 * y: DEVICE double [N]; l, r: DEVICE int32 [N*R]; occ: DEVICE uint8 [N];
 * z: DEVICE float [nv] (out).  Leaf pairs are meant to satisfy
 * 0 <= l <= r <= C; other values are not rejected: a row then exposes the
 * columns c in [0, C) with l <= c < r (no memory is touched outside the
 * arrays).                                                                   */
vmat_status vmat_dose(vmat_handle h, const double* y, const int32_t* l, const int32_t* r,
                      const uint8_t* occ, float* z, hipStream_t stream);

/* Cost and gradient of a plan (eq. 1-3; the KKT prices of Sec. 2.2):
 *   cost[0] = F(z), cost[1] = gamma G(y)                 DEVICE double [2]
 *   z    (nullable) DEVICE float  [nv] dose
 *   dFdz (nullable) DEVICE float  [nv] F'(z_j) = 2b(z-T)+ - 2a(T-z)+
 *   g    (nullable) DEVICE double [nb] beamlet prices g_i = sum_j D_ij F'(z_j)
 *   dfdy (nullable) DEVICE double [N]  sum_{i in A_k} g_i + gamma dG/dy_k
 * Inputs as for vmat_dose.  With g and dfdy both null no adjoint product runs. */
vmat_status vmat_grad(vmat_handle h, const double* y, const int32_t* l, const int32_t* r,
                      const uint8_t* occ, double* cost, float* z, float* dFdz, double* g,
                      double* dfdy, hipStream_t stream);

/* Gradient in the aperture intensities for a given dose derivative w = F'(z):
 *   dfdy[k] = sum_{i in A_k} (D w)_i + gamma dG/dy_k   (eq. 2, eq. 3)
 *   w: DEVICE float [nv]; g (nullable): DEVICE double [nb] receives D w;
 *   dfdy: DEVICE double [N].  This is the backward of vmat_grad's cost.      */
vmat_status vmat_grad_apertures(vmat_handle h, const double* y, const int32_t* l, const int32_t* r,
                                const uint8_t* occ, const float* w, double* g, double* dfdy,
                                hipStream_t stream);

/* Fluence-space forms (beamlet intensities x instead of apertures):
 *   vmat_dose_fluence:  z = D^T x                   x: DEVICE double [nb]
 *   vmat_grad_fluence:  cost[0] = F(D^T x); z, dFdz, g as in vmat_grad (nullable)
 * These carry the derivative of the dose and cost with respect to x.          */
vmat_status vmat_dose_fluence(vmat_handle h, const double* x, float* z, hipStream_t stream);
vmat_status vmat_grad_fluence(vmat_handle h, const double* x, double* cost, float* z,
                              float* dFdz, double* g, hipStream_t stream);

/* Raw products (the adjoint of the tiled layout adds a per-beamlet reduction;
 * FP8 storage adds a scaling pass to the forward):
 *   vmat_forward:  z = D^T x      x: DEVICE double [nb],  z: DEVICE double [nv]
 *   vmat_adjoint:  g = D w        w: DEVICE float  [nv],  g: DEVICE double [nb]
 * FP64 accumulation; the forward is the dose of eq. 3 for beamlet
 * intensities x, the adjoint gives the beamlet prices of Sec. 2.2 for w = F'(z). */
vmat_status vmat_forward(vmat_handle h, const double* x, double* z, hipStream_t stream);
vmat_status vmat_adjoint(vmat_handle h, const float* w, double* g, hipStream_t stream);

/* Plan variants sharing one D (many right-hand sides, one SpMM per product).
 * The variants differ in the voxel weights and thresholds of eq. 1; the dose
 * of eq. 3 and the beamlet prices of Sec. 2.2 are the same linear maps applied
 * to B columns at once.  RHS-contiguous layout: element (row, b) at row*B + b.
 *   vmat_forward_batched:  Z = D^T X   X: DEVICE float [nb*B], Z: DEVICE double [nv*B]
 *   vmat_adjoint_batched:  G = D W     W: DEVICE float [nv*B], G: DEVICE double [nb*B]
 *   vmat_grad_batched:     Z = D^T X; cost[b] = F_b(Z[:, b]) (eq. 1 with the
 *       weights of variant b); dF[j*B+b] = F_b'(Z[j, b]) (float); G = D dF
 *       (skipped when G is null).
 *       label: DEVICE uint8 [nv], the structure of each voxel, 0..n_struct-1
 *              (larger labels are read as n_struct-1);
 *       table: DEVICE float [B][n_struct][3] = (alpha, beta, T) per variant
 *              and structure; cost: DEVICE double [B]; dF: DEVICE float [nv*B]
 *   vmat_tune_batched: times every product variant for both products on the
 *       given buffers, reps launches each, and keeps the fastest of each for
 *       later calls with this B.  A variant is (TB, RPW): TB right-hand sides
 *       per pass over a row of D and RPW rows per wavefront (64 / RPW lanes
 *       per row, each with TB * RPW / 64 consecutive right-hand sides), in
 *       this order: (1,64) (2,32) (4,16) (8,8) (16,4) (16,8) (32,2) (32,4)
 *       (32,8) (64,1) (64,2) (64,4) (64,8).  Variants with TB >= 2B, or whose
 *       per-lane count does not divide B, are skipped (time +inf); the plain
 *       layout has one variant per TB (RPW = 64 / TB).
 *       best: HOST int32 [4] (forward TB, RPW, adjoint TB, RPW);
 *       times_ms: HOST float [26] (nullable): forward then adjoint, per variant.
 *   vmat_set_batched_tile: sets the variants used at B right-hand sides
 *       ((0, 0) = default; otherwise a listed pair), e.g. from an earlier tuning.
 * 1 <= B <= 64, 1 <= n_struct <= 16, FP64 accumulation, any storage format.
 * Results are deterministic (no atomics).  Variants change no result.  In
 * the tiled layout the adjoint sums each beamlet per voxel block first, which
 * needs the state of vmat_reserve_batched (without it the plain beamlet-major
 * rows are used: rounding-level differences).  Each XCD of the GPU walks its
 * own range of voxel blocks, so the right-hand sides a block gathers stay in
 * that XCD's L2.                                                              */
vmat_status vmat_forward_batched(vmat_handle h, int32_t B, const float* X, double* Z,
                                 hipStream_t stream);
vmat_status vmat_adjoint_batched(vmat_handle h, int32_t B, const float* W, double* G,
                                 hipStream_t stream);
vmat_status vmat_grad_batched(vmat_handle h, int32_t B, int32_t n_struct, const uint8_t* label,
                              const float* table, const float* X, double* Z, double* cost,
                              float* dF, double* G, hipStream_t stream);
vmat_status vmat_set_batched_tile(vmat_handle h, int32_t B, int32_t fwd_tile, int32_t fwd_rpw, int32_t adj_tile,
                                  int32_t adj_rpw);
vmat_status vmat_tune_batched(vmat_handle h, int32_t B, const float* X, double* Z, const float* W,
                              double* G, int32_t reps, int32_t* best, float* times_ms,
                              hipStream_t stream);

/* Pricing (Sec. 2.2): the best deliverable aperture over the unoccupied beams.
 * Per unoccupied beam and leaf row, one left-to-right pass minimises
 * S(l,r) = sum_{c=l}^{r-1} g_c over leaf pairs within delta*(index distance)
 * of the nearest occupied beam on each side (key (S, r-l, l); the best left
 * end for a right end is the largest running prefix sum, ties to the later l).
 * Beam price p_k = sum_rho S*_rho + gamma dG/dy_k at y_k = 0; the chosen beam
 * is the smallest k with the least p_k.
 *   g: DEVICE double [nb]; y, l, r, occ: current plan (DEVICE, as above)
 *   out_beam:  DEVICE int32 [1 + 2R]: k* (-1 if all occupied), l*[R], r*[R]
 *   out_price: DEVICE double [3]: p_k*, second-best p minus p_k* (inf if none),
 *              least gap in any row of k* between S* and a different S value
 *   beam_prices (nullable): DEVICE double [N], +inf for occupied beams          */
vmat_status vmat_price(vmat_handle h, const double* g, const double* y, const int32_t* l,
                       const int32_t* r, const uint8_t* occ, int32_t* out_beam,
                       double* out_price, double* beam_prices, hipStream_t stream);

/* Pricing without a handle and without allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  The same computation and results, bit
 * for bit, as vmat_price on a handle built with the same beams, gamma,
 * circular and max_leaf_step; the beam geometry comes in this struct.
 * Per-row and per-beam intermediate results live in a static device array
 * of the library (about 1.6 MB per GPU, held until the process ends), so:
 *   - n_beams * n_rows <= VMAT_PRICE_NOALLOC_MAX_ROWS and
 *     n_beams <= VMAT_PRICE_NOALLOC_MAX_BEAMS, else VMAT_ERR_INVALID_ARG
 *     (nothing launched);
 *   - calls that overlap on one GPU (two streams, or two threads) race on
 *     that array: serialise them;
 *   - nothing needs clearing between calls (each call writes every entry it
 *     reads first).
 * theta_deg is DEVICE double [N] here, strictly increasing in [0, 360) (not
 * checked: the call is asynchronous).  g, y, l, r, occ and the outputs as for
 * vmat_price.  The first call on a device looks up the array's address there;
 * no call allocates.                                                          */
#define VMAT_PRICE_NOALLOC_MAX_ROWS 65536
#define VMAT_PRICE_NOALLOC_MAX_BEAMS 4096
typedef struct vmat_beams {
    int32_t n_beams, n_rows, n_cols;  /* N, R, C (C <= 64)                          */
    int32_t circular;                 /* as vmat_problem.circular                    */
    int32_t max_leaf_step;            /* delta, < 0 unconstrained                    */
    int32_t reserved;
    double gamma;                     /* finite, >= 0                                */
    const double* theta_deg;          /* DEVICE [N]                                  */
} vmat_beams;
vmat_status vmat_price_noalloc(const vmat_beams* beams, const double* g, const double* y, const int32_t* l,
                               const int32_t* r, const uint8_t* occ, int32_t* out_beam, double* out_price,
                               double* beam_prices, hipStream_t stream);

typedef struct vmat_master_opts {
    int32_t max_iter;       /* iteration cap (default 200)                              */
    int32_t ls_max_steps;   /* Newton/bisection steps per line search (default 50)     */
    double tol_rel;         /* stop when max_k |min(y_k, grad_k)| <= tol_rel * ref      */
    double kkt_ref;         /* ref; <= 0: max_k |grad_k| at the start point             */
} vmat_master_opts;

typedef struct vmat_master_report {
    int32_t iters, converged, n_forward, n_adjoint, n_ls_evals, reserved;
    double F, gG, kkt, kkt_ref;
} vmat_master_report;

/* Master problem (Sec. 2.2): min F(z) + gamma G(y), y >= 0, over the intensities
 * of the given apertures, by gradient projection: steepest descent on the free
 * face after each face change, Polak-Ribiere(+) conjugate directions while the
 * face holds, exact line search (safeguarded Newton) up to the first blocking
 * bound.  y: DEVICE double [N], in: start point (unoccupied entries ignored),
 * out: solution (0 for unoccupied beams).  opts (HOST, nullable: defaults),
 * rep (HOST, nullable).  Returns VMAT_ERR_NOT_CONVERGED at the iteration cap.  */
vmat_status vmat_master(vmat_handle h, const int32_t* l, const int32_t* r, const uint8_t* occ,
                        double* y, const vmat_master_opts* opts, vmat_master_report* rep,
                        hipStream_t stream);

typedef struct vmat_solve_opts {
    int32_t max_cg_iter;     /* apertures to add (<= 0 or > free beams: until all occupied) */
    int32_t master_mode;     /* 0: the master's products stream D (one forward per
                              *    direction, one adjoint per step);
                              * 1: aperture doses d_k = D^T 1_{A_k} are stored when an
                              *    aperture opens (one forward each) and the master works
                              *    on them alone; one adjoint per column-generation
                              *    iteration gives the prices.  Same iterates up to
                              *    rounding (values stored in FP32, sums in FP64); needs
                              *    the store of vmat_reserve_solve (else
                              *    VMAT_ERR_UNSUPPORTED).                              */
    vmat_master_opts master; /* master.kkt_ref <= 0: |p| of the first priced aperture       */
} vmat_solve_opts;

typedef struct vmat_solve_report {
    /* n_forward, n_adjoint: products with D (either master mode)                */
    int32_t cg_iters, master_iters, n_forward, n_adjoint, n_ls_evals, not_converged;
    double F, gG, kkt_ref;
} vmat_solve_report;

/* Per-iteration record (HOST arrays, each nullable, length max iterations;
 * cost has one more entry: cost[0] is the cost before the first aperture).
 * y holds N entries per iteration: the intensities the pricing of that
 * iteration saw (the solution of the previous master, before the new
 * aperture opened at 0).  With the beam order and the final leaf pairs
 * (apertures never change once opened) it gives the plan state at every
 * iteration, so a reference can re-price each decision from the same state. */
typedef struct vmat_solve_trace {
    int32_t* beam;
    double* price;          /* p_k* of the chosen beam                        */
    double* margin;         /* second-best beam price minus p_k*             */
    double* row_margin;     /* least gap to a different row sum in beam k*   */
    double* cost;           /* F + gamma G after each master                 */
    int32_t* master_iters;
    double* y;              /* [iterations * N]                               */
} vmat_solve_trace;

/* Storage for master_mode 1 of vmat_solve (the master over the generated
 * apertures, Sec. 2.2): allocates the aperture-dose store at its final size,
 * 28 bytes per entry for U + nv entries, where U = sum over beams of the voxels
 * a beam reaches (no set of one aperture per beam stores more), and captures
 * the aperture-dose master's iteration.  Once per handle (later calls return
 * VMAT_OK at once); synchronises the device.                                  */
vmat_status vmat_reserve_solve(vmat_handle h);

/* Column generation (abstract; Sec. 2.2): repeat pricing -> add the aperture
 * (y = 0) -> master, until every beam has an aperture or max_cg_iter.
 * l, r, occ, y: DEVICE, in: start state (occ all zero: empty plan; otherwise a
 * resumed plan whose y is re-optimised first), out: final plan.
 * A resumed plan is checked before anything is launched (VMAT_ERR_INVALID_ARG,
 * outputs untouched): every occupied beam has 0 <= l <= r <= C in each row and
 * a finite y >= 0, and with max_leaf_step delta >= 0 every leaf of an occupied
 * beam lies within delta * (index distance) of the same leaf of the next
 * occupied beam (around the circle when circular; Sec. 2.2 leaf motion), as
 * column generation leaves a plan.  Entries of unoccupied beams are ignored.
 * z (nullable): DEVICE float [nv] final dose.  opts, rep, trace: HOST, nullable.
 * Returns VMAT_OK even if some master solve hit its cap (rep->not_converged).   */
vmat_status vmat_solve(vmat_handle h, const vmat_solve_opts* opts, int32_t* l, int32_t* r,
                       uint8_t* occ, double* y, float* z, vmat_solve_report* rep,
                       vmat_solve_trace* trace, hipStream_t stream);

/* Dose-rate feasibility of a final plan (Sec. 3): the smoothing term of eq. 3
 * only penalises intensity changes between neighbouring angles; when the
 * final plan still changes faster than the machine allows, gamma is raised
 * and the intensities are re-optimised with the apertures fixed, until the
 * plan is feasible.  Rate = max over the eq. 2 pairs (a, b) of
 * |y_b - y_a| / (theta_b - theta_a), per degree.  Each round multiplies gamma
 * by `factor` and runs vmat_master from the previous intensities; the first
 * check is on y as given (a feasible y is returned unchanged, rounds = 0).
 * The handle's gamma is left as created.
 *   y: DEVICE double [N], in: the plan's intensities, out: re-optimised;
 *   l, r, occ: DEVICE, the fixed apertures; rep: HOST.                      */
typedef struct {
    double rate_max;        /* largest allowed change per degree, >= 0        */
    double factor;          /* gamma multiplier per round, > 1                 */
    int32_t max_rounds;     /* >= 0                                            */
    int32_t reserved;
    vmat_master_opts master;/* options of every re-optimisation; fields <= 0
                             * take the defaults (200, 50, 1e-5, reference 0) */
} vmat_rate_opts;

typedef struct {
    int32_t rounds;         /* re-optimisations run                            */
    int32_t feasible;       /* 1 if the returned y meets rate_max               */
    int32_t master_iters;   /* summed over the rounds                          */
    int32_t not_converged;  /* rounds whose master hit its iteration cap       */
    double gamma;           /* gamma of the last round                         */
    double rate;            /* max rate of the returned y                      */
    double F, gG;           /* cost terms at the returned y (gG at `gamma`)    */
} vmat_rate_report;

vmat_status vmat_enforce_rate(vmat_handle h, const vmat_rate_opts* opts, const int32_t* l,
                              const int32_t* r, const uint8_t* occ, double* y,
                              vmat_rate_report* rep, hipStream_t stream);

/* Batched column generation: B plan variants (the objective of eq. 1 with
 * per-variant weights and thresholds, as in vmat_grad_batched) sharing D,
 * each solved by the column-generation loop of vmat_solve, in lockstep: every
 * dose and adjoint product is one SpMM over all variants; pricing and the
 * master's control run per variant; a variant whose master has stopped keeps
 * its state while the others iterate, and a variant opens its next aperture
 * as soon as its own master stops.  Each lockstep iteration replays two
 * captured kernel sequences (direction + dose SpMM + line search; step +
 * adjoint SpMM + gradients).  Directions enter the products in FP32
 * (rounded before the step, so y and the carried dose stay consistent).
 *   vmat_reserve_batched: allocates the work state for up to max_variants
 *       (1..64) variants (about (12 nb + 20 nv) * max_variants bytes); once,
 *       before vmat_solve_batched.
 *   vmat_solve_batched: plans start empty (occ all 0, else UNSUPPORTED) and
 *       run min(N, opts->max_cg_iter or N) iterations.
 *       l, r: DEVICE int32 [B][N*R]; occ: DEVICE uint8 [B][N]; y: DEVICE
 *       double [B][N] (outputs: the plans); label/table as in
 *       vmat_grad_batched; rep: HOST [B] reports; trace: HOST [B] (nullable,
 *       each field nullable, arrays as in vmat_solve); n_spmm: HOST int64 [2]
 *       (nullable): forward and adjoint SpMM launches.                        */
vmat_status vmat_reserve_batched(vmat_handle h, int32_t max_variants);
vmat_status vmat_solve_batched(vmat_handle h, const vmat_solve_opts* opts, int32_t B, int32_t n_struct,
                               const uint8_t* label, const float* table, int32_t* l, int32_t* r,
                               uint8_t* occ, double* y, vmat_solve_report* rep,
                               vmat_solve_trace* trace, int64_t* n_spmm, hipStream_t stream);

/* Plan variants sharing one D, K at a time: B plans, variant b with the
 * weights and thresholds table[b] (label/table as in vmat_grad_batched;
 * n_struct in [1, 256]), each a full vmat_solve from an empty plan.  The call
 * makes K plan contexts from h (vmat_create_plan), one host thread and one
 * stream each; worker t takes variants t, t + K, ... in turn, sets their
 * weights (vmat_set_weights) and solves.  Every plan is bit for bit the plan
 * vmat_solve gives on h with that variant's weights; h itself is not changed.
 * The plans of one worker follow each other; the workers' plans overlap on
 * the device (a plan with the aperture-dose master is bound by the latency of
 * its small launches).  opts: as in vmat_solve (nullable: defaults); with
 * master_mode 1 each context reserves its aperture-dose store.  K in
 * [1, 16] (more workers than the device's hardware queues add nothing).
 * l, r: DEVICE int32 [B][N*R]; occ: DEVICE uint8 [B][N]; y: DEVICE double
 * [B][N] (outputs: the plans); rep: HOST [B] reports.  Synchronises `stream`
 * before it starts; returns when every plan is done.  Allocates the K
 * contexts (their plan state and, in mode 1, their stores), K streams and
 * 12 nv bytes per worker, and releases all of it before it returns.         */
vmat_status vmat_solve_variants(vmat_handle h, const vmat_solve_opts* opts, int32_t B, int32_t n_struct,
                                const uint8_t* label, const float* table, int32_t K, int32_t* l,
                                int32_t* r, uint8_t* occ, double* y, vmat_solve_report* rep,
                                hipStream_t stream);

/* Measurement aid, not a step of the method: one streaming read of a device
 * buffer (non-temporal 16-byte loads, eight in flight per lane), timed by the
 * caller as the practical HBM read ceiling beside the products' rates.
 * buf: DEVICE [bytes], bytes a positive multiple of 16; partials: DEVICE
 * float [grid] (out: per-block sums that keep the loads live); grid in
 * [1, 65536] blocks of 256 lanes.  Asynchronous; allocates nothing.        */
vmat_status vmat_read_stream(const void* buf, int64_t bytes, float* partials, int32_t grid, hipStream_t stream);

/* Measurement aid, not a step of the method: the read of vmat_read_stream
 * with wbytes of writes mixed in, spread evenly over the read (512-byte
 * chunks, 64 lanes x 8 bytes, each wave writing its share as it goes): the
 * ceiling of a kernel that streams its input and writes a given share of
 * its traffic, as the products write their outputs.  wbuf: DEVICE double
 * [wbytes / 8] (out: overwritten with running sums), may be NULL when
 * wbytes is 0; wbytes a non-negative multiple of 512; other arguments as
 * vmat_read_stream.  Asynchronous; allocates nothing.                      */
vmat_status vmat_read_write_stream(const void* buf, int64_t bytes, double* wbuf, int64_t wbytes, float* partials,
                                   int32_t grid, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* VMAT_H */
