// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <string>
#include <vector>

#include "vmat.h"

namespace vmat {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
vmat_status fail(vmat_status code, const std::string& msg);

#define VMAT_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::vmat::fail(VMAT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define VMAT_LAUNCH_CHECK() VMAT_HIP(hipGetLastError())

// ---------------------------------------------------------------- layouts
// A sparse matrix in "quad CSR": each row padded to a multiple of 4 entries so
// that a lane reads 4 values and 4 column indices with one 16-byte (values:
// 16/8/4-byte) load each.  Padding entries have value 0 and repeat a valid
// column of the row (or column 0 for an empty row), so they are harmless.
struct QuadCsr {
    int64_t n_rows = 0;
    int64_t n_quads = 0;        // padded entries / 4
    uint32_t* qptr = nullptr;   // [n_rows+1] row start in quads
    int32_t* col = nullptr;     // [4*n_quads]
    void* val = nullptr;        // [4*n_quads] of the storage type
    float* scale = nullptr;     // [n_rows] per-row scale (FP8 only), else null
    int lanes_per_row = 16;     // lanes cooperating on one row (power of 2, <= 64)
};

// Tiled layouts of D.  The voxels are cut into blocks of consecutive indices
// (at most TILE_VOXELS each) such that the distinct beamlets reaching a block
// (its list) number at most TILE_LIST.  Per block:
//   forward: the block's voxel rows (voxel-major quad CSR, as `vm`) with 16-bit
//            indices into the block's beamlet list; the list's x values are
//            staged in LDS (FP64) and gathered from there;
//   adjoint: one row per list entry (slot) holding that beamlet's entries in
//            the block, with 16-bit voxel offsets from the block start; the
//            block's slice of the gathered vector is staged in LDS (FP32); the
//            slot results are summed per beamlet over its blocks in block order.
constexpr int WTAB_CAP = 256;     // distinct (alpha, beta, T) held as voxel labels
constexpr int TILE_VOXELS = 16384;
constexpr int TILE_LIST = 8192;
constexpr int TILE_THREADS = 512;
// Most rows of one work item (32 slices); their sums are staged in LDS, and
// 64 KB of staged values + TILE_ROWS doubles + a counter fit two 512-thread
// workgroups in a compute unit's 160 KB.
constexpr int TILE_ROWS = 2040;
// Quads in flight per lane in the sliced forward.
constexpr int SELL_U = 4;

struct Tiled {
    bool on = false;
    int nblk = 0;
    int64_t S = 0;                // total list length (slots)
    int32_t* bounds = nullptr;    // [nblk+1] voxel boundaries
    uint32_t* loff = nullptr;     // [nblk+1] list offsets
    uint32_t* list = nullptr;     // [S] beamlet of each slot
    // forward
    uint16_t* fcol = nullptr;     // [4 * vm.n_quads]
    int4* fwork = nullptr;        // (block, first row, end row, first slice)
    int n_fwork = 0;
    // forward, sliced: each work item's rows sorted by length (longest first)
    // and cut into slices of 64 rows; a slice stores its quads column-major
    // (quad k of its 64 rows contiguous), padded to its longest row
    int64_t n_slices = 0;
    int64_t s_quads = 0;          // stored quads including padding
    uint32_t* s_off = nullptr;    // [n_slices] first quad of each slice
    uint32_t* s_len = nullptr;    // [n_slices] quads per row of each slice
    uint32_t* s_row = nullptr;    // [64 * n_slices] voxel of each slice row, ~0 for padding
    uint16_t* s_col = nullptr;    // [4 * s_quads] local column indices
    void* s_val = nullptr;        // [4 * s_quads] values (storage format)
    // adjoint, sliced the same way over the slot rows of each work item
    int64_t an_slices = 0, as_quads = 0;
    uint32_t *as_off = nullptr, *as_len = nullptr, *as_row = nullptr;
    uint16_t* as_col = nullptr;
    void* as_val = nullptr;
    // adjoint
    uint32_t* aqptr = nullptr;    // [S+1] slot row starts in quads
    uint16_t* acol = nullptr;     // [4 * a_quads]
    void* aval = nullptr;         // [4 * a_quads]
    int64_t a_quads = 0;
    int4* awork = nullptr;        // (block, first slot, end slot, 0)
    int n_awork = 0;
    double* part = nullptr;       // [S] slot sums
    uint32_t* red_ptr = nullptr;  // [nb+1]
    uint32_t* red_slot = nullptr; // [S] slots of each beamlet, in block order
    // batched products: the slices of each block (forward and adjoint), and
    // for each of the 8 XCDs a contiguous range of blocks [x[i], x[i+1])
    // balanced by stored quads
    uint32_t* fb_ptr = nullptr;   // [nblk+1]
    uint32_t* fb_sl = nullptr;    // [n_slices]
    uint32_t* ab_ptr = nullptr;   // [nblk+1]
    uint32_t* ab_sl = nullptr;    // [an_slices]
    int32_t fx[9] = {}, ax[9] = {};
};

// Launch gate: a kernel given a gate returns at once unless the device-side
// value *p is one of the values in `mask` (bit v set: value v admitted).
// A default gate (p == nullptr) always runs.
struct Gate {
    const int32_t* p = nullptr;
    uint32_t mask = 0;
    __host__ __device__ bool closed() const { return p && !((1u << *p) & mask); }
};

// The sum of part[red_slot[k] * stride + b] over k in [k0, k1), added in k
// order: a beamlet's slot sums.  The slot indices of up to four slots are
// loaded at once, then their sums, so a beamlet with up to four slots costs
// two dependent loads after its range instead of two per slot.
__device__ __forceinline__ double slot_sum(uint32_t k0, uint32_t k1, const uint32_t* __restrict__ red_slot,
                                           const double* __restrict__ part, int64_t stride, int b) {
    double s = 0.0;
    for (uint32_t k = k0; k < k1; k += 4) {
        uint32_t sl[4];
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) sl[j] = k + j < k1 ? red_slot[k + j] : 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = k + j < k1 ? part[(int64_t)sl[j] * stride + b] : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (k + j < k1) s += v[j];
    }
    return s;
}

// Scalars and small vectors of the master iteration, resident on the device.
struct MasterState {
    // line search
    double t_max, t_eval, t, lo, hi, p0, h0, p, h, t_star, slope0, curv;
    // two-point passes: second point, and phi', phi'' at the bracket ends
    double t_eval2, plo, hlo, phi, hhi;
    // master
    double kkt, kkt_ref, tol, F, gG, beta_cg;
    // done: 0 while iterating, 1 when the solve has ended, 2 while an
    // iteration waits for its line search (the step found it unfinished: the
    // kernels of that iteration skip, the line-search evaluations go on)
    int32_t it, max_iter, done, converged;
    int32_t ls_phase, ls_steps, ls_max, ls_done;
    int32_t n_fwd, n_adj, n_ls, have_prev;
    int32_t n_eval;               // points in the next line-search pass (1 or 2)
    uint32_t seq;                 // line-search chains completed since the master began
};

// Host-visible copy of the master state (pinned host memory): the last
// line-search pass of the chain with count v stores the state in slot v % 2,
// then seq = v (release at system scope), so a host that sees seq >= v finds
// chain v's state in slot v % 2.  The host waits for chain v with at most chain
// v + 1 enqueued after it, so no chain writes that slot while the host copies
// it (chain v + 2, the next writer of the slot, is enqueued after the copy).
struct MasterMirror {
    MasterState s[2];
    uint32_t seq;
};

// Per-iteration record of vmat_solve, resident on the device.
struct SolveTraceDev {
    int32_t* beam;       // [N]
    double* price;       // [N]
    double* margin;      // [N]
    double* row_margin;  // [N]
    double* cost;        // [N+1]
    int32_t* miters;     // [N]
    double* y;           // [N*N] intensities each pricing saw (the previous master's solution)
};

}  // namespace vmat

namespace vmat {
// Work state of batched plan solves (plan variants sharing D), allocated by
// vmat_reserve_batched for up to `cap` variants.  Large vectors are RHS-
// contiguous ([rows][B]); per-beam and per-row arrays are variant-major.
struct BatchState {
    int cap = 0;
    float* X = nullptr;       // [nb][cap] fluence of the search direction
    double* Z = nullptr;      // [nv][cap] dose
    double* dZ = nullptr;     // [nv][cap] dose of the direction
    float* RZ = nullptr;      // [nv][cap] F'(z)
    double* G = nullptr;      // [nb][cap] beamlet prices
    double *grad = nullptr, *grad_prev = nullptr, *d = nullptr, *d_prev = nullptr, *gF = nullptr;  // [cap][N]
    uint8_t *W = nullptr, *W_prev = nullptr;                                                    // [cap][N]
    MasterState* ms = nullptr;       // [cap]
    MasterState* ms_host = nullptr;  // [cap], pinned
    double *pp = nullptr, *qq = nullptr, *pf = nullptr;  // [cap][n_part] partial sums
    double *pp2 = nullptr, *qq2 = nullptr;               // [cap][n_part] second line-search point
    double *rowS = nullptr, *rowm = nullptr;             // [cap][N*R]
    int32_t *rowl = nullptr, *rowr = nullptr;            // [cap][N*R]
    double* bprice = nullptr;                            // [cap][N]
    int32_t* pbeam = nullptr;                            // [cap][1+2R]
    double* pscore = nullptr;                            // [cap][3]
    double* kref = nullptr;                              // [cap]
    double* cost = nullptr;                              // [cap]
    double* spart = nullptr;                             // [S][cap] slot sums of the 64-wide tiled adjoint
    uint8_t* vmask = nullptr;                            // [cap] variants opening an aperture now
    int32_t* viter = nullptr;                            // [cap] their aperture counts
    uint8_t* mask_host = nullptr;                        // [cap], pinned
    int32_t* iter_host = nullptr;                        // [cap], pinned
    SolveTraceDev tr{};                                  // [cap][N] each
    int64_t bytes = 0;
};
}  // namespace vmat

namespace vmat {
constexpr int GRAPH_KEY_LEN = 10;  // words identifying a captured sequence

// Device-side view of the aperture-dose store, read by the master's kernels,
// so that a captured master iteration stays valid while the store grows.
// One aperture-major entry of the aperture doses: voxel and value, loaded
// as one 8-byte word.
struct alignas(8) ApEntry {
    uint32_t vox;
    float val;
};

struct ApView {
    const uint32_t* vx_ptr;
    const uint16_t* vx_beam;
    const float* vx_val;
    const uint32_t* col_ptr;
    const ApEntry* col;
    const int32_t* beam_slot;
};

// Aperture doses (master over the generated apertures): d_k = D^T 1_{A_k} for
// every occupied beam, built once when the aperture is opened.  Two copies:
// aperture-major (col, col_ptr: entries of slot s in [col_ptr[s], col_ptr[s+1]),
// voxels ascending) for the per-aperture sums of F'(z), and voxel-major
// (vx_*: ping-pong pair rebuilt by merging each new aperture, entries of a
// voxel in opening order) for the dose of an intensity vector.
struct ApDose {
    int64_t cap = 0;               // entries each array can hold
    int64_t top = 0;               // entries in use, up to the last counted aperture
    int pending = 0;               // 1: the last aperture's count is still in total_host
    int n_slots = 0;               // apertures stored
    int cur = 0;                   // voxel-major copy in use (0/1)
    ApEntry* col = nullptr;        // [cap]
    uint32_t* col_ptr = nullptr;   // [N+1]
    int32_t* beam_slot = nullptr;  // [N], -1 for beams without a stored aperture
    uint32_t* vx_ptr[2] = {nullptr, nullptr};  // [nv+1]
    uint16_t* vx_beam[2] = {nullptr, nullptr}; // [cap]
    float* vx_val[2] = {nullptr, nullptr};     // [cap]
    uint32_t* vx_vox[2] = {nullptr, nullptr};  // [cap] voxel of each entry (read only by the merge)
    uint32_t* chunk = nullptr;     // [n_chunks + 1] non-zero counts, then offsets; [n_chunks+1] = total
    uint32_t* shift = nullptr;     // [nv] new entries before each voxel in the last merge
    double* unit = nullptr;        // [N] unit intensity vector of the aperture being stored
    ApView* view = nullptr;        // device copy of the current pointers
    uint32_t* total_host = nullptr;// pinned: non-zeros of the last stored aperture
    hipEvent_t counted = nullptr;  // recorded after that count's copy
    int64_t bytes = 0;
};
}  // namespace vmat

struct vmat_ctx {
    int32_t N, R, C;
    int64_t nb, nv, nnz;
    int32_t d_store;
    double gamma;
    int32_t circular, delta;
    int device;

    std::vector<double> theta;     // host copy
    double* d_theta = nullptr;     // [N]

    vmat::QuadCsr bm;              // beamlet-major (rows = beamlets): adjoint g = D r
    vmat::QuadCsr vm;              // voxel-major (rows = voxels): forward z = D^T x
    vmat::Tiled tl;                // tiled forms of both (used when tl.on)
    int32_t layout_req = 0;
    // quads in flight per lane of the sliced forward and adjoint (4 or 8),
    // the faster of the two as timed on this handle at creation
    int sell_u_fwd = 4, sell_u_adj = 4;
    float4* abT = nullptr;         // [nv] (alpha, beta, T, 0)
    // the same weights as a one-byte label per voxel into a table of the
    // distinct (alpha, beta, T), kept when there are at most 256 of them (one
    // per structure in the usual case); n_wtab == 0: none
    uint8_t* wlab = nullptr;       // [nv]
    float4* wtab = nullptr;        // [WTAB_CAP], entries past n_wtab zero
    int n_wtab = 0;
    int* vflag = nullptr;          // [1] validation flags of vmat_set_weights

    // work buffers
    double* x = nullptr;           // [nb] fluence
    double* xl = nullptr;          // [tl.S] fluence in block-list order (tiled layout)
    double* z = nullptr;           // [nv] dose (FP64)
    double* dz = nullptr;          // [nv] dose of the search direction
    float* rz = nullptr;           // [nv] F'(z) for the adjoint gather
    double* g = nullptr;           // [nb] beamlet prices
    double* bpart = nullptr;       // [N * max(8, ceil(R*C/256))] beam gradient in parts
    double* part = nullptr;        // [n_part * 8] block partial sums
    int n_part = 0;
    double* part_b = nullptr;      // [64 * n_part] per-variant partial sums (batched cost)
    int32_t tune_fwd[65] = {};     // tuned RHS tile width of the batched products, by B (0: default)
    int32_t tune_adj[65] = {};
    vmat::BatchState* bs = nullptr; // batched solves (vmat_reserve_batched)
    vmat::ApDose* ap = nullptr;     // aperture doses (aperture-dose master)
    // one master iteration's kernels as a replayable graph, per master kind
    // (captured once on cap_stream: the streaming master's at creation, the
    // aperture-dose master's by vmat_reserve_solve); the batched sequences are
    // keyed by the pointers their kernels take
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t iter_graph[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t iter_key[4][vmat::GRAPH_KEY_LEN] = {};
    // the plan the master and column generation work on: the handle's own
    // copies of the caller's leaf pairs, occupancy and intensities (my), so
    // that the captured master iterations take fixed pointers
    int32_t* pl = nullptr;         // [N*R]
    int32_t* pr = nullptr;         // [N*R]
    uint8_t* pocc = nullptr;       // [N]
    // gamma on the device, read by the captured control kernels (so a new
    // gamma needs no new capture); h->gamma is its host copy
    double* d_gamma = nullptr;
    // master vectors [N]
    double *my = nullptr, *mgrad = nullptr, *mgrad_prev = nullptr, *md = nullptr, *md_prev = nullptr,
           *mgF = nullptr;
    uint8_t *mW = nullptr, *mW_prev = nullptr;
    vmat::MasterState* ms = nullptr;      // device
    vmat::MasterState* ms2 = nullptr;     // device, second buffer of the line-search chain
    vmat::MasterState* ms_host = nullptr; // pinned host mirror
    // pinned host copy of the state written by the device after every
    // line-search chain, read by the host one iteration behind
    vmat::MasterMirror* mirror = nullptr;
    vmat::MasterMirror* mirror_dev = nullptr;  // its device address
    // line-search chains enqueued on this handle; every master start sets the
    // device's chain count to it, and each chain's last pass advances both
    uint32_t chains = 0;
    // pricing
    double* row_S = nullptr;       // [N*R]
    int32_t* row_l = nullptr;      // [N*R]
    int32_t* row_r = nullptr;      // [N*R]
    double* row_m = nullptr;       // [N*R] row margins
    double* bprice = nullptr;      // [N]
    int32_t* pbeam = nullptr;      // [1 + 2R]
    double* pscore = nullptr;      // [3]
    double* cost2 = nullptr;       // [2]
    vmat::SolveTraceDev tr{};
    int64_t bytes = 0;
    // plan contexts (vmat_create_plan): d_owner is the handle whose layouts
    // of D this one reads (null: it built its own); n_plans counts the live
    // contexts reading this handle's layouts
    vmat_ctx* d_owner = nullptr;
    std::atomic<int> n_plans{0};
};
