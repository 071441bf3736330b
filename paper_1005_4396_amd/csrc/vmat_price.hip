// Pricing (Sec. 2.2): for every unoccupied beam and leaf row, the best leaf
// pair in one left-to-right pass over the beamlet prices; then the beam price
// and the chosen beam.
//
// One wavefront per (beam, row): lane c holds the prefix sum P[c] (summed in
// column order, as a sequential pass would); an inclusive max-scan of (P[l], l)
// across the lanes gives every right end r its best left end inside the
// leaf-speed window (the running best of a left-to-right pass); lane r forms
// the candidate for right end r, and a shuffle tree picks the least key
// (S, r-l, l).  C <= 64 columns fit one wave.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "vmat_block.h"
#include "vmat_internal.h"
#include "vmat_kernels.h"

#include <string>

namespace vmat {

struct Cand {
    double S;
    int len, l, r;
};

__device__ __forceinline__ bool less_key(const Cand& a, const Cand& b) {
    if (a.S != b.S) return a.S < b.S;
    if (a.len != b.len) return a.len < b.len;
    return a.l < b.l;
}

// Plan variants (blockIdx.y = variant b of B): g is RHS-contiguous (beamlet
// i of variant b at i*B + b), the plan and row arrays are variant-major.
// vmask (nullable): variants to price; the others' blocks return at once.
__global__ __launch_bounds__(256) void k_price_rows(int N, int R, int C, int delta, int circ, int B,
                                                    const double* __restrict__ g, const int32_t* __restrict__ l,
                                                    const int32_t* __restrict__ r, const uint8_t* __restrict__ occ,
                                                    double* __restrict__ rowS, int32_t* __restrict__ rowl,
                                                    int32_t* __restrict__ rowr, double* __restrict__ rowm,
                                                    const uint8_t* __restrict__ vmask) {
    __shared__ double P[4][65];
    __shared__ double gs[4][64];   // the wave's row of prices
    __shared__ uint8_t socc[4096]; // occupancy (N <= 4096), for the neighbour search
    if (vmask && !vmask[blockIdx.y]) return;
    {
        const int b = blockIdx.y;
        const int64_t NR = (int64_t)N * R;
        g += b;
        l += b * NR;
        r += b * NR;
        occ += (int64_t)b * N;
        rowS += b * NR;
        rowl += b * NR;
        rowr += b * NR;
        rowm += b * NR;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t kr = (int64_t)blockIdx.x * 4 + w;
    const bool valid = kr < (int64_t)N * R;
    const int k = valid ? (int)(kr / R) : 0;
    const int rho = valid ? (int)(kr - (int64_t)k * R) : 0;
    for (int i = threadIdx.x; i < N; i += 256) socc[i] = occ[i];
    if (valid && lane < C) gs[w][lane] = g[(kr * C + lane) * B];
    __syncthreads();
    const bool active = valid && !socc[k];

    // leaf windows from the nearest occupied beam on each side: the wave
    // tests 64 index distances at once (lane t: distance base + t, wrapping
    // round the circle when circular, else ending at the first or last beam)
    // and the lowest lane with an occupied beam gives the nearest
    int Llo = 0, Lhi = C, Rlo = 0, Rhi = C;
    if (active && delta >= 0) {
        for (int side = 0; side < 2; ++side) {
            for (int base = 1; base < N; base += 64) {
                const int dist = base + lane;
                int kk = side == 0 ? k - dist : k + dist;
                bool hit = false;
                if (dist < N) {
                    if (kk < 0 || kk >= N) {
                        if (circ) kk = kk < 0 ? kk + N : kk - N;
                    }
                    hit = kk >= 0 && kk < N && socc[kk];
                }
                const uint64_t m = __ballot(hit);
                if (m) {
                    const int first = __ffsll((unsigned long long)m) - 1;
                    const int d = base + first;
                    const int kn = __shfl(kk, first, 64);
                    const int reach = (int)min((int64_t)delta * d, (int64_t)(1 << 20));
                    const int64_t a = (int64_t)kn * R + rho;
                    Llo = max(Llo, l[a] - reach);
                    Lhi = min(Lhi, l[a] + reach);
                    Rlo = max(Rlo, r[a] - reach);
                    Rhi = min(Rhi, r[a] + reach);
                    break;
                }
            }
        }
    }
    // prefix sums P[0..C] in column order; lane t holds P[t] and P[t+64]
    if (active) {
        for (int pos = lane; pos <= C; pos += 64) {
            double acc = 0.0;
            for (int c = 0; c < pos; ++c) acc = acc + gs[w][c];
            P[w][pos] = acc;
        }
    }
    __syncthreads();

    // Best left end for every right end r: the largest P[l] over
    // Llo <= l <= min(r, Lhi), ties to the larger l.  The upper end grows
    // with r, so this is a prefix maximum of the key (P[l], l) from Llo on:
    // an inclusive max-scan across the wave's lanes (positions 0..63), with
    // position 64 (C = 64 only) folded in for r = 64.  Maxima are exact, so
    // the choice is that of a sequential left-to-right pass.
    double kp = -INFINITY;
    int kl = -1;
    if (active && lane >= Llo && lane <= min(Lhi, C)) {
        kp = P[w][lane];
        kl = lane;
    }
    for (int off = 1; off < 64; off <<= 1) {
        const double op = __shfl_up(kp, off, 64);
        const int ol = __shfl_up(kl, off, 64);
        if (lane >= off && ol >= 0 && (kl < 0 || op > kp)) {
            kp = op;
            kl = ol;
        }
    }
    // lane t evaluates the right ends t and t+64 (C <= 64, so at most r = 64)
    Cand best;
    best.S = INFINITY;
    best.len = 1 << 30;
    best.l = -1;
    best.r = -1;
    for (int rr = lane, pass = 0; pass < 2; rr += 64, ++pass) {
        // the prefix maximum at position min(rr, Lhi) (every lane takes part in the shuffle)
        const int src = min(min(rr, Lhi), 63);
        double bp = __shfl(kp, src < 0 ? 0 : src, 64);
        int bl = __shfl(kl, src < 0 ? 0 : src, 64);
        if (!active || rr > C || rr < Rlo || rr > Rhi || min(rr, Lhi) < Llo) continue;
        if (min(rr, Lhi) == 64 && P[w][64] >= bp) {
            bp = P[w][64];
            bl = 64;
        }
        if (bl >= 0) {
            Cand c;
            c.S = P[w][rr] - bp;
            c.len = rr - bl;
            c.l = bl;
            c.r = rr;
            if (less_key(c, best)) best = c;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        Cand o;
        o.S = __shfl_xor(best.S, off, 64);
        o.len = __shfl_xor(best.len, off, 64);
        o.l = __shfl_xor(best.l, off, 64);
        o.r = __shfl_xor(best.r, off, 64);
        if (less_key(o, best)) best = o;
    }
    // least gap between S* and any feasible pair with a different S
    double gap = INFINITY;
    for (int rr = lane; active && rr <= C; rr += 64) {
        if (rr < Rlo || rr > Rhi) continue;
        const int lmax = min(Lhi, rr);
        for (int ll = Llo; ll <= lmax; ++ll) {
            const double S = P[w][rr] - P[w][ll];
            if (S != best.S) gap = fmin(gap, S - best.S);
        }
    }
    for (int off = 32; off > 0; off >>= 1) gap = fmin(gap, __shfl_xor(gap, off, 64));
    if (valid && lane == 0) {
        rowS[kr] = active ? best.S : INFINITY;
        rowl[kr] = best.l;
        rowr[kr] = best.r;
        rowm[kr] = gap;
    }
}

// Beam prices, the chosen beam, and (apply) the update of the plan state.
__device__ __forceinline__ void better(double& p, int& k, double p2, int k2) {
    if (k2 >= 0 && (k < 0 || p2 < p || (p2 == p && k2 < k))) {
        p = p2;
        k = k2;
    }
}

__global__ __launch_bounds__(CTRL) void k_price_beams(int N, int R, double gamma, int circ,
                                                      const double* __restrict__ th, const double* __restrict__ y,
                                                      const uint8_t* __restrict__ occ,
                                                      const double* __restrict__ rowS, const int32_t* __restrict__ rowl,
                                                      const int32_t* __restrict__ rowr, const double* __restrict__ rowm,
                                                      double* __restrict__ bprice, int32_t* __restrict__ out_beam,
                                                      double* __restrict__ out_price, double* __restrict__ user_bp,
                                                      int apply, int iter, int32_t* __restrict__ lw,
                                                      int32_t* __restrict__ rw, uint8_t* __restrict__ occw,
                                                      double* __restrict__ yw, SolveTraceDev tr,
                                                      const uint8_t* __restrict__ vmask,
                                                      const int32_t* __restrict__ iter_v) {
    if (vmask && !vmask[blockIdx.x]) return;
    if (iter_v) iter = iter_v[blockIdx.x];
    {
        // variant blockIdx.x: variant-major plan, row and trace arrays
        const int b = blockIdx.x;
        const int64_t NR = (int64_t)N * R;
        y += (int64_t)b * N;
        occ += (int64_t)b * N;
        rowS += b * NR;
        rowl += b * NR;
        rowr += b * NR;
        rowm += b * NR;
        bprice += (int64_t)b * N;
        out_beam += (int64_t)b * (1 + 2 * R);
        out_price += (int64_t)b * 3;
        if (user_bp) user_bp += (int64_t)b * N;
        if (apply) {
            lw += b * NR;
            rw += b * NR;
            occw += (int64_t)b * N;
            yw += (int64_t)b * N;
            tr.beam += (int64_t)b * N;
            tr.price += (int64_t)b * N;
            tr.margin += (int64_t)b * N;
            tr.row_margin += (int64_t)b * N;
            tr.y += (int64_t)b * N * N;
        }
    }
    __shared__ double shp[4];
    __shared__ int shk[4];
    __shared__ double sh[4];
    double pb = INFINITY;
    int kb = -1;
    for (int k = threadIdx.x; k < N; k += CTRL) {
        double p = INFINITY;
        if (!occ[k]) {
            double tot = 0.0;
            for (int rho = 0; rho < R; ++rho) tot = tot + rowS[(int64_t)k * R + rho];
            // gamma dG/dy_k at y_k = 0 (eq. 2): -2 y_{k-1}/gap^- - 2 y_{k+1}/gap^+
            double dG = 0.0;
            const bool has_prev = k > 0 || (circ && N > 1);
            const bool has_next = k < N - 1 || (circ && N > 1);
            if (has_prev) {
                const int a = k > 0 ? k - 1 : N - 1;
                const double w = k > 0 ? th[k] - th[k - 1] : th[0] + 360.0 - th[N - 1];
                dG += 2.0 * (0.0 - y[a]) / w;
            }
            if (has_next) {
                const int b = k < N - 1 ? k + 1 : 0;
                const double w = k < N - 1 ? th[k + 1] - th[k] : th[0] + 360.0 - th[N - 1];
                dG -= 2.0 * (y[b] - 0.0) / w;
            }
            p = tot + gamma * dG;
            better(pb, kb, p, k);
        }
        bprice[k] = p;
        if (user_bp) user_bp[k] = p;
        if (apply) tr.y[(int64_t)iter * N + k] = y[k];
    }
    // block argmin with ties to the smallest k
    for (int off = 32; off > 0; off >>= 1) {
        const double p2 = __shfl_down(pb, off, 64);
        const int k2 = __shfl_down(kb, off, 64);
        better(pb, kb, p2, k2);
    }
    if ((threadIdx.x & 63) == 0) {
        shp[threadIdx.x >> 6] = pb;
        shk[threadIdx.x >> 6] = kb;
    }
    __syncthreads();
    double pbest = shp[0];
    int ks = shk[0];
    for (int i = 1; i < 4; ++i) better(pbest, ks, shp[i], shk[i]);
    __syncthreads();
    double second = INFINITY;
    for (int k = threadIdx.x; k < N; k += CTRL)
        if (!occ[k] && k != ks) second = fmin(second, bprice[k]);
    second = bmin(second, sh);
    double rm = INFINITY;
    if (ks >= 0)
        for (int rho = threadIdx.x; rho < R; rho += CTRL) rm = fmin(rm, rowm[(int64_t)ks * R + rho]);
    rm = bmin(rm, sh);
    for (int rho = threadIdx.x; rho < R; rho += CTRL) {
        const int32_t lv = ks >= 0 ? rowl[(int64_t)ks * R + rho] : 0;
        const int32_t rv = ks >= 0 ? rowr[(int64_t)ks * R + rho] : 0;
        out_beam[1 + rho] = lv;
        out_beam[1 + R + rho] = rv;
        if (apply && ks >= 0) {
            lw[(int64_t)ks * R + rho] = lv;
            rw[(int64_t)ks * R + rho] = rv;
        }
    }
    if (threadIdx.x != 0) return;
    const double margin = ks >= 0 && isfinite(second) ? second - pbest : INFINITY;
    out_beam[0] = ks;
    out_price[0] = ks >= 0 ? pbest : INFINITY;
    out_price[1] = margin;
    out_price[2] = rm;
    if (apply && ks >= 0) {
        occw[ks] = 1;
        yw[ks] = 0.0;
        tr.beam[iter] = ks;
        tr.price[iter] = pbest;
        tr.margin[iter] = margin;
        tr.row_margin[iter] = rm;
    }
}

vmat_status launch_price(const vmat_ctx* h, const double* g, const double* y, const int32_t* l, const int32_t* r,
                         const uint8_t* occ, int32_t* out_beam, double* out_price, double* beam_prices, int apply,
                         int iter, int32_t* lw, int32_t* rw, uint8_t* occw, double* yw, hipStream_t st) {
    return launch_price_variants(h, 1, g, y, l, r, occ, h->row_S, h->row_l, h->row_r, h->row_m, h->bprice, out_beam,
                                 out_price, beam_prices, apply, iter, lw, rw, occw, yw, h->tr, st, nullptr, nullptr);
}

vmat_status launch_price_variants(const vmat_ctx* h, int B, const double* g, const double* y, const int32_t* l,
                                  const int32_t* r, const uint8_t* occ, double* rowS, int32_t* rowl, int32_t* rowr,
                                  double* rowm, double* bprice, int32_t* out_beam, double* out_price,
                                  double* beam_prices, int apply, int iter, int32_t* lw, int32_t* rw, uint8_t* occw,
                                  double* yw, SolveTraceDev tr, hipStream_t st, const uint8_t* vmask,
                                  const int32_t* iter_v) {
    const int64_t NR = (int64_t)h->N * h->R;
    k_price_rows<<<dim3((unsigned)((NR + 3) / 4), (unsigned)B), 256, 0, st>>>(h->N, h->R, h->C, h->delta,
                                                                             h->circular, B, g, l, r, occ, rowS,
                                                                             rowl, rowr, rowm, vmask);
    VMAT_LAUNCH_CHECK();
    k_price_beams<<<(unsigned)B, CTRL, 0, st>>>(h->N, h->R, h->gamma, h->circular, h->d_theta, y, occ, rowS, rowl,
                                               rowr, rowm, bprice, out_beam, out_price, beam_prices, apply, iter,
                                               lw, rw, occw, yw, tr, vmask, iter_v);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

// ---------------------------------------------------------------- pricing without allocation
// Scratch of vmat_price_noalloc: the per-row results (S*, margin, l*, r*) of
// up to PRICE_NA_ROWS leaf rows and the prices of up to PRICE_NA_BEAMS beams,
// in one file-scope device array.  Every GPU the library runs on holds its own
// copy until the process ends.  Kernels get its address from
// hipGetSymbolAddress (per device, at the first call on that device); the
// array's name is not a device address in host code.
constexpr int64_t PRICE_NA_ROWS = VMAT_PRICE_NOALLOC_MAX_ROWS;
constexpr int64_t PRICE_NA_BEAMS = VMAT_PRICE_NOALLOC_MAX_BEAMS;
constexpr size_t PRICE_NA_BYTES = (size_t)PRICE_NA_ROWS * (8 + 8 + 4 + 4) + (size_t)PRICE_NA_BEAMS * 8;
static __device__ __align__(256) unsigned char scratch[PRICE_NA_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of this device's scratch array (looked up once).
vmat_status scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(VMAT_ERR_UNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VMAT_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return VMAT_OK;
}
}  // namespace

}  // namespace vmat

using namespace vmat;

extern "C" vmat_status vmat_price_noalloc(const vmat_beams* b, const double* g, const double* y, const int32_t* l,
                                          const int32_t* r, const uint8_t* occ, int32_t* out_beam,
                                          double* out_price, double* beam_prices, hipStream_t st) {
    set_error("");
    if (!b) return fail(VMAT_ERR_INVALID_ARG, "null beam description");
    if (b->n_beams < 1 || b->n_rows < 1 || b->n_cols < 1)
        return fail(VMAT_ERR_INVALID_ARG, "n_beams, n_rows and n_cols must be >= 1");
    if (b->n_cols > 64) return fail(VMAT_ERR_UNSUPPORTED, "n_cols > 64 is not supported");
    const int64_t NR = (int64_t)b->n_beams * b->n_rows;
    if (NR > PRICE_NA_ROWS || b->n_beams > PRICE_NA_BEAMS)
        return fail(VMAT_ERR_INVALID_ARG, "vmat_price_noalloc: n_beams * n_rows exceeds " +
                                              std::to_string(PRICE_NA_ROWS) + " or n_beams exceeds " +
                                              std::to_string(PRICE_NA_BEAMS) + " (the size of its static scratch)");
    if (!std::isfinite(b->gamma) || b->gamma < 0.0) return fail(VMAT_ERR_INVALID_ARG, "gamma must be finite and >= 0");
    if (!b->theta_deg || !g || !y || !l || !r || !occ || !out_beam || !out_price)
        return fail(VMAT_ERR_INVALID_ARG, "null array");
    int dev = -1;
    VMAT_HIP(hipGetDevice(&dev));
    unsigned char* base = nullptr;
    vmat_status rc = scratch_address(dev, &base);
    if (rc != VMAT_OK) return rc;
    double* rowS = reinterpret_cast<double*>(base);
    double* rowm = rowS + PRICE_NA_ROWS;
    int32_t* rowl = reinterpret_cast<int32_t*>(rowm + PRICE_NA_ROWS);
    int32_t* rowr = rowl + PRICE_NA_ROWS;
    double* bprice = reinterpret_cast<double*>(rowr + PRICE_NA_ROWS);
    // every entry the kernels read is written first in the same call (rows
    // and beams of this problem): nothing needs clearing
    k_price_rows<<<dim3((unsigned)((NR + 3) / 4), 1u), 256, 0, st>>>(b->n_beams, b->n_rows, b->n_cols,
                                                                    b->max_leaf_step, b->circular ? 1 : 0, 1, g, l,
                                                                    r, occ, rowS, rowl, rowr, rowm, nullptr);
    VMAT_LAUNCH_CHECK();
    k_price_beams<<<1u, CTRL, 0, st>>>(b->n_beams, b->n_rows, b->gamma, b->circular ? 1 : 0, b->theta_deg, y, occ,
                                       rowS, rowl, rowr, rowm, bprice, out_beam, out_price, beam_prices, 0, 0,
                                       nullptr, nullptr, nullptr, nullptr, SolveTraceDev{}, nullptr, nullptr);
    VMAT_LAUNCH_CHECK();
    return VMAT_OK;
}

