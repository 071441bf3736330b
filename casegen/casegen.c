/*
 * Seeded synthetic pencil-beam dose-deposition generator.
 *
 * Builds the sparse matrix D (row i = beamlet, column j = voxel, the paper's
 * D_ij of Sec. 2.1) for a coplanar 360-degree arc.  This is input synthesis
 * only: it holds none of the optimiser's arithmetic and is shared, as a data
 * source, by the CPU reference and the GPU library tests.
 *
 * Geometry
 *   voxel (ix,iy,iz) has centre ((ix+0.5-nx/2)h, (iy+0.5-ny/2)h, (iz+0.5-nz/2)h),
 *   linear index j = (iz*ny + iy)*nx + ix.
 *   beam k at angle th_k = 2*pi*k/N travels along d = (cos th, sin th, 0);
 *   lateral axis u = (-sin th, cos th, 0).  Leaf rows run along z, columns along u.
 *   beamlet i = (k*R + rho)*C + c has its central ray at lateral offset
 *   u_c = (c+0.5-C/2)*pitch and height z_rho = (rho+0.5-R/2)*pitch.
 *
 * Coefficient
 *   D_ij = exp(-mu*depth_j) * exp(-q^2/(2 s^2)) * (1 + jitter*xi_ij)
 *   depth_j = distance from the voxel centre back along -d to the grid box,
 *   q = perpendicular distance of the voxel centre from the central ray,
 *   s = sigma_vox*h, xi_ij in [-1,1) from SplitMix64 (Steele, Lea, Flood 2014)
 *   keyed by (seed, i, j).  An entry exists iff exp(-q^2/(2 s^2)) >= thr.
 *
 * Columns come out sorted within each row; values are rounded to fp32.
 * OpenMP parallelises over beams; the result does not depend on thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    double h;          /* voxel edge (mm) */
    int32_t n_beams, n_rows, n_cols;
    double pitch;      /* beamlet pitch at isocentre (mm) */
    double sigma_vox;  /* lateral Gaussian sigma in voxels */
    double mu_per_mm;  /* attenuation coefficient (1/mm) */
    double thr;        /* lateral cut, 0 < thr <= 1 */
    double jitter;     /* relative jitter amplitude */
    uint64_t seed;
} cg_spec;

static inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* xi in [-1, 1) keyed by (seed, i, j) */
double cg_xi(uint64_t seed, int64_t i, int64_t j) {
    uint64_t key = ((uint64_t)i << 32) | (uint64_t)(uint32_t)j;
    uint64_t v = splitmix64(seed ^ splitmix64(key));
    return (double)(v >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

/*
 * Enumerate the entries of one leaf row (beam k, row rho) for all its C
 * columns.  If col/val are NULL only counts are written into cnt[C].
 * Otherwise entries for column c go to col/val starting at off[c].
 */
static void enum_leaf_row(const cg_spec* s, int k, int rho, int64_t* cnt,
                          const int64_t* off, int32_t* col, float* val) {
    const double th = 2.0 * M_PI * (double)k / (double)s->n_beams;
    const double dx = cos(th), dy = sin(th);
    const double ux = -dy, uy = dx;
    const double h = s->h;
    const double X = 0.5 * s->nx * h, Y = 0.5 * s->ny * h;
    const double sig = s->sigma_vox * h;
    const double qmax2 = 2.0 * sig * sig * log(1.0 / s->thr);
    const double qmax = sqrt(qmax2);
    const double zr = ((double)rho + 0.5 - 0.5 * s->n_rows) * s->pitch;
    const int64_t nb_row0 = ((int64_t)k * s->n_rows + rho) * s->n_cols;

    for (int c = 0; c < s->n_cols; ++c) {
        const double uc = ((double)c + 0.5 - 0.5 * s->n_cols) * s->pitch;
        const int64_t i = nb_row0 + c;
        int64_t n = 0;
        int64_t pos = off ? off[c] : 0;
        /* z slices within reach, ascending */
        int iz0 = (int)ceil((zr - qmax) / h + 0.5 * s->nz - 0.5);
        int iz1 = (int)floor((zr + qmax) / h + 0.5 * s->nz - 0.5);
        if (iz0 < 0) iz0 = 0;
        if (iz1 > s->nz - 1) iz1 = s->nz - 1;
        for (int iz = iz0; iz <= iz1; ++iz) {
            const double vz = ((double)iz + 0.5 - 0.5 * s->nz) * h;
            const double dz = vz - zr;
            const double w2 = qmax2 - dz * dz;
            if (w2 < 0.0) continue;
            const double w = sqrt(w2);
            for (int iy = 0; iy < s->ny; ++iy) {
                const double vy = ((double)iy + 0.5 - 0.5 * s->ny) * h;
                /* |vx*ux + vy*uy - uc| <= w  -> range of vx */
                int ix0, ix1;
                const double rest = vy * uy - uc;
                if (fabs(ux) < 1e-12) {
                    if (fabs(rest) > w) continue;
                    ix0 = 0;
                    ix1 = s->nx - 1;
                } else {
                    double a = (-w - rest) / ux, b = (w - rest) / ux;
                    if (a > b) { double t = a; a = b; b = t; }
                    /* widen by one voxel; the exact test below decides */
                    ix0 = (int)floor(a / h + 0.5 * s->nx - 0.5) - 1;
                    ix1 = (int)ceil(b / h + 0.5 * s->nx - 0.5) + 1;
                    if (ix0 < 0) ix0 = 0;
                    if (ix1 > s->nx - 1) ix1 = s->nx - 1;
                }
                for (int ix = ix0; ix <= ix1; ++ix) {
                    const double vx = ((double)ix + 0.5 - 0.5 * s->nx) * h;
                    const double lat = vx * ux + vy * uy - uc;
                    const double q2 = lat * lat + dz * dz;
                    if (q2 > qmax2) continue;
                    if (col) {
                        double sx = INFINITY, sy = INFINITY;
                        if (dx > 1e-12) sx = (vx + X) / dx;
                        else if (dx < -1e-12) sx = (X - vx) / (-dx);
                        if (dy > 1e-12) sy = (vy + Y) / dy;
                        else if (dy < -1e-12) sy = (Y - vy) / (-dy);
                        double depth = sx < sy ? sx : sy;
                        if (depth < 0.0) depth = 0.0;
                        const int64_t j = ((int64_t)iz * s->ny + iy) * s->nx + ix;
                        const double xi = cg_xi(s->seed, i, j);
                        const double d = exp(-s->mu_per_mm * depth) *
                                         exp(-q2 / (2.0 * sig * sig)) *
                                         (1.0 + s->jitter * xi);
                        col[pos + n] = (int32_t)j;
                        val[pos + n] = (float)d;
                    }
                    ++n;
                }
            }
        }
        if (cnt) cnt[c] = n;
    }
}

/* row_nnz[nb]: entries per beamlet row.  Returns total nnz. */
int64_t cg_count(const cg_spec* s, int64_t* row_nnz) {
    const int nrow = s->n_beams * s->n_rows;
#pragma omp parallel for schedule(dynamic, 4)
    for (int kr = 0; kr < nrow; ++kr) {
        const int k = kr / s->n_rows, rho = kr % s->n_rows;
        enum_leaf_row(s, k, rho, row_nnz + (int64_t)kr * s->n_cols, NULL, NULL, NULL);
    }
    int64_t tot = 0;
    const int64_t nb = (int64_t)nrow * s->n_cols;
    for (int64_t i = 0; i < nb; ++i) tot += row_nnz[i];
    return tot;
}

/* row_ptr[nb+1] from cg_count's prefix sum; fills col/val. */
void cg_fill(const cg_spec* s, const int64_t* row_ptr, int32_t* col, float* val) {
    const int nrow = s->n_beams * s->n_rows;
#pragma omp parallel for schedule(dynamic, 4)
    for (int kr = 0; kr < nrow; ++kr) {
        const int k = kr / s->n_rows, rho = kr % s->n_rows;
        enum_leaf_row(s, k, rho, NULL, row_ptr + (int64_t)kr * s->n_cols, col, val);
    }
}
