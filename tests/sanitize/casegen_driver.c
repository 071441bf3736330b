/* Drives the case generator on small seeded specs for a sanitizer build:
 * counts, fills, and checks the CSR it produced (row pointers consistent,
 * columns in range and strictly ascending within a row, values finite and
 * positive).  Exit status 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t nx, ny, nz;
    double h;
    int32_t n_beams, n_rows, n_cols;
    double pitch, sigma_vox, mu_per_mm, thr, jitter;
    uint64_t seed;
} cg_spec;

int64_t cg_count(const cg_spec* s, int64_t* row_nnz);
void cg_fill(const cg_spec* s, const int64_t* row_ptr, int32_t* col, float* val);

static int run(cg_spec s) {
    const int64_t nb = (int64_t)s.n_beams * s.n_rows * s.n_cols;
    const int64_t nv = (int64_t)s.nx * s.ny * s.nz;
    int64_t* cnt = calloc((size_t)nb, sizeof(int64_t));
    const int64_t nnz = cg_count(&s, cnt);
    int64_t* rp = malloc((size_t)(nb + 1) * sizeof(int64_t));
    rp[0] = 0;
    for (int64_t i = 0; i < nb; ++i) rp[i + 1] = rp[i] + cnt[i];
    if (rp[nb] != nnz) return 1;
    int32_t* col = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    float* val = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(float));
    cg_fill(&s, rp, col, val);
    for (int64_t i = 0; i < nb; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= nv) return 2;
            if (e > rp[i] && col[e] <= col[e - 1]) return 3;
            if (!(val[e] > 0.0f) || !isfinite(val[e])) return 4;
        }
    printf("nb %lld nv %lld nnz %lld\n", (long long)nb, (long long)nv, (long long)nnz);
    free(cnt);
    free(rp);
    free(col);
    free(val);
    return 0;
}

int main(void) {
    cg_spec a = {12, 12, 8, 4.0, 8, 4, 6, 6.0, 1.0, 0.005, 0.3, 0.02, 0};
    cg_spec b = {9, 7, 5, 2.5, 5, 3, 64, 5.0, 1.5, 0.005, 0.1, 0.02, 7};   /* odd grid, 64 columns */
    cg_spec c = {8, 8, 6, 4.0, 1, 1, 1, 6.0, 1.0, 0.005, 0.2, 0.0, 3};     /* one beamlet */
    int rc = run(a);
    if (!rc) rc = run(b);
    if (!rc) rc = run(c);
    return rc;
}
