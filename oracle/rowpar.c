/*
 * Row-parallel sparse products of the dose model (Sec. 2.1, the constraint
 * of eq. 3): out_i = sum_j A_ij x_j over the rows of a CSR matrix, one row per
 * OpenMP iteration, each row summed in order in FP64.  With A = D
 * (beamlet-major) this is the beamlet price g = D r of Sec. 2.2; with A = D^T
 * (voxel-major) the dose z = D^T x.
 *
 * TEST INFRASTRUCTURE ONLY: the all-cores CPU baseline of the two products
 * (bench.py) and its pin against the plain reference product (tests/).  The
 * GPU library never calls it.  Built with plain IEEE arithmetic (no
 * fast-math).
 */
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_rowpar_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_rowpar_spmv(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const double* val,
                        const double* x, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += val[e] * x[col[e]];
        out[i] = s;
    }
}
