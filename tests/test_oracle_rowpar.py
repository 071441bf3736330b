"""The all-cores product of the CPU baseline (oracle/rowpar.c) against the
definition of the dose model's products (Sec. 2.1): exact on small-integer
data (dense brute force), and equal to the plain reference product of the
FP64 oracle on a generated case, for both orientations of D."""
import numpy as np
import scipy.sparse as sp

import oracle as O
from oracle import rowpar
from _cases import small_case


def test_rowpar_exact_on_small_integers():
    rng = np.random.default_rng(3)
    A = rng.integers(0, 4, (37, 53)) * (rng.random((37, 53)) < 0.3)
    x = rng.integers(-5, 6, 53).astype(np.float64)
    got = rowpar.spmv(sp.csr_matrix(A.astype(np.float64)), x)
    want = np.array([sum(int(A[i, j]) * int(x[j]) for j in range(53)) for i in range(37)], dtype=np.float64)
    assert np.array_equal(got, want)


def test_rowpar_matches_reference_products():
    c = small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8))
    D = O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels)
    rng = np.random.default_rng(4)
    x = rng.random(c.n_beamlets)
    w = rng.standard_normal(c.n_voxels)
    z = rowpar.spmv(D.T.tocsr(), x)       # dose z = D^T x, rows = voxels
    g = rowpar.spmv(D, w)                  # prices g = D w, rows = beamlets
    z_ref, g_ref = O.dose(D, x), D @ w
    assert np.abs(z - z_ref).max() <= 1e-14 * np.abs(z_ref).max()
    assert np.abs(g - g_ref).max() <= 1e-14 * np.abs(g_ref).max()
    assert rowpar.threads() >= 1
