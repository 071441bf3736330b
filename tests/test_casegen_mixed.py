"""Mixed voxel resolution (Sec. 3: unspecified tissue at twice the voxel size
per dimension): construction checks against the full-resolution case."""
import numpy as np
import scipy.sparse as sp

import casegen
import oracle as O


def _cases():
    c = casegen.make_case(casegen.tiny_case(n_beams=6, n_rows=4, n_cols=8, grid=(16, 16, 10)))
    m, owner = casegen.mixed_resolution(c)
    return c, m, owner


def test_mixed_voxels_partition_the_grid():
    c, m, owner = _cases()
    nx, ny, nz = c.spec.grid
    count = np.bincount(owner, minlength=m.n_voxels)
    assert owner.min() == 0 and owner.max() == m.n_voxels - 1 and np.all(count >= 1)
    # every labelled voxel keeps its own voxel, weights and label
    lab = np.flatnonzero(c.label != 0)
    assert np.all(count[owner[lab]] == 1)
    np.testing.assert_array_equal(m.label[owner[lab]], c.label[lab])
    np.testing.assert_array_equal(m.T[owner[lab]], c.T[lab])
    np.testing.assert_array_equal(m.alpha[owner[lab]], c.alpha[lab])
    # a coarse voxel weighs as much as its members together
    merged = np.flatnonzero(count > 1)
    first = np.array([np.flatnonzero(owner == v)[0] for v in merged[:50]])
    np.testing.assert_allclose(m.beta[merged[:50]], c.beta[first] * count[merged[:50]], rtol=1e-6)
    # merged voxels are body-only 2x2x2 blocks of the grid
    j = np.arange(c.n_voxels)
    ix, iy, iz = j % nx, (j // nx) % ny, j // (nx * ny)
    for v in np.flatnonzero(count > 1)[:50]:
        mem = np.flatnonzero(owner == v)
        assert len(mem) == 8 and np.all(c.label[mem] == 0)
        assert len({(a // 2, b // 2, d // 2) for a, b, d in zip(ix[mem], iy[mem], iz[mem])}) == 1
    assert m.n_voxels < c.n_voxels and m.nnz < c.nnz


def test_mixed_columns_are_member_means():
    c, m, owner = _cases()
    Df = O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels).toarray()
    Dm = O.dose_matrix(m.row_ptr, m.col, m.val, m.n_voxels).toarray()
    for v in range(m.n_voxels):
        mem = np.flatnonzero(owner == v)
        ref = Df[:, mem].mean(axis=1)
        np.testing.assert_allclose(Dm[:, v], ref, rtol=2 ** -23, atol=0)


def test_mixed_dose_is_group_average_of_full_dose():
    c, m, owner = _cases()
    rng = np.random.default_rng(0)
    x = rng.random(c.n_beamlets)
    zf = O.dose(O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels), x)
    zm = O.dose(O.dose_matrix(m.row_ptr, m.col, m.val, m.n_voxels), x)
    avg = np.bincount(owner, weights=zf) / np.bincount(owner)
    np.testing.assert_allclose(zm, avg, rtol=1e-6, atol=1e-12 * np.abs(zf).max())
