"""Shared test fixtures: seeded cases, the FP64 reference matrices, random plans.

Seeded inputs only; no expected value here comes from the GPU library.
"""
from __future__ import annotations

import functools

import numpy as np

import casegen
import oracle as O


@functools.lru_cache(maxsize=None)
def preset_case(name: str):
    return casegen.make_case(casegen.preset(name))


@functools.lru_cache(maxsize=None)
def small_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8), thr=0.3, circular=1, max_leaf_step=2, seed=0):
    return casegen.make_case(casegen.tiny_case(n_beams=n_beams, n_rows=n_rows, n_cols=n_cols, grid=grid, thr=thr,
                                               circular=circular, max_leaf_step=max_leaf_step, seed=seed))


def oracle_D(c, vals=None):
    return O.dose_matrix(c.row_ptr, c.col, c.val if vals is None else vals, c.n_voxels)


def random_plan(c, seed, p_occ=0.6, y_scale=3.0):
    """Random apertures (row intervals), occupancy and intensities."""
    rng = np.random.default_rng(seed)
    N, R, C = c.n_beams, c.n_rows, c.n_cols
    occ = (rng.random(N) < p_occ).astype(np.uint8)
    if not occ.any():
        occ[0] = 1
    a = rng.integers(0, C + 1, N * R)
    b = rng.integers(0, C + 1, N * R)
    l = np.minimum(a, b).astype(np.int32)
    r = np.maximum(a, b).astype(np.int32)
    y = (rng.random(N) * y_scale * occ).astype(np.float64)
    return l, r, occ, y


def hand_case(seed=0):
    """A hand-built case with edge structure: empty beamlet rows, empty voxel
    rows, beamlet rows longer than one wave, a voxel hit by every beamlet, and
    a voxel count that is not a multiple of 64."""
    rng = np.random.default_rng(seed)
    N, R, C = 5, 3, 7
    nb = N * R * C
    nv = 301
    rows = []
    for i in range(nb):
        kind = i % 9
        if kind == 0:
            cols = np.array([], dtype=np.int64)                 # empty beamlet row
        elif kind == 1:
            cols = np.sort(rng.choice(nv - 1, 150, replace=False))  # long row
        else:
            cols = np.sort(rng.choice(nv - 1, int(rng.integers(1, 12)), replace=False))
        cols = cols[cols != 17]                                  # voxel 17 stays empty
        cols = np.union1d(cols, [nv - 1])                        # voxel nv-1 hit by all
        rows.append(cols)
    row_ptr = np.zeros(nb + 1, np.int64)
    row_ptr[1:] = np.cumsum([len(c) for c in rows])
    col = np.concatenate(rows).astype(np.int32)
    val = (rng.random(len(col)) * 0.9 + 0.1).astype(np.float32)
    spec = casegen.tiny_case(n_beams=N, n_rows=R, n_cols=C)
    alpha = (rng.random(nv) < 0.3).astype(np.float32)
    beta = (rng.random(nv) * 0.5 + 0.01).astype(np.float32)
    T = (rng.random(nv) * 3).astype(np.float32)
    theta = np.sort(rng.choice(360, N, replace=False)).astype(np.float64)
    return casegen.Case(spec, N, R, C, nv, theta, row_ptr, col, val, alpha, beta, T, np.zeros(nv, np.uint8))


def scatter_case(nb_rows=30, n_cols=40, n_beams=10, nv=300, per_row=3, seed=0):
    """Beamlets that each touch a few random voxels of a small voxel set: a
    voxel block then reaches more beamlets than fit one tile, so the tiled
    layout has to split blocks (or, for tiny nv, cannot tile at all)."""
    rng = np.random.default_rng(seed)
    N, R, C = n_beams, nb_rows, n_cols
    nb = N * R * C
    rows = [np.sort(rng.choice(nv, min(per_row, nv), replace=False)) for _ in range(nb)]
    row_ptr = np.zeros(nb + 1, np.int64)
    row_ptr[1:] = np.cumsum([len(c) for c in rows])
    col = np.concatenate(rows).astype(np.int32)
    val = (rng.random(len(col)) * 0.9 + 0.1).astype(np.float32)
    spec = casegen.tiny_case(n_beams=N, n_rows=R, n_cols=C)
    alpha = np.ones(nv, np.float32)
    beta = np.full(nv, 0.5, np.float32)
    T = (rng.random(nv) * 50 + 10).astype(np.float32)
    theta = np.arange(N, dtype=np.float64) * (360.0 / N)
    return casegen.Case(spec, N, R, C, nv, theta, row_ptr, col, val, alpha, beta, T, np.zeros(nv, np.uint8))
