"""Seeded synthetic VMAT cases: pencil-beam D, voxel structures, beam angles.

Input synthesis only, shared as a data source by the CPU reference
(``oracle/``) and the GPU library tests and benchmark.  Nothing here computes
any part of the optimiser (dose, penalty, gradient, pricing, master).

The C core (``casegen.c``) enumerates the sparse dose-deposition matrix D
(row = beamlet, column = voxel; Sec. 2.1 of the paper).  This module adds
the voxel structures (targets / organs at risk / body with their weights
alpha_j, beta_j and thresholds T_j of eq. 1) and the case presets.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcasegen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C generator in-tree (gcc, OpenMP)."""
    src = os.path.join(_HERE, "casegen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(src) > os.path.getmtime(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Spec(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("n_beams", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
        ("pitch", ctypes.c_double), ("sigma_vox", ctypes.c_double),
        ("mu_per_mm", ctypes.c_double), ("thr", ctypes.c_double),
        ("jitter", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.cg_count.restype = ctypes.c_int64
        lib.cg_count.argtypes = [ctypes.POINTER(_Spec), ctypes.c_void_p]
        lib.cg_fill.restype = None
        lib.cg_fill.argtypes = [ctypes.POINTER(_Spec), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.cg_xi.restype = ctypes.c_double
        lib.cg_xi.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        _lib = lib
    return _lib


# --------------------------------------------------------------------------
# Structures.  Each shape is a dict; precedence is the list order (first wins).
#   kind "ellipsoid": centre (mm), semi (mm, 3)
#   kind "cyl_z" / "cyl_x": centre, radius, half_len (mm); axis along z / x
#   kind "shell_y": cylinder about z, r_in..r_out, y > centre_y, |z - cz| <= half_len
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Shape:
    name: str
    kind: str
    centre: tuple
    T: float
    alpha: float
    beta: float
    semi: tuple = (0.0, 0.0, 0.0)
    radius: float = 0.0
    r_in: float = 0.0
    half_len: float = 0.0


@dataclasses.dataclass
class CaseSpec:
    name: str
    grid: tuple            # (nx, ny, nz)
    h: float               # voxel edge (mm)
    n_beams: int
    n_rows: int            # leaf rows (along z)
    n_cols: int            # columns (along leaf travel)
    pitch: float           # beamlet pitch (mm)
    sigma_vox: float
    mu_per_mm: float
    thr: float
    shapes: list
    body: tuple = (0.0, 0.0, 0.01)     # (T, alpha, beta) of unlabelled tissue
    gamma: float = 0.1
    circular: int = 1
    max_leaf_step: int = 2
    jitter: float = 0.02
    seed: int = 0


@dataclasses.dataclass
class Case:
    spec: CaseSpec
    n_beams: int
    n_rows: int
    n_cols: int
    n_voxels: int
    theta_deg: np.ndarray   # float64 [N]
    row_ptr: np.ndarray     # int64 [nb+1]   beamlet-major CSR of D
    col: np.ndarray         # int32 [nnz]
    val: np.ndarray         # float32 [nnz]
    alpha: np.ndarray       # float32 [nv]
    beta: np.ndarray        # float32 [nv]
    T: np.ndarray           # float32 [nv]
    label: np.ndarray       # uint8 [nv]: 0 body, 1.. shapes in spec order

    @property
    def n_beamlets(self) -> int:
        return self.n_beams * self.n_rows * self.n_cols

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def gamma(self) -> float:
        return self.spec.gamma

    @property
    def circular(self) -> int:
        return self.spec.circular

    @property
    def max_leaf_step(self) -> int:
        return self.spec.max_leaf_step


def voxel_centres(nx, ny, nz, h):
    x = (np.arange(nx) + 0.5 - 0.5 * nx) * h
    y = (np.arange(ny) + 0.5 - 0.5 * ny) * h
    z = (np.arange(nz) + 0.5 - 0.5 * nz) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def _inside(shape: Shape, X, Y, Z):
    cx, cy, cz = shape.centre
    if shape.kind == "ellipsoid":
        a, b, c = shape.semi
        return ((X - cx) / a) ** 2 + ((Y - cy) / b) ** 2 + ((Z - cz) / c) ** 2 <= 1.0
    if shape.kind == "cyl_z":
        return ((X - cx) ** 2 + (Y - cy) ** 2 <= shape.radius ** 2) & (np.abs(Z - cz) <= shape.half_len)
    if shape.kind == "cyl_x":
        return ((Y - cy) ** 2 + (Z - cz) ** 2 <= shape.radius ** 2) & (np.abs(X - cx) <= shape.half_len)
    if shape.kind == "shell_y":
        rr = (X - cx) ** 2 + (Y - cy) ** 2
        return (rr <= shape.radius ** 2) & (rr >= shape.r_in ** 2) & (Y >= cy) & (np.abs(Z - cz) <= shape.half_len)
    raise ValueError(shape.kind)


def rasterise(spec: CaseSpec):
    nx, ny, nz = spec.grid
    X, Y, Z = voxel_centres(nx, ny, nz, spec.h)
    nv = nx * ny * nz
    label = np.zeros(nv, dtype=np.uint8)
    T = np.full(nv, spec.body[0], dtype=np.float32)
    alpha = np.full(nv, spec.body[1], dtype=np.float32)
    beta = np.full(nv, spec.body[2], dtype=np.float32)
    taken = np.zeros(nv, dtype=bool)
    for s_idx, sh in enumerate(spec.shapes):
        m = _inside(sh, X, Y, Z) & ~taken
        label[m] = s_idx + 1
        T[m], alpha[m], beta[m] = sh.T, sh.alpha, sh.beta
        taken |= m
    return label, alpha, beta, T


def _cspec(spec: CaseSpec) -> _Spec:
    nx, ny, nz = spec.grid
    return _Spec(nx, ny, nz, spec.h, spec.n_beams, spec.n_rows, spec.n_cols, spec.pitch,
                 spec.sigma_vox, spec.mu_per_mm, spec.thr, spec.jitter, spec.seed)


def count_nnz(spec: CaseSpec) -> int:
    lib = _load()
    nb = spec.n_beams * spec.n_rows * spec.n_cols
    cnt = np.zeros(nb, dtype=np.int64)
    cs = _cspec(spec)
    return int(lib.cg_count(ctypes.byref(cs), cnt.ctypes.data))


def make_case(spec: CaseSpec) -> Case:
    lib = _load()
    nb = spec.n_beams * spec.n_rows * spec.n_cols
    cnt = np.zeros(nb, dtype=np.int64)
    cs = _cspec(spec)
    nnz = int(lib.cg_count(ctypes.byref(cs), cnt.ctypes.data))
    if nnz >= 2 ** 31 - 1:
        raise ValueError("nnz exceeds int32 column-pointer range of this generator")
    row_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(cnt, out=row_ptr[1:])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float32)
    lib.cg_fill(ctypes.byref(cs), row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    label, alpha, beta, T = rasterise(spec)
    theta = np.arange(spec.n_beams, dtype=np.float64) * (360.0 / spec.n_beams)
    nx, ny, nz = spec.grid
    return Case(spec, spec.n_beams, spec.n_rows, spec.n_cols, nx * ny * nz, theta,
                row_ptr, col, val, alpha, beta, T, label)


def xi(seed: int, i: int, j: int) -> float:
    return float(_load().cg_xi(seed, i, j))


from .presets import PRESETS, preset, tiny_case  # noqa: E402,F401


def variant_table(case: Case, n_variants: int, seed: int = 0, spread=(0.5, 2.0), t_spread=(0.95, 1.05)):
    """Objective variants of one case: float32 [B, S, 3] of (alpha, beta, T)
    per variant and structure label (0 body, 1.. shapes).  Each weight is the
    structure's base weight times a U[spread] factor; thresholds of structures
    with an under-dose weight (targets) are scaled by U[t_spread]."""
    spec = case.spec
    base = [(spec.body[1], spec.body[2], spec.body[0])] + [(s.alpha, s.beta, s.T) for s in spec.shapes]
    base = np.asarray(base, dtype=np.float64)
    rng = np.random.default_rng(seed)
    B, S = n_variants, base.shape[0]
    tab = np.empty((B, S, 3), dtype=np.float64)
    tab[:, :, 0] = base[:, 0] * rng.uniform(*spread, (B, S))
    tab[:, :, 1] = base[:, 1] * rng.uniform(*spread, (B, S))
    t_fac = np.where(base[:, 0] > 0, rng.uniform(*t_spread, (B, S)), 1.0)
    tab[:, :, 2] = base[:, 2] * t_fac
    return tab.astype(np.float32)


def mixed_resolution(case: Case, factor: int = 2):
    """The case with unspecified tissue at `factor` times the voxel size per
    dimension: every factor^3 group of full-resolution voxels that holds only
    unlabelled voxels becomes one coarse voxel, whose dose coefficients are the
    mean of its members' (the dose at the coarse voxel as the average over its
    volume); groups that touch a target or organ keep their voxels.  A coarse
    voxel stands for the volume of its members, so its weights alpha and beta
    are the members' times their number (F keeps approximating the sum over
    the full-resolution voxels).  Mixed voxels are numbered in the order of
    their first full-resolution member.

    Returns (mixed case, owner), owner[j] = mixed voxel of full voxel j."""
    import scipy.sparse as sp
    nx, ny, nz = case.spec.grid
    j = np.arange(case.n_voxels)
    ix, iy, iz = j % nx, (j // nx) % ny, j // (nx * ny)
    gx, gy, gz = (nx + factor - 1) // factor, (ny + factor - 1) // factor, (nz + factor - 1) // factor
    group = (iz // factor) * (gy * gx) + (iy // factor) * gx + (ix // factor)
    labelled = np.zeros(gx * gy * gz, dtype=bool)
    np.logical_or.at(labelled, group, case.label != 0)
    merged = ~labelled[group]
    # key of a mixed voxel: its group for merged voxels, else its own index
    key = np.where(merged, -(group + 1), j)
    _, first_idx, inv = np.unique(key, return_index=True, return_inverse=True)
    rank = np.empty(len(first_idx), dtype=np.int64)
    rank[np.argsort(first_idx, kind="stable")] = np.arange(len(first_idx))
    owner = rank[inv.ravel()]
    n = len(first_idx)
    count = np.bincount(owner, minlength=n).astype(np.float64)
    P = sp.csr_matrix((1.0 / count[owner], (j, owner)), shape=(case.n_voxels, n))
    D = sp.csr_matrix((case.val.astype(np.float64), case.col, case.row_ptr),
                      shape=(case.n_beamlets, case.n_voxels))
    Dm = (D @ P).tocsr()
    Dm.sort_indices()
    rep = np.full(n, case.n_voxels, dtype=np.int64)
    np.minimum.at(rep, owner, j)        # first member of each mixed voxel
    vol = count.astype(np.float32)
    mixed = Case(case.spec, case.n_beams, case.n_rows, case.n_cols, n, case.theta_deg.copy(),
                 Dm.indptr.astype(np.int64), Dm.indices.astype(np.int32), Dm.data.astype(np.float32),
                 case.alpha[rep] * vol, case.beta[rep] * vol, case.T[rep].copy(), case.label[rep].copy())
    return mixed, owner
