"""Python binding of libvmat.so (the C ABI in include/vmat.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory (tensors) and the current stream.
The module raises if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmat.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vmat.h")

VMAT_OK, VMAT_ERR_INVALID_ARG, VMAT_ERR_DEVICE, VMAT_ERR_ALLOC, VMAT_ERR_NOT_CONVERGED, VMAT_ERR_UNSUPPORTED = range(6)
DTYPES = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3}
# (TB, RPW) product variants of the batched products, in the library's order
SPMM_VARIANTS = ((1, 64), (2, 32), (4, 16), (8, 8), (16, 4), (16, 8), (32, 2), (32, 4), (32, 8), (64, 1), (64, 2),
                 (64, 4), (64, 8))
LAYOUTS = {"auto": 0, "plain": 1, "tiled": 2}

_lib = None


class VmatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vmat error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_beams", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
        ("d_store", ctypes.c_int32),
        ("n_voxels", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("theta_deg", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
        ("val", ctypes.c_void_p), ("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p), ("T", ctypes.c_void_p),
        ("gamma", ctypes.c_double), ("circular", ctypes.c_int32), ("max_leaf_step", ctypes.c_int32),
        ("layout", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class LayoutInfo(ctypes.Structure):
    _fields_ = [("tiled", ctypes.c_int32), ("n_blocks", ctypes.c_int32), ("fwd_lanes", ctypes.c_int32),
                ("adj_lanes", ctypes.c_int32), ("fwd_entries", ctypes.c_int64), ("adj_entries", ctypes.c_int64),
                ("slots", ctypes.c_int64), ("fwd_bytes", ctypes.c_int64), ("adj_bytes", ctypes.c_int64),
                ("weight_labels", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Beams(ctypes.Structure):
    _fields_ = [("n_beams", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("circular", ctypes.c_int32), ("max_leaf_step", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("theta_deg", ctypes.c_void_p)]


class MasterOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("ls_max_steps", ctypes.c_int32),
                ("tol_rel", ctypes.c_double), ("kkt_ref", ctypes.c_double)]


class MasterReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("n_forward", ctypes.c_int32),
                ("n_adjoint", ctypes.c_int32), ("n_ls_evals", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("F", ctypes.c_double), ("gG", ctypes.c_double), ("kkt", ctypes.c_double),
                ("kkt_ref", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_cg_iter", ctypes.c_int32), ("master_mode", ctypes.c_int32), ("master", MasterOpts)]


class SolveReport(ctypes.Structure):
    _fields_ = [("cg_iters", ctypes.c_int32), ("master_iters", ctypes.c_int32), ("n_forward", ctypes.c_int32),
                ("n_adjoint", ctypes.c_int32), ("n_ls_evals", ctypes.c_int32), ("not_converged", ctypes.c_int32),
                ("F", ctypes.c_double), ("gG", ctypes.c_double), ("kkt_ref", ctypes.c_double)]


class SolveTrace(ctypes.Structure):
    _fields_ = [("beam", ctypes.c_void_p), ("price", ctypes.c_void_p), ("margin", ctypes.c_void_p),
                ("row_margin", ctypes.c_void_p), ("cost", ctypes.c_void_p), ("master_iters", ctypes.c_void_p),
                ("y", ctypes.c_void_p)]


_TRACE_FIELDS = ("beam", "price", "margin", "row_margin", "cost", "master_iters", "y")


def _trace_arrays(n):
    """Host arrays of one plan's trace (n beams); y is [iterations, n]."""
    return {"beam": np.zeros(n, np.int32), "price": np.zeros(n), "margin": np.zeros(n),
            "row_margin": np.zeros(n), "cost": np.zeros(n + 1), "master_iters": np.zeros(n, np.int32),
            "y": np.zeros((n, n))}


class RateOpts(ctypes.Structure):
    _fields_ = [("rate_max", ctypes.c_double), ("factor", ctypes.c_double), ("max_rounds", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("master", MasterOpts)]


class RateReport(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("feasible", ctypes.c_int32), ("master_iters", ctypes.c_int32),
                ("not_converged", ctypes.c_int32), ("gamma", ctypes.c_double), ("rate", ctypes.c_double),
                ("F", ctypes.c_double), ("gG", ctypes.c_double)]


def header_symbols():
    """Names of the functions declared in include/vmat.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:vmat_status|const char\*)\s+(vmat_\w+)\s*\(", text, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python paper_1005_4396_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "vmat_create": [ctypes.POINTER(_Problem), P, ctypes.POINTER(P)],
            "vmat_destroy": [P],
            "vmat_device_bytes": [P, ctypes.POINTER(I64)],
            "vmat_layout": [P, ctypes.POINTER(LayoutInfo)],
            "vmat_dose": [P, P, P, P, P, P, P],
            "vmat_dose_fluence": [P, P, P, P],
            "vmat_forward": [P, P, P, P],
            "vmat_adjoint": [P, P, P, P],
            "vmat_grad": [P, P, P, P, P, P, P, P, P, P, P],
            "vmat_grad_fluence": [P, P, P, P, P, P, P],
            "vmat_grad_apertures": [P, P, P, P, P, P, P, P, P],
            "vmat_price": [P, P, P, P, P, P, P, P, P, P],
            "vmat_forward_batched": [P, I32, P, P, P],
            "vmat_adjoint_batched": [P, I32, P, P, P],
            "vmat_grad_batched": [P, I32, I32, P, P, P, P, P, P, P, P],
            "vmat_tune_batched": [P, I32, P, P, P, P, I32, P, P, P],
            "vmat_set_batched_tile": [P, I32, I32, I32, I32, I32],
            "vmat_reserve_batched": [P, I32],
            "vmat_reserve_solve": [P],
            "vmat_set_weights": [P, P, P, P, P],
            "vmat_create_plan": [P, P, ctypes.POINTER(P)],
            "vmat_solve_variants": [P, ctypes.POINTER(SolveOpts), I32, I32, P, P, I32, P, P, P, P,
                                    ctypes.POINTER(SolveReport), P],
            "vmat_price_noalloc": [ctypes.POINTER(Beams), P, P, P, P, P, P, P, P, P],
            "vmat_read_stream": [P, ctypes.c_int64, P, I32, P],
            "vmat_read_write_stream": [P, ctypes.c_int64, P, ctypes.c_int64, P, I32, P],
            "vmat_enforce_rate": [P, ctypes.POINTER(RateOpts), P, P, P, P, ctypes.POINTER(RateReport), P],
            "vmat_solve_batched": [P, ctypes.POINTER(SolveOpts), I32, I32, P, P, P, P, P, P,
                                   ctypes.POINTER(SolveReport), ctypes.POINTER(SolveTrace), P, P],
            "vmat_master": [P, P, P, P, P, ctypes.POINTER(MasterOpts), ctypes.POINTER(MasterReport), P],
            "vmat_solve": [P, ctypes.POINTER(SolveOpts), P, P, P, P, P, ctypes.POINTER(SolveReport),
                           ctypes.POINTER(SolveTrace), P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = I32
        L.vmat_last_error.restype = ctypes.c_char_p
        L.vmat_last_error.argtypes = []
        _lib = L
    return _lib


def last_error() -> str:
    return lib().vmat_last_error().decode()


def _check(code, allow=()):
    if code != VMAT_OK and code not in allow:
        raise VmatError(code, last_error())
    return code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def read_stream(buf, partials, grid: int) -> None:
    """One streaming read of the device tensor buf (a measurement aid: the
    HBM read ceiling); partials: float32 device tensor of at least grid."""
    assert partials.numel() >= grid and partials.dtype.itemsize == 4
    _check(lib().vmat_read_stream(_ptr(buf), buf.numel() * buf.element_size(), _ptr(partials), grid, _stream()))


def read_write_stream(buf, wbuf, partials, grid: int) -> None:
    """The read of read_stream with all of the float64 device tensor wbuf
    written while it runs (a measurement aid: the ceiling of a stream with
    that share of writes); wbuf's byte size must be a multiple of 512."""
    assert partials.numel() >= grid and partials.dtype.itemsize == 4 and wbuf.dtype.itemsize == 8
    _check(lib().vmat_read_write_stream(_ptr(buf), buf.numel() * buf.element_size(), _ptr(wbuf),
                                        wbuf.numel() * 8, _ptr(partials), grid, _stream()))


def price_noalloc(theta, n_rows, n_cols, gamma, circular, max_leaf_step, g, y, l, r, occ, out_beam, out_price,
                  beam_prices=None) -> int:
    """vmat_price_noalloc on caller tensors (theta: float64 device [N]);
    returns the status code (outputs are written on the device)."""
    b = Beams(int(theta.numel()), int(n_rows), int(n_cols), int(circular), int(max_leaf_step), 0, float(gamma),
              theta.data_ptr())
    return lib().vmat_price_noalloc(ctypes.byref(b), _ptr(g), _ptr(y), _ptr(l), _ptr(r), _ptr(occ),
                                    _ptr(out_beam), _ptr(out_price), _ptr(beam_prices), _stream())


def master_opts(max_iter=200, ls_max_steps=50, tol_rel=1e-5, kkt_ref=0.0) -> MasterOpts:
    return MasterOpts(max_iter, ls_max_steps, tol_rel, kkt_ref)


@dataclasses.dataclass
class PriceOut:
    beam: int
    l: np.ndarray
    r: np.ndarray
    price: float
    margin: float
    row_margin: float
    beam_prices: np.ndarray


class Problem:
    """A handle over one problem (D, voxel weights, beams) on the current GPU."""

    def __init__(self, n_beams, n_rows, n_cols, n_voxels, theta_deg, row_ptr, col, val, alpha, beta, T,
                 gamma, circular=1, max_leaf_step=2, d_store="f32", layout="auto"):
        import torch
        self.N, self.R, self.C, self.nv = int(n_beams), int(n_rows), int(n_cols), int(n_voxels)
        self.nb = self.N * self.R * self.C
        self.device = row_ptr.device
        self._theta = np.ascontiguousarray(theta_deg, dtype=np.float64)
        for t, dt in ((row_ptr, torch.int64), (col, torch.int32), (val, torch.float32),
                      (alpha, torch.float32), (beta, torch.float32), (T, torch.float32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError("problem arrays must be contiguous CUDA tensors of the documented dtypes")
        p = _Problem(self.N, self.R, self.C, DTYPES[d_store], self.nv, int(col.numel()),
                     self._theta.ctypes.data, row_ptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                     alpha.data_ptr(), beta.data_ptr(), T.data_ptr(), float(gamma), int(circular),
                     int(max_leaf_step), LAYOUTS[layout], 0)
        h = ctypes.c_void_p()
        _check(lib().vmat_create(ctypes.byref(p), _stream(), ctypes.byref(h)))
        self._h = h
        self.d_store = d_store
        self.gamma, self.circular, self.max_leaf_step = float(gamma), int(circular), int(max_leaf_step)

    @classmethod
    def from_case(cls, case, d_store="f32", device="cuda", layout="auto"):
        import torch
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
        rp, col, val = t(case.row_ptr), t(case.col), t(case.val)
        a, b, T = t(case.alpha), t(case.beta), t(case.T)
        prob = cls(case.n_beams, case.n_rows, case.n_cols, case.n_voxels, case.theta_deg, rp, col, val, a, b, T,
                   case.gamma, case.circular, case.max_leaf_step, d_store, layout)
        torch.cuda.synchronize()
        return prob

    def solve_variants(self, label, table, K=4, opts: SolveOpts | None = None):
        """B full plans, variant b with weights table[b] (float [B, S, 3] of
        (alpha, beta, T) per structure; label uint8 [nv]), K at a time on K
        plan contexts over this problem's D (vmat_solve_variants).  Returns
        (reports, l [B, N*R], r, occ [B, N], y [B, N])."""
        import torch
        dev = self.device
        B, S = int(table.shape[0]), int(table.shape[1])
        l = torch.zeros(B, self.N * self.R, dtype=torch.int32, device=dev)
        r = torch.zeros_like(l)
        occ = torch.zeros(B, self.N, dtype=torch.uint8, device=dev)
        y = torch.zeros(B, self.N, dtype=torch.float64, device=dev)
        reps = (SolveReport * B)()
        _check(lib().vmat_solve_variants(self._h, ctypes.byref(opts) if opts else None, B, S, _ptr(label),
                                         _ptr(table), int(K), _ptr(l), _ptr(r), _ptr(occ), _ptr(y), reps,
                                         _stream()))
        return list(reps), l, r, occ, y

    def new_plan(self) -> "Problem":
        """A plan context on this problem's D (vmat_create_plan): its own
        weights (a copy of the current ones), plan, master state and stores;
        D is read from this handle, which must stay open while the context
        lives (closing it first raises)."""
        h = ctypes.c_void_p()
        _check(lib().vmat_create_plan(self._h, _stream(), ctypes.byref(h)))
        ctx = Problem.__new__(Problem)
        ctx.__dict__.update({k: v for k, v in self.__dict__.items() if k not in ("_h", "_src")})
        ctx._h = h
        ctx._src = self            # keeps the owner of D alive
        return ctx

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None):
            _check(lib().vmat_destroy(self._h))
            self._h = None
            self._src = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self) -> int:
        v = ctypes.c_int64()
        _check(lib().vmat_device_bytes(self._h, ctypes.byref(v)))
        return int(v.value)

    def layout(self) -> dict:
        info = LayoutInfo()
        _check(lib().vmat_layout(self._h, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in LayoutInfo._fields_ if k != "reserved"}

    # ------------------------------------------------------------ helpers
    def empty_plan(self):
        import torch
        dev = self.device
        return (torch.zeros(self.N * self.R, dtype=torch.int32, device=dev),
                torch.zeros(self.N * self.R, dtype=torch.int32, device=dev),
                torch.zeros(self.N, dtype=torch.uint8, device=dev),
                torch.zeros(self.N, dtype=torch.float64, device=dev))

    # ------------------------------------------------------------ calls
    def dose(self, y, l, r, occ, z=None):
        import torch
        if z is None:
            z = torch.empty(self.nv, dtype=torch.float32, device=self.device)
        _check(lib().vmat_dose(self._h, _ptr(y), _ptr(l), _ptr(r), _ptr(occ), _ptr(z), _stream()))
        return z

    def dose_fluence(self, x, z=None):
        import torch
        if z is None:
            z = torch.empty(self.nv, dtype=torch.float32, device=self.device)
        _check(lib().vmat_dose_fluence(self._h, _ptr(x), _ptr(z), _stream()))
        return z

    def forward(self, x, z=None):
        """z = D^T x (FP64 in, FP64 out), one kernel."""
        import torch
        if z is None:
            z = torch.empty(self.nv, dtype=torch.float64, device=self.device)
        _check(lib().vmat_forward(self._h, _ptr(x), _ptr(z), _stream()))
        return z

    def adjoint(self, w, g=None):
        """g = D w (FP32 w, FP64 g), one kernel."""
        import torch
        if g is None:
            g = torch.empty(self.nb, dtype=torch.float64, device=self.device)
        _check(lib().vmat_adjoint(self._h, _ptr(w), _ptr(g), _stream()))
        return g

    def forward_batched(self, X, Z=None):
        """Z = D^T X for B right-hand sides: X float [nb, B] -> Z double [nv, B]."""
        import torch
        B = X.shape[1]
        if Z is None:
            Z = torch.empty(self.nv, B, dtype=torch.float64, device=self.device)
        _check(lib().vmat_forward_batched(self._h, B, _ptr(X), _ptr(Z), _stream()))
        return Z

    def adjoint_batched(self, W, G=None):
        """G = D W for B right-hand sides: W float [nv, B] -> G double [nb, B]."""
        import torch
        B = W.shape[1]
        if G is None:
            G = torch.empty(self.nb, B, dtype=torch.float64, device=self.device)
        _check(lib().vmat_adjoint_batched(self._h, B, _ptr(W), _ptr(G), _stream()))
        return G

    def grad_batched(self, label, table, X, with_g=True):
        """Eq. 1 for B objective variants at once.  label uint8 [nv]; table
        float [B, S, 3] of (alpha, beta, T); X float [nb, B].  Returns cost
        double [B], Z double [nv, B], dF float [nv, B] and G double [nb, B]."""
        import torch
        B, S = table.shape[0], table.shape[1]
        dev = self.device
        Z = torch.empty(self.nv, B, dtype=torch.float64, device=dev)
        dF = torch.empty(self.nv, B, dtype=torch.float32, device=dev)
        cost = torch.empty(B, dtype=torch.float64, device=dev)
        G = torch.empty(self.nb, B, dtype=torch.float64, device=dev) if with_g else None
        _check(lib().vmat_grad_batched(self._h, B, S, _ptr(label), _ptr(table), _ptr(X), _ptr(Z), _ptr(cost),
                                       _ptr(dF), _ptr(G), _stream()))
        return {"cost": cost, "Z": Z, "dF": dF, "G": G}

    def enforce_rate(self, l, r, occ, y, rate_max, factor=10.0, max_rounds=8, master=None) -> RateReport:
        """Dose-rate feasibility of a final plan: raise gamma by `factor` and
        re-optimise y (in place) until the largest change per degree between
        neighbouring angles is at most rate_max."""
        o = RateOpts(rate_max, factor, max_rounds, 0, master if master is not None else MasterOpts(0, 0, 0.0, 0.0))
        rep = RateReport()
        _check(lib().vmat_enforce_rate(self._h, ctypes.byref(o), _ptr(l), _ptr(r), _ptr(occ), _ptr(y),
                                       ctypes.byref(rep), _stream()))
        return rep

    def reserve_batched(self, max_variants):
        _check(lib().vmat_reserve_batched(self._h, max_variants))

    def solve_batched(self, label, table, opts: SolveOpts | None = None, want_trace=True):
        """Column generation for B objective variants at once (table float
        [B, S, 3] of (alpha, beta, T) per structure label).  Returns the plans
        (l [B, N*R], r, occ [B, N], y [B, N]), the B reports, the B traces and
        the numbers of forward and adjoint SpMM launches."""
        import torch
        B, S = table.shape[0], table.shape[1]
        dev, N, R = self.device, self.N, self.R
        l = torch.zeros(B, N * R, dtype=torch.int32, device=dev)
        r = torch.zeros(B, N * R, dtype=torch.int32, device=dev)
        occ = torch.zeros(B, N, dtype=torch.uint8, device=dev)
        y = torch.zeros(B, N, dtype=torch.float64, device=dev)
        reps = (SolveReport * B)()
        trs, tr_c = None, None
        if want_trace:
            trs = [_trace_arrays(N) for _ in range(B)]
            tr_c = (SolveTrace * B)(*[SolveTrace(*(t[k].ctypes.data for k in _TRACE_FIELDS)) for t in trs])
        cnt = (ctypes.c_int64 * 2)()
        _check(lib().vmat_solve_batched(self._h, ctypes.byref(opts) if opts is not None else None, B, S,
                                        _ptr(label), _ptr(table), _ptr(l), _ptr(r), _ptr(occ), _ptr(y), reps,
                                        tr_c, cnt, _stream()))
        reports = [reps[b] for b in range(B)]
        if trs is not None:
            trs = [{k: (v[:rep.cg_iters + 1] if k == "cost" else v[:rep.cg_iters]) for k, v in t.items()}
                   for t, rep in zip(trs, reports)]
        return (l, r, occ, y), reports, trs, (cnt[0], cnt[1])

    def set_batched_tile(self, B, fwd, adj):
        """Product variants at B right-hand sides: fwd, adj = (TB, RPW) pairs
        ((0, 0): default)."""
        _check(lib().vmat_set_batched_tile(self._h, B, fwd[0], fwd[1], adj[0], adj[1]))

    def tune_batched(self, B, reps=5, seed=0):
        """Times every product variant (TB right-hand sides per pass, RPW rows
        per wave) for both products at B right-hand sides and keeps the
        fastest.  Returns (forward (TB, RPW), adjoint (TB, RPW), times in ms
        by variant)."""
        import torch
        dev = self.device
        g = torch.Generator(device="cpu").manual_seed(seed)
        X = torch.rand(self.nb, B, generator=g).to(dev, torch.float32)
        W = torch.randn(self.nv, B, generator=g).to(dev, torch.float32)
        Z = torch.empty(self.nv, B, dtype=torch.float64, device=dev)
        G = torch.empty(self.nb, B, dtype=torch.float64, device=dev)
        best = (ctypes.c_int32 * 4)()
        n = len(SPMM_VARIANTS)
        times = (ctypes.c_float * (2 * n))()
        _check(lib().vmat_tune_batched(self._h, B, _ptr(X), _ptr(Z), _ptr(W), _ptr(G), reps, best, times,
                                       _stream()))
        return ((best[0], best[1]), (best[2], best[3]),
                {"forward": dict(zip(SPMM_VARIANTS, times[:n])), "adjoint": dict(zip(SPMM_VARIANTS, times[n:]))})

    def grad(self, y, l, r, occ, want=("z", "dF", "g", "dfdy")):
        import torch
        dev = self.device
        cost = torch.empty(2, dtype=torch.float64, device=dev)
        z = torch.empty(self.nv, dtype=torch.float32, device=dev) if "z" in want else None
        dF = torch.empty(self.nv, dtype=torch.float32, device=dev) if "dF" in want else None
        g = torch.empty(self.nb, dtype=torch.float64, device=dev) if "g" in want else None
        dfdy = torch.empty(self.N, dtype=torch.float64, device=dev) if "dfdy" in want else None
        _check(lib().vmat_grad(self._h, _ptr(y), _ptr(l), _ptr(r), _ptr(occ), _ptr(cost), _ptr(z), _ptr(dF),
                               _ptr(g), _ptr(dfdy), _stream()))
        return {"cost": cost, "z": z, "dF": dF, "g": g, "dfdy": dfdy}

    def grad_apertures(self, y, l, r, occ, w, want_g=False):
        """dfdy = sum over each aperture of (D w) + gamma dG/dy (w: FP32 dose derivative)."""
        import torch
        g = torch.empty(self.nb, dtype=torch.float64, device=self.device) if want_g else None
        dfdy = torch.empty(self.N, dtype=torch.float64, device=self.device)
        _check(lib().vmat_grad_apertures(self._h, _ptr(y), _ptr(l), _ptr(r), _ptr(occ), _ptr(w), _ptr(g),
                                         _ptr(dfdy), _stream()))
        return dfdy, g

    def grad_fluence(self, x, want=("z", "dF", "g")):
        import torch
        dev = self.device
        cost = torch.empty(2, dtype=torch.float64, device=dev)
        z = torch.empty(self.nv, dtype=torch.float32, device=dev) if "z" in want else None
        dF = torch.empty(self.nv, dtype=torch.float32, device=dev) if "dF" in want else None
        g = torch.empty(self.nb, dtype=torch.float64, device=dev) if "g" in want else None
        _check(lib().vmat_grad_fluence(self._h, _ptr(x), _ptr(cost), _ptr(z), _ptr(dF), _ptr(g), _stream()))
        return {"cost": cost, "z": z, "dF": dF, "g": g}

    def price(self, g, y, l, r, occ) -> PriceOut:
        import torch
        dev = self.device
        ob = torch.empty(1 + 2 * self.R, dtype=torch.int32, device=dev)
        op = torch.empty(3, dtype=torch.float64, device=dev)
        bp = torch.empty(self.N, dtype=torch.float64, device=dev)
        _check(lib().vmat_price(self._h, _ptr(g), _ptr(y), _ptr(l), _ptr(r), _ptr(occ), _ptr(ob), _ptr(op),
                                _ptr(bp), _stream()))
        ob, op, bp = ob.cpu().numpy(), op.cpu().numpy(), bp.cpu().numpy()
        R = self.R
        return PriceOut(int(ob[0]), ob[1:1 + R].copy(), ob[1 + R:].copy(), float(op[0]), float(op[1]),
                        float(op[2]), bp)

    def master(self, l, r, occ, y, opts: MasterOpts | None = None):
        rep = MasterReport()
        code = lib().vmat_master(self._h, _ptr(l), _ptr(r), _ptr(occ), _ptr(y),
                                 ctypes.byref(opts) if opts is not None else None, ctypes.byref(rep), _stream())
        _check(code, allow=(VMAT_ERR_NOT_CONVERGED,))
        return rep

    def set_weights(self, alpha, beta, T):
        """New voxel weights and thresholds of eq. 1 (float32 device tensors [nv])
        on this handle: a plan variant with the same D."""
        for t in (alpha, beta, T):
            if t.dtype.itemsize != 4 or not t.is_cuda or not t.is_contiguous() or t.numel() != self.nv:
                raise ValueError("alpha, beta, T must be contiguous float32 CUDA tensors of n_voxels")
        _check(lib().vmat_set_weights(self._h, _ptr(alpha), _ptr(beta), _ptr(T), _stream()))

    def reserve_solve(self):
        """Aperture-dose store and captured iteration for master_mode 1."""
        _check(lib().vmat_reserve_solve(self._h))

    def solve(self, l, r, occ, y, opts: SolveOpts | None = None, z=None, want_trace=True):
        if opts is not None and opts.master_mode == 1:
            self.reserve_solve()
        rep = SolveReport()
        n = self.N
        tr_arrays = None
        tr = None
        if want_trace:
            tr_arrays = _trace_arrays(n)
            tr = SolveTrace(*(tr_arrays[k].ctypes.data for k in _TRACE_FIELDS))
        _check(lib().vmat_solve(self._h, ctypes.byref(opts) if opts is not None else None, _ptr(l), _ptr(r),
                                _ptr(occ), _ptr(y), _ptr(z), ctypes.byref(rep),
                                ctypes.byref(tr) if tr is not None else None, _stream()))
        if tr_arrays is not None:
            k = rep.cg_iters
            tr_arrays = {key: (v[:k + 1] if key == "cost" else v[:k]) for key, v in tr_arrays.items()}
        return rep, tr_arrays
