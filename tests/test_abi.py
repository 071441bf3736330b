"""The C-ABI library without a GPU: it loads, exports every function that
include/vmat.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os

import pytest

import paper_1005_4396_amd as P
from paper_1005_4396_amd import vmat as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(V.LIB_PATH):
        pytest.skip("libvmat.so not built (run __graft_entry__.build())")
    return V.lib()


def test_header_declares_the_paper_entry_points():
    names = V.header_symbols()
    for n in ("vmat_dose", "vmat_grad", "vmat_price", "vmat_master", "vmat_solve", "vmat_create",
              "vmat_destroy", "vmat_forward_batched", "vmat_adjoint_batched", "vmat_grad_batched",
              "vmat_tune_batched"):
        assert n in names, n


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in V.header_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_null_handle_rejected():
    L = _lib()
    assert L.vmat_dose(None, None, None, None, None, None, None) == V.VMAT_ERR_INVALID_ARG
    assert "handle" in V.last_error()
    assert L.vmat_forward_batched(None, 4, None, None, None) == V.VMAT_ERR_INVALID_ARG
    assert L.vmat_set_batched_tile(None, 4, 8, 8, 8, 8) == V.VMAT_ERR_INVALID_ARG
    h = ctypes.c_void_p(1)
    assert L.vmat_create_plan(None, None, ctypes.byref(h)) == V.VMAT_ERR_INVALID_ARG
    assert h.value is None            # the output is cleared on every path out
    assert L.vmat_destroy(None) in (V.VMAT_OK, V.VMAT_ERR_INVALID_ARG)


def test_create_rejects_bad_problem_without_device():
    L = _lib()
    h = ctypes.c_void_p()
    assert L.vmat_create(None, None, ctypes.byref(h)) == V.VMAT_ERR_INVALID_ARG
    p = V._Problem()
    p.n_beams, p.n_rows, p.n_cols = 0, 4, 4     # no beams
    assert L.vmat_create(ctypes.byref(p), None, ctypes.byref(h)) == V.VMAT_ERR_INVALID_ARG
    assert V.last_error()


def test_status_codes_match_header():
    with open(os.path.join(ROOT, "include", "vmat.h")) as f:
        text = f.read()
    for name in ("VMAT_OK", "VMAT_ERR_INVALID_ARG", "VMAT_ERR_DEVICE", "VMAT_ERR_ALLOC",
                 "VMAT_ERR_NOT_CONVERGED", "VMAT_ERR_UNSUPPORTED"):
        assert name in text
        assert hasattr(V, name)


def test_product_path_has_no_fallback(monkeypatch):
    """Without the built library the binding raises instead of computing."""
    monkeypatch.setattr(V, "_lib", None)
    monkeypatch.setattr(V, "LIB_PATH", os.path.join(ROOT, "no_such_libvmat.so"))
    with pytest.raises(RuntimeError):
        V.lib()
    assert not hasattr(P, "oracle")


def test_create_without_a_device_reports_an_error():
    """Without a GPU every device step fails: vmat_create must return an error
    status with a message (never crash or abort).  Skipped where a GPU is
    present, since the arrays here are host memory."""
    import numpy as np
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    L = _lib()
    N, R, C, nv = 2, 1, 2, 3
    theta = np.array([0.0, 180.0])
    row_ptr = np.array([0, 1, 1, 2, 2], np.int64)
    col = np.array([0, 2], np.int32)
    val = np.array([1.0, 0.5], np.float32)
    ab = np.ones(nv, np.float32)
    p = V._Problem()
    p.n_beams, p.n_rows, p.n_cols, p.n_voxels, p.nnz = N, R, C, nv, 2
    p.theta_deg = theta.ctypes.data
    p.row_ptr, p.col, p.val = row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data
    p.alpha = p.beta = p.T = ab.ctypes.data
    h = ctypes.c_void_p()
    rc = L.vmat_create(ctypes.byref(p), None, ctypes.byref(h))
    assert rc in (V.VMAT_ERR_ALLOC, V.VMAT_ERR_DEVICE)
    assert V.last_error()
    assert not h.value


def test_read_stream_rejects_bad_arguments_before_launch():
    """The measurement aid checks its arguments on the host: nothing is
    launched for a null buffer, a size that is not a positive multiple of
    16, or a grid outside [1, 65536] (the pointers below are never touched)."""
    L = _lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.vmat_read_stream(None, 1024, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert L.vmat_read_stream(fake, 1000, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert L.vmat_read_stream(fake, 0, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert L.vmat_read_stream(fake, 1024, fake, 0, None) == V.VMAT_ERR_INVALID_ARG
    assert L.vmat_read_stream(fake, 1024, fake, 65537, None) == V.VMAT_ERR_INVALID_ARG
    assert "grid" in V.last_error()


def test_read_write_stream_rejects_bad_arguments_before_launch():
    """The read-with-writes aid checks its arguments on the host: a null read
    buffer or partials, a read size that is not a positive multiple of 16, a
    write size that is negative or not a multiple of 512, a null write buffer
    with writes asked for, a grid outside [1, 65536]."""
    L = _lib()
    fake = ctypes.c_void_p(0x1000)
    rw = L.vmat_read_write_stream
    assert rw(None, 1024, fake, 512, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert rw(fake, 1024, fake, 512, None, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert rw(fake, 1000, fake, 512, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert rw(fake, 1024, fake, -512, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert rw(fake, 1024, fake, 100, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert "512" in V.last_error()
    assert rw(fake, 1024, None, 512, fake, 8, None) == V.VMAT_ERR_INVALID_ARG
    assert rw(fake, 1024, fake, 512, fake, 0, None) == V.VMAT_ERR_INVALID_ARG
    assert rw(fake, 1024, fake, 512, fake, 65537, None) == V.VMAT_ERR_INVALID_ARG
