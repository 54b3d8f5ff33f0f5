"""The C-ABI library loads and exports every function include/lskum.h declares
(no GPU work is done here), and rejects bad inputs on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lskum.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lskum_[A-Za-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2406_07441_amd import build, lskum
    if build.stale():
        build.build()
    return lskum.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lskum_cloud_create", "lskum_state_create", "lskum_residual",
                 "lskum_lusgs_step", "lskum_solve", "lskum_forces", "lskum_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing


def test_binding_covers_every_declared_symbol():
    from paper_2406_07441_amd import lskum
    assert set(declared_functions()) == set(lskum._SIGS)


def test_default_params(lib):
    from paper_2406_07441_amd import lskum
    p = lskum.default_params()
    assert p.gamma == 1.4 and p.cfl == 100.0 and p.inner_iters == 1
    assert p.tol_rel == 1e-8 and p.jvp_mode == 0 and p.precision == 0


def _create(lib, n, off, idx, typ=None):
    x = np.arange(n, dtype=np.float64)
    y = np.zeros(n)
    typ = np.ones(n, dtype=np.int8) if typ is None else typ
    h = C.c_void_p()
    code = lib.lskum_cloud_create(n, x.ctypes.data, y.ctypes.data, typ.ctypes.data, None, None,
                                  off.ctypes.data, idx.ctypes.data, None, C.byref(h))
    return code, lib.lskum_last_error().decode()


def test_asymmetric_connectivity_is_rejected_before_any_device_work(lib):
    off = np.array([0, 1, 1], dtype=np.int32)
    idx = np.array([1], dtype=np.int32)
    code, msg = _create(lib, 2, off, idx)
    assert code == -2 and "symmetric" in msg


def test_out_of_range_and_self_edges_are_rejected(lib):
    off = np.array([0, 1, 2], dtype=np.int32)
    code, msg = _create(lib, 2, off, np.array([5, 0], dtype=np.int32))
    assert code == -2 and "range" in msg
    code, msg = _create(lib, 2, off, np.array([0, 1], dtype=np.int32))
    assert code == -2 and "self" in msg


def test_wall_points_need_a_frame(lib):
    off = np.array([0, 1, 2], dtype=np.int32)
    code, msg = _create(lib, 2, off, np.array([1, 0], dtype=np.int32),
                        typ=np.array([0, 1], dtype=np.int8))
    assert code == -1 and "frame" in msg


def test_empty_and_malformed_inputs_are_rejected(lib):
    off = np.array([0], dtype=np.int32)
    code, msg = _create(lib, 0, off, np.zeros(0, dtype=np.int32))
    assert code == -1 and "range" in msg
    # offsets that do not start at zero, or decrease
    code, msg = _create(lib, 2, np.array([1, 1, 1], dtype=np.int32), np.zeros(1, dtype=np.int32))
    assert code == -2 and "nbr_off[0]" in msg
    code, msg = _create(lib, 3, np.array([0, 2, 1, 2], dtype=np.int32),
                        np.array([1, 2], dtype=np.int32))
    assert code == -2 and "monotone" in msg
    # an invalid point type and a non-finite coordinate
    off = np.array([0, 1, 2], dtype=np.int32)
    code, msg = _create(lib, 2, off, np.array([1, 0], dtype=np.int32),
                        typ=np.array([1, 7], dtype=np.int8))
    assert code == -1 and "type" in msg
    h = C.c_void_p()
    x = np.array([0.0, np.nan])
    code = lib.lskum_cloud_create(2, x.ctypes.data, np.zeros(2).ctypes.data,
                                  np.ones(2, dtype=np.int8).ctypes.data, None, None,
                                  off.ctypes.data, np.array([1, 0], dtype=np.int32).ctypes.data,
                                  None, C.byref(h))
    assert code == -1 and "finite" in lib.lskum_last_error().decode()
