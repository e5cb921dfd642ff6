"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and validates arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmrf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def g(built_library):
    from paper_1606_00980_amd import gmrf
    return gmrf


def test_every_declared_symbol_is_exported(g):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(g.lib, n), n
    assert sorted(g.EXPORTS) == names


def test_opts_default(g):
    o = g.gp_opts_default()
    assert o.tol == 1e-8 and o.inner_tol == 1e-4
    assert o.max_iter == 2000 and o.max_outer == 30
    assert o.precond == g.GP_PRECOND_BLOCK_JACOBI and o.precision == g.GP_PREC_FP32_REFINE64
    assert g.gp_version() >= 10000


def test_null_arguments_rejected_before_device_use(g):
    L = g.lib
    vp = ctypes.c_void_p
    assert L.gp_ctx_create(0, None, 0, None) == g.GP_ERR_INVALID_ARG
    out = vp()
    assert L.gp_op_create(None, None, 4, 4, 1, 4, 2, ctypes.byref(out)) == g.GP_ERR_INVALID_ARG
    assert L.gp_solve(None, 1, None, None, None, None) == g.GP_ERR_INVALID_ARG
    assert L.gp_apply(None, 1, None, None) == g.GP_ERR_INVALID_ARG
    assert L.gp_sample(None, 1, None, None, None, None, None, None) == g.GP_ERR_INVALID_ARG
    assert L.gp_trace(None, 1, None, None, None, None, None, None, None) == g.GP_ERR_INVALID_ARG
    assert L.gp_solve_batch(None, 0, None, None, None) == g.GP_ERR_INVALID_ARG
    assert L.gp_op_query(None, None, None, None, None) == g.GP_ERR_INVALID_ARG
    assert "NULL" in g.gp_last_error() or "null" in g.gp_last_error()
    assert L.gp_ctx_destroy(None) == g.GP_OK
    assert L.gp_op_destroy(None) == g.GP_OK


def test_ctx_without_device_reports_device_error(g):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert g.lib.gp_ctx_create(0, None, 0, ctypes.byref(h)) == g.GP_ERR_DEVICE
    assert h.value is None


def test_stats_view_reads_the_c_array(g):
    """Per-right-hand-side statistics come back as a read-only view over the
    gp_stats array the library filled: fields, negative indices, slices,
    concatenation with lists and equality behave like a list of dicts."""
    arr = g._stats_array(5)
    for i in range(5):
        arr[i].status, arr[i].inner_iters, arr[i].outer_steps = -i, 10 + i, 3
        arr[i].relres, arr[i].time_us = 1e-9 * (i + 1), 2.5
    s = g._stats_list(arr, 4)   # only the first four were solved
    assert len(s) == 4
    assert s[1] == {"status": -1, "inner_iters": 11, "outer_steps": 3, "relres": 2e-9, "time_us": 2.5}
    assert s[-1]["inner_iters"] == 13 and [e["status"] for e in s] == [0, -1, -2, -3]
    assert s[1:3] == [s[1], s[2]]
    both = s + g._stats_list(arr, 2)
    assert isinstance(both, list) and len(both) == 6 and both[4] == s[0]
    assert [] + s == list(s) and s == list(s)
    with pytest.raises(IndexError):
        s[4]
