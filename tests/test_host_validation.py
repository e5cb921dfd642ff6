"""Argument validation of every C-ABI entry point on the host, before any
device work: NULL handles and out-of-range sizes are refused with
GP_ERR_INVALID_ARG and a message, NULL destroys are no-ops, and the
host-only helpers compute their documented results.  Needs no GPU; the
sanitizer test runs this module against the host-sanitized build too."""
import ctypes
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def g(built_library):
    from paper_1606_00980_amd import gmrf
    return gmrf


def default_args(argtypes):
    out = []
    for t in argtypes:
        if t in (ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint64):
            out.append(1)
        elif t is ctypes.c_double:
            out.append(1.0)
        elif t is ctypes.c_char_p:
            out.append(b"/nonexistent/gmrf_tune.json")
        else:   # handles and pointers
            out.append(None)
    return out


HANDLE_FIRST = ["gp_ctx_set_stream", "gp_ctx_memory", "gp_ctx_profile", "gp_ctx_profile_read", "gp_op_create",
                "gp_op_set_blocks", "gp_op_set_alpha", "gp_op_query", "gp_op_voxel_index", "gp_apply", "gp_solve",
                "gp_solve_batch", "gp_perturb_rhs", "gp_sample", "gp_probe_rhs", "gp_trace_reduce",
                "gp_trace_reduce_static", "gp_trace", "gp_rng_normal", "gp_rng_rademacher", "gp_rng_raw",
                "gp_rng_gamma", "gp_server_create", "gp_server_submit", "gp_server_poll", "gp_server_drain",
                "gp_server_get_stats", "gp_server_cancel", "gp_server_step", "gp_autotune", "gp_tune_save",
                "gp_tune_load", "gp_data_create", "gp_data_assemble", "gp_data_lambda", "gp_alpha_posterior",
                "gp_svb_step", "gp_data_assemble_ar", "gp_gibbs_step", "gp_svb_step_ar"]


@pytest.mark.parametrize("name", HANDLE_FIRST)
def test_null_handle_is_refused(g, name):
    f = getattr(g.lib, name)
    assert f(*default_args(f.argtypes)) == g.GP_ERR_INVALID_ARG, name
    msg = g.gp_last_error()
    assert msg and len(msg) < 1000


@pytest.mark.parametrize("name", ["gp_ctx_destroy", "gp_op_destroy", "gp_data_destroy", "gp_server_destroy"])
def test_null_destroy_is_a_no_op(g, name):
    assert getattr(g.lib, name)(None) == g.GP_OK


def test_ctx_create_needs_an_out_pointer(g):
    assert g.lib.gp_ctx_create(0, None, 0, None) == g.GP_ERR_INVALID_ARG


def test_defaults_fill_every_field(g):
    o = g.GpOpts()
    g.lib.gp_opts_default(ctypes.byref(o))
    assert o.tol == 1e-8 and o.max_iter > 0 and o.max_outer > 0
    c = g.GpServerCfg()
    g.lib.gp_server_cfg_default(ctypes.byref(c))
    assert c.hbm_budget > 0 and c.max_active_rhs >= c.probes >= 1 and c.chunk >= 1 and c.manual == 0
    assert c.opts.tol == o.tol
    h = g.GpHyper()
    g.lib.gp_hyper_default(ctypes.byref(h))
    assert all(math.isfinite(getattr(h, f)) and getattr(h, f) > 0 for f, _ in g.GpHyper._fields_)


def test_alpha_extrapolation_on_the_host(g):
    """gp_alpha_extrapolate validates K and its pointers; on sequences that
    are constant or linear in the iteration number (no curvature) the rule
    gives a_jm1 + 20 (a_j - a_jm1), limited to [a_j / 5, 5 a_j]."""
    K = 5
    a2 = (ctypes.c_double * K)(*[1.0, 2.0, 3.0, 4.0, 5.0])
    a1 = (ctypes.c_double * K)(*[1.5, 2.0, 2.5, 4.0, 6.0])
    aj = (ctypes.c_double * K)(*[2.0, 2.0, 2.0, 4.0, 7.0])
    assert g.lib.gp_alpha_extrapolate(0, a2, a1, aj) == g.GP_ERR_INVALID_ARG
    assert g.lib.gp_alpha_extrapolate(K, None, a1, aj) == g.GP_ERR_INVALID_ARG
    assert g.lib.gp_alpha_extrapolate(K, a2, None, aj) == g.GP_ERR_INVALID_ARG
    assert g.lib.gp_alpha_extrapolate(K, a2, a1, None) == g.GP_ERR_INVALID_ARG
    assert g.lib.gp_alpha_extrapolate(K, a2, a1, aj) == g.GP_OK
    # 11.5 capped at 5 * 2; constant; -7.5 raised to 2 / 5; constant; 26
    assert list(aj) == [10.0, 2.0, 0.4, 4.0, 26.0]


def test_tune_load_of_a_missing_or_malformed_file(g, tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text('{"gmrf_tune": 1, "entries": [\n {"key": "K6_N15_R64_p1_c2", "rhs_tile": 99}\n]}\n')
    assert g.lib.gp_tune_load(None, str(bad).encode()) == g.GP_ERR_INVALID_ARG
    assert g.lib.gp_tune_load(None, None) == g.GP_ERR_INVALID_ARG
    assert g.lib.gp_tune_save(None, None) == g.GP_ERR_INVALID_ARG


def test_last_error_survives_many_failures(g):
    for i in range(2000):
        g.lib.gp_apply(None, i, None, None)
    assert "NULL" in g.gp_last_error() or "null" in g.gp_last_error()
