"""Serving loop: every result equals the oracle's, and is bitwise the same
whether the request ran alone or among others (continuous batching with
batch-invariant reductions), with the block-Jacobi and the red-black
incomplete Cholesky preconditioners; admission by HBM budget; requests that
join while others are running (manual rounds make the schedule exact);
failing, cancelled and timed-out requests retire alone."""
import time

import numpy as np
import pytest

from oracle import gmrf_oracle as orc
from oracle import philox
from paper_1606_00980_amd import synth

pytestmark = pytest.mark.gpu

PRECONDS = ["block_jacobi", "rb_ic0"]


@pytest.fixture(scope="module")
def env(built_library):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_00980_amd import gmrf as g
    ctx = g.gp_ctx_create(0, torch.cuda.current_stream().cuda_stream, 0)
    ws = [synth.tiny((13, 11, 7), 6, 2, seed=31), synth.tiny((16, 12, 8), 6, 5, seed=32),
          synth.tiny((12, 10, 1), 4, 3, seed=33)]
    ops, bws, keep = [], [], []
    for w in ws:
        op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
        B = torch.from_numpy(w.B).cuda()
        g.gp_op_set_blocks(op, B)
        g.gp_op_set_alpha(op, w.alpha)
        bw = torch.from_numpy(w.bw).cuda()
        ops.append(op)
        bws.append(bw)
        keep.append(B)
    yield g, torch, ctx, ws, ops, bws
    for op in ops:
        g.gp_op_destroy(op)
    g.gp_ctx_destroy(ctx)


PROBES = 4


def pc_of(g, name):
    return {"block_jacobi": g.GP_PRECOND_BLOCK_JACOBI, "rb_ic0": g.GP_PRECOND_RB_IC0}[name]


def server_cfg(g, precond, budget=1 << 30, **kw):
    opts = g.gp_opts_default(tol=1e-9, precond=pc_of(g, precond), **kw.pop("opts", {}))
    return g.gp_server_cfg_default(probes=PROBES, hbm_budget=budget, opts=opts, **kw)


def run(g, torch, ctx, ws, ops, bws, reqs, precond="block_jacobi", budget=1 << 30):
    srv = g.gp_server_create(ctx, ops, bws, server_cfg(g, precond, budget))
    outs, tickets = [], []
    try:
        for kind, oi, seed in reqs:
            w = ws[oi]
            R = PROBES if kind == g.GP_REQ_TRACE else 1
            out = torch.zeros((R, w.K, w.N), dtype=torch.float64, device="cuda")
            outs.append(out)
            tickets.append(g.gp_server_submit(srv, kind, oi, seed, out))
        g.gp_server_drain(srv, 60000)
        res = {r["ticket"]: r for r in g.gp_server_poll(srv, 1024)}
        stats = g.gp_server_get_stats(srv)
    finally:
        g.gp_server_destroy(srv)
    torch.cuda.synchronize()
    return [res[t] for t in tickets], [o.cpu().numpy() for o in outs], stats


def oracle_result(g, w, kind, seed, probes=PROBES):
    grid = orc.grid(w.mask, w.conn)
    Q = orc.precision(grid, w.alpha, w.B)
    n = w.K * w.N
    if kind == g.GP_REQ_SOLVE:
        b = w.bw + philox.normal(seed, 4, n).reshape(w.K, w.N)
        return orc.solve(Q, b[None]), None
    if kind == g.GP_REQ_SAMPLE:
        z1 = philox.normal(seed, 1, grid.ndirs * n).reshape(1, w.K, grid.ndirs, w.N)
        z2 = philox.normal(seed, 2, n).reshape(1, w.K, w.N)
        return orc.sample(grid, w.alpha, w.B, w.bw, z1, z2), None
    v = philox.rademacher(seed, 3, probes * n).reshape(probes, w.K, w.N)
    t, tk, gk, u = orc.hutchinson(grid, Q, v)
    return u, (t, tk, gk)


@pytest.mark.parametrize("precond", PRECONDS)
def test_server_mix_matches_alone_and_oracle(env, precond):
    g, torch, ctx, ws, ops, bws = env
    kinds = [g.GP_REQ_SOLVE, g.GP_REQ_SAMPLE, g.GP_REQ_TRACE]
    reqs = [(kinds[i % 3], (i * 7) % 3, 1000 + i) for i in range(15)]
    res, outs, stats = run(g, torch, ctx, ws, ops, bws, reqs, precond)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0 and stats["p99_us"] >= stats["p50_us"] > 0
    assert all(r["status"] == 0 and r["relres_max"] <= 1e-9 for r in res)
    for (kind, oi, seed), r, out in zip(reqs, res, outs):
        alone_res, alone_out, _ = run(g, torch, ctx, ws, ops, bws, [(kind, oi, seed)], precond)
        assert np.array_equal(alone_out[0], out), (kind, oi, seed)
        if kind == g.GP_REQ_TRACE:
            assert alone_res[0]["trace_total"] == r["trace_total"]
    for (kind, oi, seed), r, out in list(zip(reqs, res, outs))[:6]:
        w = ws[oi]
        ref, tr = oracle_result(g, w, kind, seed)
        ref = ref.reshape(out.shape)
        for i in range(out.shape[0]):
            assert np.linalg.norm(out[i] - ref[i]) <= 1e-6 * np.linalg.norm(ref[i])
        if tr is not None:
            assert abs(r["trace_total"] - tr[0]) <= 1e-6 * abs(tr[0])
            assert np.allclose(r["trace_kk"][:w.K], tr[1], rtol=1e-6)
            assert np.allclose(r["trace_Gkk"][:w.K], tr[2], rtol=1e-6)


@pytest.mark.parametrize("precond", PRECONDS)
def test_server_admission_budget(env, precond):
    g, torch, ctx, ws, ops, bws = env
    reqs = [(g.GP_REQ_SAMPLE, i % 3, 2000 + i) for i in range(6)]
    full, full_out, _ = run(g, torch, ctx, ws, ops, bws, reqs, precond)
    # a budget that holds about one request at a time still completes all of them
    # (a red-black request holds the split system's vectors besides b and x)
    tight_budget = {"block_jacobi": 300_000, "rb_ic0": 400_000}[precond]
    tight, tight_out, st = run(g, torch, ctx, ws, ops, bws, reqs, precond, budget=tight_budget)
    assert st["completed"] == 6 and st["peak_active_rhs"] <= 2
    for a, b in zip(full_out, tight_out):
        assert np.array_equal(a, b)
    srv = g.gp_server_create(ctx, ops, bws, server_cfg(g, precond, budget=1000))
    try:
        with pytest.raises(g.GmrfError) as e:
            g.gp_server_submit(srv, g.GP_REQ_SOLVE, 0, 1)
        assert e.value.status == g.GP_ERR_OOM
    finally:
        g.gp_server_destroy(srv)


@pytest.mark.parametrize("precond", PRECONDS)
def test_server_trace_on_k20_operator(env, precond):
    """A trace request on an operator with K = 20 (more regressors than 16):
    every t_k and g_k of Section 3.3's trace term is returned and matches the
    oracle with the same Philox probes; the entries past K stay zero."""
    g, torch, ctx, _, _, _ = env
    w = synth.tiny((12, 10, 6), 6, 20, seed=34, T=80)
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    B = torch.from_numpy(w.B).cuda()
    bw = torch.from_numpy(w.bw).cuda()
    try:
        g.gp_op_set_blocks(op, B)
        g.gp_op_set_alpha(op, w.alpha)
        res, outs, _ = run(g, torch, ctx, [w], [op], [bw], [(g.GP_REQ_TRACE, 0, 4242)], precond)
    finally:
        torch.cuda.synchronize()
        g.gp_op_destroy(op)
    r = res[0]
    assert r["status"] == 0 and r["kind"] == g.GP_REQ_TRACE and r["op_index"] == 0 and r["rhs"] == PROBES
    u_ref, (t, tk, gk) = oracle_result(g, w, g.GP_REQ_TRACE, 4242)
    for i in range(PROBES):
        assert np.linalg.norm(outs[0][i] - u_ref[i]) <= 1e-6 * np.linalg.norm(u_ref[i])
    assert abs(r["trace_total"] - t) <= 1e-6 * abs(t)
    assert len(r["trace_kk"]) == g.GP_KMAX and len(r["trace_Gkk"]) == g.GP_KMAX
    assert np.allclose(r["trace_kk"][:w.K], tk, rtol=1e-6)
    assert np.allclose(r["trace_Gkk"][:w.K], gk, rtol=1e-6)
    assert all(v == 0.0 for v in r["trace_kk"][w.K:]) and all(v == 0.0 for v in r["trace_Gkk"][w.K:])


def manual_server(g, ctx, ops, bws, precond, chunk=1, probes=PROBES, fp64=True):
    opts = {"precision": g.GP_PREC_FP64} if fp64 else {}
    cfg = server_cfg(g, precond, manual=1, chunk=chunk, opts=opts)
    cfg.probes = probes
    return g.gp_server_create(ctx, ops, bws, cfg)


def step_until_done(g, srv, n_expected, limit=5000):
    got = []
    for _ in range(limit):
        got += g.gp_server_poll(srv, 64)
        if len(got) >= n_expected:
            return {r["ticket"]: r for r in got}
        g.gp_server_step(srv, 1)
    raise AssertionError("requests did not finish")


@pytest.mark.parametrize("precond", PRECONDS)
def test_request_joins_while_another_runs(env, precond):
    """Continuous batching, deterministically: with rounds granted one at a
    time (one FP64 iteration each), trace request A is admitted in round 0
    and still running when solve request B is submitted after two rounds; B
    is admitted in round 2, before A retires, and both results are bitwise
    those of the same requests served alone."""
    g, torch, ctx, ws, ops, bws = env
    wa, wb = ws[1], ws[0]
    outs = {}

    def serve(schedule):
        srv = manual_server(g, ctx, ops, bws, precond)
        try:
            tickets = {}
            for name, kind, oi, seed, at_round in schedule:
                while g.gp_server_get_stats(srv)["rounds"] < at_round:
                    g.gp_server_step(srv, 1)
                w = ws[oi]
                R = PROBES if kind == g.GP_REQ_TRACE else 1
                out = torch.zeros((R, w.K, w.N), dtype=torch.float64, device="cuda")
                outs[name] = out
                tickets[name] = g.gp_server_submit(srv, kind, oi, seed, out)
            res = step_until_done(g, srv, len(schedule))
        finally:
            g.gp_server_destroy(srv)
        torch.cuda.synchronize()
        return {name: res[t] for name, t in tickets.items()}, {k: v.cpu().numpy() for k, v in outs.items()}

    A = ("A", g.GP_REQ_TRACE, 1, 777, 0)
    Bq = ("B", g.GP_REQ_SOLVE, 0, 778, 2)
    mix, mix_out = serve([A, Bq])
    ra, rb = mix["A"], mix["B"]
    assert ra["status"] == 0 and rb["status"] == 0
    assert ra["admit_round"] == 0 and rb["admit_round"] == 2
    assert rb["admit_round"] < ra["retire_round"], (ra, rb)   # B joined while A was running
    assert ra["iters_max"] > 2
    alone_a, out_a = serve([("A",) + A[1:4] + (0,)])
    alone_b, out_b = serve([("B",) + Bq[1:4] + (0,)])
    assert np.array_equal(mix_out["A"], out_a["A"]) and mix["A"]["trace_total"] == alone_a["A"]["trace_total"]
    assert np.array_equal(mix_out["B"], out_b["B"])
    ref, _ = oracle_result(g, wb, g.GP_REQ_SOLVE, 778)
    assert np.linalg.norm(mix_out["B"][0] - ref[0]) <= 1e-6 * np.linalg.norm(ref[0])


@pytest.mark.parametrize("precond", PRECONDS)
def test_failed_request_leaves_the_others_unchanged(env, precond):
    """An operator whose b_w holds a NaN: its solve request breaks down alone
    (GP_ERR_BREAKDOWN, nothing written to its output), while the requests it
    shared rounds with return bitwise what they return without it."""
    g, torch, ctx, ws, ops, bws = env
    bad = bws[2].clone()
    bad[0, 3] = float("nan")
    bws_bad = [bws[0], bws[1], bad]
    reqs = [(g.GP_REQ_SOLVE, 0, 3001), (g.GP_REQ_SOLVE, 2, 3002), (g.GP_REQ_TRACE, 1, 3003),
            (g.GP_REQ_SAMPLE, 2, 3004), (g.GP_REQ_SAMPLE, 0, 3005)]
    res, outs, st = run(g, torch, ctx, ws, ops, bws_bad, reqs, precond)
    assert st["completed"] == 5 and st["failed"] == 2
    for (kind, oi, seed), r, out in zip(reqs, res, outs):
        if oi == 2:
            assert r["status"] == g.GP_ERR_BREAKDOWN, r
            assert np.all(out == 0.0)
        else:
            assert r["status"] == 0
    good = [(q, o) for q, o in zip(reqs, outs) if q[1] != 2]
    ref_res, ref_outs, _ = run(g, torch, ctx, ws, ops, bws, [q for q, _ in good], precond)
    for (q, o), ro in zip(good, ref_outs):
        assert np.array_equal(o, ro), q


@pytest.mark.parametrize("precond", PRECONDS)
def test_cancel_and_timeout(env, precond):
    """Cancellation of a waiting and of a running request, and deadlines that
    pass before admission and while running: each retires with its status
    (nothing written to its output), the others complete unchanged."""
    g, torch, ctx, ws, ops, bws = env
    srv = manual_server(g, ctx, ops, bws, precond)
    outs = {}
    try:
        def submit(name, kind, oi, seed, timeout_ms=0.0):
            w = ws[oi]
            R = PROBES if kind == g.GP_REQ_TRACE else 1
            outs[name] = torch.zeros((R, w.K, w.N), dtype=torch.float64, device="cuda")
            return g.gp_server_submit(srv, kind, oi, seed, outs[name], timeout_ms)

        t_run = submit("running_cancel", g.GP_REQ_TRACE, 1, 4001)
        t_keep = submit("keep", g.GP_REQ_SOLVE, 0, 4002)
        t_late = submit("running_timeout", g.GP_REQ_TRACE, 1, 4003, timeout_ms=200.0)
        g.gp_server_step(srv, 1)                      # all three admitted and iterating
        t_wait = submit("waiting_cancel", g.GP_REQ_SOLVE, 2, 4004)
        t_exp = submit("waiting_timeout", g.GP_REQ_SOLVE, 2, 4005, timeout_ms=1.0)
        g.gp_server_cancel(srv, t_run)
        g.gp_server_cancel(srv, t_wait)
        time.sleep(0.25)                              # both deadlines pass
        res = step_until_done(g, srv, 5)
        with pytest.raises(g.GmrfError):
            g.gp_server_cancel(srv, t_keep)           # already finished
        st = g.gp_server_get_stats(srv)
    finally:
        g.gp_server_destroy(srv)
    torch.cuda.synchronize()
    assert res[t_run]["status"] == g.GP_ERR_CANCELLED and res[t_run]["admit_round"] == 0
    assert res[t_wait]["status"] == g.GP_ERR_CANCELLED and res[t_wait]["admit_round"] == -1
    assert res[t_late]["status"] == g.GP_ERR_TIMEOUT and res[t_late]["admit_round"] == 0
    assert res[t_exp]["status"] == g.GP_ERR_TIMEOUT and res[t_exp]["admit_round"] == -1
    assert res[t_keep]["status"] == 0
    assert st["failed"] == 4 and st["completed"] == 5
    for name in ("running_cancel", "waiting_cancel", "running_timeout", "waiting_timeout"):
        assert np.all(outs[name].cpu().numpy() == 0.0), name
    ref, _ = oracle_result(g, ws[0], g.GP_REQ_SOLVE, 4002)
    keep = outs["keep"].cpu().numpy()
    assert np.linalg.norm(keep[0] - ref[0]) <= 1e-6 * np.linalg.norm(ref[0])
