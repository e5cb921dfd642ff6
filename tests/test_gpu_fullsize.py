"""Full-size parity: the measured workloads at their real sizes and in the
launch configuration the benchmark times, every right-hand side compared
element by element with the FP64 oracle.

* 64 right-hand sides on the whole-brain operator (N = 52,740, K = 6): 32
  Algorithm-2 samples and 32 Rademacher probes, FP32 inner PCG with FP64
  refinement to relative residual 1e-8, with the red-black incomplete
  Cholesky factor and with block Jacobi;
* 16 uneven operators (N = 16,515 .. 283,572, K = 2 .. 10), 4 samples and 4
  probes each, in one batched solve, both preconditioners;
* a Poisson stream of served requests over the 24 resident operators of the
  serving workload, a seeded 1% sample of the results against the oracle.

Gate (Section 3.1 relative-residual criterion with delta = 1e-8; Algorithm 2;
the Section 3.3 trace term): per right-hand side, the oracle's recomputed FP64
relative residual <= 1e-8, ||x - x_ref|| <= 1e-6 ||x_ref|| over all K*N
entries and for every regressor block k, ||x_k - x_ref,k|| <= 1e-6 ||x_ref||;
the Hutchinson estimates t, t_k, g_k within 1e-6 (relative) of the oracle's
from the same probes.  The oracle runs in worker processes (oracle/jobs.py) to
relative residual 1e-12, so its own error is far below the gate.
"""
import numpy as np
import pytest

from oracle import gmrf_oracle as orc
from oracle import jobs
from paper_1606_00980_amd import synth

pytestmark = pytest.mark.gpu

REL_ERR = 1e-6
TOL = 1e-8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def g(built_library, torch_cuda):
    from paper_1606_00980_amd import gmrf
    return gmrf


@pytest.fixture(scope="module")
def ctx(g, torch_cuda):
    h = g.gp_ctx_create(0, torch_cuda.cuda.current_stream().cuda_stream, 0)
    yield h
    torch_cuda.cuda.synchronize()
    g.gp_ctx_destroy(h)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def precond_of(g, name):
    return {"rb_ic0": g.GP_PRECOND_RB_IC0, "block_jacobi": g.GP_PRECOND_BLOCK_JACOBI}[name]


def assert_close(x, ref, what):
    whole, block = jobs.rel_errors(x, ref)
    assert np.all(whole <= REL_ERR), (what, "whole", float(whole.max()), int(whole.argmax()))
    assert np.all(block <= REL_ERR), (what, "block", float(block.max()), int(block.argmax()))
    return float(whole.max()), float(block.max())


def assert_trace(t, tk, gk, ref, what):
    t_ref, tk_ref, gk_ref = ref
    assert abs(t - t_ref) <= REL_ERR * abs(t_ref), (what, t, t_ref)
    assert np.all(np.abs(np.asarray(tk) - tk_ref) <= REL_ERR * np.abs(tk_ref)), what
    assert np.all(np.abs(np.asarray(gk) - gk_ref) <= REL_ERR * np.abs(gk_ref)), what


# ------------------------------------------------ whole brain, 64 right-hand sides
S_BRAIN = M_BRAIN = 32


@pytest.fixture(scope="module")
def brain_ref():
    """Oracle solutions of all 32 samples and all 32 probes, 4 per job."""
    js = [(("brain",), S_BRAIN, range(i, i + 4), M_BRAIN, [], False) for i in range(0, S_BRAIN, 4)]
    js += [(("brain",), S_BRAIN, [], M_BRAIN, range(i, i + 4), False) for i in range(0, M_BRAIN, 4)]
    out, _, _ = jobs.run_parallel(jobs.solutions, js)
    xs = np.concatenate([o["samples"] for o in out[:S_BRAIN // 4]])
    bs = np.concatenate([o["sample_rhs"] for o in out[:S_BRAIN // 4]])
    u = np.concatenate([o["probes"] for o in out[S_BRAIN // 4:]])
    return xs, bs, u


@pytest.mark.parametrize("precond", ["rb_ic0", "block_jacobi"])
def test_whole_brain_64_rhs_every_rhs_vs_oracle(g, ctx, torch_cuda, brain_ref, precond):
    torch = torch_cuda
    xs_ref, b_ref, u_ref = brain_ref
    w = synth.brain_3d()
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    try:
        g.gp_op_set_blocks(op, dev(torch, w.B))
        g.gp_op_set_alpha(op, w.alpha)
        z1, z2 = w.z(S_BRAIN)
        v = w.probes(M_BRAIN)
        bs = torch.empty((S_BRAIN, w.K, w.N), dtype=torch.float64, device="cuda")
        g.gp_perturb_rhs(op, S_BRAIN, dev(torch, w.bw), dev(torch, z1), dev(torch, z2), bs)
        vd = dev(torch, v)
        bp = torch.empty((M_BRAIN, w.K, w.N), dtype=torch.float64, device="cuda")
        g.gp_probe_rhs(op, M_BRAIN, vd, bp)
        o = g.gp_opts_default(tol=TOL, zero_guess=1, precond=precond_of(g, precond),
                              precision=g.GP_PREC_FP32_REFINE64)
        xs = torch.zeros_like(bs)
        xp = torch.zeros_like(bp)
        _, stats = g.gp_solve_batch(ctx, [(op, S_BRAIN, bs, xs), (op, M_BRAIN, bp, xp)], o)
        assert all(s["status"] == g.GP_OK and s["relres"] <= TOL for s in stats)
        t, tk, gk = g.gp_trace_reduce(op, M_BRAIN, vd, xp, w.K)
        xs_h, xp_h = xs.cpu().numpy(), xp.cpu().numpy()
    finally:
        torch.cuda.synchronize()
        g.gp_op_destroy(op)
    grid = orc.grid(w.mask, w.conn)
    Q = orc.precision(grid, w.alpha, w.B)
    assert np.max(np.abs(bs.cpu().numpy() - b_ref)) <= 1e-12 * np.max(np.abs(b_ref))
    assert np.all(orc.relres(Q, xs_h, b_ref) <= TOL)
    assert np.all(orc.relres(Q, xp_h, v.astype(np.float64)) <= TOL)
    assert_close(xs_h, xs_ref, "samples")
    assert_close(xp_h, u_ref, "probes")
    tr_ref = orc.hutchinson(grid, Q, v, u=u_ref)[:3]
    assert_trace(t, tk, gk, tr_ref, "trace")


# ------------------------------------------------- 16 uneven operators, 8 RHS each
N_UNEVEN, R_HALF = 16, 4


@pytest.fixture(scope="module")
def uneven_ref():
    """Oracle solutions of every sample and probe of the 16 operators (one job
    for an operator's samples, one for its probes and traces), started first
    so that the workers run while this process makes the operators."""
    specs = [("uneven", synth.CFG_UNEVEN, i) for i in range(N_UNEVEN)]
    cost = [synth.uneven_params(synth.CFG_UNEVEN, i) for i in range(N_UNEVEN)]
    order = sorted(range(N_UNEVEN), key=lambda i: -np.prod(cost[i][0]) * cost[i][1] * cost[i][2])
    js, keys = [], []
    for i in order:
        js.append((specs[i], R_HALF, range(R_HALF), R_HALF, [], False))
        keys.append((i, "s"))
        js.append((specs[i], R_HALF, [], R_HALF, range(R_HALF), True))
        keys.append((i, "p"))
    pend = jobs.start_parallel(jobs.solutions, js)
    ws = [synth.from_spec(s) for s in specs]
    out, _, _ = pend.get()
    ref = {k: o for k, o in zip(keys, out)}
    return ws, ref


@pytest.mark.parametrize("precond", ["rb_ic0", "block_jacobi"])
def test_uneven_16_operators_every_rhs_vs_oracle(g, ctx, torch_cuda, uneven_ref, precond):
    torch = torch_cuda
    ws, ref = uneven_ref
    ops, items, keep = [], [], []
    try:
        for w in ws:
            op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
            ops.append(op)
            B = dev(torch, w.B)
            keep.append(B)
            g.gp_op_set_blocks(op, B)
            g.gp_op_set_alpha(op, w.alpha)
            z1, z2 = w.z(R_HALF)
            vd = dev(torch, w.probes(R_HALF))
            bs = torch.empty((R_HALF, w.K, w.N), dtype=torch.float64, device="cuda")
            bp = torch.empty_like(bs)
            g.gp_perturb_rhs(op, R_HALF, dev(torch, w.bw), dev(torch, z1), dev(torch, z2), bs)
            g.gp_probe_rhs(op, R_HALF, vd, bp)
            xs, xp = torch.zeros_like(bs), torch.zeros_like(bp)
            keep += [vd, bs, bp]
            items += [(op, R_HALF, bs, xs), (op, R_HALF, bp, xp)]
        o = g.gp_opts_default(tol=TOL, zero_guess=1, precond=precond_of(g, precond),
                              precision=g.GP_PREC_FP32_REFINE64)
        _, stats = g.gp_solve_batch(ctx, items, o)
        assert len(stats) == N_UNEVEN * 2 * R_HALF
        assert all(s["status"] == g.GP_OK and s["relres"] <= TOL for s in stats)
        traces = [g.gp_trace_reduce(op, R_HALF, keep[4 * i + 1], items[2 * i + 1][3], w.K)
                  for i, (op, w) in enumerate(zip(ops, ws))]
        host = [(it[2].cpu().numpy(), it[3].cpu().numpy()) for it in items]
    finally:
        torch.cuda.synchronize()
        for op in ops:
            g.gp_op_destroy(op)
    for i, w in enumerate(ws):
        (bs_h, xs_h), (bp_h, xp_h) = host[2 * i], host[2 * i + 1]
        rs, rp = ref[(i, "s")], ref[(i, "p")]
        assert np.max(np.abs(bs_h - rs["sample_rhs"])) <= 1e-12 * np.max(np.abs(rs["sample_rhs"])), i
        Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
        assert np.all(orc.relres(Q, xs_h, bs_h) <= TOL), i
        assert np.all(orc.relres(Q, xp_h, bp_h) <= TOL), i
        del Q
        assert_close(xs_h, rs["samples"], ("samples", i, w.N, w.K))
        assert_close(xp_h, rp["probes"], ("probes", i, w.N, w.K))
        assert_trace(*traces[i], rp["trace"], ("trace", i))


# ------------------------------------------------------ served stream, 1% sample
SERVE_OPS, SERVE_PROBES = 24, 16


def test_served_stream_sample_vs_oracle(g, ctx, torch_cuda):
    """A 2 s Poisson stream at 200 requests/s (solve, sample, 16-probe trace,
    uniform) over the 24 resident serving operators; a seeded 1% sample of the
    requests (at least one of each kind) returns its result, which is compared
    with the oracle's for the same Philox-drawn vectors (trace probes split
    over workers, the estimates formed from all 16 oracle solutions)."""
    torch = torch_cuda
    specs = [("uneven", synth.CFG_SERVE, 100 + i) for i in range(SERVE_OPS)]
    ws = synth.generate(specs)
    rng = np.random.default_rng([synth.CFG_SERVE, 6, 1])
    t, sched = 0.0, []
    while True:
        t += rng.exponential(1.0 / 200.0)
        if t >= 2.0:
            break
        sched.append((int(rng.integers(0, 3)), int(rng.integers(0, SERVE_OPS)), 50_000 + len(sched), t))
    n_pick = max(3, int(round(0.01 * len(sched))))
    pick = [int(rng.choice([j for j, s_ in enumerate(sched) if s_[0] == k])) for k in range(3)]
    rest = [j for j in range(len(sched)) if j not in pick]
    pick += [int(j) for j in rng.choice(rest, size=n_pick - 3, replace=False)]
    # the oracle: one job per solve/sample, one per probe of a trace
    js, keys = [], []
    for j in pick:
        kind, oi, seed, _ = sched[j]
        if kind == 2:
            for p in range(SERVE_PROBES):
                js.append((specs[oi], kind, seed, SERVE_PROBES, [p]))
                keys.append((j, p))
        else:
            js.append((specs[oi], kind, seed, SERVE_PROBES, None))
            keys.append((j, 0))
    pend = jobs.start_parallel(jobs.served, js)
    ops, bws, keep, outs = [], [], [], {}
    try:
        for w in ws:
            op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
            ops.append(op)
            B = dev(torch, w.B)
            keep.append(B)
            g.gp_op_set_blocks(op, B)
            g.gp_op_set_alpha(op, w.alpha)
            bws.append(dev(torch, w.bw))
        cfg = g.gp_server_cfg_default(probes=SERVE_PROBES, hbm_budget=64 << 30, max_active_rhs=4096,
                                      opts=g.gp_opts_default(tol=TOL))
        srv = g.gp_server_create(ctx, ops, bws, cfg)
        try:
            import time
            tickets = {}
            t0 = time.perf_counter()
            for j, (kind, oi, seed, ta) in enumerate(sched):
                now = time.perf_counter() - t0
                if ta > now:
                    time.sleep(ta - now)
                out = None
                if j in pick:
                    R = SERVE_PROBES if kind == 2 else 1
                    out = torch.zeros((R, ws[oi].K, ws[oi].N), dtype=torch.float64, device="cuda")
                    outs[j] = out
                tickets[j] = g.gp_server_submit(srv, kind, oi, seed, out)
            g.gp_server_drain(srv, 120000)
            res = {r["ticket"]: r for r in g.gp_server_poll(srv, len(sched) + 8)}
            st = g.gp_server_get_stats(srv)
        finally:
            g.gp_server_destroy(srv)
        torch.cuda.synchronize()
        host = {j: o.cpu().numpy() for j, o in outs.items()}
    finally:
        torch.cuda.synchronize()
        for op in ops:
            g.gp_op_destroy(op)
    assert st["completed"] == len(sched)
    assert all(r["status"] == 0 and r["relres_max"] <= TOL for r in res.values())
    oref, _, _ = pend.get()
    got = {}
    for k, o in zip(keys, oref):
        got.setdefault(k[0], []).append(o["x"])
    for j in pick:
        kind, oi, seed, _ = sched[j]
        ref = np.concatenate(got[j])
        assert_close(host[j], ref, ("served", j, kind, oi))
        if kind == 2:
            w = ws[oi]
            v = jobs.served_probes(seed, SERVE_PROBES, w.K, w.N)
            tr_ref = orc.hutchinson(orc.grid(w.mask, w.conn), None, v, u=ref)[:3]
            r = res[tickets[j]]
            assert_trace(r["trace_total"], r["trace_kk"][:w.K], r["trace_Gkk"][:w.K], tr_ref, ("served", j))
