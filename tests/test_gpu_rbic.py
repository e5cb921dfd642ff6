"""GPU parity of the red-black incomplete Cholesky preconditioner (block IC(0)
on the two-colour voxel order, the M of Algorithm 2, steps 6-7), through the
C ABI, against the oracle.

Tolerances: each right-hand side must reach an FP64 relative residual
||b - Qx|| / ||b|| <= tol, recomputed here by the oracle, and a relative error
<= 1e-6 against the oracle's direct solution (tol 1e-10 on operators whose
condition number is far below 1e4).  The iteration counts of the device's
half-size Schur-complement iteration and of the oracle's PCG with the explicit
incomplete factor agree within one step (the two are the same iteration in
exact arithmetic; they differ only in rounding)."""
import numpy as np
import pytest

from oracle import gmrf_oracle as orc
from paper_1606_00980_amd import synth

pytestmark = pytest.mark.gpu

REL_ERR = 1e-6


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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def make_op(g, ctx, torch, w):
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    g.gp_op_set_blocks(op, dev(torch, w.B))
    g.gp_op_set_alpha(op, w.alpha)
    return op


def rhs(w, R, seed):
    b = np.random.default_rng(seed).standard_normal((R, w.K, w.N)) * 3.0
    b[R - 1] = 0.0                           # one right-hand side b = 0 (solution 0)
    return b


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,conn,K", [((23, 19, 9), 6, 3), ((41, 33, 1), 4, 2), ((13, 11, 7), 6, 6)])
def test_solve_matches_oracle(g, ctx, torch_cuda, precision, dims, conn, K):
    """Several voxel tiles of each colour with ragged tails, a random start
    value, and b = 0 in the last right-hand side."""
    w = synth.tiny(dims, conn, K, seed=5 + K)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        R, tol = 4, 1e-10
        b = rhs(w, R, 1)
        x0 = np.random.default_rng(2).standard_normal(b.shape)
        x = dev(torch_cuda, x0)
        prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
        o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0, precision=prec)
        st, stats = g.gp_solve(op, R, dev(torch_cuda, b), x, o)
        xs = x.cpu().numpy()
        grid = orc.grid(w.mask, w.conn)
        Q = orc.precision(grid, w.alpha, w.B)
        rel = orc.relres(Q, xs, b)
        assert np.all(rel <= tol), rel
        assert all(s["status"] == g.GP_OK for s in stats)
        assert np.all(xs[R - 1] == 0.0)
        ref = orc.solve_direct(Q, b)
        for r in range(R - 1):
            assert np.linalg.norm(xs[r] - ref[r]) <= REL_ERR * np.linalg.norm(ref[r]), r
        # the reported residual is the whole system's
        for r in range(R - 1):
            assert stats[r]["relres"] <= tol and abs(stats[r]["relres"] - rel[r]) <= 0.1 * tol + 1e-3 * rel[r]
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


@pytest.mark.parametrize("dims,conn,K", [((11, 9, 7), 6, 3), ((26, 21, 1), 4, 2)])
def test_iterations_match_pcg_with_the_incomplete_factor(g, ctx, torch_cuda, dims, conn, K):
    """FP64 inner solves stop at half the tolerance on the recursive residual
    (then an FP64 residual confirms), so the oracle's PCG with M = L L' runs to
    tol / 2 from the same start value (its red entries solved from the red
    rows, as the device does)."""
    w = synth.tiny(dims, conn, K, seed=17)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        R, tol = 3, 1e-9
        b = np.random.default_rng(3).standard_normal((R, w.K, w.N))
        x0 = np.random.default_rng(4).standard_normal(b.shape)
        x = dev(torch_cuda, x0)
        o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0, precision=g.GP_PREC_FP64)
        st, stats = g.gp_solve(op, R, dev(torch_cuda, b), x, o)
        grid = orc.grid(w.mask, w.conn)
        Q = orc.precision(grid, w.alpha, w.B)
        L, perm = orc.ic0_redblack(grid, w.alpha, w.B)
        for r in range(R):
            xs = orc.redblack_start(grid, Q, b[r], x0[r])
            _, it, _ = orc.solve_pcg_ic0(Q, b[r], L, perm, tol=0.5 * tol, x0=xs)
            assert abs(stats[r]["inner_iters"] - it) <= 1, (r, stats[r]["inner_iters"], it)
            assert stats[r]["outer_steps"] == 2
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_zero_start_value_ignores_x(g, ctx, torch_cuda):
    w = synth.tiny((17, 15, 8), 6, 4, seed=23)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        R, tol = 3, 1e-10
        b = rhs(w, R, 7)
        x = torch_cuda.full((R, w.K, w.N), float("nan"), dtype=torch_cuda.float64, device="cuda")
        o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0, zero_guess=1)
        g.gp_solve(op, R, dev(torch_cuda, b), x, o)
        xs = x.cpu().numpy()
        Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
        assert np.all(np.isfinite(xs)) and np.all(orc.relres(Q, xs, b) <= tol)
        assert np.all(xs[R - 1] == 0.0)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_alpha_and_blocks_changes_rebuild_the_factor(g, ctx, torch_cuda):
    w = synth.tiny((15, 13, 9), 6, 3, seed=29)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        R, tol = 2, 1e-10
        b = rhs(w, R + 1, 8)[:R]
        grid = orc.grid(w.mask, w.conn)
        o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0)
        for alpha, scaleB in ((w.alpha, 1.0), (w.alpha * 7.0, 1.0), (w.alpha * 7.0, 0.25)):
            g.gp_op_set_alpha(op, alpha)
            g.gp_op_set_blocks(op, dev(torch_cuda, w.B * scaleB))
            x = torch_cuda.zeros((R, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            g.gp_solve(op, R, dev(torch_cuda, b), x, o)
            Q = orc.precision(grid, alpha, w.B * scaleB)
            assert np.all(orc.relres(Q, x.cpu().numpy(), b) <= tol)
        # switching back to block Jacobi and again to the incomplete factor
        for pc in (g.GP_PRECOND_BLOCK_JACOBI, g.GP_PRECOND_RB_IC0):
            x = torch_cuda.zeros((R, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            g.gp_solve(op, R, dev(torch_cuda, b), x, g.gp_opts_default(tol=tol, precond=pc))
            assert np.all(orc.relres(Q, x.cpu().numpy(), b) <= tol)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_sampling_and_batch_with_the_incomplete_factor(g, ctx, torch_cuda):
    """Algorithm 2 samples with the incomplete factor, and a batch over two
    operators of different K (solved operator by operator)."""
    w = synth.tiny((14, 12, 8), 6, 3, seed=31)
    w2 = synth.tiny((19, 16, 1), 4, 5, seed=37)
    op = make_op(g, ctx, torch_cuda, w)
    op2 = make_op(g, ctx, torch_cuda, w2)
    try:
        R, tol = 2, 1e-10
        z1, z2 = w.z(R)
        out = torch_cuda.zeros((R, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
        o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0)
        g.gp_sample(op, R, dev(torch_cuda, w.bw), dev(torch_cuda, z1), dev(torch_cuda, z2), out, o)
        grid = orc.grid(w.mask, w.conn)
        ref = orc.sample(grid, w.alpha, w.B, w.bw, z1, z2)
        for r in range(R):
            assert np.linalg.norm(out[r].cpu().numpy() - ref[r]) <= REL_ERR * np.linalg.norm(ref[r])
        b1, b2 = rhs(w, 3, 11), rhs(w2, 2, 12)
        x1 = torch_cuda.zeros(b1.shape, dtype=torch_cuda.float64, device="cuda")
        x2 = torch_cuda.zeros(b2.shape, dtype=torch_cuda.float64, device="cuda")
        st, stats = g.gp_solve_batch(ctx, [(op, 3, dev(torch_cuda, b1), x1), (op2, 2, dev(torch_cuda, b2), x2)], o)
        assert len(stats) == 5 and all(s["status"] == g.GP_OK for s in stats)
        Q1 = orc.precision(grid, w.alpha, w.B)
        Q2 = orc.precision(orc.grid(w2.mask, w2.conn), w2.alpha, w2.B)
        assert np.all(orc.relres(Q1, x1.cpu().numpy(), b1) <= tol)
        assert np.all(orc.relres(Q2, x2.cpu().numpy(), b2) <= tol)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)
        g.gp_op_destroy(op2)


def test_whole_brain_fewer_iterations_than_block_jacobi(g, ctx, torch_cuda):
    """The whole-brain operator (N = 52,740, K = 6): residual recomputed by
    the oracle, and the iteration counts of the two preconditioners in FP64."""
    w = synth.brain_3d()
    op = make_op(g, ctx, torch_cuda, w)
    try:
        R, tol = 4, 1e-8
        b = w.rhs(R)
        Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
        its = {}
        for name, pc in (("rb", g.GP_PRECOND_RB_IC0), ("bj", g.GP_PRECOND_BLOCK_JACOBI)):
            x = torch_cuda.zeros((R, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            o = g.gp_opts_default(tol=tol, precond=pc, precision=g.GP_PREC_FP64)
            st, stats = g.gp_solve(op, R, dev(torch_cuda, b), x, o)
            assert np.all(orc.relres(Q, x.cpu().numpy(), b) <= tol)
            its[name] = [s["inner_iters"] for s in stats]
        print("iterations", its)
        assert max(its["rb"]) < min(its["bj"])
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_autotune_with_the_incomplete_factor(g, ctx, torch_cuda):
    """The autotuner times right-hand sides per work item for the red-black
    solver and later solves use the tuned value; the results do not depend
    on it."""
    w = synth.tiny((29, 23, 17), 6, 3, seed=41)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        o = g.gp_opts_default(tol=1e-10, precond=g.GP_PRECOND_RB_IC0, zero_guess=1)
        best = g.gp_autotune(op, 8, o)
        assert best.rhs_tile in (1, 2, 4, 8) and best.precond == g.GP_PRECOND_RB_IC0
        b = rhs(w, 8, 42)
        x = torch_cuda.zeros(b.shape, dtype=torch_cuda.float64, device="cuda")
        _, stats = g.gp_solve(op, 8, dev(torch_cuda, b), x, o)
        assert all(s["status"] == g.GP_OK for s in stats)
        Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
        assert np.all(orc.relres(Q, x.cpu().numpy(), b) <= 1e-10)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_items_of_one_operator_are_solved_together(g, ctx, torch_cuda, precision):
    """Two batch items of one operator (stacked into one run), a zero start
    value with x holding NaN on entry, b = 0 in the last right-hand side of
    each item, and a stats array in item order."""
    w = synth.tiny((21, 17, 9), 6, 3, seed=43)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        tol = 1e-10
        b1, b2 = rhs(w, 2, 13), rhs(w, 3, 14)
        nan = float("nan")
        x1 = torch_cuda.full(b1.shape, nan, dtype=torch_cuda.float64, device="cuda")
        x2 = torch_cuda.full(b2.shape, nan, dtype=torch_cuda.float64, device="cuda")
        prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
        o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0, precision=prec, zero_guess=1)
        st, stats = g.gp_solve_batch(ctx, [(op, 2, dev(torch_cuda, b1), x1), (op, 3, dev(torch_cuda, b2), x2)], o)
        assert len(stats) == 5 and all(s["status"] == g.GP_OK for s in stats)
        assert stats[1]["inner_iters"] == 0 and stats[4]["inner_iters"] == 0   # b = 0
        Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
        for b, x in ((b1, x1), (b2, x2)):
            xs = x.cpu().numpy()
            assert np.all(np.isfinite(xs)) and np.all(orc.relres(Q, xs, b) <= tol)
            assert np.all(xs[-1] == 0.0)
            ref = orc.solve_direct(Q, b)
            for r in range(b.shape[0] - 1):
                assert np.linalg.norm(xs[r] - ref[r]) <= REL_ERR * np.linalg.norm(ref[r])
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_replayed_round_shape_continues_and_repeats_exactly(g, ctx, torch_cuda, precision):
    """The first round of a solve replays the previous solve's outer-step
    positions.  After a solve of b = 0 only (one outer step each) the next
    solve needs far more than that shape and must go on in planned rounds to
    the same answer; a third solve of the same right-hand sides, now replayed
    in one round, must give the same x bit for bit (each right-hand side takes
    the same steps whatever the round boundaries)."""
    w = synth.tiny((23, 19, 9), 6, 3, seed=29)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        R, tol = 4, 1e-10
        prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
        o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0, precision=prec, zero_guess=1)
        zero = np.zeros((R, w.K, w.N))
        x = dev(torch_cuda, zero)
        _, stats0 = g.gp_solve(op, R, dev(torch_cuda, zero), x, o)
        assert all(s["outer_steps"] == 1 and s["inner_iters"] == 0 for s in stats0)
        b = rhs(w, R, 31)
        xs = []
        stats = []
        for _ in range(2):
            x = dev(torch_cuda, zero)
            _, st = g.gp_solve(op, R, dev(torch_cuda, b), x, o)
            xs.append(x.cpu().numpy())
            stats.append(st)
        Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
        ref = orc.solve_direct(Q, b)
        assert np.all(orc.relres(Q, xs[0], b) <= tol)
        for r in range(R - 1):
            assert np.linalg.norm(xs[0][r] - ref[r]) <= REL_ERR * np.linalg.norm(ref[r]), r
        assert np.all(xs[0][R - 1] == 0.0)
        assert np.array_equal(xs[0], xs[1])
        for a, c in zip(stats[0], stats[1]):
            assert (a["inner_iters"], a["outer_steps"]) == (c["inner_iters"], c["outer_steps"])
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_whole_brain_step_in_the_benchmark_configuration(g, ctx, torch_cuda):
    """The benchmark's solve at full size and in its launch configuration:
    whole-brain operator (N = 52,740, K = 6), 32 Algorithm-2 samples and 32
    Rademacher probes in one grouped solve, red-black incomplete Cholesky, FP32
    inner iterations with FP64 refinement to 1e-8 from a zero start, graphs
    on.  Every right-hand side's residual is recomputed by the oracle; sampled
    solutions and the trace estimates are checked against the oracle's; the
    repeated solve (its first round replayed from the first) gives the same x."""
    torch = torch_cuda
    w = synth.brain_3d()
    op = make_op(g, ctx, torch, w)
    try:
        S = M = 32
        z1, z2 = w.z(S)
        v = w.probes(M)
        bs = torch.empty((S, w.K, w.N), dtype=torch.float64, device="cuda")
        g.gp_perturb_rhs(op, S, dev(torch, w.bw), dev(torch, z1), dev(torch, z2), bs)
        vd = torch.from_numpy(np.ascontiguousarray(v)).cuda()
        bp = torch.empty((M, w.K, w.N), dtype=torch.float64, device="cuda")
        g.gp_probe_rhs(op, M, vd, bp)
        o = g.gp_opts_default(tol=1e-8, zero_guess=1, precond=g.GP_PRECOND_RB_IC0,
                              precision=g.GP_PREC_FP32_REFINE64)
        runs = []
        for _ in range(2):
            xs = torch.zeros_like(bs)
            xp = torch.zeros_like(bp)
            _, stats = g.gp_solve_batch(ctx, [(op, S, bs, xs), (op, M, bp, xp)], o)
            assert all(s["status"] == g.GP_OK and s["relres"] <= 1e-8 for s in stats)
            t = g.gp_trace_reduce(op, M, vd, xp, w.K)
            runs.append((xs.cpu().numpy(), xp.cpu().numpy(), t))
        grid = orc.grid(w.mask, w.conn)
        Q = orc.precision(grid, w.alpha, w.B)
        b_ref = orc.perturbation_rhs(grid, w.alpha, w.B, w.bw, z1, z2)
        xs_h, xp_h, (t, tk, gk) = runs[0]
        assert np.max(np.abs(bs.cpu().numpy() - b_ref)) <= 1e-12 * np.max(np.abs(b_ref))
        assert np.all(orc.relres(Q, xs_h, b_ref) <= 1e-8)
        assert np.all(orc.relres(Q, xp_h, v.astype(np.float64)) <= 1e-8)
        pick = [0, 13, 31]
        xs_ref = orc.solve(Q, b_ref[pick], tol=1e-13)
        u_ref = orc.solve(Q, v.astype(np.float64), tol=1e-12)
        for r_i, r in enumerate(pick):
            assert np.linalg.norm(xs_h[r] - xs_ref[r_i]) <= 1e-6 * np.linalg.norm(xs_ref[r_i]), r
            assert np.linalg.norm(xp_h[r] - u_ref[r]) <= 1e-6 * np.linalg.norm(u_ref[r]), r
        t_ref, tk_ref, gk_ref, _ = orc.hutchinson(grid, Q, v, u=u_ref)
        assert abs(t - t_ref) <= 1e-6 * abs(t_ref)
        assert np.all(np.abs(np.asarray(tk) - tk_ref) <= 1e-6 * np.abs(tk_ref))
        assert np.all(np.abs(np.asarray(gk) - gk_ref) <= 1e-6 * np.abs(gk_ref))
        assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    finally:
        torch.cuda.synchronize()
        g.gp_op_destroy(op)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cells", [[(1, 1, 1)], [(2, 1, 1)], [(1, 1, 1), (2, 1, 1)],
                                   [(1, 1, 1), (2, 1, 1), (1, 2, 1), (2, 2, 1), (1, 1, 2)]])
def test_degenerate_colourings(g, ctx, torch_cuda, precision, cells):
    """Masks with no red voxel (one odd voxel), no black voxel (one even
    voxel), one of each, and a small cluster: the black system may be empty
    (the red voxels are then solved directly by the recovery) or the red one
    may be (nothing to eliminate).  Compared with the oracle's direct solve."""
    mask = np.zeros((4, 4, 4), dtype=np.uint8)   # [z][y][x]
    for (x, y, z) in cells:
        mask[z, y, x] = 1
    K = 3
    rng = np.random.default_rng(len(cells))
    N = int(mask.sum())
    M = rng.standard_normal((N, K, K))
    B = np.einsum("nij,nkj->nik", M, M) + 2.0 * np.eye(K)
    alpha = np.array([0.5, 1.5, 3.0])
    op = g.gp_op_create(ctx, mask, 6, K)
    try:
        g.gp_op_set_blocks(op, dev(torch_cuda, B))
        g.gp_op_set_alpha(op, alpha)
        R = 3
        b = rng.standard_normal((R, K, N))
        b[R - 1] = 0.0
        x = dev(torch_cuda, np.zeros((R, K, N)))
        prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
        o = g.gp_opts_default(tol=1e-10, precond=g.GP_PRECOND_RB_IC0, precision=prec, zero_guess=1)
        _, stats = g.gp_solve(op, R, dev(torch_cuda, b), x, o)
        assert all(s["status"] == g.GP_OK for s in stats)
        Q = orc.precision(orc.grid(mask, 6), alpha, B)
        ref = orc.solve_direct(Q, b)
        xs = x.cpu().numpy()
        for r in range(R - 1):
            assert np.linalg.norm(xs[r] - ref[r]) <= REL_ERR * np.linalg.norm(ref[r]), r
        assert np.all(xs[R - 1] == 0.0)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,conn,K", [((29, 23, 17), 6, 3), ((37, 35, 1), 4, 2), ((21, 19, 13), 6, 10)])
def test_rhs_per_work_item_does_not_change_results(g, ctx, torch_cuda, precision, dims, conn, K):
    """The work decomposition (1, 2, 3, 4 or 8 right-hand sides per workgroup
    of the solver-round launches; with 3 a pair of the paired red-stage vector
    is split between two work items) changes neither the arithmetic nor its
    order: bitwise equal solutions and iteration counts, which match the
    oracle's direct solve."""
    w = synth.tiny(dims, conn, K, seed=70 + K)
    op = make_op(g, ctx, torch_cuda, w)
    try:
        R, tol = 5, 1e-10
        b = rhs(w, R, 71)
        prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
        out = {}
        for rt in (1, 2, 3, 4, 8):
            x = torch_cuda.zeros(b.shape, dtype=torch_cuda.float64, device="cuda")
            o = g.gp_opts_default(tol=tol, precond=g.GP_PRECOND_RB_IC0, precision=prec, rhs_tile=rt, zero_guess=1)
            _, stats = g.gp_solve(op, R, dev(torch_cuda, b), x, o)
            assert all(s["status"] == g.GP_OK for s in stats)
            out[rt] = (x.cpu().numpy(), [(s["inner_iters"], s["outer_steps"]) for s in stats])
        for rt in (2, 3, 4, 8):
            assert np.array_equal(out[rt][0], out[1][0]), rt
            assert out[rt][1] == out[1][1], rt
        Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
        ref = orc.solve_direct(Q, b)
        for r in range(R - 1):
            assert np.linalg.norm(out[1][0][r] - ref[r]) <= REL_ERR * np.linalg.norm(ref[r]), r
        assert np.all(out[1][0][R - 1] == 0.0)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grouped_operators_match_alone_bitwise(g, ctx, torch_cuda, precision):
    """Five operators of three different K (two launch groups share K = 3)
    solved in one grouped batch give bitwise the solutions each gives alone
    (the reductions are per right-hand side and tile, whatever the company),
    and match the oracle."""
    ws = [synth.tiny((31, 27, 14), 6, 3, seed=81), synth.tiny((18, 16, 11), 6, 5, seed=82),
          synth.tiny((25, 21, 12), 6, 3, seed=83), synth.tiny((44, 39, 1), 4, 2, seed=84),
          synth.tiny((15, 14, 13), 6, 5, seed=85)]
    ops = [make_op(g, ctx, torch_cuda, w) for w in ws]
    try:
        prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
        o = g.gp_opts_default(tol=1e-10, precond=g.GP_PRECOND_RB_IC0, precision=prec, zero_guess=1)
        Rs = [3, 2, 4, 1, 2]
        bs = [rhs(w, R, 90 + i) if R > 1 else np.random.default_rng(9).standard_normal((1, w.K, w.N))
              for i, (w, R) in enumerate(zip(ws, Rs))]
        alone = []
        for op, b, R in zip(ops, bs, Rs):
            x = torch_cuda.zeros(b.shape, dtype=torch_cuda.float64, device="cuda")
            g.gp_solve(op, R, dev(torch_cuda, b), x, o)
            alone.append(x.cpu().numpy())
        xs = [torch_cuda.zeros(b.shape, dtype=torch_cuda.float64, device="cuda") for b in bs]
        bd = [dev(torch_cuda, b) for b in bs]
        _, stats = g.gp_solve_batch(ctx, [(op, R, b, x) for op, R, b, x in zip(ops, Rs, bd, xs)], o)
        assert len(stats) == sum(Rs) and all(s["status"] == g.GP_OK for s in stats)
        for i, (w, b, x, a) in enumerate(zip(ws, bs, xs, alone)):
            xh = x.cpu().numpy()
            assert np.array_equal(xh, a), i
            Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
            assert np.all(orc.relres(Q, xh, b) <= 1e-10), i
            ref = orc.solve_direct(Q, b) if w.N * w.K <= 20000 else orc.solve(Q, b)
            for r in range(b.shape[0]):
                if np.any(b[r]):
                    assert np.linalg.norm(xh[r] - ref[r]) <= REL_ERR * np.linalg.norm(ref[r]), (i, r)
    finally:
        torch_cuda.cuda.synchronize()
        for op in ops:
            g.gp_op_destroy(op)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_many_operators_and_items_match_alone_bitwise(g, ctx, torch_cuda, precision):
    """Nine operators (K = 2..5) with two items each: enough set-ups and items
    that the grouped solve runs the preconditioner set-ups, the splits and the
    recoveries on branch streams side by side.  Every item's solution equals
    bitwise the one its operator gives alone (one item at a time, everything
    in order on one stream), and its residual meets the tolerance."""
    shapes = [((17, 15, 9), 2), ((13, 12, 10), 3), ((19, 11, 8), 4), ((12, 12, 12), 5), ((21, 9, 7), 3),
              ((14, 16, 6), 2), ((11, 13, 9), 5), ((16, 10, 11), 4), ((15, 15, 5), 3)]
    ws = [synth.tiny(d, 6, K, seed=120 + i) for i, (d, K) in enumerate(shapes)]
    ops = [make_op(g, ctx, torch_cuda, w) for w in ws]
    try:
        prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
        o = g.gp_opts_default(tol=1e-10, precond=g.GP_PRECOND_RB_IC0, precision=prec, zero_guess=1)
        items = []   # (operator index, b) two per operator: 3 and 2 right-hand sides
        for i, w in enumerate(ws):
            items.append((i, rhs(w, 3, 130 + 2 * i)))
            items.append((i, np.random.default_rng(131 + 2 * i).standard_normal((2, w.K, w.N))))
        alone = []
        for i, b in items:
            x = torch_cuda.zeros(b.shape, dtype=torch_cuda.float64, device="cuda")
            _, st = g.gp_solve(ops[i], b.shape[0], dev(torch_cuda, b), x, o)
            assert all(s["status"] == g.GP_OK for s in st)
            alone.append(x.cpu().numpy())
        for op, w in zip(ops, ws):
            g.gp_op_set_alpha(op, w.alpha)   # every factor rebuilt by the grouped solve
        xs = [torch_cuda.zeros(b.shape, dtype=torch_cuda.float64, device="cuda") for _, b in items]
        bd = [dev(torch_cuda, b) for _, b in items]
        _, stats = g.gp_solve_batch(ctx, [(ops[i], b.shape[0], bb, x) for (i, b), bb, x in zip(items, bd, xs)], o)
        assert len(stats) == sum(b.shape[0] for _, b in items) and all(s["status"] == g.GP_OK for s in stats)
        for n, ((i, b), x, a) in enumerate(zip(items, xs, alone)):
            xh = x.cpu().numpy()
            assert np.array_equal(xh, a), n
            w = ws[i]
            Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, w.B)
            assert np.all(orc.relres(Q, xh, b) <= 1e-10), n
    finally:
        torch_cuda.cuda.synchronize()
        for op in ops:
            g.gp_op_destroy(op)
