"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: every solution must reach FP64 relative residual <= tol (1e-10
for the 2D slice, 1e-8 otherwise) and relative error <= 1e-6 against the
oracle's solution, per right-hand side over all K*N entries; each regressor
block's error, measured against the norm of the whole right-hand side's
solution, is held to the same bound.  Index work is bit-exact; FP64 operator
products agree to 1e-12 relative."""
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
    return torch


@pytest.fixture(scope="module")
def g(built_library, torch_cuda):
    from paper_1606_00980_amd import gmrf
    return gmrf


_LIVE_OPS = []


@pytest.fixture(scope="module")
def ctx(g, torch_cuda):
    h = g.gp_ctx_create(0, torch_cuda.cuda.current_stream().cuda_stream, 0)
    yield h
    while _LIVE_OPS:
        g.gp_op_destroy(_LIVE_OPS.pop())
    g.gp_ctx_destroy(h)


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


class Op:
    def __init__(self, g, ctx, torch, w):
        self.g, self.torch, self.w = g, torch, w
        self.h = g.gp_op_create(ctx, w.mask, w.conn, w.K)
        self.B = dev(torch, w.B)
        g.gp_op_set_blocks(self.h, self.B)
        g.gp_op_set_alpha(self.h, w.alpha)
        self.grid = orc.grid(w.mask, w.conn)
        self.Q = orc.precision(self.grid, w.alpha, w.B)
        _LIVE_OPS.append(self.h)


def rel_err(x, ref):
    x = np.asarray(x).reshape(ref.shape)
    return np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300)


def check_solutions(x, ref, K, N, tol=REL_ERR):
    x = np.asarray(x).reshape(-1, K, N)
    ref = np.asarray(ref).reshape(-1, K, N)
    for r in range(ref.shape[0]):
        scale = max(np.linalg.norm(ref[r]), 1e-300)
        assert np.linalg.norm(x[r] - ref[r]) <= tol * scale, (r, rel_err(x[r], ref[r]))
        for k in range(K):
            assert np.linalg.norm(x[r, k] - ref[r, k]) <= tol * scale, (r, k)


def opts(g, **kw):
    return g.gp_opts_default(**kw)


# ----------------------------------------------------------------- operator
@pytest.mark.parametrize("maker", ["tiny3d", "tiny2d", "slice"])
def test_voxel_index_and_edges_exact(g, ctx, torch_cuda, maker):
    w = {"tiny3d": lambda: synth.tiny((13, 11, 7), 6, 3, seed=1),
         "tiny2d": lambda: synth.tiny((19, 17, 1), 4, 2, seed=2),
         "slice": synth.slice_2d}[maker]()
    op = Op(g, ctx, torch_cuda, w)
    lin = torch_cuda.empty(w.N, dtype=torch_cuda.int32, device="cuda")
    g.gp_op_voxel_index(op.h, lin)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(lin.cpu().numpy(), np.flatnonzero(w.mask.ravel()))
    q = g.gp_op_query(op.h)
    assert q["N"] == op.grid.N and q["E"] == op.grid.E and q["K"] == w.K


@pytest.mark.parametrize("maker,R", [("tiny3d", 3), ("slice", 2), ("brain", 1)])
def test_apply_matches_oracle(g, ctx, torch_cuda, maker, R):
    w = {"tiny3d": lambda: synth.tiny((13, 11, 7), 6, 3, seed=1),
         "slice": synth.slice_2d, "brain": synth.brain_3d}[maker]()
    op = Op(g, ctx, torch_cuda, w)
    x = np.random.default_rng(0).standard_normal((R, w.K, w.N))
    xd = dev(torch_cuda, x)
    yd = torch_cuda.empty_like(xd)
    g.gp_apply(op.h, R, xd, yd)
    torch_cuda.cuda.synchronize()
    y = yd.cpu().numpy()
    ref = orc.apply(op.Q, x)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


# ------------------------------------------------------------- solves
def test_slice_fp64_jacobi_solve_and_sample(g, ctx, torch_cuda):
    """2D slice, K = 2: one FP64 Jacobi solve to 1e-10 and one sample."""
    w = synth.slice_2d()
    op = Op(g, ctx, torch_cuda, w)
    o = opts(g, tol=1e-10, precond=g.GP_PRECOND_JACOBI, precision=g.GP_PREC_FP64)
    b = dev(torch_cuda, w.bw[None])
    x = torch_cuda.zeros_like(b)
    st, stats = g.gp_solve(op.h, 1, b, x, o)
    xs = x.cpu().numpy()
    ref = orc.solve(op.Q, w.bw[None])
    assert stats[0]["relres"] <= 1e-10
    assert orc.relres(op.Q, xs, w.bw[None])[0] <= 1e-10
    check_solutions(xs, ref, w.K, w.N)
    z1, z2 = w.z(1)
    wd = torch_cuda.zeros_like(b)
    st, stats = g.gp_sample(op.h, 1, dev(torch_cuda, w.bw), dev(torch_cuda, z1), dev(torch_cuda, z2), wd, o)
    ref_s = orc.sample(op.grid, w.alpha, w.B, w.bw, z1, z2)
    assert stats[0]["relres"] <= 1e-10
    check_solutions(wd.cpu().numpy(), ref_s, w.K, w.N)


def test_perturb_rhs_matches_oracle(g, ctx, torch_cuda):
    for w in (synth.tiny((9, 8, 5), 6, 3, seed=3), synth.tiny((11, 9, 1), 4, 2, seed=4), synth.slice_2d()):
        op = Op(g, ctx, torch_cuda, w)
        R = 3
        z1, z2 = w.z(R)
        b = torch_cuda.empty((R, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
        g.gp_perturb_rhs(op.h, R, dev(torch_cuda, w.bw), dev(torch_cuda, z1), dev(torch_cuda, z2), b)
        torch_cuda.cuda.synchronize()
        ref = orc.perturbation_rhs(op.grid, w.alpha, w.B, w.bw, z1, z2)
        assert np.max(np.abs(b.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("matvec", ["raster", "zmarch"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("precond", ["jacobi", "block"])
def test_small_solves_all_modes(g, ctx, torch_cuda, precision, precond, matvec):
    """Several tiles plus a ragged tail; R = 11 with 4 right-hand sides per workgroup."""
    w = synth.tiny((21, 19, 9), 6, 4, seed=5)
    assert w.N % 256 != 0 and w.N > 3 * 256
    op = Op(g, ctx, torch_cuda, w)
    R = 11
    b = w.rhs(R)
    o = opts(g, tol=1e-8, rhs_tile=4,
             precond=g.GP_PRECOND_JACOBI if precond == "jacobi" else g.GP_PRECOND_BLOCK_JACOBI,
             precision=g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64,
             matvec=g.GP_MATVEC_RASTER if matvec == "raster" else g.GP_MATVEC_ZMARCH)
    bd = dev(torch_cuda, b)
    x = torch_cuda.zeros_like(bd)
    st, stats = g.gp_solve(op.h, R, bd, x, o)
    xs = x.cpu().numpy()
    ref = orc.solve(op.Q, b)
    assert max(s["relres"] for s in stats) <= 1e-8
    assert np.all(orc.relres(op.Q, xs, b) <= 1e-8)
    check_solutions(xs, ref, w.K, w.N)


def test_brain_fp64_block_jacobi_single_rhs(g, ctx, torch_cuda):
    """Whole-brain 3D operator, K = 6, one FP64 right-hand side, block Jacobi, 1e-8."""
    w = synth.brain_3d()
    op = Op(g, ctx, torch_cuda, w)
    o = opts(g, tol=1e-8, precond=g.GP_PRECOND_BLOCK_JACOBI, precision=g.GP_PREC_FP64)
    b = dev(torch_cuda, w.bw[None])
    x = torch_cuda.zeros_like(b)
    st, stats = g.gp_solve(op.h, 1, b, x, o)
    xs = x.cpu().numpy()
    ref = orc.solve(op.Q, w.bw[None], tol=1e-13)
    assert stats[0]["relres"] <= 1e-8
    assert orc.relres(op.Q, xs, w.bw[None])[0] <= 1e-8
    check_solutions(xs, ref, w.K, w.N)


def test_brain_batched_mixed_samples_and_probes(g, ctx, torch_cuda):
    """Same operator, 64 right-hand sides in one grouped solve: 32 perturbation
    samples and 32 Rademacher probes, FP32 inner PCG with FP64 refinement to
    1e-8; trace estimates against the oracle's with the same probes."""
    torch = torch_cuda
    w = synth.brain_3d()
    op = Op(g, ctx, torch, w)
    S = M = 32
    z1, z2 = w.z(S, stream=CFG_STREAM)
    v = w.probes(M, stream=CFG_STREAM)
    bs = torch.empty((S, w.K, w.N), dtype=torch.float64, device="cuda")
    g.gp_perturb_rhs(op.h, S, dev(torch, w.bw), dev(torch, z1), dev(torch, z2), bs)
    vd = dev(torch, v)
    bp = torch.empty((M, w.K, w.N), dtype=torch.float64, device="cuda")
    g.gp_probe_rhs(op.h, M, vd, bp)
    xs = torch.zeros_like(bs)
    xp = torch.zeros_like(bp)
    o = opts(g, tol=1e-8)
    st, stats = g.gp_solve_batch(ctx, [(op.h, S, bs, xs), (op.h, M, bp, xp)], o)
    assert all(s["status"] == 0 and s["relres"] <= 1e-8 for s in stats)
    t, tk, gk = g.gp_trace_reduce(op.h, M, vd, xp, w.K)
    xs_h, xp_h = xs.cpu().numpy(), xp.cpu().numpy()
    b_ref = orc.perturbation_rhs(op.grid, w.alpha, w.B, w.bw, z1, z2)
    assert np.max(np.abs(bs.cpu().numpy() - b_ref)) <= 1e-12 * np.max(np.abs(b_ref))
    assert np.all(orc.relres(op.Q, xs_h, b_ref) <= 1e-8)
    assert np.all(orc.relres(op.Q, xp_h, v.astype(np.float64)) <= 1e-8)
    # full oracle comparison on a sample of the right-hand sides
    pick = [0, 7, 31]
    check_solutions(xs_h[pick], orc.solve(op.Q, b_ref[pick], tol=1e-13), w.K, w.N)
    u_ref = orc.solve(op.Q, v.astype(np.float64), tol=1e-12)
    check_solutions(xp_h[pick], u_ref[pick], w.K, w.N)
    t_ref, tk_ref, gk_ref, _ = orc.hutchinson(op.grid, op.Q, v, u=u_ref)
    assert abs(t - t_ref) <= REL_ERR * abs(t_ref)
    assert np.all(np.abs(tk - tk_ref) <= REL_ERR * np.abs(tk_ref))
    assert np.all(np.abs(gk - gk_ref) <= REL_ERR * np.abs(gk_ref))


CFG_STREAM = 0


def test_trace_small_vs_oracle(g, ctx, torch_cuda):
    w = synth.tiny((12, 10, 6), 6, 3, seed=6)
    op = Op(g, ctx, torch_cuda, w)
    m = 9
    v = w.probes(m)
    u = torch_cuda.empty((m, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
    t, tk, gk, stats = g.gp_trace(op.h, m, dev(torch_cuda, v), u, w.K, opts(g, tol=1e-10))
    t_ref, tk_ref, gk_ref, _ = orc.hutchinson(op.grid, op.Q, v)
    assert abs(t - t_ref) <= REL_ERR * abs(t_ref)
    assert np.allclose(tk, tk_ref, rtol=REL_ERR)
    assert np.allclose(gk, gk_ref, rtol=REL_ERR)


# --------------------------------------------------------------- uneven batch
def test_uneven_batch_grouped(g, ctx, torch_cuda):
    """Operators of different K and N advanced together in grouped launches."""
    torch = torch_cuda
    ws = [synth.tiny((11, 9, 7), 6, 2, seed=7), synth.tiny((15, 13, 8), 6, 5, seed=8),
          synth.tiny((9, 9, 9), 6, 2, seed=9), synth.tiny((17, 11, 1), 4, 3, seed=10)]
    ops = [Op(g, ctx, torch, w) for w in ws]
    items, bs, xs = [], [], []
    for i, (w, op) in enumerate(zip(ws, ops)):
        R = 2 + i
        b = w.rhs(R)
        bd = dev(torch, b)
        xd = torch.zeros_like(bd)
        items.append((op.h, R, bd, xd))
        bs.append(b)
        xs.append(xd)
    st, stats = g.gp_solve_batch(ctx, items, opts(g, tol=1e-8, rhs_tile=2))
    assert all(s["status"] == 0 for s in stats)
    for w, op, b, xd in zip(ws, ops, bs, xs):
        check_solutions(xd.cpu().numpy(), orc.solve(op.Q, b), w.K, w.N)


# ------------------------------------------------------------------ edges
def test_zero_rhs_gives_zero(g, ctx, torch_cuda):
    w = synth.tiny((8, 7, 5), 6, 2, seed=11)
    op = Op(g, ctx, torch_cuda, w)
    b = np.zeros((2, w.K, w.N))
    b[1] = w.bw
    bd = dev(torch_cuda, b)
    x = torch_cuda.full_like(bd, 3.0)
    st, stats = g.gp_solve(op.h, 2, bd, x, opts(g))
    xs = x.cpu().numpy()
    assert np.all(xs[0] == 0.0)
    assert stats[0]["inner_iters"] == 0 and stats[0]["status"] == 0
    check_solutions(xs[1:], orc.solve(op.Q, b[1:]), w.K, w.N)


def test_single_voxel_and_k1(g, ctx, torch_cuda):
    mask = np.zeros((3, 3, 3), dtype=np.uint8)
    mask[1, 1, 1] = 1
    torch = torch_cuda
    h = g.gp_op_create(ctx, mask, 6, 3)
    B = np.array([[[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]]])
    Bd = dev(torch, B)
    g.gp_op_set_blocks(h, Bd)
    g.gp_op_set_alpha(h, [1.0, 2.0, 3.0])
    b = np.array([[[1.0], [2.0], [3.0]]])
    bd = dev(torch, b)
    x = torch.zeros_like(bd)
    g.gp_solve(h, 1, bd, x, opts(g, precision=g.GP_PREC_FP64))
    assert np.allclose(x.cpu().numpy().ravel(), np.linalg.solve(B[0], b.ravel()), rtol=1e-8)
    g.gp_op_destroy(h)
    w = synth.tiny((10, 9, 6), 6, 1, seed=12)
    op = Op(g, ctx, torch, w)
    bd = dev(torch, w.bw[None])
    x = torch.zeros_like(bd)
    g.gp_solve(op.h, 1, bd, x, opts(g))
    check_solutions(x.cpu().numpy(), orc.solve(op.Q, w.bw[None]), 1, w.N)


def test_k16_and_slices_without_z_coupling(g, ctx, torch_cuda):
    w = synth.tiny((9, 8, 4), 6, 16, seed=13)
    op = Op(g, ctx, torch_cuda, w)
    b = w.rhs(2)
    bd = dev(torch_cuda, b)
    x = torch_cuda.zeros_like(bd)
    g.gp_solve(op.h, 2, bd, x, opts(g))
    check_solutions(x.cpu().numpy(), orc.solve(op.Q, b), w.K, w.N)
    # a 4-neighbour operator over several slices: the slices do not interact
    w2 = synth.tiny((9, 8, 5), 6, 2, seed=14)
    h = g.gp_op_create(ctx, w2.mask, 4, 2)
    Bd = dev(torch_cuda, w2.B)
    g.gp_op_set_blocks(h, Bd)
    g.gp_op_set_alpha(h, w2.alpha)
    gr = orc.grid(w2.mask, 6)
    G4 = orc.grid(w2.mask[:1], 4)
    assert G4.N > 0
    bd = dev(torch_cuda, w2.bw[None])
    x = torch_cuda.zeros_like(bd)
    g.gp_solve(h, 1, bd, x, opts(g))
    # oracle: block-diagonal over slices
    xs = x.cpu().numpy()[0]
    z = gr.coords[:, 2]
    for zz in np.unique(z):
        sel = np.flatnonzero(z == zz)
        gs = orc.grid(w2.mask[zz:zz + 1], 4)
        Qs = orc.precision(gs, w2.alpha, w2.B[sel])
        ref = orc.solve(Qs, w2.bw[:, sel])
        assert rel_err(xs[:, sel], ref) <= REL_ERR
    g.gp_op_destroy(h)


@pytest.mark.parametrize("K", [15, 23])
def test_large_k_every_preconditioner_and_precision(g, ctx, torch_cuda, K):
    """The paper's real-data regressor counts: solves with each
    preconditioner in both precisions, an Algorithm-2 sample, and the data
    term assembled on the device with AR(2), against the oracle."""
    w = synth.tiny((9, 8, 4), 6, K, seed=13 + K, T=120, P=2)
    op = Op(g, ctx, torch_cuda, w)
    b = w.rhs(3)
    ref = orc.solve(op.Q, b)
    bd = dev(torch_cuda, b)
    for pc in (g.GP_PRECOND_JACOBI, g.GP_PRECOND_BLOCK_JACOBI, g.GP_PRECOND_RB_IC0):
        for prec in (g.GP_PREC_FP64, g.GP_PREC_FP32_REFINE64):
            x = torch_cuda.zeros_like(bd)
            g.gp_solve(op.h, 3, bd, x, opts(g, precond=pc, precision=prec))
            check_solutions(x.cpu().numpy(), ref, w.K, w.N)
    z1, z2 = w.z(2)
    out = torch_cuda.zeros((2, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
    g.gp_sample(op.h, 2, dev(torch_cuda, w.bw), dev(torch_cuda, z1), dev(torch_cuda, z2), out, opts(g))
    check_solutions(out.cpu().numpy(), orc.sample(op.grid, w.alpha, w.B, w.bw, z1, z2), w.K, w.N)
    d = g.gp_data_create(op.h, w.X.shape[0], 2, w.X, dev(torch_cuda, w.Y))
    try:
        lam = 1.0 / w.sigma2
        bw = torch_cuda.empty((w.K, w.N), dtype=torch_cuda.float64, device="cuda")
        g.gp_data_assemble(d, dev(torch_cuda, lam), 1, dev(torch_cuda, w.ar[None, :2]), bw)
        B_ref, b_ref = orc.data_term_mc(w.X, w.Y, w.ar[None, :2], lam)
        assert np.abs(bw.cpu().numpy() - b_ref).max() <= 1e-10 * np.abs(b_ref).max()
        Q = orc.precision(op.grid, w.alpha, B_ref)
        xv = np.random.default_rng(3).standard_normal((1, w.K, w.N))
        y = torch_cuda.empty((1, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
        g.gp_apply(op.h, 1, dev(torch_cuda, xv), y)
        yr = orc.apply(Q, xv)
        assert np.abs(y.cpu().numpy() - yr).max() <= 1e-10 * np.abs(yr).max()
    finally:
        g.gp_data_destroy(d)


def test_not_spd_block_is_reported(g, ctx, torch_cuda):
    w = synth.tiny((8, 7, 5), 6, 3, seed=15)
    B = w.B.copy()
    B[17] = -np.eye(3)
    h = g.gp_op_create(ctx, w.mask, 6, 3)
    Bd = dev(torch_cuda, B)
    with pytest.raises(g.GmrfError) as e:
        g.gp_op_set_blocks(h, Bd)
    assert e.value.status == g.GP_ERR_NOT_SPD and e.value.bad_voxel == 17
    g.gp_op_destroy(h)


def test_iteration_cap_and_breakdown(g, ctx, torch_cuda):
    w = synth.tiny((10, 9, 6), 6, 3, seed=16)
    op = Op(g, ctx, torch_cuda, w)
    bd = dev(torch_cuda, w.bw[None])
    x = torch_cuda.zeros_like(bd)
    st, stats = g.gp_solve(op.h, 1, bd, x, opts(g, max_iter=1), check=False)
    assert st == g.GP_ERR_NOT_CONVERGED and stats[0]["status"] == g.GP_ERR_NOT_CONVERGED
    assert stats[0]["inner_iters"] == 1
    assert np.all(np.isfinite(x.cpu().numpy()))
    b = w.bw[None].copy()
    b[0, 1, 5] = np.nan
    x = torch_cuda.zeros_like(bd)
    st, stats = g.gp_solve(op.h, 1, dev(torch_cuda, b), x, opts(g), check=False)
    assert st == g.GP_ERR_BREAKDOWN


def test_warm_start_converges_immediately(g, ctx, torch_cuda):
    w = synth.tiny((12, 10, 6), 6, 3, seed=17)
    op = Op(g, ctx, torch_cuda, w)
    ref = orc.solve(op.Q, w.bw[None])
    x = dev(torch_cuda, ref)
    st, stats = g.gp_solve(op.h, 1, dev(torch_cuda, w.bw[None]), x, opts(g))
    assert stats[0]["inner_iters"] == 0 and stats[0]["outer_steps"] == 1


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_zero_guess_ignores_x_on_entry(g, ctx, torch_cuda, precision):
    """zero_guess = 1: x is never read, so NaN on entry changes nothing; the
    result equals the solve from an explicit zero start value bit for bit, and
    right-hand sides that end at their first refinement (b = 0; a cap of one
    refinement) leave zeros."""
    w = synth.tiny((13, 11, 7), 6, 3, seed=23)
    op = Op(g, ctx, torch_cuda, w)
    prec = g.GP_PREC_FP64 if precision == "fp64" else g.GP_PREC_FP32_REFINE64
    b = w.rhs(5)
    b[3] = 0.0
    bd = dev(torch_cuda, b)
    x0 = torch_cuda.zeros_like(bd)
    g.gp_solve(op.h, 5, bd, x0, opts(g, precision=prec), check=False)
    xg = torch_cuda.full_like(bd, float("nan"))
    st, stats = g.gp_solve(op.h, 5, bd, xg, opts(g, precision=prec, zero_guess=1), check=False)
    assert torch_cuda.equal(xg, x0)
    assert all(s["status"] == g.GP_OK for s in stats)
    assert torch_cuda.count_nonzero(xg[3]).item() == 0
    check_solutions(xg.cpu().numpy(), orc.solve(op.Q, b), w.K, w.N)
    # one refinement allowed: every right-hand side stops at it, x = 0
    xc = torch_cuda.full_like(bd, float("nan"))
    st, stats = g.gp_solve(op.h, 5, bd, xc, opts(g, precision=prec, zero_guess=1, max_outer=1), check=False)
    assert st == g.GP_ERR_NOT_CONVERGED
    assert torch_cuda.count_nonzero(xc).item() == 0


def test_invalid_arguments_and_budget(g, torch_cuda):
    h = g.gp_ctx_create(0, torch_cuda.cuda.current_stream().cuda_stream, 4096)
    mask = np.ones((4, 4, 4), dtype=np.uint8)
    with pytest.raises(g.GmrfError) as e:
        g.gp_op_create(h, mask, 6, 2)
    assert e.value.status == g.GP_ERR_OOM
    with pytest.raises(g.GmrfError) as e:
        g.gp_op_create(h, mask, 5, 2)
    assert e.value.status == g.GP_ERR_INVALID_ARG
    with pytest.raises(g.GmrfError) as e:
        g.gp_op_create(h, np.zeros((3, 3, 3), np.uint8), 6, 2)
    assert e.value.status == g.GP_ERR_INVALID_ARG
    with pytest.raises(g.GmrfError) as e:
        g.gp_op_create(h, mask, 6, 25)
    assert e.value.status == g.GP_ERR_INVALID_ARG
    assert g.gp_ctx_memory(h)[0] == 0
    g.gp_ctx_destroy(h)


def test_deterministic_and_batch_invariant(g, ctx, torch_cuda):
    """A right-hand side gives bitwise the same result alone and among others."""
    w = synth.tiny((14, 12, 8), 6, 3, seed=18)
    op = Op(g, ctx, torch_cuda, w)
    b = w.rhs(6)
    bd = dev(torch_cuda, b)
    xa = torch_cuda.zeros_like(bd)
    g.gp_solve(op.h, 6, bd, xa, opts(g, rhs_tile=3))
    xb = torch_cuda.zeros_like(bd)
    g.gp_solve(op.h, 6, bd, xb, opts(g, rhs_tile=3))
    assert torch_cuda.equal(xa, xb)
    alone = torch_cuda.zeros_like(bd[2:3])
    g.gp_solve(op.h, 1, bd[2:3].contiguous(), alone, opts(g))
    assert torch_cuda.equal(alone[0], xa[2])


def test_graph_replays_match_eager(g, ctx, torch_cuda):
    """Solver rounds replayed from captured graphs (profiling off) give bitwise
    the eager result (profiling on launches kernel by kernel), over several
    alternating calls with other device work in between."""
    torch = torch_cuda
    w = synth.tiny((15, 12, 9), 6, 3, seed=19)
    op = Op(g, ctx, torch, w)
    b = w.rhs(5)
    bd = dev(torch, b)
    o = opts(g, tol=1e-8, rhs_tile=2)
    g.gp_ctx_profile(ctx, True)
    xe = torch.zeros_like(bd)
    g.gp_solve(op.h, 5, bd, xe, o)
    g.gp_ctx_profile(ctx, False)
    for rep in range(4):
        xg = torch.zeros_like(bd)
        g.gp_solve(op.h, 5, bd, xg, o)
        assert torch.equal(xg, xe), rep
        _ = (bd * 2.0).sum().item()          # unrelated eager work and a sync
        g.gp_ctx_profile(ctx, True)
        xe2 = torch.zeros_like(bd)
        g.gp_solve(op.h, 5, bd, xe2, o)
        g.gp_ctx_profile(ctx, False)
        assert torch.equal(xe2, xe), rep
    check_solutions(xe.cpu().numpy(), orc.solve(op.Q, b), w.K, w.N)


# ----------------------------------------------------------- random vectors
def test_philox_matches_oracle_twin(g, ctx, torch_cuda):
    from oracle import philox
    torch = torch_cuda
    for seed, stream, n in ((0, 0, 1), (12345, 7, 1001), (2 ** 40 + 3, 2 ** 33 + 5, 70001)):
        nb = (n + 3) // 4
        raw = torch.empty(4 * nb, dtype=torch.int32, device="cuda")
        g.gp_rng_raw(ctx, seed, stream, nb, raw)
        ref = philox.philox4x32_10(np.arange(nb, dtype=np.uint64), seed, stream).ravel()
        torch.cuda.synchronize()
        assert np.array_equal(raw.cpu().numpy().view(np.uint32), ref)
        z = torch.empty(n, dtype=torch.float64, device="cuda")
        g.gp_rng_normal(ctx, seed, stream, n, z)
        zr = philox.normal(seed, stream, n)
        torch.cuda.synchronize()
        assert np.allclose(z.cpu().numpy(), zr, rtol=1e-12, atol=1e-13)
        v = torch.empty(n, dtype=torch.int8, device="cuda")
        g.gp_rng_rademacher(ctx, seed, stream, n, v)
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), philox.rademacher(seed, stream, n))


def test_sample_and_trace_with_device_random_vectors(g, ctx, torch_cuda):
    from oracle import philox
    torch = torch_cuda
    w = synth.tiny((11, 10, 7), 6, 3, seed=20)
    op = Op(g, ctx, torch, w)
    R, seed = 3, 777
    o = opts(g, tol=1e-9, seed=seed)
    ws = torch.zeros((R, w.K, w.N), dtype=torch.float64, device="cuda")
    g.gp_sample(op.h, R, dev(torch, w.bw), None, None, ws, o)
    n1 = R * w.K * 3 * w.N
    z1 = philox.normal(seed, 1, n1).reshape(R, w.K, 3, w.N)
    z2 = philox.normal(seed, 2, R * w.K * w.N).reshape(R, w.K, w.N)
    ref = orc.sample(op.grid, w.alpha, w.B, w.bw, z1, z2)
    check_solutions(ws.cpu().numpy(), ref, w.K, w.N)
    m = 7
    u = torch.empty((m, w.K, w.N), dtype=torch.float64, device="cuda")
    t, tk, gk, _ = g.gp_trace(op.h, m, None, u, w.K, o)
    v = philox.rademacher(seed, 3, m * w.K * w.N).reshape(m, w.K, w.N)
    t_ref, tk_ref, gk_ref, _ = orc.hutchinson(op.grid, op.Q, v)
    assert abs(t - t_ref) <= REL_ERR * abs(t_ref)
    assert np.allclose(tk, tk_ref, rtol=REL_ERR) and np.allclose(gk, gk_ref, rtol=REL_ERR)


@pytest.mark.parametrize("zslices", [None, "1", "2", "5"])
@pytest.mark.parametrize("K", [1, 3, 10])
def test_zmarch_tiling_edges(g, ctx, torch_cuda, zslices, K):
    """Footprints wider than one x tile (x halo), rows not a multiple of the
    footprint height, z segments of 1..5 slices, 2D masks; z-march and raster
    kernels both reach the oracle."""
    import os
    torch = torch_cuda
    w = synth.tiny((70, 9, 13), 6, K, seed=22) if K != 1 else synth.tiny((70, 9, 13), 6, 1, seed=22)
    w2 = synth.tiny((67, 11, 1), 4, 2, seed=23)
    old = os.environ.get("GMRF_ZSLICES")
    try:
        if zslices is None:
            os.environ.pop("GMRF_ZSLICES", None)
        else:
            os.environ["GMRF_ZSLICES"] = zslices
        for ww in (w, w2):
            op = Op(g, ctx, torch, ww)
            b = ww.rhs(5)
            bd = dev(torch, b)
            ref = orc.solve(op.Q, b)
            for mv in (g.GP_MATVEC_ZMARCH, g.GP_MATVEC_RASTER):
                for prec in (g.GP_PREC_FP32_REFINE64, g.GP_PREC_FP64):
                    x = torch.zeros_like(bd)
                    st, stats = g.gp_solve(op.h, 5, bd, x, opts(g, tol=1e-9, matvec=mv, precision=prec))
                    assert all(s["relres"] <= 1e-9 for s in stats)
                    check_solutions(x.cpu().numpy(), ref, ww.K, ww.N)
    finally:
        if old is None:
            os.environ.pop("GMRF_ZSLICES", None)
        else:
            os.environ["GMRF_ZSLICES"] = old


def test_autotune_and_table_round_trip(g, ctx, torch_cuda, tmp_path):
    torch = torch_cuda
    w = synth.tiny((20, 16, 9), 6, 4, seed=24)
    op = Op(g, ctx, torch, w)
    best = g.gp_autotune(op.h, 6, g.gp_opts_default(tol=1e-8))
    assert best.rhs_tile in (1, 2, 4, 8, 16) and best.wg_per_cu in (4, 8)
    assert best.matvec in (g.GP_MATVEC_RASTER, g.GP_MATVEC_ZMARCH)
    path = str(tmp_path / "tune.json")
    g.gp_tune_save(ctx, path)
    text = open(path).read()
    assert '"rhs_tile": %d' % best.rhs_tile in text
    ctx2 = g.gp_ctx_create(0, torch.cuda.current_stream().cuda_stream, 0)
    try:
        g.gp_tune_load(ctx2, path)
    finally:
        g.gp_ctx_destroy(ctx2)
    # a solve with automatic launch options now uses the tuned entry
    b = w.rhs(6)
    x = torch.zeros((6, w.K, w.N), dtype=torch.float64, device="cuda")
    g.gp_solve(op.h, 6, dev(torch, b), x, opts(g, tol=1e-8))
    check_solutions(x.cpu().numpy(), orc.solve(op.Q, b), w.K, w.N)
