"""GPU parity, through the C ABI, of the data term assembled on the device
(Appendix A.2 tensors, Appendix B Monte Carlo expectation) against the
oracle's explicit-whitening definition, and of the hyperparameter updates
(alpha and lambda posteriors, one SVB iteration) against the oracle's."""
import numpy as np
import pytest

from oracle import gmrf_oracle as orc
from paper_1606_00980_amd import synth

pytestmark = pytest.mark.gpu


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


def check_operator(g, torch, op, w, B_ref, tol=1e-11):
    """gp_apply with the installed blocks against the oracle's precision."""
    Q = orc.precision(orc.grid(w.mask, w.conn), w.alpha, B_ref)
    x = np.random.default_rng(2).standard_normal((2, w.K, w.N))
    y = torch.empty((2, w.K, w.N), dtype=torch.float64, device="cuda")
    g.gp_apply(op, 2, dev(torch, x), y)
    ref = orc.apply(Q, x)
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < tol, err


@pytest.mark.parametrize("P", [0, 1, 3])
def test_assembly_matches_whitening_definition(g, ctx, torch_cuda, P):
    w = synth.tiny((13, 11, 7), 6, 5, seed=31 + P, T=70, P=max(P, 1))
    ar = w.ar[:P] if P > 0 else np.zeros((0, w.N))
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    try:
        g.gp_op_set_alpha(op, w.alpha)
        d = g.gp_data_create(op, w.X.shape[0], P, w.X, dev(torch_cuda, w.Y))
        try:
            lam = 1.0 / w.sigma2
            bw = torch_cuda.empty((w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            A = dev(torch_cuda, ar[None]) if P > 0 else None
            g.gp_data_assemble(d, dev(torch_cuda, lam), 1, A, bw)
            B_ref, b_ref = orc.data_term_mc(w.X, w.Y, ar[None], lam)
            assert np.allclose(bw.cpu().numpy(), b_ref, rtol=1e-11, atol=1e-11 * np.abs(b_ref).max())
            check_operator(g, torch_cuda, op, w, B_ref)
            # SVB expectation: three draws of A, lambda perturbed per voxel
            if P > 0:
                rng = np.random.default_rng(7)
                A3 = ar[None] + 0.05 * rng.standard_normal((3,) + ar.shape)
                lam3 = lam * rng.uniform(0.5, 2.0, w.N)
                g.gp_data_assemble(d, dev(torch_cuda, lam3), 3, dev(torch_cuda, A3), bw)
                B3, b3 = orc.data_term_mc(w.X, w.Y, A3, lam3)
                assert np.allclose(bw.cpu().numpy(), b3, rtol=1e-11, atol=1e-11 * np.abs(b3).max())
                check_operator(g, torch_cuda, op, w, B3)
            # a solve with the assembled operator
            x = torch_cuda.zeros((1, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            g.gp_solve(op, 1, bw[None].contiguous(), x, g.gp_opts_default(tol=1e-10))
            B_now = B3 if P > 0 else B_ref
            b_now = (b3 if P > 0 else b_ref)[None]
            ref = orc.solve(orc.precision(orc.grid(w.mask, w.conn), w.alpha, B_now), b_now)
            assert np.linalg.norm(x.cpu().numpy() - ref) <= 1e-7 * np.linalg.norm(ref)
        finally:
            g.gp_data_destroy(d)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_assembly_reports_non_spd_voxel(g, ctx, torch_cuda):
    w = synth.tiny((9, 8, 5), 6, 3, seed=41, T=40, P=2)
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    try:
        d = g.gp_data_create(op, w.X.shape[0], 2, w.X, dev(torch_cuda, w.Y))
        try:
            lam = 1.0 / w.sigma2
            lam[17] = -1.0
            with pytest.raises(g.GmrfError) as e:
                g.gp_data_assemble(d, dev(torch_cuda, lam), 1, dev(torch_cuda, w.ar[None]))
            assert e.value.status == g.GP_ERR_NOT_SPD and e.value.bad_voxel == 17
            with pytest.raises(g.GmrfError) as e:
                g.gp_data_assemble(d, dev(torch_cuda, lam), 0, dev(torch_cuda, w.ar[None]))
            assert e.value.status == g.GP_ERR_INVALID_ARG
        finally:
            g.gp_data_destroy(d)
        with pytest.raises(g.GmrfError) as e:
            g.gp_data_create(op, 40, 5, w.X, dev(torch_cuda, w.Y))
        assert e.value.status == g.GP_ERR_INVALID_ARG
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_assembly_whole_brain(g, ctx, torch_cuda):
    """The whole-brain operator (N = 52,740, K = 6, T = 200, AR(3)): b_w for every
    voxel against the generator's data term (pinned to the whitening definition
    on the CPU), and the blocks through an FP64 matvec against the oracle."""
    w = synth.brain_3d(keep_y=True)
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    try:
        g.gp_op_set_alpha(op, w.alpha)
        d = g.gp_data_create(op, w.X.shape[0], 3, w.X, dev(torch_cuda, w.Y))
        try:
            bw = torch_cuda.empty((w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            g.gp_data_assemble(d, dev(torch_cuda, 1.0 / w.sigma2), 1, dev(torch_cuda, w.ar[None]), bw)
            assert np.allclose(bw.cpu().numpy(), w.bw, rtol=1e-10, atol=1e-10 * np.abs(w.bw).max())
            check_operator(g, torch_cuda, op, w, w.B, tol=1e-10)
        finally:
            g.gp_data_destroy(d)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


# --------------------------------------------------- hyperparameter statistics
def test_alpha_posterior_matches_oracle(g, ctx, torch_cuda):
    for dims, conn in (((15, 12, 9), 6), ((20, 17, 1), 4)):
        w = synth.tiny(dims, conn, 4, seed=51)
        op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
        try:
            W = np.random.default_rng(3).standard_normal((3, w.K, w.N)) + w.W_true[None]
            qf, scale, mean = g.gp_alpha_posterior(op, 3, dev(torch_cuda, W), 10.0, 0.1, w.K)
            grid = orc.grid(w.mask, w.conn)
            qf_ref = orc.quadform(grid, W)
            assert np.allclose(qf, qf_ref, rtol=1e-12)
            s1, s2 = orc.alpha_posterior(qf_ref.mean(axis=0), w.N, 10.0, 0.1)
            assert np.allclose(scale, s1, rtol=1e-12) and np.allclose(mean, s1 * s2, rtol=1e-12)
        finally:
            torch_cuda.cuda.synchronize()
            g.gp_op_destroy(op)


@pytest.mark.parametrize("P", [0, 1, 3])
def test_lambda_posterior_matches_oracle(g, ctx, torch_cuda, P):
    w = synth.tiny((12, 10, 6), 6, 5, seed=61 + P, T=64, P=max(P, 1))
    ar = w.ar[:P] if P > 0 else np.zeros((0, w.N))
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    try:
        d = g.gp_data_create(op, w.X.shape[0], P, w.X, dev(torch_cuda, w.Y))
        try:
            rng = np.random.default_rng(9)
            Ns = 2
            W = w.W_true[None] + 0.1 * rng.standard_normal((Ns, w.K, w.N))
            A = ar[None] + 0.05 * rng.standard_normal((Ns,) + ar.shape)
            rss = torch_cuda.empty(w.N, dtype=torch_cuda.float64, device="cuda")
            scale, mean = torch_cuda.empty_like(rss), torch_cuda.empty_like(rss)
            g.gp_data_lambda(d, Ns, dev(torch_cuda, W), dev(torch_cuda, A) if P > 0 else None, 10.0, 0.1,
                             rss, scale, mean)
            ref = np.mean([orc.residual_ss(w.X, w.Y, W[j], A[j]) for j in range(Ns)], axis=0)
            assert np.allclose(rss.cpu().numpy(), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
            s1, s2 = orc.lambda_posterior(ref, w.X.shape[0], P, 10.0, 0.1)
            assert np.allclose(scale.cpu().numpy(), s1, rtol=1e-9)
            assert np.allclose(mean.cpu().numpy(), s1 * s2, rtol=1e-9)
        finally:
            g.gp_data_destroy(d)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)


def test_svb_steps_match_oracle(g, ctx, torch_cuda):
    """Two SVB iterations (fixed random vectors, warm starts, AR draws held)
    against the oracle's steps fed the same inputs."""
    w = synth.tiny((14, 11, 7), 6, 3, seed=71, T=60, P=2)
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    try:
        d = g.gp_data_create(op, w.X.shape[0], 2, w.X, dev(torch_cuda, w.Y))
        try:
            rng = np.random.default_rng(5)
            Ns = 3
            A = w.ar[None] + 0.05 * rng.standard_normal((Ns,) + w.ar.shape)
            z1 = rng.standard_normal((Ns, w.K, 3, w.N))
            z2 = rng.standard_normal((Ns, w.K, w.N))
            alpha = np.array([1.0, 1.0, 1.0])
            lam = 1.0 / w.sigma2.copy()
            grid = orc.grid(w.mask, w.conn)
            Wd = torch_cuda.zeros((Ns, w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            lam_d = dev(torch_cuda, lam)
            bw = torch_cuda.empty((w.K, w.N), dtype=torch_cuda.float64, device="cuda")
            a_gpu = alpha.copy()
            a_ref, l_ref = alpha.copy(), lam.copy()
            opts = g.gp_opts_default(tol=1e-10)
            for it in range(2):
                st, stats = g.gp_svb_step(d, Ns, dev(torch_cuda, A), dev(torch_cuda, z1), dev(torch_cuda, z2), Wd,
                                          lam_d, a_gpu, bw, opts=opts)
                assert all(s["status"] == g.GP_OK for s in stats)
                W_ref, a_ref, l_ref = orc.svb_step(grid, w.X, w.Y, A, z1, z2, a_ref, l_ref)
                assert np.linalg.norm(Wd.cpu().numpy() - W_ref) <= 1e-7 * np.linalg.norm(W_ref), it
                assert np.allclose(a_gpu, a_ref, rtol=1e-6), (it, a_gpu, a_ref)
                assert np.allclose(lam_d.cpu().numpy(), l_ref, rtol=1e-6), it
        finally:
            g.gp_data_destroy(d)
    finally:
        torch_cuda.cuda.synchronize()
        g.gp_op_destroy(op)
