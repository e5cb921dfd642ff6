"""Pins of the oracle's AR-coefficient system (Appendix A.2, full conditional
of A; Appendix B, its SVB expectation) against facts that do not re-use its
code: the tensor form of the paper equals the lagged-residual regression; the
whitened residual sum of squares (pinned elsewhere by brute force) is, as a
function of A, the quadratic with that precision and linear term; the
posterior mean under the spatial prior makes the gradient of the log
posterior vanish; and one SVB iteration over W and A lands on the
conditional modes for zero random vectors."""
import numpy as np
import pytest

from oracle import gmrf_oracle as orc
from paper_1606_00980_amd import synth


def workload(P, seed=3):
    w = synth.tiny((6, 5, 4), 6, 3, seed=seed, T=50, P=max(P, 1))
    rng = np.random.default_rng(seed)
    lam = (1.0 / w.sigma2) * rng.uniform(0.5, 2.0, w.N)
    return w, lam, rng


@pytest.mark.parametrize("P", [1, 2, 3])
@pytest.mark.parametrize("Ns", [1, 3])
def test_residual_regression_equals_the_tensor_form(P, Ns):
    w, lam, rng = workload(P)
    Wd = w.W_true[None] + 0.2 * rng.standard_normal((Ns, w.K, w.N))
    J1, b1 = orc.ar_term_mc(w.X, w.Y, Wd, lam, P)
    J2, b2 = orc.ar_term_from_tensors(orc.data_tensors(w.X, w.Y, P), orc.data_tensors_noise(w.Y, P), Wd, lam)
    assert np.abs(J1 - J2).max() <= 1e-9 * np.abs(J1).max()
    assert np.abs(b1 - b2).max() <= 1e-9 * np.abs(b1).max()
    assert np.allclose(J1, J1.transpose(0, 2, 1))
    assert np.all(np.linalg.eigvalsh(J1) > 0)


@pytest.mark.parametrize("P", [1, 3])
def test_ar_term_is_the_quadratic_of_the_residual_sum_of_squares(P):
    """rss_n(a) = c - 2 (b_n/lambda_n)'a + a'(J_n/lambda_n)a, read off by exact
    second differences of the whitened residual sum of squares."""
    w, lam, rng = workload(P, seed=5)
    W = w.W_true + 0.3 * rng.standard_normal((w.K, w.N))
    J, b = orc.ar_term_residuals(w.X, w.Y, W, lam, P)
    rss = lambda a: orc.residual_ss(w.X, w.Y, W, a)
    zero = np.zeros((P, w.N))
    r0 = rss(zero)
    E = [np.zeros((P, w.N)) for _ in range(P)]
    for p in range(P):
        E[p][p] = 1.0
    Jt = np.empty((w.N, P, P))
    bt = np.empty((P, w.N))
    for p in range(P):
        rp, rm = rss(E[p]), rss(-E[p])
        Jt[:, p, p] = 0.5 * (rp + rm - 2 * r0)
        bt[p] = 0.25 * (rm - rp)
        for q in range(p):
            Jt[:, p, q] = Jt[:, q, p] = 0.5 * (rss(E[p] + E[q]) - rp - rss(E[q]) + r0)
    scale = np.abs(J).max()
    assert np.abs(J - lam[:, None, None] * Jt).max() <= 1e-8 * scale
    assert np.abs(b - lam * bt).max() <= 1e-8 * np.abs(b).max()


def test_posterior_mean_of_a_zeroes_the_gradient():
    """With the spatial prior diag(beta) (x) D_w, Q_a^{-1} b_a maximises
    -1/2 sum_n lambda_n rss_n(a_n) - 1/2 sum_p beta_p A_p D_w A_p'."""
    P = 2
    w, lam, rng = workload(P, seed=7)
    g = orc.grid(w.mask, w.conn)
    W = w.W_true + 0.1 * rng.standard_normal((w.K, w.N))
    beta = np.array([3.0, 0.5])
    J, b = orc.ar_term_residuals(w.X, w.Y, W, lam, P)
    a = orc.solve_direct(orc.precision(g, beta, J), b)            # (P, N)
    h = 1e-3
    for p in range(P):
        d = np.zeros_like(a)
        d[p] = h
        # rss_n depends on a_n alone: one central difference per row p gives every voxel
        grad_like = -0.5 * lam * (orc.residual_ss(w.X, w.Y, W, a + d) - orc.residual_ss(w.X, w.Y, W, a - d)) / (2 * h)
        grad_prior = -beta[p] * (g.G @ a[p])
        assert np.abs(grad_like + grad_prior).max() <= 1e-6 * np.abs(grad_prior).max()


def test_svb_step_ar_lands_on_conditional_modes_for_zero_vectors():
    """With zero random vectors the Algorithm-2 samples are the conditional
    means: W makes the gradient of the W log posterior (given the input A)
    vanish, A that of the A log posterior (given the new W); the
    hyperparameter outputs are the Gamma posterior means of those draws."""
    P, K = 2, 3
    w, lam, rng = workload(P, seed=11)
    g = orc.grid(w.mask, w.conn)
    N = w.N
    A0 = w.ar[None, :P] if w.ar.shape[0] >= P else np.zeros((1, P, N))
    A0 = A0 + 0.05 * rng.standard_normal((1, P, N))
    alpha, beta = np.array([0.7, 2.0, 1.3]), np.array([4.0, 1.5])
    z1w, z2w = np.zeros((1, K, 3, N)), np.zeros((1, K, N))
    z1a, z2a = np.zeros((1, P, 3, N)), np.zeros((1, P, N))
    Wn, An, am, bm, lm = orc.svb_step_ar(g, w.X, w.Y, A0, z1w, z2w, z1a, z2a,
                                         alpha, beta, lam)
    h = 1e-3
    for k in range(K):
        d = np.zeros((K, N)); d[k] = h
        gl = -0.5 * lam * (orc.residual_ss(w.X, w.Y, Wn[0] + d, A0[0]) - orc.residual_ss(w.X, w.Y, Wn[0] - d, A0[0])) / (2 * h)
        gp = -alpha[k] * (g.G @ Wn[0, k])
        assert np.abs(gl + gp).max() <= 1e-6 * max(np.abs(gl).max(), 1.0)
    for p in range(P):
        d = np.zeros((P, N)); d[p] = h
        gl = -0.5 * lam * (orc.residual_ss(w.X, w.Y, Wn[0], An[0] + d) - orc.residual_ss(w.X, w.Y, Wn[0], An[0] - d)) / (2 * h)
        gp = -beta[p] * (g.G @ An[0, p])
        assert np.abs(gl + gp).max() <= 1e-6 * max(np.abs(gl).max(), 1.0)
    T = w.X.shape[0]
    qa = np.array([np.sum((g.D @ Wn[0, k]) ** 2) for k in range(K)])
    qb = np.array([np.sum((g.D @ An[0, p]) ** 2) for p in range(P)])
    assert np.allclose(am, (N / 2 + 0.1) / (qa / 2 + 1 / 10.0), rtol=1e-12)
    assert np.allclose(bm, (N / 2 + 0.1) / (qb / 2 + 1 / 10000.0), rtol=1e-12)
    rss = orc.residual_ss(w.X, w.Y, Wn[0], An[0])
    assert np.allclose(lm, ((T - P) / 2 + 0.1) / (rss / 2 + 1 / 10.0), rtol=1e-12)


# ------------------------------------------------- SVB convergence device
def test_alpha_extrapolation_against_a_fitted_parabola():
    """The vertex branch against numpy's least-squares parabola through the
    three points (exact for three points), the linear branch, and the factor-5
    limits."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        a = rng.uniform(0.5, 5.0, 3)
        out = orc.alpha_extrapolate(a[:1], a[1:2], a[2:])[0]
        c2, c1, c0 = np.polyfit([0.0, 1.0, 2.0], a, 2)
        tv = -c1 / (2 * c2) if c2 != 0 else -np.inf
        pred = np.polyval([c2, c1, c0], tv) if tv > 2.0 else a[1] + 20.0 * (a[2] - a[1])
        want = min(max(pred, a[2] / 5), 5 * a[2])
        assert out == pytest.approx(want, rel=1e-9, abs=1e-12)
    # a parabola whose vertex lies ahead: 1 + 1.75 t - 0.25 t^2 through (0, 1), (1, 2.5),
    # (2, 3.5) peaks at t = 3.5 with the value 4.0625
    a = np.array([1.0, 2.5, 3.5])
    assert orc.alpha_extrapolate(a[:1], a[1:2], a[2:])[0] == pytest.approx(4.0625)
    # a straight line: the factor-20 step, limited to 5 a_j
    assert orc.alpha_extrapolate([1.0], [2.0], [3.0])[0] == pytest.approx(15.0)
    assert orc.alpha_extrapolate([3.0], [2.0], [1.0])[0] == pytest.approx(0.2)
