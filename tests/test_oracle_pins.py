"""Pins of the FP64 oracle against things other than itself: hand-derived closed
forms (tests/golden), brute force, exact rational arithmetic, the DCT
diagonalisation of box-grid Laplacians, the Papandreou-Yuille identity behind
Algorithm 2, Algorithm 1 (dense Cholesky), the paper's tensor form of the AR
data term, and statistical tests of samples and Hutchinson estimates."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import gmrf_oracle as orc
from paper_1606_00980_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = [float(t) for t in v.split()]
    return out


def brute_laplacian(mask, conn):
    """Degree/adjacency by explicit loops over grid cells (no sparse algebra)."""
    m = np.asarray(mask).astype(bool)
    nz, ny, nx = m.shape
    order = {}
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if m[z, y, x]:
                    order[(x, y, z)] = len(order)
    N = len(order)
    G = np.zeros((N, N))
    steps = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0)]
    if conn == 6:
        steps += [(0, 0, 1), (0, 0, -1)]
    for (x, y, z), n in order.items():
        for dx, dy, dz in steps:
            q = (x + dx, y + dy, z + dz)
            if q in order:
                G[n, n] += 1
                G[n, order[q]] = -1
    return G


def exact_solve(Q, b):
    """Gauss-Jordan elimination over the rationals."""
    n = len(b)
    A = [[Fraction(Q[i][j]) for j in range(n)] + [Fraction(b[i])] for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        piv = A[c][c]
        A[c] = [v / piv for v in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [a - f * bb for a, bb in zip(A[r], A[c])]
    return [A[i][n] for i in range(n)]


def masks_small():
    rng = np.random.default_rng(5)
    yield synth.ellipsoid_mask((5, 4, 3), (2.5, 2.0, 1.5)), 6
    yield synth.ellipsoid_mask((6, 5, 1), (3.0, 2.5, 1.0)), 4
    yield (rng.random((3, 4, 5)) < 0.6).astype(np.uint8), 6
    yield (rng.random((1, 6, 7)) < 0.6).astype(np.uint8), 4
    yield np.ones((2, 3, 4), dtype=np.uint8), 6


# ------------------------------------------------------------------ Laplacian
@pytest.mark.parametrize("case", range(5))
def test_laplacian_matches_bruteforce(case):
    mask, conn = list(masks_small())[case]
    g = orc.grid(mask, conn)
    G = g.G.toarray()
    assert np.array_equal(G, brute_laplacian(mask, conn))
    assert np.allclose(G, G.T)
    assert np.allclose(G @ np.ones(g.N), 0.0)
    # one incidence row per adjacent pair
    assert g.E == int(-(np.triu(G, 1)).sum())
    D = g.D.toarray()
    assert np.all(D.sum(axis=1) == 0) and np.all(np.abs(D).sum(axis=1) == 2)


def test_paper_facts():
    f = read_golden("paper_facts.txt")
    box3 = np.ones((7, 7, 7), dtype=np.uint8)
    g3 = orc.grid(box3, 6)
    centre = g3.index[3 + 7 * (3 + 7 * 3)]
    assert g3.G[centre, centre] == f["interior_degree_3d"][0]
    box2 = np.ones((1, 7, 7), dtype=np.uint8)
    g2 = orc.grid(box2, 4)
    centre = g2.index[3 + 7 * 3]
    assert g2.G[centre, centre] == f["interior_degree_2d"][0]
    K = 4
    B = np.stack([np.eye(K) * 2.0 + 0.5] * g3.N)
    Q = orc.precision(g3, np.ones(K), B)
    assert np.diff(Q.indptr).max() == K + f["max_row_nnz_3d_extra"][0]
    for key, dims in (("box_10x10x10", (10, 10, 10)), ("box_25x20x20", (25, 20, 20))):
        m = np.ones(dims[::-1], dtype=np.uint8)
        assert orc.grid(m, 6).N == f[key][0]
    assert int(np.prod((50, 50, 40))) == f["box_50x50x40"][0]


# -------------------------------------------------------------- golden cases
def _golden_operator(fx):
    nx, ny, nz = (int(fx[k][0]) for k in ("nx", "ny", "nz"))
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    K = int(fx["K"][0])
    g = orc.grid(mask, int(fx["conn"][0]))
    B = np.array(fx["B"]).reshape(g.N, K, K) if K > 1 else np.array(fx["B"]).reshape(g.N, 1, 1)
    return g, np.array(fx["alpha"]), B, K


@pytest.mark.parametrize("name", ["line3_k1.txt", "pair_k2.txt"])
def test_golden_solve(name):
    fx = read_golden(name)
    g, alpha, B, K = _golden_operator(fx)
    Q = orc.precision(g, alpha, B)
    b = np.array(fx["b"]).reshape(K, g.N)
    want = np.array(fx["x_num"]) / fx["x_den"][0]
    x = orc.solve(Q, b)
    assert np.allclose(x.ravel(), want, rtol=1e-14, atol=1e-15)
    x2, _, rr = orc.solve_pcg(Q, b.ravel(), tol=1e-14)
    assert np.allclose(x2, want, rtol=1e-12)
    # and the rational solve of the oracle's own matrix agrees exactly
    exact = exact_solve(Q.toarray().astype(int).tolist(), [int(v) for v in fx["b"]])
    assert [float(v) for v in exact] == pytest.approx(list(want), rel=1e-15)
    if "trace_num" in fx:
        tr = np.trace(np.linalg.inv(Q.toarray()))
        assert tr == pytest.approx(fx["trace_num"][0] / fx["trace_den"][0], rel=1e-14)


def test_golden_perturbation():
    fx = read_golden("line3_perturb.txt")
    g, alpha, B, K = _golden_operator(fx)
    z1 = np.stack([np.array(fx["z1_x"]), np.array(fx["z1_y"])])[None, None]   # (1,1,2,3)
    z2 = np.array(fx["z2"]).reshape(1, 1, 3)
    b = orc.perturbation_rhs(g, alpha, B, np.zeros((1, 3)), z1, z2)
    assert np.allclose(b.ravel(), fx["b_num"], atol=1e-14)
    w = orc.sample(g, alpha, B, np.zeros((1, 3)), z1, z2)
    assert np.allclose(w.ravel(), np.array(fx["w_num"]) / fx["w_den"][0], rtol=1e-14)


# ------------------------------------------------------------------ data term
@pytest.mark.parametrize("P", [1, 3])
def test_data_term_whitening_equals_tensor_route(P):
    w = synth.tiny((6, 5, 4), 6, 4, seed=P, T=50, P=P)
    B1, b1 = orc.data_term_whitening(w.X, w.Y, w.ar, w.sigma2)
    B2, b2 = orc.data_term_from_tensors(orc.data_tensors(w.X, w.Y, P), w.ar[None], 1.0 / w.sigma2)
    assert np.allclose(B1, B2, rtol=1e-12, atol=1e-12 * np.abs(B1).max())
    assert np.allclose(b1, b2, rtol=1e-12, atol=1e-12 * np.abs(b1).max())
    # the generator's data term is the same quantity
    assert np.allclose(w.B, B1, rtol=1e-11, atol=1e-11 * np.abs(B1).max())
    assert np.allclose(w.bw, b1, rtol=1e-11, atol=1e-11 * np.abs(b1).max())


def test_data_tensors_by_brute_force():
    """Each tensor entry as a plain double loop over scans (t, p, q)."""
    w = synth.tiny((4, 3, 2), 6, 3, seed=5, T=30, P=2)
    P, (T, K) = 2, w.X.shape
    XX, R, S, YX, Bt, Dt = orc.data_tensors(w.X, w.Y, P)
    X, Y = w.X, w.Y
    for k in range(K):
        for j in range(K):
            assert np.isclose(XX[k, j], sum(X[t, k] * X[t, j] for t in range(P, T)))
            for p in range(P):
                assert np.isclose(R[k, j, p], sum(X[t, k] * X[t - p - 1, j] for t in range(P, T)))
                for q in range(P):
                    assert np.isclose(S[p, k, j, q], sum(X[t - p - 1, k] * X[t - q - 1, j] for t in range(P, T)))
    for n in (0, w.N - 1):
        for k in range(K):
            assert np.isclose(YX[n, k], sum(Y[t, n] * X[t, k] for t in range(P, T)))
            for p in range(P):
                assert np.isclose(Bt[n, p, k], sum(Y[t, n] * X[t - p - 1, k] + Y[t - p - 1, n] * X[t, k]
                                                   for t in range(P, T)))
                for q in range(P):
                    assert np.isclose(Dt[n, p, k, q], sum(Y[t - p - 1, n] * X[t - q - 1, k] for t in range(P, T)))


def test_data_term_mc_average():
    """The SVB expectation over draws is the mean of the full-conditional data
    terms: equal draws give the single-draw term, and it is linear in lambda;
    the tensor route gives the same average."""
    w = synth.tiny((5, 4, 3), 6, 3, seed=8, T=40, P=3)
    lam = 1.0 / w.sigma2
    A = np.stack([w.ar, w.ar, w.ar])
    B1, b1 = orc.data_term_mc(w.X, w.Y, A, lam)
    B0, b0 = orc.data_term_whitening(w.X, w.Y, w.ar, w.sigma2)
    assert np.allclose(B1, B0, rtol=1e-13) and np.allclose(b1, b0, rtol=1e-13)
    rng = np.random.default_rng(3)
    A = w.ar[None] + 0.1 * rng.standard_normal((4,) + w.ar.shape)
    B2, b2 = orc.data_term_mc(w.X, w.Y, A, 2.0 * lam)
    B3, b3 = orc.data_term_mc(w.X, w.Y, A, lam)
    assert np.allclose(B2, 2 * B3, rtol=1e-13) and np.allclose(b2, 2 * b3, rtol=1e-13)
    B4, b4 = orc.data_term_from_tensors(orc.data_tensors(w.X, w.Y, 3), A, lam)
    assert np.allclose(B4, B3, rtol=1e-11, atol=1e-11 * np.abs(B3).max())
    assert np.allclose(b4, b3, rtol=1e-11, atol=1e-11 * np.abs(b3).max())


# ----------------------------------------------------- hyperparameter statistics
def test_quadform_brute_force_over_grid_cells():
    """W_k D_w W_k' as a loop over in-mask cells and their +x, +y, +z
    neighbours in the mask (one term per adjacent pair)."""
    for dims, conn in (((6, 5, 4), 6), ((7, 6, 1), 4)):
        w = synth.tiny(dims, conn, 3, seed=11)
        g = orc.grid(w.mask, conn)
        W = np.random.default_rng(0).standard_normal((2, 3, w.N))
        mask = w.mask.astype(bool)
        idx = -np.ones(mask.shape, int)
        idx[mask] = np.arange(w.N)
        nz, ny, nx = mask.shape
        ref = np.zeros((2, 3))
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    if not mask[z, y, x]:
                        continue
                    for dz, dy, dx in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
                        z2, y2, x2 = z + dz, y + dy, x + dx
                        if z2 < nz and y2 < ny and x2 < nx and mask[z2, y2, x2]:
                            ref += (W[:, :, idx[z, y, x]] - W[:, :, idx[z2, y2, x2]]) ** 2
        assert np.allclose(orc.quadform(g, W), ref, rtol=1e-13)


@pytest.mark.parametrize("P", [1, 3])
def test_residual_ss_identities(P):
    """rss_n = yw'yw - 2 (b_n/lambda)'w + w'(B_n/lambda) w with the whitening data
    term; the tensor form of the lambda full conditional gives the same; and a
    noise-free Y = XW gives zero."""
    w = synth.tiny((5, 4, 3), 6, 4, seed=20 + P, T=45, P=P)
    Wt = np.random.default_rng(P).standard_normal((w.K, w.N)) + w.W_true
    rss = orc.residual_ss(w.X, w.Y, Wt, w.ar)
    B, bw = orc.data_term_whitening(w.X, w.Y, w.ar, np.ones(w.N))
    T = w.X.shape[0]
    for n in range(0, w.N, 7):
        A = np.zeros((T - P, T))
        for i, t in enumerate(range(P, T)):
            A[i, t] = 1.0
            for p in range(1, P + 1):
                A[i, t - p] = -w.ar[p - 1, n]
        yw = A @ w.Y[:, n]
        ref = yw @ yw - 2 * bw[:, n] @ Wt[:, n] + Wt[:, n] @ B[n] @ Wt[:, n]
        assert np.isclose(rss[n], ref, rtol=1e-10)
    tens = orc.data_tensors(w.X, w.Y, P)
    extra = orc.data_tensors_noise(w.Y, P)
    assert np.allclose(orc.residual_ss_from_tensors(tens, extra, Wt, w.ar), rss, rtol=1e-9,
                       atol=1e-9 * np.abs(rss).max())
    assert np.allclose(orc.residual_ss(w.X, w.X @ Wt, Wt, w.ar), 0.0, atol=1e-12)


def test_gamma_posteriors_by_numerical_integration():
    """Mean of the unnormalised full conditional, integrated on a fine grid:
    p(alpha | W) ~ alpha^(q2-1) e^(-alpha/q1) * alpha^(N/2) e^(-alpha qf/2);
    p(lambda | .) ~ lambda^(u2-1) e^(-lambda/u1) * lambda^((T-P)/2) e^(-lambda rss/2).
    Ga(scale, shape) has mean scale * shape."""
    for qf, N, c1, c2 in ((37.5, 120, 10.0, 0.1), (2.0, 9, 10.0, 0.1), (400.0, 1000, 3.0, 2.0)):
        s1, s2 = orc.alpha_posterior(np.array([qf]), N, c1, c2)
        x = np.linspace(1e-9, 60 * s1[0] * s2, 400001)
        logp = (c2 - 1 + N / 2.0) * np.log(x) - x / c1 - x * qf / 2.0
        wgt = np.exp(logp - logp.max())
        assert np.isclose((x * wgt).sum() / wgt.sum(), s1[0] * s2, rtol=1e-6)
    for rss, T, P in ((55.0, 200, 3), (3.0, 30, 1)):
        s1, s2 = orc.lambda_posterior(np.array([rss]), T, P, 10.0, 0.1)
        x = np.linspace(1e-9, 60 * s1[0] * s2, 400001)
        logp = (0.1 - 1 + (T - P) / 2.0) * np.log(x) - x / 10.0 - x * rss / 2.0
        wgt = np.exp(logp - logp.max())
        assert np.isclose((x * wgt).sum() / wgt.sum(), s1[0] * s2, rtol=1e-6)


def test_svb_step_against_dense_recomputation():
    """One SVB step on a tiny grid, recomputed densely and independently: the
    precision assembled entry by entry from (alpha, B, D_w), the perturbed
    right-hand side from an explicit incidence matrix and Cholesky factors,
    dense solves, and the statistics by plain loops."""
    w = synth.tiny((4, 3, 2), 6, 2, seed=13, T=30, P=1)
    g = orc.grid(w.mask, 6)
    N, K, T, P = w.N, w.K, w.X.shape[0], 1
    rng = np.random.default_rng(4)
    Ns = 2
    A = w.ar[None] + 0.05 * rng.standard_normal((Ns, P, N))
    lam = 1.0 / w.sigma2
    alpha = np.array([0.7, 2.5])
    z1 = rng.standard_normal((Ns, K, 3, N))
    z2 = rng.standard_normal((Ns, K, N))
    W, a_mean, l_mean = orc.svb_step(g, w.X, w.Y, A, z1, z2, alpha, lam)
    # dense recomputation
    mask = w.mask.astype(bool)
    idx = -np.ones(mask.shape, int); idx[mask] = np.arange(N)
    nz, ny, nx = mask.shape
    edges = []      # (n, m, slot d) for m = n + e_d in the mask
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if mask[z, y, x]:
                    for d, (dz, dy, dx) in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
                        z2_, y2, x2 = z + dz, y + dy, x + dx
                        if z2_ < nz and y2 < ny and x2 < nx and mask[z2_, y2, x2]:
                            edges.append((idx[z, y, x], idx[z2_, y2, x2], d))
    Dm = np.zeros((len(edges), N))
    for e, (n, m, _) in enumerate(edges):
        Dm[e, n], Dm[e, m] = 1.0, -1.0
    Lap = Dm.T @ Dm
    Bd = np.zeros((N, K, K)); bd = np.zeros((K, N))
    for j in range(Ns):
        for n in range(N):
            Aw = np.zeros((T - P, T))
            for i, t in enumerate(range(P, T)):
                Aw[i, t], Aw[i, t - 1] = 1.0, -A[j, 0, n]
            Xw, yw = Aw @ w.X, Aw @ w.Y[:, n]
            Bd[n] += lam[n] * Xw.T @ Xw / Ns
            bd[:, n] += lam[n] * Xw.T @ yw / Ns
    Qd = np.zeros((K * N, K * N))
    for k in range(K):
        Qd[k * N:(k + 1) * N, k * N:(k + 1) * N] += alpha[k] * Lap
        for l in range(K):
            Qd[k * N + np.arange(N), l * N + np.arange(N)] += Bd[:, k, l]
    Wd = np.empty((Ns, K, N))
    for j in range(Ns):
        rhs = bd.copy()
        for k in range(K):
            ze = np.array([z1[j, k, dd, n] for (n, m, dd) in edges])
            rhs[k] += np.sqrt(alpha[k]) * Dm.T @ ze
        for n in range(N):
            rhs[:, n] += np.linalg.cholesky(Bd[n]) @ z2[j, :, n]
        Wd[j] = np.linalg.solve(Qd, rhs.ravel()).reshape(K, N)
    assert np.allclose(W, Wd, rtol=1e-9, atol=1e-9 * np.abs(Wd).max())
    qf = np.array([[Wd[j, k] @ Lap @ Wd[j, k] for k in range(K)] for j in range(Ns)]).mean(axis=0)
    assert np.allclose(a_mean, (N / 2 + 0.1) / (qf / 2 + 1 / 10.0), rtol=1e-9)
    rss = np.zeros(N)
    for j in range(Ns):
        e = w.Y - w.X @ Wd[j]
        for n in range(N):
            r = e[1:, n] - A[j, 0, n] * e[:-1, n]
            rss[n] += r @ r / Ns
    assert np.allclose(l_mean, ((T - P) / 2 + 0.1) / (rss / 2 + 1 / 10.0), rtol=1e-8)


def test_slice_workload_data_term():
    w = synth.slice_2d()
    idx = np.random.default_rng(1).choice(w.N, 40, replace=False)
    B1, b1 = orc.data_term_whitening(w.X, w.Y[:, idx], w.ar[:, idx], w.sigma2[idx])
    assert np.allclose(w.B[idx], B1, rtol=1e-11)
    assert np.allclose(w.bw[:, idx], b1, rtol=1e-11)


# ------------------------------------------------------------------- operator
def test_alpha_zero_is_per_voxel_solve():
    w = synth.tiny((7, 6, 5), 6, 3, seed=2)
    g = orc.grid(w.mask, 6)
    Q = orc.precision(g, np.zeros(w.K), w.B)
    x = orc.solve(Q, w.bw)
    want = np.stack([np.linalg.solve(w.B[n], w.bw[:, n]) for n in range(w.N)], axis=1)
    assert np.allclose(x, want, rtol=1e-11)


def test_precision_spd_and_symmetric():
    w = synth.tiny((6, 6, 4), 6, 3, seed=3)
    g = orc.grid(w.mask, 6)
    Q = orc.precision(g, w.alpha, w.B).toarray()
    assert np.allclose(Q, Q.T)
    np.linalg.cholesky(Q)


def dct_solve(dims_xyz, alpha, beta, b):
    """Closed form on a full box with B_n = beta*I: the path-graph Laplacian with
    free ends is diagonalised by the orthonormal DCT-II, eigenvalues
    2 - 2 cos(pi j / n) per axis (a textbook fact)."""
    nx, ny, nz = dims_xyz
    lam = (2 - 2 * np.cos(np.pi * np.arange(nz) / nz))[:, None, None] \
        + (2 - 2 * np.cos(np.pi * np.arange(ny) / ny))[None, :, None] \
        + (2 - 2 * np.cos(np.pi * np.arange(nx) / nx))[None, None, :]
    K = len(alpha)
    x = np.empty_like(b)
    for k in range(K):
        c = sfft.dctn(b[k].reshape(nz, ny, nx), type=2, norm="ortho")
        x[k] = sfft.idctn(c / (alpha[k] * lam + beta), type=2, norm="ortho").ravel()
    tr = sum(float(np.sum(1.0 / (alpha[k] * lam + beta))) for k in range(K))
    trG = np.array([float(np.sum(lam / (alpha[k] * lam + beta))) for k in range(K)])
    trk = np.array([float(np.sum(1.0 / (alpha[k] * lam + beta))) for k in range(K)])
    return x, tr, trk, trG


@pytest.mark.parametrize("dims,conn", [((9, 7, 5), 6), ((16, 12, 1), 4)])
def test_dct_closed_form_small(dims, conn):
    nx, ny, nz = dims
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    g = orc.grid(mask, conn)
    alpha = np.array([0.7, 2.5, 4.0])
    beta = 1.3
    B = np.stack([np.eye(3) * beta] * g.N)
    b = np.random.default_rng(0).standard_normal((3, g.N))
    Q = orc.precision(g, alpha, B)
    want, tr, trk, trG = dct_solve(dims, alpha, beta, b)
    assert np.allclose(orc.solve(Q, b), want, rtol=1e-10, atol=1e-12)
    x2, _, rr = orc.solve_pcg(Q, b.ravel(), tol=1e-13)
    assert np.allclose(x2.reshape(3, -1), want, rtol=1e-9, atol=1e-11)
    Qi = np.linalg.inv(Q.toarray())
    assert np.trace(Qi) == pytest.approx(tr, rel=1e-11)
    N = g.N
    G = g.G.toarray()
    for k in range(3):
        blk = Qi[k * N:(k + 1) * N, k * N:(k + 1) * N]
        assert np.trace(blk) == pytest.approx(trk[k], rel=1e-11)
        assert np.trace(G @ blk) == pytest.approx(trG[k], rel=1e-11)


@pytest.mark.slow
def test_dct_closed_form_large():
    """A 64x64x33 box (135,168 voxels), K = 2: the oracle's iterative path."""
    dims = (64, 64, 33)
    mask = np.ones(dims[::-1], dtype=np.uint8)
    g = orc.grid(mask, 6)
    alpha = np.array([0.5, 3.0])
    beta = 2.0
    B = np.broadcast_to(np.eye(2) * beta, (g.N, 2, 2)).copy()
    b = np.random.default_rng(1).standard_normal((2, g.N))
    Q = orc.precision(g, alpha, B)
    want, *_ = dct_solve(dims, alpha, beta, b)
    x = orc.solve(Q, b, tol=1e-13)
    assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-11


# ------------------------------------------------------------ Algorithm 1
@pytest.mark.parametrize("dims,conn,K", [((4, 4, 1), 4, 2), ((4, 3, 3), 6, 3)])
def test_solve_matches_cholesky_algorithm1(dims, conn, K):
    w = synth.tiny(dims, conn, K, seed=4, shape="box")
    g = orc.grid(w.mask, conn)
    Q = orc.precision(g, w.alpha, w.B)
    z = np.random.default_rng(3).standard_normal((K, g.N))
    mu, wsamp = orc.cholesky_mean_and_sample(Q, w.bw, z)
    assert np.allclose(orc.solve(Q, w.bw), mu, rtol=1e-11)
    x, _, _ = orc.solve_pcg(Q, w.bw.ravel(), tol=1e-14)
    assert np.allclose(x.reshape(K, -1), mu, rtol=1e-10)
    # Algorithm 1 sample: L' v = z  =>  Q v = L z
    L = np.linalg.cholesky(Q.toarray())
    v = (wsamp - mu).ravel()
    assert np.allclose(Q.toarray() @ v, L @ z.ravel(), atol=1e-10)


# --------------------------------------------------------------- Algorithm 2
@pytest.mark.parametrize("dims,conn,K", [((4, 3, 1), 4, 2), ((3, 3, 3), 6, 2), ((4, 4, 2), 6, 3)])
def test_perturbation_identity(dims, conn, K):
    """S S' = Q with S = [(blkdiag sqrt(alpha_k) G_w)' | H'L_data H]."""
    w = synth.tiny(dims, conn, K, seed=5)
    g = orc.grid(w.mask, conn)
    Q = orc.precision(g, w.alpha, w.B).toarray()
    S = orc.perturbation_factor(g, w.alpha, w.B)
    assert np.allclose(S @ S.T, Q, rtol=1e-12, atol=1e-12 * np.abs(Q).max())
    # perturbation_rhs applies S to z (edges mapped from the padded slots)
    rng = np.random.default_rng(9)
    z1, z2 = rng.standard_normal((1, K, g.ndirs, g.N)), rng.standard_normal((1, K, g.N))
    slots = orc.edge_slots(g)
    zE = np.concatenate([z1[0, k].ravel()[slots] for k in range(K)])
    b = orc.perturbation_rhs(g, w.alpha, w.B, w.bw, z1, z2)
    assert np.allclose(b[0].ravel(), w.bw.ravel() + S @ np.r_[zE, z2[0].ravel()], atol=1e-10)
    # unused slots do not matter
    used = np.zeros(g.ndirs * g.N, bool); used[slots] = True
    z1b = z1.copy()
    z1b[0].reshape(K, -1)[:, ~used] = 123.0
    assert np.array_equal(orc.perturbation_rhs(g, w.alpha, w.B, w.bw, z1b, z2), b)
    # z = 0 gives the mean
    zero = orc.perturbation_rhs(g, w.alpha, w.B, w.bw, 0 * z1, 0 * z2)
    assert np.array_equal(zero[0], w.bw)


def test_sample_covariance_converges_to_inverse_precision():
    w = synth.tiny((3, 3, 1), 4, 2, seed=6)
    g = orc.grid(w.mask, 4)
    Q = orc.precision(g, w.alpha, w.B)
    Sigma = np.linalg.inv(Q.toarray())
    M = 20000
    rng = np.random.default_rng(11)
    z1 = rng.standard_normal((M, w.K, g.ndirs, g.N))
    z2 = rng.standard_normal((M, w.K, g.N))
    bw = np.zeros_like(w.bw)
    b = orc.perturbation_rhs(g, w.alpha, w.B, bw, z1, z2).reshape(M, -1)
    xs = np.linalg.solve(Q.toarray(), b.T).T
    C = xs.T @ xs / M
    sd = np.sqrt((np.outer(np.diag(Sigma), np.diag(Sigma)) + Sigma ** 2) / M)
    assert np.all(np.abs(C - Sigma) <= 4.5 * sd)
    assert np.abs(xs.mean(axis=0)).max() < 4.5 * np.sqrt(np.diag(Sigma).max() / M)


# ------------------------------------------------------------------ Hutchinson
def rademacher_var(A):
    As = 0.5 * (A + A.T)
    return 2.0 * (np.sum(As ** 2) - np.sum(np.diag(As) ** 2))


def test_hutchinson_unbiased_with_exact_variance():
    w = synth.tiny((3, 3, 2), 6, 2, seed=7)
    g = orc.grid(w.mask, 6)
    Q = orc.precision(g, w.alpha, w.B)
    Qi = np.linalg.inv(Q.toarray())
    N, K = g.N, w.K
    m = 4000
    v = (2 * np.random.default_rng(12).integers(0, 2, size=(m, K, N)) - 1).astype(np.int8)
    t, tk, gk, _ = orc.hutchinson(g, Q, v)
    assert abs(t - np.trace(Qi)) <= 4 * np.sqrt(rademacher_var(Qi) / m)
    G = g.G.toarray()
    for k in range(K):
        Pk = np.zeros((N, K * N)); Pk[:, k * N:(k + 1) * N] = np.eye(N)
        Ak = Pk.T @ Pk @ Qi                   # v' A v = v_k' [Q^{-1} v]_k
        assert abs(tk[k] - np.trace(Ak)) <= 4 * np.sqrt(rademacher_var(Ak) / m)
        Bk = Pk.T @ G @ Pk @ Qi               # v' B v = (G v_k)' [Q^{-1} v]_k
        assert abs(gk[k] - np.trace(Bk)) <= 4 * np.sqrt(rademacher_var(Bk) / m) + 1e-12


def test_hutchinson_deterministic_form():
    """With given probes the estimate is a fixed linear-algebra quantity."""
    w = synth.tiny((4, 3, 1), 4, 2, seed=8)
    g = orc.grid(w.mask, 4)
    Q = orc.precision(g, w.alpha, w.B)
    Qi = np.linalg.inv(Q.toarray())
    v = w.probes(5).astype(np.float64)
    t, tk, gk, u = orc.hutchinson(g, Q, v)
    V = v.reshape(5, -1)
    assert t == pytest.approx(np.einsum("ij,jk,ik->", V, Qi, V) / 5, rel=1e-12)


# ------------------------------------------------------- planted mistakes
def _mutants():
    """Plausible mistakes in the precision assembly, each must be caught."""
    def swapped_kron(g, alpha, B):            # voxel-major instead of k-major prior
        import scipy.sparse as sp
        return (sp.kron(g.G, sp.diags(alpha)) + orc.blocks_kmajor(B)).tocsr()

    def dropped_prior(g, alpha, B):
        return orc.blocks_kmajor(B)

    def wrong_sign(g, alpha, B):
        import scipy.sparse as sp
        Gbad = sp.diags(g.G.diagonal()) - (g.G - sp.diags(g.G.diagonal()))
        return (sp.kron(sp.diags(alpha), Gbad) + orc.blocks_kmajor(B)).tocsr()

    def transposed_blocks(g, alpha, B):       # B applied voxel-major
        import scipy.sparse as sp
        return (sp.kron(sp.diags(alpha), g.G) + sp.block_diag(list(B))).tocsr()

    return [swapped_kron, dropped_prior, wrong_sign, transposed_blocks]


@pytest.mark.parametrize("mutant", _mutants(), ids=lambda f: f.__name__)
def test_pins_catch_planted_mistakes(mutant):
    dims = (5, 4, 3)
    g = orc.grid(np.ones(dims[::-1], dtype=np.uint8), 6)
    alpha = np.array([0.7, 2.5])
    beta = 1.3
    B = np.stack([np.array([[beta, 0.0], [0.0, beta]])] * g.N)
    b = np.random.default_rng(0).standard_normal((2, g.N))
    want, *_ = dct_solve(dims, alpha, beta, b)
    caught = not np.allclose(orc.solve(mutant(g, alpha, B), b), want, rtol=1e-8)
    if not caught:                         # the DCT case cannot see B layout; the golden K=2 case can
        fx = read_golden("pair_k2.txt")
        g2, a2, B2, K2 = _golden_operator(fx)
        x = orc.solve(mutant(g2, a2, B2), np.array(fx["b"]).reshape(K2, g2.N))
        caught = not np.allclose(x.ravel(), np.array(fx["x_num"]) / fx["x_den"][0])
    assert caught
