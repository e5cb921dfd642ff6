"""Plain FP64 CPU oracle for the posterior-precision solves of the spatial GLM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; it reads only the raw
synthetic inputs (mask, design, AR coefficients, variances, data, alpha, random
vectors).

It computes, slowly and directly, what the paper (Siden, Eklund, Bolin, Villani,
"Fast Bayesian whole-brain fMRI analysis with spatial 3D priors") defines:

* the masked-grid incidence matrix G_w (here ``D``) with one row per adjacent
  voxel pair, and the unweighted graph Laplacian D_w = G_w'G_w (here ``G``)
  -- Section 2 (prior on W_k) and Section 3.1 (the G_w construction);
* the per-voxel data term B_n, b_n of the AR(P) likelihood by explicit
  whitening -- Appendix A.2 (temporal likelihood, full conditional of W);
* the time-summed data tensors of Appendix A.2 (Y_n'X, X'X, R = X'X~,
  S = X~X~, B~_n = Y_n'X~ + d_n X, D_n = d_n X~) and the data term assembled
  from them, and its SVB expectation over Monte Carlo draws of the AR
  coefficients -- Appendix A.2 (full conditional of W) and Appendix B
  (expectations b_w^SVB, B~^SVB);
* the precision of w_r = vec(W') (k-major), Q = diag(alpha) (x) D_w + H'blkdiag(B_n)H
  -- Section 3, full conditional of w_r, and Appendix A.2;
* mean solves x = Q^{-1} b -- Section 3.1 (PCG paragraph, relative residual
  criterion);
* perturbation samples w = Q^{-1}(b_w + (blkdiag_k sqrt(alpha_k) G_w)' z1
  + H'L_data H z2) -- Algorithm 2;
* Cholesky-based mean and sample -- Algorithm 1 (dense, tiny grids only);
* the hyperparameter statistics and conjugate Gamma posteriors: the spatial
  quadratic forms W_k D_w W_k' and 1/q~1k = W_k D_w W_k'/2 + 1/q1,
  q~2 = N/2 + q2 (Section 3.2 full conditionals, Section 3.3 / Appendix B SVB
  with the Monte Carlo mean over samples), and the whitened residual sum of
  squares with 1/u~1n = rss_n/2 + 1/u1, u~2 = (T-P)/2 + u2 (Appendix A.2,
  full conditional of lambda), Ga(scale, shape) with mean scale * shape;
* the incomplete Cholesky preconditioner M of Algorithm 2 (steps 6-7) as a
  block IC(0) factor (K x K voxel blocks, zero fill outside Q's block
  pattern) under a given voxel order, here the red-black two-colour order,
  and PCG with it (Section 3.1);
* the full conditional of the AR coefficients A (Appendix A.2): its data
  part from the lagged residuals of Y - XW (an AR(P) regression per voxel)
  and in the tensor form, its Monte Carlo SVB expectation over draws of W, the
  operator with K = P, prior precisions beta and D_a = D_w, and one SVB
  iteration over W, A and the hyperparameters (Section 3.3, Appendix B);
* one Gibbs iteration of Section 3.2 (W, alpha, lambda) with the Gamma
  draws of the Philox twin;
* Hutchinson estimates with Rademacher probes of tr(Q^{-1}), of tr([Q^{-1}]_kk)
  and of tr(D_w [Q^{-1}]_kk), the trace inside E[W_k D_w W_k'] of Section 3.3
  (quadratic-form expectation).

Readings where the paper is silent (all repeated in the design notes):
voxel order is x-fastest raster over in-mask voxels; the stencil has a free
boundary (the diagonal of D_w is the in-mask degree); edge (n, n+e_d) is
oriented +1 at n and -1 at n+e_d; z1 carries one N(0,1) entry per regressor
and edge (K*E in total); the relative residual uses the Euclidean norm over all
K*N entries of one right-hand side.

Parity status: every function here is pinned by a test that does not re-use it
(closed forms, brute force, exact rational arithmetic, identities, statistics);
none is "parity unpinned".
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

__all__ = [
    "Grid", "grid", "data_term_whitening", "data_term_mc", "data_tensors", "data_term_from_tensors",
    "data_tensors_noise", "quadform", "residual_ss", "residual_ss_from_tensors", "alpha_posterior",
    "lambda_posterior", "svb_step", "ar_term_residuals", "ar_term_mc", "ar_term_from_tensors", "svb_step_ar",
    "alpha_extrapolate", "gibbs_step",
    "precision", "apply", "relres",
    "solve", "solve_direct", "solve_pcg", "perturbation_rhs", "perturbation_factor",
    "sample", "hutchinson", "cholesky_mean_and_sample",
    "redblack_order", "ic0_block", "ic0_redblack", "ic0_solve", "redblack_start", "solve_pcg_ic0",
]


# ------------------------------------------------------------------ grid / prior
class Grid:
    """Mask bookkeeping plus the incidence matrix D and Laplacian G = D'D."""

    def __init__(self, mask: np.ndarray, conn: int):
        if conn not in (4, 6):
            raise ValueError("conn must be 4 or 6")
        m = np.asarray(mask).astype(bool)
        if m.ndim == 2:
            m = m[None]
        self.mask = m
        self.conn = conn
        nz, ny, nx = m.shape
        self.nx, self.ny, self.nz = nx, ny, nz
        flat = m.ravel()
        self.lin = np.flatnonzero(flat)                  # compact n -> linear l
        self.N = int(self.lin.size)
        self.index = -np.ones(flat.size, dtype=np.int64)  # linear l -> compact n
        self.index[self.lin] = np.arange(self.N)
        x = self.lin % nx
        y = (self.lin // nx) % ny
        z = self.lin // (nx * ny)
        self.coords = np.stack([x, y, z], axis=1)
        dirs = [(1, 0, 0), (0, 1, 0)] + ([(0, 0, 1)] if conn == 6 else [])
        self.ndirs = len(dirs)
        # Edge list: for each direction d and voxel n with n+e_d inside the mask,
        # one edge (n, n+e_d).  Edges are ordered direction-major, then by n.
        self.edge_dir, self.edge_lo, self.edge_hi = [], [], []
        for d, (dx, dy, dz) in enumerate(dirs):
            xx, yy, zz = x + dx, y + dy, z + dz
            ok = (xx < nx) & (yy < ny) & (zz < nz)
            far = np.full(self.N, -1, dtype=np.int64)
            far[ok] = self.index[xx[ok] + nx * (yy[ok] + ny * zz[ok])]
            keep = far >= 0
            self.edge_dir.append(np.full(int(keep.sum()), d))
            self.edge_lo.append(np.flatnonzero(keep))
            self.edge_hi.append(far[keep])
        self.edge_dir = np.concatenate(self.edge_dir)
        self.edge_lo = np.concatenate(self.edge_lo)
        self.edge_hi = np.concatenate(self.edge_hi)
        self.E = int(self.edge_lo.size)
        e = np.arange(self.E)
        # G_w: one row per adjacent pair, +1 at the first voxel, -1 at the second
        # (Section 3.1, increments of adjacent voxels are iid normal).
        self.D = sp.csr_matrix(
            (np.r_[np.ones(self.E), -np.ones(self.E)],
             (np.r_[e, e], np.r_[self.edge_lo, self.edge_hi])),
            shape=(self.E, self.N))
        # D_w = G_w'G_w: in-mask degree on the diagonal, -1 for adjacent pairs
        # (Section 2, unweighted graph Laplacian).
        self.G = (self.D.T @ self.D).tocsr()


def grid(mask, conn) -> Grid:
    return Grid(mask, conn)


# --------------------------------------------------------------------- data term
def data_term_whitening(X: np.ndarray, Y: np.ndarray, ar: np.ndarray, sigma2: np.ndarray):
    """B_n and b_n of the AR(P) likelihood, conditional on the first P scans.

    Appendix A.2: the residual at scan t is (y_t - x_t W) minus the AR
    prediction from the P previous residuals, with noise precision
    lambda_n = 1/sigma2_n.  Written out: the whitening matrix A_n ((T-P) x T)
    has rows [-a_P .. -a_1, 1]; Xw = A_n X, yw = A_n y_n; B_n = lambda_n Xw'Xw
    and b_n = lambda_n Xw'yw.  Returns B (N, K, K) and b_w (K, N), the latter in
    the k-major layout of w_r = vec(W').
    """
    T, K = X.shape
    P, N = ar.shape
    B = np.empty((N, K, K))
    bw = np.empty((K, N))
    for n in range(N):
        A = np.zeros((T - P, T))
        for i, t in enumerate(range(P, T)):
            A[i, t] = 1.0
            for p in range(1, P + 1):
                A[i, t - p] = -ar[p - 1, n]
        Xw = A @ X
        yw = A @ Y[:, n]
        lam = 1.0 / sigma2[n]
        B[n] = lam * (Xw.T @ Xw)
        bw[:, n] = lam * (Xw.T @ yw)
    return B, bw


def data_term_mc(X: np.ndarray, Y: np.ndarray, A: np.ndarray, lam: np.ndarray):
    """Average of the whitening data term over Monte Carlo draws of the AR
    coefficients with the noise precision held at lam -- the SVB expectations
    b_w^SVB and the data part of B~^SVB of Appendix B, which are the plain
    mean of the full-conditional quantities over the draws A[j] (P, N) because
    lambda enters linearly.  A has shape (Ns, P, N)."""
    Ns = A.shape[0]
    B = 0.0
    bw = 0.0
    for j in range(Ns):
        Bj, bj = data_term_whitening(X, Y, A[j], 1.0 / lam)
        B = B + Bj
        bw = bw + bj
    return B / Ns, bw / Ns


def data_tensors(X: np.ndarray, Y: np.ndarray, P: int):
    """The time-summed data of Appendix A.2, conditional on the first P scans.

    With the lagged design X~[t] (P x K, row p = X[t-p]) and lagged data
    d_t (P, entry p = y[t-p]) over scans t = P..T-1 (0-based), and X, y at
    those scans:
      XX = X'X (K x K); R = X'X~ (K x K x P); S = X~X~ (P x K x K x P);
      YX[n] = Y_n'X (K); Bt[n] = Y_n'X~ + d_n X (P x K); Dt[n] = d_n X~ (P x K x P).
    Returns (XX, R, S, YX (N, K), Bt (N, P, K), Dt (N, P, K, P)).
    """
    T, K = X.shape
    N = Y.shape[1]
    ts = np.arange(P, T)
    Xt = np.stack([X[ts - p] for p in range(1, P + 1)], axis=1)          # (T-P, P, K)
    Xc = X[ts]                                                             # (T-P, K)
    XX = Xc.T @ Xc
    R = np.einsum("tk,tpj->kjp", Xc, Xt)
    S = np.einsum("tpk,tqj->pkjq", Xt, Xt)
    YX = np.empty((N, K)); Bt = np.empty((N, P, K)); Dt = np.empty((N, P, K, P))
    for n in range(N):
        y = Y[ts, n]
        d = np.stack([Y[ts - p, n] for p in range(1, P + 1)], axis=1)     # (T-P, P)
        YX[n] = y @ Xc
        Bt[n] = np.einsum("t,tpk->pk", y, Xt) + d.T @ Xc
        Dt[n] = np.einsum("tp,tqk->pkq", d, Xt)
    return XX, R, S, YX, Bt, Dt


def data_tensors_noise(Y: np.ndarray, P: int):
    """Per-voxel data tensors of the lambda full conditional (Appendix A.2),
    over scans t = P..T-1: YY_n = y'y, dY_n[p] = sum_t y[t-1-p] y[t],
    dd_n[p][q] = sum_t y[t-1-p] y[t-1-q].  Returns (YY (N), dY (N, P), dd (N, P, P))."""
    T, N = Y.shape
    ts = np.arange(P, T)
    YY = np.einsum("tn,tn->n", Y[ts], Y[ts])
    d = np.stack([Y[ts - p] for p in range(1, P + 1)], axis=1) if P > 0 else np.zeros((len(ts), 0, N))
    dY = np.einsum("tpn,tn->np", d, Y[ts])
    dd = np.einsum("tpn,tqn->npq", d, d)
    return YY, dY, dd


def data_term_from_tensors(tensors, A: np.ndarray, lam: np.ndarray):
    """Appendix A.2 (and its Appendix B expectation over draws A (Ns, P, N)):
    B_n = lambda_n (X'X - mean_j [R A_n + (R A_n)' - A_n' S A_n]),
    b_n = lambda_n (Y_n'X - mean_j [A_n' B~_n - A_n' D_n A_n])."""
    XX, R, S, YX, Bt, Dt = tensors
    N, K = YX.shape
    Ns = A.shape[0]
    B = np.empty((N, K, K)); bw = np.empty((K, N))
    for n in range(N):
        Bd = np.zeros((K, K)); bd = np.zeros(K)
        for j in range(Ns):
            a = A[j, :, n]
            RA = np.einsum("kjp,p->kj", R, a)
            Bd += RA + RA.T - np.einsum("p,pkjq,q->kj", a, S, a)
            bd += a @ Bt[n] - np.einsum("p,pkq,q->k", a, Dt[n], a)
        B[n] = lam[n] * (XX - Bd / Ns)
        bw[:, n] = lam[n] * (YX[n] - bd / Ns)
    return B, bw


# ------------------------------------------------------- hyperparameter statistics
def quadform(g: Grid, W: np.ndarray) -> np.ndarray:
    """W_k D_w W_k' = ||G_w W_k'||^2 for every sample r and regressor k of
    W (R, K, N) in the k-major layout: the statistic of the alpha_k full
    conditional (Section 3.2) and of its SVB Monte Carlo approximation."""
    R, K, _ = W.shape
    out = np.empty((R, K))
    for r in range(R):
        for k in range(K):
            e = g.D @ W[r, k]
            out[r, k] = e @ e
    return out


def residual_ss(X: np.ndarray, Y: np.ndarray, W: np.ndarray, ar: np.ndarray) -> np.ndarray:
    """Whitened residual sum of squares per voxel, conditional on the first P
    scans (Appendix A.2): rss_n = ||A_n (y_n - X w_n)||^2 with the whitening
    rows [-a_P .. -a_1 1]; W is (K, N), ar is (P, N)."""
    T, K = X.shape
    P, N = ar.shape
    e = Y - X @ W                                   # (T, N) residuals
    out = np.empty(N)
    for n in range(N):
        w = e[P:, n].copy()
        for p in range(1, P + 1):
            w -= ar[p - 1, n] * e[P - p:T - p, n]
        out[n] = w @ w
    return out


def residual_ss_from_tensors(tensors, extra, W: np.ndarray, ar: np.ndarray) -> np.ndarray:
    """The bracket of the lambda full conditional in the tensor form of
    Appendix A.2: Y'Y - 2Y'XW + W'X'XW - 2Y'd'A + A'dd'A + 2A'B~W
    - 2W'(RA)W - 2A'(DW)A + W'(A'SA)W, with the extra per-voxel tensors
    extra = (YY (N), dY (N, P) = d_n y_n, dd (N, P, P) = d_n d_n')."""
    XX, R, S, YX, Bt, Dt = tensors
    YY, dY, dd = extra
    N = YY.shape[0]
    out = np.empty(N)
    for n in range(N):
        w, a = W[:, n], ar[:, n]
        RA = np.einsum("kjp,p->kj", R, a)
        DW = np.einsum("pkq,k->pq", Dt[n], w)
        ASA = np.einsum("p,pkjq,q->kj", a, S, a)
        out[n] = (YY[n] - 2 * YX[n] @ w + w @ XX @ w - 2 * dY[n] @ a + a @ dd[n] @ a
                  + 2 * a @ Bt[n] @ w - 2 * w @ RA @ w - 2 * a @ DW @ a + w @ ASA @ w)
    return out


def alpha_posterior(qf_mean: np.ndarray, N: int, q1: float, q2: float):
    """Ga(q~1k, q~2) of alpha_k: 1/q~1k = qf_k/2 + 1/q1, q~2 = N/2 + q2
    (qf_k = W_k D_w W_k', or its mean over samples for SVB)."""
    q1t = 1.0 / (0.5 * np.asarray(qf_mean, dtype=float) + 1.0 / q1)
    return q1t, N / 2.0 + q2


def lambda_posterior(rss_mean: np.ndarray, T: int, P: int, u1: float, u2: float):
    """Ga(u~1n, u~2) of lambda_n: 1/u~1n = rss_n/2 + 1/u1, u~2 = (T-P)/2 + u2."""
    u1t = 1.0 / (0.5 * np.asarray(rss_mean, dtype=float) + 1.0 / u1)
    return u1t, (T - P) / 2.0 + u2


def gibbs_step(g: Grid, X, Y, A, z1, z2, alpha, lam, seed: int, iteration: int, q1=10.0, q2=0.1, u1=10.0,
               u2=0.1, tol: float = 1e-13):
    """One iteration of the Gibbs sampler of Section 3.2 with the AR
    coefficients held at A (P, N): W from its full conditional by Algorithm 2
    with the random vectors z1 (1, K, dirs, N), z2 (1, K, N); then
    alpha_k ~ Ga(q~1k, N/2 + q2) and lambda_n ~ Ga(u~1n, (T-P)/2 + u2) from
    their full conditionals, drawn from the Philox streams 16 + 2 iteration and
    17 + 2 iteration of ``seed`` (Marsaglia-Tsang, see oracle/philox.py).
    Returns (W (K, N), alpha (K), lam (N))."""
    from oracle import philox
    T = X.shape[0]
    P = A.shape[0]
    B, bw = data_term_mc(X, Y, A[None], lam)
    W = sample(g, alpha, B, bw, z1, z2, tol)[0]
    q1t, q2t = alpha_posterior(quadform(g, W[None])[0], g.N, q1, q2)
    alpha_new = philox.gamma(seed, 16 + 2 * iteration, q2t, q1t)
    u1t, u2t = lambda_posterior(residual_ss(X, Y, W, A), T, P, u1, u2)
    lam_new = philox.gamma(seed, 17 + 2 * iteration, u2t, u1t)
    return W, alpha_new, lam_new


def alpha_extrapolate(a_jm2: np.ndarray, a_jm1: np.ndarray, a_j: np.ndarray) -> np.ndarray:
    """The first convergence device of the SVB implementation (Appendix C,
    speeding up SVB): through the posterior means of the last three
    iterations j-2, j-1, j put the quadratic in the iteration number; if its
    vertex lies after j, predict the value at the vertex, otherwise
    a_{j-1} + 20 (a_j - a_{j-1}); keep the prediction within a factor 5 of
    a_j (the value the update equation proposed).  Elementwise over k."""
    a2, a1, a0 = (np.asarray(v, dtype=np.float64) for v in (a_jm2, a_jm1, a_j))
    out = np.empty_like(a0)
    for k in range(a0.size):
        # quadratic c0 + c1 t + c2 t^2 through (0, a2), (1, a1), (2, a0)
        c2 = 0.5 * (a0[k] - 2.0 * a1[k] + a2[k])
        c1 = (a1[k] - a2[k]) - c2
        c0 = a2[k]
        pred = None
        if c2 != 0.0:
            tv = -c1 / (2.0 * c2)
            if tv > 2.0:
                pred = c0 + c1 * tv + c2 * tv * tv
        if pred is None:
            pred = a1[k] + 20.0 * (a0[k] - a1[k])
        out[k] = min(max(pred, a0[k] / 5.0), a0[k] * 5.0)
    return out


# --------------------------------------------------------- AR coefficients A
def ar_term_residuals(X: np.ndarray, Y: np.ndarray, W: np.ndarray, lam: np.ndarray, P: int):
    """Data part of the full conditional of the AR coefficients (Appendix A.2,
    full conditional of A), conditional on the first P scans: with the
    residuals e = Y - X W and, for voxel n, the P x (T-P) matrix E_n of lagged
    residuals (row p - 1 holds e[t-p] for t = P..T-1), the likelihood is
    Gaussian in A_n with precision J_n = lambda_n E_n E_n' and linear term
    b_n = lambda_n E_n e_n[P:].  W is (K, N).  Returns (J (N, P, P), b (P, N))."""
    T = X.shape[0]
    N = Y.shape[1]
    e = Y - X @ W
    J = np.empty((N, P, P))
    b = np.empty((P, N))
    for n in range(N):
        E = np.stack([e[P - p:T - p, n] for p in range(1, P + 1)])      # (P, T-P)
        J[n] = lam[n] * E @ E.T
        b[:, n] = lam[n] * E @ e[P:, n]
    return J, b


def ar_term_mc(X: np.ndarray, Y: np.ndarray, Wd: np.ndarray, lam: np.ndarray, P: int):
    """The SVB expectation of the above over Monte Carlo draws Wd (Ns, K, N) of
    W (Appendix B): the mean over draws of J_n and of b_n."""
    Js, bs = zip(*[ar_term_residuals(X, Y, Wd[j], lam, P) for j in range(Wd.shape[0])])
    return np.mean(Js, axis=0), np.mean(bs, axis=0)


def ar_term_from_tensors(tensors, extra, Wd: np.ndarray, lam: np.ndarray):
    """The tensor form of Appendix A.2 (full conditional of A), averaged over
    draws Wd (Ns, K, N):
      J_n = lambda_n mean_j [d_n d_n' - D_n W - (D_n W)' + W' S W],
      b_n = lambda_n mean_j [Y_n'd_n' - W' B~_n' + W' R W],   W = Wd[j][:, n],
    with (D_n W)[p][q] = sum_k D_n[p][k][q] W_k, (W'SW)[p][q] = sum_kl W_k S[p][k][l][q] W_l,
    (W'B~')[p] = sum_k B~_n[p][k] W_k and (W'RW)[p] = sum_kl W_k R[k][l][p] W_l."""
    XX, R, S, YX, Bt, Dt = tensors
    YY, dY, dd = extra
    N, P = dY.shape
    Ns = Wd.shape[0]
    J = np.zeros((N, P, P))
    b = np.zeros((P, N))
    for n in range(N):
        for j in range(Ns):
            w = Wd[j][:, n]
            DW = np.einsum("pkq,k->pq", Dt[n], w)
            WSW = np.einsum("k,pklq,l->pq", w, S, w)
            J[n] += dd[n] - DW - DW.T + WSW
            b[:, n] += dY[n] - Bt[n] @ w + np.einsum("k,klp,l->p", w, R, w)
        J[n] *= lam[n] / Ns
        b[:, n] *= lam[n] / Ns
    return J, b


def svb_step_ar(g: Grid, X, Y, A, z1w, z2w, z1a, z2a, alpha, beta, lam, q1=10.0, q2=0.1, r1=10000.0,
                r2=0.1, u1=10.0, u2=0.1, tol: float = 1e-13):
    """One spatial-VB iteration with the AR coefficients (Section 3.3, Appendix
    B), in the order W, A, then the hyperparameters:
      q(W): the data term with the mean lambda and the draws A (Ns, P, N); Ns
            Algorithm-2 samples with z1w, z2w and prior precisions alpha;
      q(A): the A data term with the new W draws; Ns Algorithm-2 samples on
            the operator with K = P, prior precisions beta and D_a = D_w, with
            z1a (Ns, P, dirs, N), z2a (Ns, P, N);
      alpha_k, beta_p: Gamma posterior means from the Monte Carlo mean of the
            spatial quadratic forms (r1, r2 the prior of beta);
      lambda_n: Gamma posterior mean from the Monte Carlo mean of the whitened
            residual sum of squares over the pairs (W^j, A^j).
    Returns (W, A, alpha_mean, beta_mean, lam_mean)."""
    T = X.shape[0]
    P = A.shape[1]
    B, bw = data_term_mc(X, Y, A, lam)
    Wn = sample(g, alpha, B, bw, z1w, z2w, tol)
    J, ba = ar_term_mc(X, Y, Wn, lam, P)
    An = sample(g, beta, J, ba, z1a, z2a, tol)
    q1t, q2t = alpha_posterior(quadform(g, Wn).mean(axis=0), g.N, q1, q2)
    r1t, r2t = alpha_posterior(quadform(g, An).mean(axis=0), g.N, r1, r2)
    rss = np.mean([residual_ss(X, Y, Wn[j], An[j]) for j in range(Wn.shape[0])], axis=0)
    u1t, u2t = lambda_posterior(rss, T, P, u1, u2)
    return Wn, An, q1t * q2t, r1t * r2t, u1t * u2t


# ---------------------------------------------------------------------- operator
def blocks_kmajor(B: np.ndarray) -> sp.csr_matrix:
    """H' blkdiag_n(B_n) H: the data term in the k-major (w_r) ordering.

    Entry ((k, n), (j, m)) equals B_n[k, j] when n == m (Section 3 and
    Appendix A.2, with H the permutation between vec(W) and vec(W'))."""
    N, K, _ = B.shape
    return sp.bmat([[sp.diags(B[:, k, j]) for j in range(K)] for k in range(K)]).tocsr()


def precision(g: Grid, alpha: np.ndarray, B: np.ndarray) -> sp.csr_matrix:
    """Q = diag(alpha) (x) D_w + H'blkdiag(B_n)H, size KN x KN, k-major.

    Section 3 (full conditional of w_r) and Appendix A.2 (temporal model)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    prior = sp.kron(sp.diags(alpha), g.G)
    return (prior + blocks_kmajor(B)).tocsr()


def apply(Q: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = Q x for one or many right-hand sides laid out (R, K, N) or (K, N)."""
    x = np.asarray(x, dtype=np.float64)
    flat = x.reshape(-1, Q.shape[0])
    return (Q @ flat.T).T.reshape(x.shape)


def relres(Q, x, b) -> np.ndarray:
    """||b - Qx||_2 / ||b||_2 per right-hand side (Section 3.1, PCG stopping rule)."""
    x = np.asarray(x).reshape(-1, Q.shape[0])
    b = np.asarray(b).reshape(-1, Q.shape[0])
    r = b - (Q @ x.T).T
    nb = np.linalg.norm(b, axis=1)
    out = np.linalg.norm(r, axis=1) / np.where(nb > 0, nb, 1.0)
    return np.where(nb > 0, out, 0.0)


# ------------------------------------------------------------------------- solve
def solve_direct(Q: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    """x = Q^{-1} b by a sparse direct factorisation (small operators only)."""
    lu = spl.splu(sp.csc_matrix(Q))
    flat = np.asarray(b, dtype=np.float64).reshape(-1, Q.shape[0])
    return np.stack([lu.solve(v) for v in flat]).reshape(np.shape(b))


def solve_pcg(Q: sp.csr_matrix, b: np.ndarray, tol: float = 1e-13, maxiter: int = 20000,
              x0: np.ndarray | None = None):
    """Preconditioned conjugate gradients in FP64 with the diagonal of Q as
    preconditioner, for one right-hand side, iterated until the relative
    residual ||b - Qx|| / ||b|| falls below ``tol`` (Section 3.1: PCG with a
    relative-residual tolerance delta; this is the textbook iteration of the
    Barrett et al. templates).  Returns (x, iterations, relres)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0
    dinv = 1.0 / Q.diagonal()
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    r = b - Q @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * nb and it < maxiter:
        q = Q @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        it += 1
        if it % 50 == 0:                      # guard against recursive-residual drift
            r = b - Q @ x
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    rr = np.linalg.norm(b - Q @ x) / nb
    return x, it, rr


def solve(Q: sp.csr_matrix, b: np.ndarray, tol: float = 1e-13, direct_limit: int = 20000):
    """x = Q^{-1} b for b shaped (R, K, N) or (K, N).  A sparse direct solve
    when KN <= direct_limit, otherwise FP64 PCG to relative residual ``tol``."""
    b = np.asarray(b, dtype=np.float64)
    if Q.shape[0] <= direct_limit:
        return solve_direct(Q, b)
    flat = b.reshape(-1, Q.shape[0])
    out = np.stack([solve_pcg(Q, v, tol)[0] for v in flat])
    return out.reshape(b.shape)


# ------------------------------------------------ incomplete Cholesky (block IC(0))
def redblack_order(g: Grid) -> np.ndarray:
    """Voxel order of the two-colour (red-black) numbering: voxels with even
    x + y + z ("red") in increasing n, then those with odd x + y + z ("black").
    Adjacent voxels differ by one in exactly one coordinate, so no edge joins
    two voxels of one colour."""
    red = (g.coords.sum(axis=1) % 2) == 0
    return np.r_[np.flatnonzero(red), np.flatnonzero(~red)]


def ic0_block(g: Grid, Q: sp.spmatrix, K: int, order: np.ndarray):
    """Incomplete Cholesky factor with zero fill, in K x K voxel blocks, of the
    precision Q (k-major, KN x KN) under the voxel order ``order`` -- the
    preconditioner M of Algorithm 2 (step 6), with the incomplete Cholesky of
    Section 3.1 taken blockwise on the grid graph.

    Block (n, m) of Q holds the entries ((k, n), (j, m)); it is non-zero when
    n == m or n, m are adjacent, which is the pattern L may use.  Elimination
    runs over the voxels in ``order``: the pivot block is factored by Cholesky,
    the blocks below it become A_ij L_jj^{-T}, and the Schur update
    A_il -= L_ij L_lj' is kept only where (i, l) lies in the pattern; fill
    outside it is dropped.  Dense and slow: tiny grids only.

    Returns (L, perm): L is the sparse lower-triangular factor in the permuted
    voxel-major order, row ``p*K + k`` for voxel order[p], regressor k; perm
    maps that permuted index to the k-major index ``k*N + n``."""
    N = g.N
    Qd = np.asarray(Q.todense()).reshape(K, N, K, N)
    pos = np.empty(N, dtype=np.int64)
    pos[order] = np.arange(N)
    adj = [set() for _ in range(N)]                 # adjacency in permuted positions
    for lo, hi in zip(g.edge_lo, g.edge_hi):
        adj[pos[lo]].add(pos[hi])
        adj[pos[hi]].add(pos[lo])

    def block(i, j):
        return Qd[:, order[i], :, order[j]].copy()

    A = {}
    for i in range(N):
        A[(i, i)] = block(i, i)
        for j in adj[i]:
            if j < i:
                A[(i, j)] = block(i, j)
    L = {}
    for j in range(N):
        Ljj = np.linalg.cholesky(A[(j, j)])
        L[(j, j)] = Ljj
        below = sorted(i for i in adj[j] if i > j)
        for i in below:
            # L_ij = A_ij L_jj^{-T}, i.e. L_jj L_ij' = A_ij'
            L[(i, j)] = np.linalg.solve(Ljj, A[(i, j)].T).T
        for i in below:
            for l in below:
                if l <= i and (i, l) in A:
                    A[(i, l)] -= L[(i, j)] @ L[(l, j)].T
    rows, cols, vals = [], [], []
    for (i, j), blk in L.items():
        for k in range(K):
            for c in range(K):
                if blk[k, c] != 0.0 or (i == j and k == c):
                    rows.append(i * K + k)
                    cols.append(j * K + c)
                    vals.append(blk[k, c])
    Lp = sp.csr_matrix((vals, (rows, cols)), shape=(N * K, N * K))
    perm = (np.arange(K)[None, :] * N + order[:, None]).ravel()   # p*K + k -> k*N + order[p]
    return Lp, perm


def ic0_redblack(g: Grid, alpha: np.ndarray, B: np.ndarray):
    """Block IC(0) of Q = diag(alpha) (x) D_w + H'blkdiag(B_n)H on the
    red-black voxel order.  Returns (L, perm) as ic0_block."""
    K = B.shape[1]
    return ic0_block(g, precision(g, alpha, B), K, redblack_order(g))


def ic0_solve(L: sp.csr_matrix, perm: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = M^{-1} r with M = L L': a forward solve with L and a backward solve
    with L' in the permuted order."""
    rp = np.asarray(r, dtype=np.float64).ravel()[perm]
    y = spl.spsolve_triangular(L, rp, lower=True)
    zp = spl.spsolve_triangular(sp.csr_matrix(L.T), y, lower=False)
    z = np.empty_like(zp)
    z[perm] = zp
    return z


def redblack_start(g: Grid, Q: sp.spmatrix, b: np.ndarray, x0: np.ndarray) -> np.ndarray:
    """Start value with the black entries of x0 and the red entries solved from
    the red rows of Q x = b, so that those rows of b - Q x vanish."""
    K = Q.shape[0] // g.N
    red = (g.coords.sum(axis=1) % 2) == 0
    R_idx = (np.arange(K)[:, None] * g.N + np.flatnonzero(red)[None, :]).ravel()
    B_idx = (np.arange(K)[:, None] * g.N + np.flatnonzero(~red)[None, :]).ravel()
    Qc = sp.csr_matrix(Q)
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    b = np.asarray(b, dtype=np.float64).ravel()
    rhs = b[R_idx] - Qc[R_idx][:, B_idx] @ x[B_idx]
    x[R_idx] = spl.spsolve(sp.csc_matrix(Qc[R_idx][:, R_idx]), rhs)
    return x


def solve_pcg_ic0(Q: sp.csr_matrix, b: np.ndarray, L: sp.csr_matrix, perm: np.ndarray, tol: float = 1e-13,
                  maxiter: int = 20000, x0: np.ndarray | None = None):
    """PCG (Barrett et al. templates) with the incomplete Cholesky
    preconditioner M = L L' of Algorithm 2, steps 6-7, for one right-hand side,
    until ||r|| <= tol ||b|| on the recursively updated residual (Section 3.1,
    relative-residual tolerance delta).  Returns (x, iterations, relres)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    r = b - Q @ x
    z = ic0_solve(L, perm, r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * nb and it < maxiter:
        q = Q @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        it += 1
        z = ic0_solve(L, perm, r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, np.linalg.norm(b - Q @ x) / nb


# --------------------------------------------------------------------- sampling
def edge_slots(g: Grid) -> np.ndarray:
    """For each edge, its slot (d, n_lo) in a z1 array laid out (K, dirs, N)."""
    return g.edge_dir * g.N + g.edge_lo


def perturbation_rhs(g: Grid, alpha, B, bw, z1, z2) -> np.ndarray:
    """Algorithm 2, step 4:
    b = (blkdiag_k sqrt(alpha_k) G_w)' z1 + H'L_data H z2 + b_w,
    with L_data the lower Cholesky factor of blkdiag_n(B_n).

    z1 arrives as (R, K, dirs, N) slots, one per (regressor, direction, voxel);
    the slot (k, d, n) holds the entry of edge (n, n+e_d) and slots without an
    edge are ignored.  z2 is (R, K, N); b_w is (K, N).  Returns (R, K, N)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    z1 = np.asarray(z1, dtype=np.float64)
    z2 = np.asarray(z2, dtype=np.float64)
    R, K = z2.shape[0], z2.shape[1]
    N = g.N
    slots = edge_slots(g)
    L = np.linalg.cholesky(B)                                  # (N, K, K) lower
    out = np.empty((R, K, N))
    for r in range(R):
        ze = z1[r].reshape(K, -1)[:, slots]                    # (K, E)
        prior = np.stack([np.sqrt(alpha[k]) * (g.D.T @ ze[k]) for k in range(K)])
        data = np.einsum("nkj,jn->kn", L, z2[r])
        out[r] = bw + prior + data
    return out


def perturbation_factor(g: Grid, alpha, B) -> np.ndarray:
    """Dense S = [(blkdiag_k sqrt(alpha_k) G_w)' | H'L_data H] (KN x (KE + KN));
    S S' equals Q (the identity behind Algorithm 2).  Tiny grids only."""
    alpha = np.asarray(alpha, dtype=np.float64)
    N, K, _ = B.shape
    D = g.D.toarray()
    L = np.linalg.cholesky(B)
    left = np.zeros((K * N, K * g.E))
    right = np.zeros((K * N, K * N))
    for k in range(K):
        left[k * N:(k + 1) * N, k * g.E:(k + 1) * g.E] = np.sqrt(alpha[k]) * D.T
        for j in range(K):
            right[k * N:(k + 1) * N, j * N:(j + 1) * N] = np.diag(L[:, k, j])
    return np.hstack([left, right])


def sample(g: Grid, alpha, B, bw, z1, z2, tol: float = 1e-13) -> np.ndarray:
    """Algorithm 2: w = Q^{-1} b with the perturbed right-hand side above."""
    Q = precision(g, alpha, B)
    return solve(Q, perturbation_rhs(g, alpha, B, bw, z1, z2), tol)


def cholesky_mean_and_sample(Q: sp.spmatrix, bw: np.ndarray, z: np.ndarray):
    """Algorithm 1 without reordering, dense: Q = L L', L x = b_w, L' mu = x,
    L' v = z, w = mu + v.  Returns (mu, w).  Tiny operators only."""
    from scipy.linalg import solve_triangular
    L = np.linalg.cholesky(Q.toarray())
    x = solve_triangular(L, np.asarray(bw).ravel(), lower=True)
    mu = solve_triangular(L.T, x, lower=False)
    v = solve_triangular(L.T, np.asarray(z).ravel(), lower=False)
    return mu.reshape(np.shape(bw)), (mu + v).reshape(np.shape(bw))


# ------------------------------------------------------------------ SVB iteration
def svb_step(g: Grid, X, Y, A, z1, z2, alpha, lam, q1=10.0, q2=0.1, u1=10.0, u2=0.1, tol: float = 1e-13):
    """One spatial-VB iteration with the AR coefficients held at the draws A
    (Ns, P, N) (Section 3.3, Appendix B), in the paper's order: the data term
    with the mean noise precisions lam and the draws; Ns Algorithm-2 samples
    of q(W) with the random vectors z1 (Ns, K, dirs, N), z2 (Ns, K, N); the
    posterior means of alpha (Monte Carlo mean of W_k D_w W_k') and of lambda
    (Monte Carlo mean of the whitened residual sum of squares).
    Returns (W (Ns, K, N), alpha_mean (K), lam_mean (N))."""
    T = X.shape[0]
    P = A.shape[1]
    B, bw = data_term_mc(X, Y, A, lam)
    W = sample(g, alpha, B, bw, z1, z2, tol)
    q1t, q2t = alpha_posterior(quadform(g, W).mean(axis=0), g.N, q1, q2)
    rss = np.mean([residual_ss(X, Y, W[j], A[j]) for j in range(W.shape[0])], axis=0)
    u1t, u2t = lambda_posterior(rss, T, P, u1, u2)
    return W, q1t * q2t, u1t * u2t


# ---------------------------------------------------------------------- traces
def hutchinson(g: Grid, Q: sp.csr_matrix, probes: np.ndarray, tol: float = 1e-13,
               u: np.ndarray | None = None):
    """Hutchinson estimates from Rademacher probes v_i (m, K, N):

        t   = (1/m) sum_i v_i' Q^{-1} v_i                ~ tr(Q^{-1})
        t_k = (1/m) sum_i v_ik' [Q^{-1} v_i]_k            ~ tr([Q^{-1}]_kk)
        g_k = (1/m) sum_i (D_w v_ik)' [Q^{-1} v_i]_k      ~ tr(D_w [Q^{-1}]_kk)

    The last is the trace term of E[W_k D_w W_k'] in Section 3.3.  ``u`` may
    carry precomputed solutions Q^{-1} v_i.  Returns (t, t_k, g_k, u)."""
    v = np.asarray(probes, dtype=np.float64)
    m, K, N = v.shape
    if u is None:
        u = solve(Q, v, tol)
    tk = np.einsum("ikn,ikn->k", v, u) / m
    gk = np.array([sum((g.G @ v[i, k]) @ u[i, k] for i in range(m)) for k in range(K)]) / m
    return float(tk.sum()), tk, gk, u
