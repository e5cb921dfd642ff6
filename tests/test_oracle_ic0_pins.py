"""Pins of the oracle's incomplete Cholesky preconditioner (block IC(0) on the
red-black voxel order, the M of Algorithm 2, steps 6-7) against facts that do
not re-use its code: the defining property of a zero-fill incomplete factor
(M agrees with Q on Q's pattern, L stays inside it), exactness where no fill
is dropped, the unit eigenvalues that a red-black order forces, and the
solution of a direct solve."""
import numpy as np
import pytest

from oracle import gmrf_oracle as orc
from paper_1606_00980_amd import synth


def block_pattern(g, order):
    """Permuted voxel positions (i, j) whose K x K block of Q may be non-zero."""
    pos = np.empty(g.N, dtype=np.int64)
    pos[order] = np.arange(g.N)
    pat = np.eye(g.N, dtype=bool)
    pat[pos[g.edge_lo], pos[g.edge_hi]] = True
    pat[pos[g.edge_hi], pos[g.edge_lo]] = True
    return pat


def permuted_dense(Q, perm):
    return np.asarray(Q.todense())[np.ix_(perm, perm)]


def test_redblack_order_is_a_two_colouring():
    for dims, conn in (((6, 5, 4), 6), ((9, 7, 1), 4)):
        w = synth.tiny(dims, conn, 2, seed=3)
        g = orc.grid(w.mask, w.conn)
        order = orc.redblack_order(g)
        assert sorted(order.tolist()) == list(range(g.N))
        colour = np.empty(g.N, dtype=int)
        nred = int(((g.coords.sum(axis=1) % 2) == 0).sum())
        colour[order[:nred]] = 0
        colour[order[nred:]] = 1
        assert g.E > 0 and np.all(colour[g.edge_lo] != colour[g.edge_hi])
        # red voxels come first and each colour keeps increasing n
        assert np.all(np.diff(order[:nred]) > 0) and np.all(np.diff(order[nred:]) > 0)


@pytest.mark.parametrize("dims,conn,K", [((5, 4, 3), 6, 3), ((7, 6, 1), 4, 2), ((4, 4, 3), 6, 1)])
def test_factor_is_the_zero_fill_incomplete_factor(dims, conn, K):
    """An incomplete Cholesky factor with zero fill is characterised by: L
    lower block triangular inside Q's block pattern, lower-triangular diagonal
    blocks with a positive diagonal, and (L L')_ij = Q_ij on the pattern
    (these determine L uniquely).  Off the pattern M differs from Q, which
    shows that fill was dropped."""
    w = synth.tiny(dims, conn, K, seed=11 + K)
    g = orc.grid(w.mask, w.conn)
    order = orc.redblack_order(g)
    Q = orc.precision(g, w.alpha, w.B)
    L, perm = orc.ic0_redblack(g, w.alpha, w.B)
    Ld = L.toarray()
    Qp = permuted_dense(Q, perm)
    pat = block_pattern(g, order)
    patK = np.kron(pat, np.ones((K, K), dtype=bool))
    assert np.all(np.triu(Ld, 1) == 0.0)
    assert np.all(np.diag(Ld) > 0.0)
    lower_blocks = np.kron(np.tril(pat), np.ones((K, K), dtype=bool))
    assert np.all(Ld[~lower_blocks] == 0.0)
    M = Ld @ Ld.T
    scale = np.abs(Qp).max()
    assert np.abs(M - Qp)[patK].max() <= 1e-12 * scale
    assert np.abs(M - Qp)[~patK].max() > 1e-6 * scale


@pytest.mark.parametrize("dims", [(3, 1, 1), (2, 1, 1), (1, 3, 1)])
def test_factor_is_exact_without_dropped_fill(dims):
    """On a path of at most three voxels coloured red-black-red no two black
    voxels share a red neighbour, so elimination creates no fill outside the
    pattern: M = Q and PCG converges in one step."""
    nx, ny, nz = dims
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    g = orc.grid(mask, 6)
    K = 3
    rng = np.random.default_rng(5)
    A = rng.standard_normal((g.N, K, K))
    B = A @ A.transpose(0, 2, 1) + K * np.eye(K)
    alpha = np.array([0.7, 1.9, 3.1])
    Q = orc.precision(g, alpha, B)
    L, perm = orc.ic0_redblack(g, alpha, B)
    M = (L @ L.T).toarray()
    assert np.allclose(M, permuted_dense(Q, perm), rtol=0, atol=1e-12 * abs(Q).max())
    b = rng.standard_normal(Q.shape[0])
    x, it, rel = orc.solve_pcg_ic0(Q, b, L, perm, tol=1e-12)
    assert it == 1 and rel < 1e-12


def test_redblack_factor_has_unit_eigenvalues_on_the_red_block():
    """With red voxels first, L's red diagonal blocks factor Q's red block
    exactly and L's off-diagonal blocks are Q's, so M and Q share their first
    block row: M^{-1} Q has the eigenvalue 1 at least K * (number of red
    voxels) times."""
    w = synth.tiny((5, 4, 3), 6, 2, seed=21)
    g = orc.grid(w.mask, w.conn)
    K = 2
    nred = int(((g.coords.sum(axis=1) % 2) == 0).sum())
    Q = orc.precision(g, w.alpha, w.B)
    L, perm = orc.ic0_redblack(g, w.alpha, w.B)
    Ld = L.toarray()
    Qp = permuted_dense(Q, perm)
    ev = np.linalg.eigvals(np.linalg.solve(Ld @ Ld.T, Qp)).real
    assert np.sum(np.abs(ev - 1.0) < 1e-8) >= K * nred
    assert ev.min() > 0.0


def test_ic0_solve_inverts_the_factor():
    w = synth.tiny((4, 4, 3), 6, 3, seed=23)
    g = orc.grid(w.mask, w.conn)
    L, perm = orc.ic0_redblack(g, w.alpha, w.B)
    Ld = L.toarray()
    r = np.random.default_rng(1).standard_normal(L.shape[0])
    z = orc.ic0_solve(L, perm, r)
    M = Ld @ Ld.T
    assert np.allclose(M @ z[perm], r[perm], rtol=0, atol=1e-10 * np.abs(r).max())


@pytest.mark.parametrize("dims,conn,K", [((6, 5, 4), 6, 3), ((9, 8, 1), 4, 4)])
def test_pcg_with_ic0_reaches_the_direct_solution(dims, conn, K):
    w = synth.tiny(dims, conn, K, seed=31 + K)
    g = orc.grid(w.mask, w.conn)
    Q = orc.precision(g, w.alpha, w.B)
    L, perm = orc.ic0_redblack(g, w.alpha, w.B)
    b = np.random.default_rng(2).standard_normal(Q.shape[0])
    ref = orc.solve_direct(Q, b)
    x0 = orc.redblack_start(g, Q, b, np.zeros_like(b))
    x, it, rel = orc.solve_pcg_ic0(Q, b, L, perm, tol=1e-12, x0=x0)
    assert rel < 1e-11 and np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    # fewer iterations than diagonal scaling on the same system
    _, it_jac, _ = orc.solve_pcg(Q, b, tol=1e-12)
    assert it < it_jac


def test_redblack_start_zeroes_the_red_residual():
    w = synth.tiny((6, 5, 4), 6, 3, seed=41)
    g = orc.grid(w.mask, w.conn)
    Q = orc.precision(g, w.alpha, w.B)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(Q.shape[0])
    x0 = rng.standard_normal(Q.shape[0])
    x = orc.redblack_start(g, Q, b, x0)
    red = (g.coords.sum(axis=1) % 2) == 0
    r = (b - Q @ x).reshape(3, g.N)
    xb, x0b = x.reshape(3, g.N), x0.reshape(3, g.N)
    assert np.abs(r[:, red]).max() <= 1e-12 * np.abs(b).max()
    assert np.array_equal(xb[:, ~red], x0b[:, ~red])
    assert np.abs(r[:, ~red]).max() > 1e-3


# ------------------------------------------------------- planted mistakes
def characterised(Ld, Qp, pat, K):
    """The zero-fill incomplete-factor characterisation of the test above."""
    patK = np.kron(pat, np.ones((K, K), dtype=bool))
    lower_blocks = np.kron(np.tril(pat), np.ones((K, K), dtype=bool))
    M = Ld @ Ld.T
    scale = np.abs(Qp).max()
    return (np.all(np.triu(Ld, 1) == 0.0) and np.all(np.diag(Ld) > 0.0) and np.all(Ld[~lower_blocks] == 0.0)
            and np.abs(M - Qp)[patK].max() <= 1e-12 * scale)


def test_characterisation_catches_plausible_factor_mistakes():
    """Factors that plausible mistakes produce fail the characterisation: fill
    kept (a complete Cholesky factor), the Schur updates dropped (block
    Jacobi), the off-diagonal blocks transposed, a scalar instead of a block
    pattern (the dense couplings inside a voxel block lost)."""
    K = 3
    w = synth.tiny((5, 4, 3), 6, K, seed=13)
    g = orc.grid(w.mask, w.conn)
    order = orc.redblack_order(g)
    Q = orc.precision(g, w.alpha, w.B)
    L, perm = orc.ic0_redblack(g, w.alpha, w.B)
    Ld = L.toarray()
    Qp = permuted_dense(Q, perm)
    pat = block_pattern(g, order)
    assert characterised(Ld, Qp, pat, K)
    full = np.linalg.cholesky(Qp)
    assert not characterised(full, Qp, pat, K)
    diag_only = np.zeros_like(Ld)
    for i in range(g.N):
        sl = slice(i * K, (i + 1) * K)
        diag_only[sl, sl] = np.linalg.cholesky(Qp[sl, sl])
    assert not characterised(diag_only, Qp, pat, K)
    transposed = Ld.copy()
    for i in range(g.N):
        for j in range(i):
            if pat[i, j]:
                si, sj = slice(i * K, (i + 1) * K), slice(j * K, (j + 1) * K)
                transposed[si, sj] = Ld[si, sj].T
    assert not characterised(transposed, Qp, pat, K)
    scalar = Ld * (np.kron(np.eye(g.N), np.ones((K, K))) + np.kron(np.ones((g.N, g.N)), np.eye(K)) > 0)
    assert not characterised(scalar, Qp, pat, K)
