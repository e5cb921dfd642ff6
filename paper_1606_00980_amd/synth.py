"""Seeded synthetic fMRI workloads: the inputs shared by the HIP path and the oracle.

This module only *generates inputs*.  It draws masks, design matrices, AR noise,
true activations and the random vectors (z1, z2, Rademacher probes) that the
method consumes, and it forms the per-voxel data term (B_n, b_n) that the solver
library takes as its input.  It contains no part of the solver: no precision
operator, no Laplacian, no solve, no sample, no trace.

Shapes follow the paper's workloads (Appendix D and the real-data sizes):
whole-brain voxel counts of 10^3..3*10^5, T = 160..200 scans, AR order up to 3,
an intercept with mean about 100, and block-design regressors convolved with a
haemodynamic response.  The paper's datasets are not used; these stand in.

Conventions used by every consumer:
  * a mask is a uint8 array of shape (nz, ny, nx); the linear voxel index is
    l = x + nx*(y + ny*z), i.e. ``mask.ravel()`` order, and in-mask voxels are
    numbered in increasing l;
  * per-voxel arrays are indexed by that compact voxel number n;
  * B has shape (N, K, K), b_w has shape (K, N) (k-major, the paper's
    w_r = vec(W') ordering of Section 3);
  * z1 has shape (R, K, dirs, N) with dirs = 3 in 3D (+x, +y, +z) and 2 in 2D;
    slot (k, d, n) belongs to the edge (n, n + e_d); slots whose far end lies
    outside the mask are drawn but unused;
  * z2 has shape (R, K, N); probes have shape (m, K, N), int8 in {-1, +1}.

Every random stream is ``numpy.random.default_rng([config_id, purpose, instance])``
with purposes MASK_W = 0, NOISE = 1, ALPHA = 2, Z = 3, PROBES = 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK_W, NOISE, ALPHA, Z, PROBES, OPS = 0, 1, 2, 3, 4, 5

# configuration ids of the five named workloads
CFG_SLICE, CFG_BRAIN, CFG_BATCH, CFG_UNEVEN, CFG_SERVE = 0, 1, 2, 3, 4

TR_SECONDS = 2.0
BURN_IN = 100


def _rng(config_id: int, purpose: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(config_id), int(purpose), int(instance)])


# --------------------------------------------------------------------------- masks
def circle_mask(n: int, radius: float) -> np.ndarray:
    """2D disc in an n x n grid, centre ((n-1)/2, (n-1)/2), inclusive test."""
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n]
    inside = (x - c) ** 2 + (y - c) ** 2 <= radius * radius
    return inside.astype(np.uint8)[None, :, :]          # (nz=1, ny, nx)


def ellipsoid_mask(dims_xyz, semi_axes_xyz) -> np.ndarray:
    """3D ellipsoid in an nx x ny x nz box, centred at (n_d-1)/2, inclusive test."""
    nx, ny, nz = (int(d) for d in dims_xyz)
    ax, ay, az = (float(a) for a in semi_axes_xyz)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    q = (((x - (nx - 1) / 2.0) / ax) ** 2 + ((y - (ny - 1) / 2.0) / ay) ** 2
         + ((z - (nz - 1) / 2.0) / az) ** 2)
    return (q <= 1.0).astype(np.uint8)                  # (nz, ny, nx)


# ----------------------------------------------------------------- design matrix
def gamma_hrf() -> np.ndarray:
    """Gamma density, shape 6 and scale 1 s, sampled every TR over [0, 32) s, unit sum."""
    t = np.arange(0.0, 32.0, TR_SECONDS)
    h = t ** 5 * np.exp(-t) / math.gamma(6.0)
    return h / h.sum()


def boxcar(T: int, period: int, phase: int) -> np.ndarray:
    """50% duty block design that starts in the 'off' half; ``phase`` delays it."""
    t = np.arange(T) - phase
    return (np.mod(t, period) >= period // 2).astype(np.float64) * (t >= 0)


def task_regressor(T: int, period: int, phase: int) -> np.ndarray:
    return np.convolve(boxcar(T, period, phase), gamma_hrf())[:T]


def drift(T: int, j: int) -> np.ndarray:
    t = np.arange(T)
    return np.cos(math.pi * j * (t + 0.5) / T)


def design_matrix(K: int, T: int, kind: str):
    """Returns (X, roles) with roles[k] in {'task', 'const', 'drift'}."""
    cols, roles = [], []
    if kind == "slice":                      # one task regressor plus a constant
        cols = [task_regressor(T, 20, 0), np.ones(T)]
        roles = ["task", "const"]
    elif kind == "brain":                    # three task regressors plus three drifts
        for per, ph in zip((20, 30, 40), (0, 5, 10)):
            cols.append(task_regressor(T, per, ph)); roles.append("task")
        for j in (1, 2, 3):
            cols.append(drift(T, j)); roles.append("drift")
    elif kind == "uneven":                   # min(K-1, 4) tasks, constant, then drifts
        ntask = min(K - 1, 4)
        for per, ph in list(zip((20, 30, 40, 50), (0, 5, 10, 15)))[:ntask]:
            cols.append(task_regressor(T, per, ph)); roles.append("task")
        cols.append(np.ones(T)); roles.append("const")
        j = 1
        while len(cols) < K:
            cols.append(drift(T, j)); roles.append("drift"); j += 1
    else:
        raise ValueError(kind)
    X = np.stack(cols[:K], axis=1)
    assert X.shape == (T, K)
    return X, roles[:K]


# ------------------------------------------------------------------------- noise
def pacf_to_ar(kappa: np.ndarray) -> np.ndarray:
    """Durbin-Levinson map from partial autocorrelations (P, N) to AR coefficients.

    With |kappa_p| < 1 the resulting AR(P) process is stationary.  Convention:
    e_t = sum_p a_p e_{t-p} + eps_t.
    """
    P = kappa.shape[0]
    a = np.zeros_like(kappa)
    for p in range(P):
        prev = a[:p].copy()
        a[p] = kappa[p]
        for j in range(p):
            a[j] = prev[j] - kappa[p] * prev[p - 1 - j]
    return a


def simulate_ar(a: np.ndarray, sigma2: np.ndarray, T: int, rng) -> np.ndarray:
    """AR(P) noise (T, N) after BURN_IN scans, innovations N(0, sigma2_n)."""
    P, N = a.shape
    tot = T + BURN_IN
    eps = rng.standard_normal((tot, N)) * np.sqrt(sigma2)[None, :]
    e = np.zeros((tot, N))
    for t in range(tot):
        acc = eps[t].copy()
        for p in range(1, P + 1):
            if t - p >= 0:
                acc += a[p - 1] * e[t - p]
        e[t] = acc
    return e[BURN_IN:]


# ---------------------------------------------------------------------- workload
@dataclass
class Workload:
    """One synthetic operator plus the raw data it was made from."""
    name: str
    mask: np.ndarray            # (nz, ny, nx) uint8
    conn: int                   # 4 (2D) or 6 (3D)
    K: int
    T: int
    P: int
    X: np.ndarray               # (T, K)
    ar: np.ndarray              # (P, N) AR coefficients
    sigma2: np.ndarray          # (N,) innovation variances (lambda_n = 1/sigma2_n)
    W_true: np.ndarray          # (K, N)
    Y: np.ndarray | None        # (T, N) or None when not kept
    B: np.ndarray               # (N, K, K)
    bw: np.ndarray              # (K, N)
    alpha: np.ndarray           # (K,)
    config_id: int = 0
    instance: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.B.shape[0])

    @property
    def dims(self):
        nz, ny, nx = self.mask.shape
        return nx, ny, nz

    @property
    def dirs(self) -> int:
        return 3 if self.conn == 6 else 2

    def z(self, R: int, stream: int = 0):
        """z1 (R, K, dirs, N) and z2 (R, K, N), N(0,1)."""
        g = _rng(self.config_id, Z, self.instance * 1000 + stream)
        z1 = g.standard_normal((R, self.K, self.dirs, self.N))
        z2 = g.standard_normal((R, self.K, self.N))
        return z1, z2

    def probes(self, m: int, stream: int = 0) -> np.ndarray:
        """Rademacher probes (m, K, N) int8, +1/-1 with probability 1/2."""
        g = _rng(self.config_id, PROBES, self.instance * 1000 + stream)
        bits = g.integers(0, 2, size=(m, self.K, self.N), dtype=np.int8)
        return (2 * bits - 1).astype(np.int8)

    def rhs(self, R: int, stream: int = 0) -> np.ndarray:
        """R right-hand sides b_w + N(0, 1) noise, (R, K, N)."""
        g = _rng(self.config_id, NOISE, 7_000_000 + self.instance * 1000 + stream)
        return self.bw[None] + g.standard_normal((R, self.K, self.N))


def _blob(mask: np.ndarray, centre_lin: int, sigma: float, amp: float) -> np.ndarray:
    nz, ny, nx = mask.shape
    lin = np.flatnonzero(mask.ravel())
    x = lin % nx; y = (lin // nx) % ny; z = lin // (nx * ny)
    cx = centre_lin % nx; cy = (centre_lin // nx) % ny; cz = centre_lin // (nx * ny)
    d2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
    return amp * np.exp(-0.5 * d2 / (sigma * sigma))


def _data_term(X, ar, sigma2, Y, P):
    """B_n = Xw'Xw/sigma2_n and b_n = Xw'yw/sigma2_n with the AR(P) whitening
    c = (1, -a_1, .., -a_P), conditional on the first P scans.  Written as a
    quadratic form in c over lagged cross products, so no per-voxel T-length
    arrays are formed."""
    T, K = X.shape
    N = sigma2.shape[0]
    c = np.concatenate([np.ones((1, N)), -ar], axis=0)          # (P+1, N)
    lam = 1.0 / sigma2
    lagX = [X[P - p:T - p] for p in range(P + 1)]                # (T-P, K) each
    lagY = [Y[P - p:T - p] for p in range(P + 1)]                # (T-P, N) each
    B = np.zeros((N, K, K))
    bw = np.zeros((K, N))
    for p in range(P + 1):
        for q in range(P + 1):
            cc = c[p] * c[q] * lam                              # (N,)
            Cpq = lagX[p].T @ lagX[q]                           # (K, K)
            B += cc[:, None, None] * Cpq[None]
            bw += cc[None, :] * (lagX[p].T @ lagY[q])            # (K, N)
    B = 0.5 * (B + B.transpose(0, 2, 1))
    return B, bw


def make_workload(name: str, mask: np.ndarray, conn: int, K: int, T: int, P: int,
                  kind: str, config_id: int, instance: int, alpha: np.ndarray,
                  ar_kind: str, keep_y: bool) -> Workload:
    g_mw = _rng(config_id, MASK_W, instance)
    g_noise = _rng(config_id, NOISE, instance)
    N = int(mask.sum())
    X, roles = design_matrix(K, T, kind)
    lin = np.flatnonzero(mask.ravel())
    W = np.zeros((K, N))
    for k, role in enumerate(roles):
        if role == "task":
            W[k] = _blob(mask, int(lin[g_mw.integers(0, N)]), 4.0, 2.0)
        elif role == "const":
            W[k] = g_mw.normal(100.0, 14.4, size=N)
    if ar_kind == "ar1":
        ar = g_noise.uniform(0.2, 0.5, size=(1, N))
    else:
        ar = pacf_to_ar(g_noise.uniform(-0.5, 0.5, size=(P, N)))
    sigma2 = g_noise.uniform(0.5, 2.0, size=N)
    B = np.zeros((N, K, K)); bw = np.zeros((K, N))
    Ykeep = np.zeros((T, N)) if keep_y else None
    chunk = 65536
    for s in range(0, N, chunk):
        e = slice(s, min(N, s + chunk))
        noise = simulate_ar(ar[:, e], sigma2[e], T, g_noise)
        Yc = X @ W[:, e] + noise
        B[e], bw[:, e] = _data_term(X, ar[:, e], sigma2[e], Yc, P)
        if keep_y:
            Ykeep[:, e] = Yc
    return Workload(name=name, mask=mask, conn=conn, K=K, T=T, P=P, X=X, ar=ar,
                    sigma2=sigma2, W_true=W, Y=Ykeep, B=B, bw=bw,
                    alpha=np.asarray(alpha, dtype=np.float64),
                    config_id=config_id, instance=instance,
                    meta={"roles": roles, "kind": kind})


def slice_2d(keep_y: bool = True) -> Workload:
    """64x64 slice, disc of radius 28, 4-neighbour, K = 2, T = 160, AR(1), alpha = (1, 1)."""
    return make_workload("slice2d_64x64_r28_K2", circle_mask(64, 28.0), 4, 2, 160, 1,
                         "slice", CFG_SLICE, 0, np.array([1.0, 1.0]), "ar1", keep_y)


def brain_3d(keep_y: bool = False) -> Workload:
    """64x64x33 grid, ellipsoid (28, 30, 15), 6-neighbour, K = 6, T = 200, AR(3),
    alpha_k ~ Gamma(shape 2, scale 1)."""
    alpha = _rng(CFG_BRAIN, ALPHA, 0).gamma(2.0, 1.0, size=6)
    return make_workload("brain3d_64x64x33_K6", ellipsoid_mask((64, 64, 33), (28, 30, 15)),
                         6, 6, 200, 3, "brain", CFG_BRAIN, 0, alpha, "ar3", keep_y)


def uneven_params(config_id: int, instance: int):
    """Grid dims, fill fraction and K of one uneven instance."""
    g = _rng(config_id, OPS, instance)
    s = g.uniform(1.0, 3.0)
    f = g.uniform(0.4, 0.6)
    K = int(g.integers(2, 11))
    dims = tuple(int(round(s * d)) for d in (32, 32, 20))
    return dims, f, K


def uneven_instance(config_id: int, instance: int, keep_y: bool = False,
                    dims=None, fill=None, K=None) -> Workload:
    """One operator of the uneven batch: grid between 32x32x20 and 96x96x60,
    ellipsoid at 40-60% fill, K in 2..10, T = 200, AR(3)."""
    d0, f0, K0 = uneven_params(config_id, instance)
    dims = d0 if dims is None else dims
    fill = f0 if fill is None else fill
    K = K0 if K is None else K
    c = (6.0 * fill / math.pi) ** (1.0 / 3.0)
    semi = [min(0.5 * d * c, 0.5 * d) for d in dims]
    mask = ellipsoid_mask(dims, semi)
    alpha = _rng(config_id, ALPHA, instance).gamma(2.0, 1.0, size=K)
    return make_workload(f"uneven{config_id}_{instance}_{dims[0]}x{dims[1]}x{dims[2]}_K{K}",
                         mask, 6, K, 200, 3, "uneven", config_id, instance, alpha, "ar3", keep_y)


def tiny(dims_xyz, conn: int, K: int, seed: int = 0, T: int = 60, P: int = 1,
         shape: str = "ellipsoid") -> Workload:
    """Small operators for exhaustive checks (oracle pins and edge cases)."""
    nx, ny, nz = dims_xyz
    if shape == "box":
        mask = np.ones((nz, ny, nx), dtype=np.uint8)
    elif conn == 4:
        mask = ellipsoid_mask((nx, ny, 1), (nx / 2.0, ny / 2.0, 1.0))
    else:
        mask = ellipsoid_mask((nx, ny, nz), (nx / 2.0, ny / 2.0, nz / 2.0))
    kind = "uneven" if K >= 2 else "single"
    if kind == "single":
        X = np.ones((T, 1))
    alpha = _rng(900 + seed, ALPHA, 0).gamma(2.0, 1.0, size=K)
    if K >= 2:
        return make_workload(f"tiny{nx}x{ny}x{nz}_K{K}_s{seed}", mask, conn, K, T, P,
                             "uneven", 900 + seed, 0, alpha, "ar1" if P == 1 else "ar3",
                             keep_y=True)
    # K = 1: intercept-only model
    return _intercept_only(mask, conn, T, P, seed, alpha)


def _intercept_only(mask, conn, T, P, seed, alpha) -> Workload:
    g_mw = _rng(900 + seed, MASK_W, 0); g_noise = _rng(900 + seed, NOISE, 0)
    N = int(mask.sum())
    X = np.ones((T, 1))
    W = g_mw.normal(100.0, 14.4, size=(1, N))
    ar = g_noise.uniform(0.2, 0.5, size=(1, N)) if P == 1 else \
        pacf_to_ar(g_noise.uniform(-0.5, 0.5, size=(P, N)))
    sigma2 = g_noise.uniform(0.5, 2.0, size=N)
    Y = X @ W + simulate_ar(ar, sigma2, T, g_noise)
    B, bw = _data_term(X, ar, sigma2, Y, P)
    return Workload(name=f"tiny_K1_s{seed}", mask=mask, conn=conn, K=1, T=T, P=P, X=X,
                    ar=ar, sigma2=sigma2, W_true=W, Y=Y, B=B, bw=bw,
                    alpha=np.asarray(alpha, dtype=np.float64), config_id=900 + seed)


# ----------------------------------------------------------- named workloads
def from_spec(spec) -> Workload:
    """The workload a spec names: ("slice",), ("brain",) or
    ("uneven", config_id, instance)."""
    kind = spec[0]
    if kind == "slice":
        return slice_2d(keep_y=False)
    if kind == "brain":
        return brain_3d()
    if kind == "uneven":
        return uneven_instance(int(spec[1]), int(spec[2]))
    raise ValueError(f"unknown workload spec {spec!r}")


def generate(specs, workers: int | None = None) -> list:
    """[from_spec(s) for s in specs], made by a pool of ``spawn`` worker
    processes (at most 16, and at most the cores this process may use)."""
    import multiprocessing as mp
    import os
    specs = list(specs)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:                     # pragma: no cover
        cores = os.cpu_count() or 1
    workers = max(1, min(workers or 16, cores, len(specs)))
    if workers == 1:
        return [from_spec(s) for s in specs]
    with mp.get_context("spawn").Pool(workers, maxtasksperchild=1) as pool:
        return pool.map(from_spec, specs, chunksize=1)

