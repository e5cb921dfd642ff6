"""Parallel runs of the FP64 oracle over many right-hand sides (test
infrastructure only, like the rest of ``oracle/``: the test suite and the
CPU-baseline leg of the benchmark use it; the product path never does).

Each job regenerates its seeded synthetic workload inside a worker process
(``paper_1606_00980_amd.synth``, the input generator shared by both sides; it
holds none of the method's arithmetic) and calls ``gmrf_oracle`` on it:
Algorithm 2 right-hand sides and their solves, Rademacher probe solves and the
Hutchinson estimates of Section 3.3, or the Philox-drawn vectors of a served
request.  Workers are started with the ``spawn`` method: they never touch a
GPU, and a parent that has initialised one is not forked.  This mirrors the
paper's independent samples on separate cores (Section 3.3): one process per
right-hand-side group.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np


def pool_size(limit: int = 16) -> int:
    """Worker processes: the cores this process may use, at most ``limit``."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:                     # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def _single_thread():
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(limits=1)
    except ImportError:                        # pragma: no cover
        return None


class Pending:
    """Jobs running in a spawn pool; get() waits and returns (results in job
    order, wall seconds since the start, workers used)."""

    def __init__(self, fn, jobs, workers: int | None = None):
        self.workers = min(workers or pool_size(), max(1, len(jobs)))
        self.t0 = time.perf_counter()
        self.pool = mp.get_context("spawn").Pool(self.workers, initializer=_single_thread, maxtasksperchild=1)
        self.res = self.pool.starmap_async(fn, jobs, chunksize=1)

    def get(self):
        try:
            out = self.res.get()
        finally:
            self.pool.close()
            self.pool.join()
        return out, time.perf_counter() - self.t0, self.workers


def start_parallel(fn, jobs, workers: int | None = None) -> Pending:
    """Start [fn(*job) for job in jobs] in a spawn pool of single-threaded
    worker processes and return at once."""
    return Pending(fn, jobs, workers)


def run_parallel(fn, jobs, workers: int | None = None):
    """[fn(*job) for job in jobs] by a spawn pool of single-threaded worker
    processes (or in this process when workers == 1).  Returns (results in job
    order, wall seconds, workers used)."""
    if (workers or pool_size()) == 1 or len(jobs) <= 1:
        t0 = time.perf_counter()
        lim = _single_thread()
        try:
            out = [fn(*j) for j in jobs]
        finally:
            if lim is not None:
                lim.unregister()
        return out, time.perf_counter() - t0, 1
    return start_parallel(fn, jobs, workers).get()


# ------------------------------------------------------------------------ jobs
def _workload(spec):
    from paper_1606_00980_amd import synth
    return synth.from_spec(spec)


def solutions(spec, n_samples: int, sample_idx, n_probes: int, probe_idx, trace: bool = False,
              tol: float = 1e-12):
    """Oracle solutions for the workload ``spec`` (("brain",), ("slice",) or
    ("uneven", config_id, instance)): the Algorithm-2 samples ``sample_idx`` of
    the seeded draws ``w.z(n_samples)`` and the probe solutions ``probe_idx`` of
    ``w.probes(n_probes)``, each solved to relative residual ``tol``; with
    ``trace`` (all probes requested) also the Hutchinson estimates t, t_k, g_k.
    Returns a dict of arrays and the job's seconds."""
    from oracle import gmrf_oracle as orc
    t0 = time.perf_counter()
    w = _workload(spec)
    g = orc.grid(w.mask, w.conn)
    Q = orc.precision(g, w.alpha, w.B)
    out = {"N": w.N, "K": w.K}
    sample_idx = list(sample_idx)
    probe_idx = list(probe_idx)
    if sample_idx:
        z1, z2 = w.z(n_samples)
        b = orc.perturbation_rhs(g, w.alpha, w.B, w.bw, z1[sample_idx], z2[sample_idx])
        out["samples"] = orc.solve(Q, b, tol)
        out["sample_rhs"] = b
    if probe_idx:
        v = w.probes(n_probes)[probe_idx]
        if trace:
            t, tk, gk, u = orc.hutchinson(g, Q, v, tol)
            out["trace"] = (t, tk, gk)
        else:
            u = orc.solve(Q, v.astype(np.float64), tol)
        out["probes"] = u
    out["seconds"] = time.perf_counter() - t0
    return out


def solve_rhs(mask, conn: int, alpha, B, rhs, tol: float = 1e-12):
    """Oracle solutions Q^{-1} rhs (rhs: (R, K, N) FP64) of the operator given
    by its raw inputs (mask, connectivity, alpha, blocks B (N, K, K)).
    Returns (x, oracle seconds: assembly and solves)."""
    from oracle import gmrf_oracle as orc
    t0 = time.perf_counter()
    g = orc.grid(mask, conn)
    Q = orc.precision(g, alpha, B)
    x = orc.solve(Q, np.asarray(rhs, dtype=np.float64), tol)
    return x, time.perf_counter() - t0


def algorithm2_solutions(mask, conn: int, alpha, B, bw, z1, z2, probes, tol: float = 1e-12):
    """The oracle on raw inputs: Algorithm-2 right-hand sides from z1
    (R, K, dirs, N) and z2 (R, K, N) and their solutions, and the solutions of
    the Rademacher probes (m, K, N) (either part may be empty).  Returns
    (samples (R, K, N), probe solutions (m, K, N), oracle seconds: assembly,
    right-hand sides and solves)."""
    from oracle import gmrf_oracle as orc
    t0 = time.perf_counter()
    g = orc.grid(mask, conn)
    Q = orc.precision(g, alpha, B)
    K, N = np.shape(B)[1], np.shape(B)[0]
    xs = np.zeros((0, K, N))
    u = np.zeros((0, K, N))
    if z2 is not None and len(z2):
        b = orc.perturbation_rhs(g, alpha, B, bw, z1, z2)
        xs = orc.solve(Q, b, tol)
    if probes is not None and len(probes):
        u = orc.solve(Q, np.asarray(probes, dtype=np.float64), tol)
    return xs, u, time.perf_counter() - t0


def perturbation_rhs(mask, conn: int, alpha, B, bw, z1, z2):
    """The oracle's Algorithm-2 right-hand sides for raw inputs (see
    gmrf_oracle.perturbation_rhs)."""
    from oracle import gmrf_oracle as orc
    return orc.perturbation_rhs(orc.grid(mask, conn), alpha, B, bw, z1, z2)


def hutchinson_from(mask, conn: int, probes, u):
    """t, t_k, g_k of the oracle's Hutchinson estimator from given probe
    solutions u (see gmrf_oracle.hutchinson)."""
    from oracle import gmrf_oracle as orc
    return orc.hutchinson(orc.grid(mask, conn), None, probes, u=u)[:3]


def served(spec, kind: int, seed: int, probes: int, probe_idx=None, tol: float = 1e-12):
    """Oracle result of one served request on workload ``spec`` with the
    request's Philox-drawn vectors: kind 0 solves b_w + n (n from stream 4),
    kind 1 is the Algorithm-2 sample with z1, z2 from streams 1 and 2, kind 2
    solves the Rademacher probes ``probe_idx`` (all when None) of the
    ``probes`` drawn from stream 3 (the estimates t, t_k, g_k follow from all
    of them with ``hutchinson(..., u=...)``).  Returns {"x": (R, K, N)}."""
    from oracle import gmrf_oracle as orc
    from oracle import philox
    w = _workload(spec)
    g = orc.grid(w.mask, w.conn)
    Q = orc.precision(g, w.alpha, w.B)
    n = w.K * w.N
    if kind == 0:
        b = w.bw + philox.normal(seed, 4, n).reshape(w.K, w.N)
        return {"x": orc.solve(Q, b[None], tol)}
    if kind == 1:
        z1 = philox.normal(seed, 1, g.ndirs * n).reshape(1, w.K, g.ndirs, w.N)
        z2 = philox.normal(seed, 2, n).reshape(1, w.K, w.N)
        return {"x": orc.sample(g, w.alpha, w.B, w.bw, z1, z2, tol)}
    v = served_probes(seed, probes, w.K, w.N)
    idx = range(probes) if probe_idx is None else list(probe_idx)
    return {"x": orc.solve(Q, v[list(idx)].astype(np.float64), tol)}


def served_probes(seed: int, probes: int, K: int, N: int) -> np.ndarray:
    """The Rademacher probes (probes, K, N) of a served trace request."""
    from oracle import philox
    return philox.rademacher(seed, 3, probes * K * N).reshape(probes, K, N)


# ------------------------------------------------------------------ comparison
def rel_errors(x, ref):
    """Per right-hand side: ||x - ref|| / ||ref|| over all K*N entries, and the
    largest regressor block's ||x_k - ref_k|| / ||ref|| (the parity gate of
    both is 1e-6).  x, ref: (R, K, N).  Returns two arrays of length R."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1), 1e-300)
    whole = np.linalg.norm((x - ref).reshape(ref.shape[0], -1), axis=1) / scale
    block = np.linalg.norm(x - ref, axis=2).max(axis=1) / scale
    return whole, block
