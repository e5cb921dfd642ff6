#!/usr/bin/env python3
"""Throughput benchmark of the posterior-precision hot path on one MI355X.

One step is one pass of the whole path over one batch of synthetic input on
the 52,740-voxel whole-brain operator (64x64x33 ellipsoid, K = 6, AR(3)):
assemble the data term on the device (blocks packed and factored), set alpha
(preconditioner set-up), form 32 perturbed right-hand sides (Algorithm 2) and
32 Rademacher probe right-hand sides, solve all 64 in one batch (FP32 inner
PCG, FP64 refinement to relative residual 1e-8, every right-hand side from
zero) preconditioned by the incomplete Cholesky factor on the red-black voxel
order (--precond block_jacobi for the block-Jacobi solver), and reduce the
Hutchinson trace estimates.  `value` is solves/s over the
timed steps with inputs resident in HBM.

    python bench.py [--steps K] [--warmup W] [--workload batch64|brain_fp64|uneven]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pmc.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1606_00980_amd", "csrc", f)
                  for f in ("pcg.hpp", "device.hpp", "common.hpp", "rbic.hpp", "k_rbic_f32.hip", "k_rbic_f64.hip",
                            "spd.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64", choices=["batch64", "brain_fp64", "uneven", "serve"])
    ap.add_argument("--precond", default="rb_ic0", choices=["rb_ic0", "block_jacobi"],
                    help="batch64 and uneven: the incomplete Cholesky factor on the red-black order "
                         "(default) or block Jacobi (autotuned)")
    ap.add_argument("--no-precond-compare", action="store_true",
                    help="batch64: skip the solve-only comparison of preconditioners and precisions")
    ap.add_argument("--no-ar-step", action="store_true",
                    help="batch64: skip the timing of the AR-coefficient step")
    ap.add_argument("--duration", type=float, default=20.0,
                    help="serve: seconds of Poisson arrivals (the full stream is 300)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: requests per second")
    ap.add_argument("--no-sequential", action="store_true",
                    help="serve: skip the sequential FP64 replay of the same stream")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default launch configuration instead of autotuning it first")
    ap.add_argument("--no-baseline-gpu", action="store_true",
                    help="skip the plain FP64 single-right-hand-side comparison run")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, copy a buffer of this size 5 times (counter calibration)")
    ap.add_argument("--no-bandwidth-sweep", action="store_true",
                    help="skip the working-set sweep on the largest uneven operator")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="reduce two rocprofv3 --pmc counter files (FETCH_SIZE, WRITE_SIZE) of a "
                         "'--copy-probe-mib' run to per-launch HBM bytes per kernel kind, write "
                         "profiles/traffic_pmc.json and exit")
    ap.add_argument("--copy-mib", type=int, default=1024, help="with --traffic-from: the copy probe size")
    return ap.parse_args()


def load_library():
    from paper_1606_00980_amd import build
    if not os.path.exists(build.OUT):
        build.build(verbose=False)
    from paper_1606_00980_amd import gmrf
    return gmrf


class Workload:
    """Device-resident inputs and the step function of one benchmark workload."""

    def __init__(self, name, g, torch, ctx, precond="block_jacobi"):
        from paper_1606_00980_amd import synth
        self.name, self.g, self.torch, self.ctx = name, g, torch, ctx
        self.precond = precond
        pc = g.GP_PRECOND_RB_IC0 if precond == "rb_ic0" else g.GP_PRECOND_BLOCK_JACOBI
        dev = lambda a: torch.from_numpy(a).cuda()
        self.data = None
        if name in ("batch64", "brain_fp64"):
            w = synth.brain_3d(keep_y=(name == "batch64"))
            self.ws = [w]
            self.op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
            self.ops = [self.op]
            self.B = [dev(w.B)]
            self.alpha = [w.alpha]
            if name == "batch64":
                # the data term is assembled on the device in every step from
                # tensors precomputed once (lambda = 1/sigma^2, the AR(3) draw)
                self.data = g.gp_data_create(self.op, w.X.shape[0], w.ar.shape[0], w.X, dev(w.Y))
                self.lam = dev(1.0 / w.sigma2)
                self.A = dev(np.ascontiguousarray(w.ar[None]))
                w.Y = None
                self.S = self.M = 32
                z1, z2 = w.z(self.S)
                self.v = dev(w.probes(self.M))
                self.bw, self.z1, self.z2 = dev(w.bw), dev(z1), dev(z2)
                self.bs = torch.empty((self.S, w.K, w.N), dtype=torch.float64, device="cuda")
                self.bp = torch.empty((self.M, w.K, w.N), dtype=torch.float64, device="cuda")
                self.xs = torch.zeros_like(self.bs)
                self.xp = torch.zeros_like(self.bp)
                self.opts = g.gp_opts_default(tol=1e-8, zero_guess=1, precond=pc)
                self.solves = self.S + self.M
            else:
                self.b = dev(w.bw[None].copy())
                self.x = torch.zeros_like(self.b)
                self.opts = g.gp_opts_default(tol=1e-8, precision=g.GP_PREC_FP64, zero_guess=1)
                self.solves = 1
        else:   # 16 uneven operators, 8 right-hand sides each (4 samples + 4 probes)
            self.ws = []
            for i in range(16):
                self.ws.append(synth.uneven_instance(synth.CFG_UNEVEN, i))
                log(f"operator {i + 1}/16 generated: N={self.ws[-1].N} K={self.ws[-1].K}")
            self.ops, self.B, self.alpha, self.items = [], [], [], []
            self.pert = []
            for w in self.ws:
                op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
                self.ops.append(op)
                self.B.append(dev(w.B))
                self.alpha.append(w.alpha)
                z1, z2 = w.z(4)
                v = dev(w.probes(4))
                bs = torch.empty((4, w.K, w.N), dtype=torch.float64, device="cuda")
                bp = torch.empty_like(bs)
                xs, xp = torch.zeros_like(bs), torch.zeros_like(bp)
                self.pert.append((op, dev(w.bw), dev(z1), dev(z2), v, bs, bp, xs, xp))
                self.items += [(op, 4, bs, xs), (op, 4, bp, xp)]
            self.opts = g.gp_opts_default(tol=1e-8, zero_guess=1, precond=pc)
            self.solves = 16 * 8
        self.last_stats = []
        self.trace = None

    def step(self):
        g = self.g
        if self.data is not None:
            g.gp_data_assemble(self.data, self.lam, 1, self.A, self.bw)
            g.gp_op_set_alpha(self.op, self.alpha[0])
        else:
            for op, B, a in zip(self.ops, self.B, self.alpha):
                g.gp_op_set_blocks(op, B)
                g.gp_op_set_alpha(op, a)
        if self.name == "batch64":
            g.gp_perturb_rhs(self.op, self.S, self.bw, self.z1, self.z2, self.bs)
            g.gp_probe_rhs(self.op, self.M, self.v, self.bp)
            _, self.last_stats = g.gp_solve_batch(
                self.ctx, [(self.op, self.S, self.bs, self.xs), (self.op, self.M, self.bp, self.xp)],
                self.opts, check=False)
            self.trace = g.gp_trace_reduce(self.op, self.M, self.v, self.xp, self.ws[0].K)
        elif self.name == "brain_fp64":
            _, self.last_stats = g.gp_solve(self.op, 1, self.b, self.x, self.opts, check=False)
        else:
            for (op, bw, z1, z2, v, bs, bp, xs, xp) in self.pert:
                g.gp_perturb_rhs(op, 4, bw, z1, z2, bs)
                g.gp_probe_rhs(op, 4, v, bp)
            _, self.last_stats = g.gp_solve_batch(self.ctx, self.items, self.opts, check=False)
            for (op, bw, z1, z2, v, bs, bp, xs, xp), w in zip(self.pert, self.ws):
                g.gp_trace_reduce(op, 4, v, xp, w.K)

    def autotune(self):
        """Tune the launch configuration for each (operator, right-hand-side
        count) this workload solves; later solves pick it up."""
        g = self.g
        for op, B, a in zip(self.ops, self.B, self.alpha):
            g.gp_op_set_blocks(op, B)
            g.gp_op_set_alpha(op, a)
        R = {"batch64": 32, "brain_fp64": 1, "uneven": 4}[self.name]
        out = []
        for op in self.ops:
            b = g.gp_autotune(op, R, self.opts)
            out.append({"rhs_tile": b.rhs_tile, "wg_per_cu": b.wg_per_cu,
                        "matvec": "zmarch" if b.matvec == g.GP_MATVEC_ZMARCH else "raster"})
        return out[0] if len(out) == 1 else out

    def config(self):
        if self.name == "uneven":
            Ns = [w.N for w in self.ws]
            Ks = [w.K for w in self.ws]
            return {"workload": "uneven16_ellipsoids_32x32x20_to_96x96x60_K2to10_R8",
                    "operators": 16, "N_total": int(sum(Ns)), "N_min": int(min(Ns)),
                    "N_max": int(max(Ns)), "K": Ks, "R_per_operator": 8,
                    "tol": 1e-8, "precond": self.precond, "precision": "fp32_inner_fp64_refine"}
        w = self.ws[0]
        if self.name == "brain_fp64":
            return {"workload": "brain3d_64x64x33_ellipsoid_K6_R1_fp64", "N": w.N, "K": w.K, "R": 1,
                    "tol": 1e-8, "precond": "block_jacobi", "precision": "fp64"}
        return {"workload": "brain3d_64x64x33_ellipsoid_K6_R64_fp32refine64", "N": w.N, "K": w.K,
                "R": 64, "samples": 32, "probes": 32, "tol": 1e-8, "precond": self.precond,
                "precision": "fp32_inner_fp64_refine",
                "step": "data_assemble+set_alpha+perturb_rhs(32)+probe_rhs(32)+solve_batch(64)+trace_reduce"}


def roofline(prof):
    """Roofline entry for the kernel kind with the largest total time."""
    kinds = {k: v for k, v in prof.items() if v["launches"] > 0}
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    d = kinds[dom]
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    # measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated), while
    # the kernel sources are those the counters were taken on
    traffic, detail = None, None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tf = json.load(f)
        if tf.get("kernel_source_hash") == kernel_source_hash() and dom in tf.get("kernels", {}):
            detail = tf["kernels"][dom]
            traffic = detail["bytes_per_launch"]
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "traffic_detail": detail,
            "avg_launch_us": round(d["ms"] * 1e3 / d["launches"], 2),
            "bytes_per_launch": round(d["bytes"] / d["launches"])}


KERNEL_KIND_OF = [("k_rb_red<double", "rb_red64"), ("k_rb_red", "rb_red"), ("k_rb_matvec", "rb_matvec"),
                  ("k_rb_update", "rb_update"),
                  ("k_rb_refine", "rb_refine"), ("k_rb_addsol", "rb_addsol"), ("k_rb_split", "rb_edge"),
                  ("k_rb_recover", "rb_edge"), ("k_rb_setup", "precond"),
                  ("k_matvec_zm", "matvec"), ("k_matvec", "matvec"), ("k_update", "update"),
                  ("k_refine", "refine"), ("k_addsol", "addsol"), ("k_perturb", "perturb"),
                  ("k_probe_rhs", "probe"), ("k_precond", "precond"), ("k_pack_blocks", "pack")]


def traffic_from(fetch_csv, write_csv, copy_mib):
    """Per-launch HBM traffic of each kernel kind from rocprofv3 counter files.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
    counters read for the calibration copy (copy_mib MiB read and written per
    dispatch); the launches of a kind are averaged as the profiler's
    bytes-per-launch figure is.
    """
    import csv

    def load(path):
        per = {}
        for r in csv.DictReader(open(path)):
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return per

    fetch, write = load(fetch_csv), load(write_csv)
    copy_bytes = copy_mib * float(1 << 20)

    def factor(per):
        big = [v for k, vs in per.items() if "copyBuffer" in k for v in vs if v > 0.25 * copy_bytes]
        if not big:
            raise SystemExit("no calibration copy dispatches found")
        big.sort()
        return copy_bytes / big[len(big) // 2]

    ff, fw = factor(fetch), factor(write)
    kinds = {}
    for name, vs in fetch.items():
        kind = next((kd for pat, kd in KERNEL_KIND_OF if pat in name), None)
        if kind is None:
            continue
        ws = write.get(name, [])
        d = kinds.setdefault(kind, {"fetch": [], "write": []})
        d["fetch"] += vs
        d["write"] += ws
    out = {}
    for kind, d in kinds.items():
        fb = ff * sum(d["fetch"]) / len(d["fetch"])
        wb = fw * sum(d["write"]) / max(1, len(d["write"]))
        out[kind] = {"bytes_per_launch": round(fb + wb), "fetch_bytes": round(fb), "write_bytes": round(wb),
                     "launches": len(d["fetch"])}
    res = {"kernel_source_hash": kernel_source_hash(), "fetch_factor": round(ff, 4), "write_factor": round(fw, 4),
           "copy_mib": copy_mib, "kernels": out,
           "note": "FETCH_SIZE / WRITE_SIZE per dispatch x (copy bytes / counter reading of the copy), "
                   "averaged over a kind's launches"}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def bandwidth_sweep(g, torch, ctx):
    """Matvec and update bandwidth over a working-set sweep on the largest
    uneven operator (96x96x60 grid, 60% ellipsoid fill, K = 10), R = 1..64
    right-hand sides b = b_w + N(0, 1) drawn on the device; the 256 MB MALL
    boundary is marked.  One full FP32+FP64 solve per R, profiled."""
    from paper_1606_00980_amd import synth
    w = synth.uneven_instance(synth.CFG_UNEVEN, 0, dims=(96, 96, 60), fill=0.6, K=10)
    log(f"bandwidth sweep operator: N={w.N} K={w.K}")
    op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
    g.gp_op_set_blocks(op, torch.from_numpy(w.B).cuda())
    g.gp_op_set_alpha(op, w.alpha)
    bw = torch.from_numpy(w.bw).cuda()
    opts = g.gp_opts_default(tol=1e-8, zero_guess=1)
    rows = []
    for R in (1, 4, 16, 64):
        b = torch.empty((R, w.K, w.N), dtype=torch.float64, device="cuda")
        g.gp_rng_normal(ctx, 7, 4, b.numel(), b)
        b += bw
        x = torch.empty_like(b)
        g.gp_solve(op, R, b, x, opts, check=False)
        torch.cuda.synchronize()
        g.gp_ctx_profile(ctx, True)
        _, stats = g.gp_solve(op, R, b, x, opts, check=False)
        prof = g.gp_ctx_profile_read(ctx)
        g.gp_ctx_profile(ctx, False)
        row = {"R": R, "converged": all(s_["status"] == 0 for s_ in stats)}
        for kind in ("matvec", "update", "refine"):
            v = prof[kind]
            if v["launches"]:
                gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9
                row[kind] = {"avg_us": round(v["ms"] * 1e3 / v["launches"], 2),
                             "bytes_per_launch": round(v["bytes"] / v["launches"]),
                             "GBps": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
        row["beyond_mall"] = row["matvec"]["bytes_per_launch"] > 256e6
        rows.append(row)
        log(f"bandwidth sweep R={R}: matvec {row['matvec']['GBps']} GB/s, update {row['update']['GBps']} GB/s")
        del b, x
    g.gp_op_destroy(op)
    return {"workload": f"uneven_largest_96x96x60_fill0.6_K10_N{w.N}", "N": w.N, "K": w.K,
            "mall_bytes": 256e6, "sweep": rows}


def precond_compare(g, torch, ctx, wl):
    """The step's 64-right-hand-side solve alone (graphs, no profiling) with
    each preconditioner and inner precision: time, solves/s and iterations.
    Block Jacobi runs with its autotuned launch configuration."""
    w = wl.ws[0]
    g.gp_data_assemble(wl.data, wl.lam, 1, wl.A, wl.bw)
    g.gp_op_set_alpha(wl.op, wl.alpha[0])
    g.gp_perturb_rhs(wl.op, wl.S, wl.bw, wl.z1, wl.z2, wl.bs)
    g.gp_probe_rhs(wl.op, wl.M, wl.v, wl.bp)
    out = []
    for name, pc, prec in (("rb_ic0", g.GP_PRECOND_RB_IC0, g.GP_PREC_FP32_REFINE64),
                           ("rb_ic0", g.GP_PRECOND_RB_IC0, g.GP_PREC_FP64),
                           ("block_jacobi", g.GP_PRECOND_BLOCK_JACOBI, g.GP_PREC_FP32_REFINE64),
                           ("block_jacobi", g.GP_PRECOND_BLOCK_JACOBI, g.GP_PREC_FP64)):
        o = g.gp_opts_default(tol=1e-8, zero_guess=1, precond=pc, precision=prec)
        if pc == g.GP_PRECOND_BLOCK_JACOBI:
            g.gp_autotune(wl.op, wl.S, o)
        items = [(wl.op, wl.S, wl.bs, wl.xs), (wl.op, wl.M, wl.bp, wl.xp)]
        for _ in range(3):
            g.gp_solve_batch(ctx, items, o)
        torch.cuda.synchronize()
        n = 20
        t0 = time.perf_counter()
        for _ in range(n):
            _, st = g.gp_solve_batch(ctx, items, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        out.append({"precond": name, "precision": "fp32_inner_fp64_refine" if prec else "fp64",
                    "ms_per_solve_batch": round(dt * 1e3, 3), "solves_per_s": round(wl.solves / dt, 1),
                    "inner_iters_mean": round(sum(s["inner_iters"] for s in st) / len(st), 2),
                    "max_relres": max(s["relres"] for s in st)})
        log(f"compare {out[-1]}")
    return {"what": "solve_batch of the step's 64 right-hand sides alone, tol 1e-8, zero start", "runs": out}


def ar_step(g, torch, ctx, wl, n=10):
    """The AR-coefficient step of an SVB iteration on the whole-brain operator
    (P = 3): assemble the A system from the step's 32 samples of W and the
    noise precisions, set beta, draw 32 samples of A by Algorithm 2 (device
    random vectors, red-black incomplete Cholesky, FP32 inner / FP64
    refinement to 1e-8) and form beta's posterior."""
    w = wl.ws[0]
    P = wl.A.shape[1]
    op_a = g.gp_op_create(ctx, w.mask, w.conn, P)
    try:
        S = wl.S
        ba = torch.empty((P, w.N), dtype=torch.float64, device="cuda")
        A = torch.zeros((S, P, w.N), dtype=torch.float64, device="cuda")
        beta = np.full(P, 5.0)
        # from zero each time: repeating the step with the same W, lambda and
        # random vectors would make a warm start exact
        o = g.gp_opts_default(tol=1e-8, precond=g.GP_PRECOND_RB_IC0, seed=11, zero_guess=1)

        def one():
            g.gp_data_assemble_ar(wl.data, op_a, wl.lam, S, wl.xs, ba)
            g.gp_op_set_alpha(op_a, beta)
            _, st = g.gp_sample(op_a, S, ba, None, None, A, o)
            g.gp_alpha_posterior(op_a, S, A, 10000.0, 0.1, P)
            return st

        for _ in range(2):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            st = one()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        out = {"what": "assemble the A system from 32 W samples + set beta + 32 Algorithm-2 samples of A "
                       "(red-black incomplete Cholesky, FP32 inner / FP64 refinement, tol 1e-8, from zero) "
                       "+ beta posterior", "P": P, "ms_per_step": round(dt * 1e3, 3),
               "samples_per_s": round(S / dt, 1),
               "inner_iters_mean": round(sum(x["inner_iters"] for x in st) / len(st), 2),
               "converged": all(x["status"] == 0 for x in st)}
        log(f"ar step {out}")
        return out
    finally:
        torch.cuda.synchronize()
        g.gp_op_destroy(op_a)


def cpu_baseline():
    """The oracle on the host: Algorithm 2 right-hand sides and FP64 PCG to 1e-13
    for 16 samples and 16 probes of the same operator, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import gmrf_oracle as orc
    from paper_1606_00980_amd import synth
    with threadpool_limits(limits=1):
        w = synth.brain_3d()
        z1, z2 = w.z(16)
        v = w.probes(16).astype(np.float64)
        t0 = time.perf_counter()
        g = orc.grid(w.mask, w.conn)
        Q = orc.precision(g, w.alpha, w.B)
        b = orc.perturbation_rhs(g, w.alpha, w.B, w.bw, z1, z2)
        orc.solve(Q, b, tol=1e-13)
        orc.hutchinson(g, Q, v, tol=1e-13)
        dt = time.perf_counter() - t0
    return {"value": round(32 / dt, 3), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "brain3d_64x64x33 K=6: operator assembly, 16 Algorithm-2 samples and 16 "
                      "Hutchinson probes, FP64 PCG to 1e-13 (scipy, 1 thread)",
            "seconds": round(dt, 2)}


def log(msg):
    """Progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def serve_schedule(duration, rate, nops):
    """Poisson arrivals: (arrival s, kind, operator, seed) for the serving run."""
    import numpy as np
    from paper_1606_00980_amd import synth
    rng = np.random.default_rng([synth.CFG_SERVE, 6, 0])
    t, out, i = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append((t, int(rng.integers(0, 3)), int(rng.integers(0, nops)), 10_000 + i))
        i += 1


def main_serve(args, g, torch, ctx):
    """24 resident uneven operators, Poisson requests (solve / sample / 16-probe
    trace, uniform), served with continuous batching; then the same stream
    replayed one request at a time through plain FP64 PCG."""
    from paper_1606_00980_amd import synth
    ws = []
    for i in range(24):
        ws.append(synth.uneven_instance(synth.CFG_SERVE, 100 + i))
        log(f"operator {i + 1}/24 generated: N={ws[-1].N} K={ws[-1].K}")
    ops, bws, keep = [], [], []
    for w in ws:
        op = g.gp_op_create(ctx, w.mask, w.conn, w.K)
        B = torch.from_numpy(w.B).cuda()
        g.gp_op_set_blocks(op, B)
        g.gp_op_set_alpha(op, w.alpha)
        ops.append(op)
        bws.append(torch.from_numpy(w.bw).cuda())
        keep.append(B)
    sched = serve_schedule(args.duration, args.rate, len(ops))
    cfg = g.gp_server_cfg_default(probes=16, hbm_budget=64 << 30, max_active_rhs=4096)
    # warm-up: one request of each kind on the largest operator
    big = max(range(len(ws)), key=lambda i: ws[i].N * ws[i].K)
    srv = g.gp_server_create(ctx, ops, bws, cfg)
    for kind in range(3):
        g.gp_server_submit(srv, kind, big, 1 + kind)
    g.gp_server_drain(srv, 120000)
    g.gp_server_destroy(srv)
    srv = g.gp_server_create(ctx, ops, bws, cfg)
    log(f"serving {len(sched)} requests over {args.duration} s")
    t0 = time.perf_counter()
    for (t, kind, oi, seed) in sched:
        now = time.perf_counter() - t0
        if t > now:
            time.sleep(t - now)
        g.gp_server_submit(srv, kind, oi, seed)
    g.gp_server_drain(srv, 600000)
    res = g.gp_server_poll(srv, len(sched) + 16)
    st = g.gp_server_get_stats(srv)
    g.gp_server_destroy(srv)
    ok = all(r["status"] == 0 and r["relres_max"] <= 1e-8 for r in res) and len(res) == len(sched)
    out = {
        "metric": "PCG solves/s @ rel-res 1e-8 + matvec HBM GB/s %peak; served p50/p99 latency",
        "value": round(st["solves_per_s"], 2), "unit": "solves/s", "n_gpus": 1,
        "steps": len(sched), "warmup": 3, "ms_per_step": round(st["mean_us"] / 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "serve_poisson_24_uneven_operators", "rate_per_s": args.rate,
                   "duration_s": args.duration, "requests": len(sched),
                   "mix": "uniform over solve / Algorithm-2 sample / 16-probe trace",
                   "N": [w.N for w in ws], "K": [w.K for w in ws], "tol": 1e-8},
        "serving": {"p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
                    "mean_ms": round(st["mean_us"] / 1e3, 3), "max_ms": round(st["max_us"] / 1e3, 3),
                    "requests_per_s": round(st["requests_per_s"], 2),
                    "peak_active_rhs": st["peak_active_rhs"], "all_converged": ok},
    }
    log(f"served: p50 {st['p50_us'] / 1e3:.2f} ms, p99 {st['p99_us'] / 1e3:.2f} ms")
    if not args.no_sequential:
        seq = sequential_fp64(g, torch, ctx, ws, ops, bws, sched, budget_s=max(30.0, 2 * args.duration))
        out["sequential_fp64"] = seq
    print(json.dumps(out))
    sys.stdout.flush()
    if not ok:
        sys.exit(1)


def sequential_fp64(g, torch, ctx, ws, ops, bws, sched, budget_s):
    """The same arrivals handled one request at a time by plain FP64 PCG
    (block Jacobi): latency = completion - arrival, stopped after budget_s."""
    import numpy as np
    o = g.gp_opts_default(tol=1e-8, precision=g.GP_PREC_FP64)
    lat, solves, done = [], 0, 0
    t0 = time.perf_counter()
    for (t, kind, oi, seed) in sched:
        now = time.perf_counter() - t0
        if now > budget_s:
            break
        if t > now:
            time.sleep(t - now)
        w, op = ws[oi], ops[oi]
        o.seed = seed
        if kind == 0:
            b = torch.empty((1, w.K, w.N), dtype=torch.float64, device="cuda")
            g.gp_rng_normal(ctx, seed, 4, w.K * w.N, b)
            b += bws[oi]
            x = torch.zeros_like(b)
            g.gp_solve(op, 1, b, x, o)
            solves += 1
        elif kind == 1:
            x = torch.zeros((1, w.K, w.N), dtype=torch.float64, device="cuda")
            g.gp_sample(op, 1, bws[oi], None, None, x, o)
            solves += 1
        else:
            u = torch.empty((16, w.K, w.N), dtype=torch.float64, device="cuda")
            g.gp_trace(op, 16, None, u, w.K, o)
            solves += 16
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - t)
        done += 1
    el = time.perf_counter() - t0
    lat.sort()
    pct = lambda p: lat[min(len(lat) - 1, max(0, int(np.ceil(p * len(lat))) - 1))] if lat else None
    return {"requests_done": done, "requests_offered": len(sched), "elapsed_s": round(el, 2),
            "solves_per_s": round(solves / el, 2),
            "p50_ms": round(1e3 * pct(0.5), 3) if lat else None,
            "p99_ms": round(1e3 * pct(0.99), 3) if lat else None}


def main():
    args = parse()
    if args.traffic_from:
        traffic_from(args.traffic_from[0], args.traffic_from[1], args.copy_mib)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not "
                                   "supported (one process, one MI355X)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    g = load_library()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    ctx = g.gp_ctx_create(0, stream, 0)
    if args.workload == "serve":
        main_serve(args, g, torch, ctx)
        return
    wl = Workload(args.workload, g, torch, ctx, args.precond if args.workload in ("batch64", "uneven") else "block_jacobi")
    tuned = None
    if not args.no_autotune and wl.precond != "rb_ic0":
        tuned = wl.autotune()
        log(f"autotuned: {tuned}")
    for _ in range(args.warmup):
        wl.step()
    # the timed steps: the library as it runs in production (solver rounds
    # replayed as graphs, no per-launch timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        wl.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = wl.last_stats
    # the same steps again with per-launch HIP-event timing (eager launches),
    # for the per-kernel figures and the roofline
    g.gp_ctx_profile(ctx, True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        wl.step()
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - tp0
    prof = g.gp_ctx_profile_read(ctx)
    g.gp_ctx_profile(ctx, False)
    stats = stats + wl.last_stats
    ok = all(s["status"] == 0 and s["relres"] <= 1e-8 for s in stats)
    result = {
        "metric": "PCG solves/s @ rel-res 1e-8 + matvec HBM GB/s %peak; served p50/p99 latency",
        "value": round(wl.solves * args.steps / dt, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.workload == "brain_fp64" else "f32+f64",
        "data": "synthetic",
        "config": dict(wl.config(), launch=tuned if tuned is not None else "default"),
        "roofline": roofline(prof),
        "cpu_baseline": None,
        "converged": ok,
        "max_relres": max(s["relres"] for s in stats),
        "inner_iters_mean": round(sum(s["inner_iters"] for s in stats) / len(stats), 2),
        "outer_steps_mean": round(sum(s["outer_steps"] for s in stats) / len(stats), 2),
        "value_profiled": round(wl.solves * args.steps / dt_prof, 2),
        "kernels": {k: {"launches": v["launches"],
                        "avg_us": round(v["ms"] * 1e3 / v["launches"], 2),
                        "GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)}
                    for k, v in prof.items() if v["launches"] > 0},
    }
    if wl.trace is not None:
        result["trace_estimate"] = round(wl.trace[0], 6)
    if args.workload == "batch64" and not args.no_baseline_gpu:
        base = Workload("brain_fp64", g, torch, ctx)
        base.step()
        torch.cuda.synchronize()
        n = 10
        tb = time.perf_counter()
        for _ in range(n):
            base.x.zero_()
            g.gp_solve(base.op, 1, base.b, base.x, base.opts)
        torch.cuda.synchronize()
        result["gpu_fp64_single_rhs"] = {"value": round(n / (time.perf_counter() - tb), 2),
                                         "unit": "solves/s",
                                         "what": "plain FP64 single-RHS PCG, same operator, block Jacobi"}
    if args.workload == "batch64" and not args.no_ar_step:
        result["ar_step"] = ar_step(g, torch, ctx, wl)
    if args.workload == "batch64" and not args.no_precond_compare:
        result["precond_compare"] = precond_compare(g, torch, ctx, wl)
    if args.workload == "batch64" and not args.no_bandwidth_sweep:
        result["bandwidth_sweep"] = bandwidth_sweep(g, torch, ctx)
        big = result["bandwidth_sweep"]["sweep"][-1]
        result["roofline_beyond_mall"] = {"kernel": "matvec", "R": big["R"], **big["matvec"],
                                          "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline and args.workload == "batch64":
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result))
    sys.stdout.flush()
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
