"""Time-to-k-modes of the iterative sample-and-merge POD on one MI355X.

Default workload: 1,000,000 x 4,000 FP32 snapshot matrix (16 GB; 200
travelling waves, a_j = j^-1.2, N(0, 1e-3) noise, rows centred), k = 50 modes,
c = 100 column draws per iteration (merge width 150), stop at a largest
principal angle below 1e-5 between successive estimates (or when every column
has been drawn).  One step = one whole ISMA run (set-up pass with the column
norms, sample/merge iterations until the stop rule holds, final projection
with Rayleigh-Ritz) on the matrix already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c3|c2|c4|c5]

Prints one JSON line.  `value` is the plain FP64 GPU path (FP64 matrix cores,
FP64 basis).  Beside it: the split-BF16 and FP32 merge paths, each with its
time, merge count, stop reason, singular-value error and largest principal
angle against the FP64 path's modes, and its speedup over the FP64 path
(reported only where that angle is within 1e-5); the dominant m-pass kernel
class of the FP64 path against its roof, timed with HIP events during the
timed steps; the latency of the small FP64 stages; and the FP64 CPU oracle
timed on row subsamples of the same matrix at one thread and at the host's
threads (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-k-modes & HBM GB/s: mixed-prec+adjoint vs plain FP64 at θ_max≤1e-5"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
CLASSES = ["colnorms", "draw", "gram", "gram_reduce", "chol", "tall", "svd", "project", "rr", "sign"]
MPASS = ["colnorms", "gram", "tall", "project"]
SMALL = ["draw", "gram_reduce", "chol", "svd", "rr", "sign"]
ANGLE_TOL = 1e-5

WORKLOADS = {
    # travelling waves: rows, columns, modes reported, draws per iteration,
    # waves, amplitude exponent, data seed, sampling seed
    "c3": dict(m=1_000_000, n=4_000, k=50, c=100, modes=200, alpha=1.2, dseed=1003, sseed=2003),
    "c2": dict(m=200_000, n=2_000, k=20, c=40, modes=60, alpha=1.5, dseed=1002, sseed=2002),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed steps of the FP64 path")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--other-steps", type=int, default=5, help="timed steps of each reduced-precision path")
    ap.add_argument("--workload", choices=["c3", "c2", "c5", "c4"], default="c3",
                    help="c3: travelling waves 1M x 4k, k=50, c=100 (default); c2: travelling waves 200k x 2k, "
                         "k=20, c=40; c5: 64-matrix batch, forward + gradient; c4: Alg. 3 over pinned host "
                         "blocks of 2M x 512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward-with-checkpoints plus gradient timing of each path")
    ap.add_argument("--paths", default="f64,bf16,f32",
                    help="precision paths run (f64 first; the reduced ones are compared against it)")
    ap.add_argument("--no-class-breakdown", action="store_true",
                    help="skip the per-class HIP-event pre-pass (for profiler runs)")
    ap.add_argument("--cpu-rows", type=int, default=50_000, help="rows of the oracle's larger row subsample")
    ap.add_argument("--cpu-merges", type=int, default=6, help="oracle merges timed per row subsample")
    ap.add_argument("--c5-count", type=int, default=64)
    ap.add_argument("--c4-blocks", type=int, default=32, help="blocks of 512 columns (32: the full 16,000)")
    return ap.parse_args()


def kernel_work(cls, path, m, n, k, p, r, launches):
    """Algorithmic work of one launch of a kernel class on a precision path,
    averaged over the launches of one step: (bound, amount, unit, hbm_bytes,
    peak key).

    colnorms: one pass over A (m n 4 bytes; A is stored FP32).  project:
    B = U^T A, 2 m n k flops (one launch of the pair partial + reduce counts
    half), reading A once: arithmetic intensity 2 k / 4 = 25 flop/B at k = 50,
    above the FP64 (9.8) and FP32 (19.7) ridges, so matrix-core bound (FP32 on
    the split-BF16 path, whose final step runs in FP32).
    gram: symmetric Gram m p (p+1) flops, the mean of pass 1 (reading X0 =
    [U | A(:, I)]: r basis columns at the compute width e, p - r columns of
    A at 4 bytes) and pass 2 (reading Y, m p e).  tall: the mean of
    Y = X0 T1 with T1 upper triangular (m p (p+1) flops; X0 read, Y written)
    and U = Y Z2 (2 m p r flops; Y read, U written).  The
    split-BF16 path's Gram and tall transforms are HBM bound (six bf16
    products per FP32-accurate one put the matrix-core roof at 2.5 PFLOP/s / 6
    and its ridge at 52 flop/B, above (p+1)/4).  svd: FP64 flops of the p x p
    stage (Cholesky p^3/3, R = R2 R1 p^3/3, H = R R^T p^3/3,
    tridiagonalisation 4 p^3/3, triangular inverse p^3/3, back-transformation
    2 p^2 r, Z2 p^2 r, U_R^T R p^2 r); chol: G1 = P G0 P, Cholesky, inverse."""
    e = 8 if path == "f64" else 4
    if cls == "colnorms":
        return "hbm", m * n * 4, "B", m * n * 4, None
    if cls == "project":
        b = m * n * 4 / max(launches, 1)
        return "mfma", 2.0 * m * n * k / max(launches, 1), "flop", b, "f64" if path == "f64" else "f32"
    x0 = m * (r * e + (p - r) * 4)   # bytes of X0 = [U | A(:, I)]
    if cls == "gram":
        hb = (x0 + m * p * e) // 2
        if path == "bf16":
            return "hbm", hb, "B", hb, None
        return "mfma", m * p * (p + 1), "flop", hb, path
    if cls == "tall":
        hb = (x0 + m * p * e + m * p * e + m * r * e) // 2
        if path == "bf16":
            return "hbm", hb, "B", hb, None
        return "mfma", (m * p * (p + 1) + 2 * m * p * r) / 2, "flop", hb, path
    if cls == "svd":
        return "alu", (8.0 / 3.0) * p ** 3 + 4.0 * p * p * r, "flop", 0, "f64"
    if cls == "chol":
        return "alu", (2.0 / 3.0) * p ** 3, "flop", 0, "f64"
    return None, 0, None, 0, None


TRAFFIC_FILES = {"c2": "isma_waves200k_hbm_traffic.md", "c3": "isma_waves1M_hbm_traffic.md"}
TRAFFIC_SOURCES = {"svd": ["pod_small.hip", "pod_rl.h", "pod_big.h", "pod_symeig.h", "pod_internal.h"],
                   "chol": ["pod_small.hip", "pod_rl.h", "pod_big.h", "pod_symeig.h", "pod_internal.h"],
                   "gram": ["pod_gemm.hip", "pod_internal.h"], "tall": ["pod_gemm.hip", "pod_internal.h"],
                   "project": ["pod_gemm.hip", "pod_internal.h"], "colnorms": ["pod_sample.hip", "pod_internal.h"]}


def measured_traffic(cls, path, workload):
    """HBM bytes per launch of a kernel class from the committed FETCH_SIZE /
    WRITE_SIZE summary of the workload (profiles/), scaled by the copy-kernel
    factors recorded there; None when the class was not measured on that
    path and workload, or the kernel sources changed since (sha256 prefix
    mismatch)."""
    import hashlib
    fn = TRAFFIC_FILES.get(workload)
    path_md = os.path.join(ROOT, "profiles", fn) if fn else None
    if not path_md or cls not in TRAFFIC_SOURCES or not os.path.exists(path_md):
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[cls]:
        with open(os.path.join(ROOT, "paper_1905_05107_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    cur = h.hexdigest()[:16]
    for line in open(path_md):
        parts = line.split()
        if len(parts) >= 3 and parts[0] == "traffic" and parts[1] == f"{path}:{cls}":
            kv = dict(q.split("=", 1) for q in parts[2:])
            if kv.get("sources") != cur:
                return None
            kib = float(kv["fetch_kib"]) * float(kv["fetch_factor"]) + float(kv["write_kib"]) * float(kv["write_factor"])
            return round(kib * 1024.0)
    return None


RUN_CHUNK = 8   # iterations the device-driven loop enqueues between syncs
PER_MERGE_LAUNCHES = {"gram": 2, "gram_reduce": 2, "tall": 2, "chol": 1, "svd": 1, "draw": 1}


def real_launches(cls, launches, iters):
    """Launches of a class that did work in one step: the device-driven loop
    enqueues ceil(iters / RUN_CHUNK) chunks, and the iterations past the
    stop launch kernels that return at once."""
    per = PER_MERGE_LAUNCHES.get(cls)
    if per is None:
        return launches
    enq = -(-iters // RUN_CHUNK) * RUN_CHUNK
    return max(launches - per * (enq - iters), 1)


def roofline_entry(bound, amount, avg_s, hbm_bytes, peak_key):
    if bound == "hbm":
        a = amount / avg_s / 1e9
        return {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(a / HBM_PEAK_GBS, 4)}
    if bound == "mfma":
        a = amount / avg_s / 1e12
        pk = PEAK_TFLOPS[peak_key]
        e = {"bound": "mfma", "achieved": round(a, 3), "peak": pk, "unit": "TFLOP/s", "frac": round(a / pk, 4),
             "peak_dtype": peak_key}
        if hbm_bytes:
            e["hbm_gbs"] = round(hbm_bytes / avg_s / 1e9, 1)
        return e
    a = amount / avg_s / 1e12
    return {"bound": "alu", "achieved": round(a, 6), "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
            "frac": round(a / PEAK_TFLOPS["f64"], 7), "frac_of_one_cu": round(a / (PEAK_TFLOPS["f64"] / 256), 4)}


def cpu_baseline(At, wl, iters, draws, rows_big, merges):
    """The FP64 oracle on row subsamples of the same matrix (rows_big evenly
    spaced rows and every second of them), timed at one thread and at the
    host's threads: the column-norm pass over all columns, `merges` BLOCK
    MERGEs with the GPU run's own draws (the draws do not depend on the path),
    and the final projection on 1/8 of the columns.  Extrapolated to the
    whole run: norms and projection linearly in m (and n), the merge cost as
    a + b m fitted through the two subsample sizes (a: the p x p work, b: the
    m-length work), times the run's merge count."""
    import numpy as np

    import oracle

    m, n, k = wl["m"], wl["n"], wl["k"]
    stride = max(m // rows_big, 1)
    X2 = np.asfortranarray(At[:, ::stride][:, :rows_big].cpu().numpy().T.astype(np.float64))
    X1 = np.asfortranarray(X2[::2])
    m2, m1 = X2.shape[0], X1.shape[0]
    nsub = max(n // 8, 1)
    nmerge = min(merges, len(draws))
    host_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {}
    for th in sorted({1, host_threads}):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.col_sqnorms(X2, 4)
        t_norm = time.perf_counter() - t0
        per = []
        for X in (X1, X2):
            U = np.zeros((X.shape[0], 0), order="F")
            s = np.zeros(0)
            t0 = time.perf_counter()
            for it in range(nmerge):
                U, s = oracle.merge(U, s, np.asfortranarray(X[:, draws[it]]), k)
            per.append((time.perf_counter() - t0) / nmerge)
        t0 = time.perf_counter()
        oracle.project(X2[:, :nsub], U, want_v=False)
        t_proj = time.perf_counter() - t0
        b = (per[1] - per[0]) / (m2 - m1)
        a = per[1] - b * m2
        est = t_norm * (m / m2) + iters * max(a + b * m, per[1]) + t_proj * (m / m2) * (n / nsub)
        sample_s = t_norm + nmerge * (per[0] + per[1]) + t_proj
        out[th] = (est, t_norm, per, t_proj, sample_s)
    oracle.set_threads(host_threads)
    th = max(out)
    est, t_norm, per, t_proj, sample_s = out[th]
    return {
        "value": round(est * 1e3, 1),
        "unit": "ms per time-to-k-modes (extrapolated)",
        "cores": th,
        "kind": "oracle",
        "single_thread_value": round(out[1][0] * 1e3, 1),
        "sample": (f"rows {m2} (every {stride}th) and {m1}, all {n} columns, FP64: column-norm pass "
                   f"{t_norm:.2f} s, {nmerge} merges with the run's draws at {per[0]:.3f} / {per[1]:.3f} s each, "
                   f"projection on {nsub} columns {t_proj:.2f} s at {th} threads ({sample_s:.1f} s; "
                   f"{out[1][4]:.1f} s at 1 thread); extrapolated to {m} rows, {n} columns and {iters} merges "
                   f"(merge cost a + b m through the two row counts)"),
    }


def compare_modes(U, s, U64, s64):
    """(largest relative singular-value difference, sine of the largest
    principal angle) of (U, s) against the FP64 path's (U64, s64), in FP64 on
    the device: sines from the residual U - U64 (U64^T U)."""
    import torch
    kk = min(U.shape[1], U64.shape[1])
    Ud = U[:, :kk].to(torch.float64)
    P = U64[:, :kk].T @ Ud
    R = Ud - U64[:, :kk] @ P
    sin2 = torch.linalg.eigvalsh(R.T @ R).max().clamp_min(0.0)
    rel = ((s[:kk] - s64[:kk]).abs() / s64[:kk]).max()
    return float(rel), float(sin2.sqrt())


def run_single(args):
    import torch

    import paper_1905_05107_amd as pod
    import snapgen

    wl = WORKLOADS[args.workload]
    m, n, k, c = wl["m"], wl["n"], wl["k"], wl["c"]
    p = k + min(c, n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    At = snapgen.travelling_waves(m, n, wl["modes"], wl["alpha"], 1e-3, seed=wl["dseed"], device="cuda")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    A = At.T
    kw = dict(k=k, c=c, seed=wl["sseed"], theta_tol=ANGLE_TOL)
    precs = {"f64": pod.POD_F64, "bf16": pod.POD_BF16_REFINE, "f32": pod.POD_F32}

    def step(path):
        with pod.PodContext(A, precision=precs[path], **kw) as ctx:
            ctx.run(chunk=RUN_CHUNK)
            inf = ctx.info()
            U, s, _ = ctx.project(want_v=False)
        return U, s, inf

    def classes(path, iters):
        """Per-class HIP-event time of one step (one class timed per step)."""
        per = {}
        for cls in CLASSES:
            pod.profile_enable(cls)
            step(path)
            torch.cuda.synchronize()
            per[cls] = pod.profile_read()
        pod.profile_enable(None)
        rows = {}
        for cls, (ln, ms) in per.items():
            ln = real_launches(cls, ln, iters)
            b, amt, _, hb, pk = kernel_work(cls, path, m, n, k, p, k, ln)
            e = {"ms_per_step": round(ms, 3), "launches_per_step": ln, "avg_launch_us": round(ms * 1e3 / max(ln, 1), 2)}
            if b is not None and ln > 0:
                e.update(roofline_entry(b, amt, ms / 1e3 / ln, hb, pk))
            rows[cls] = e
        return rows

    def timed(path, steps, prof_cls=None):
        for _ in range(max(args.warmup, 1)):
            step(path)
        if prof_cls:
            pod.profile_enable(prof_cls)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = step(path)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        prof = pod.profile_read() if prof_cls else None
        pod.profile_enable(None)
        return sec, out, prof

    # per-class pre-pass of the FP64 path picks its dominant m-pass class
    U64, s64, inf64 = step("f64")
    iters64 = inf64.iter
    cls64 = None if args.no_class_breakdown else classes("f64", iters64)
    dominant = "tall" if cls64 is None else max(MPASS, key=lambda q: cls64[q]["ms_per_step"])

    # timed region: the plain FP64 path, its dominant class timed live
    sec64, (U64, s64, inf64), (dl, dms) = timed("f64", args.steps, dominant)
    per_step = real_launches(dominant, dl / args.steps, inf64.iter)
    avg_s = dms / 1e3 / max(per_step * args.steps, 1)
    b, amt, _, hb, pk = kernel_work(dominant, "f64", m, n, k, p, k, per_step)
    roof = roofline_entry(b, amt, avg_s, hb, pk)
    roof["traffic"] = measured_traffic(dominant, "f64", args.workload)
    roof.update({"kernel_class": dominant, "path": "f64", "avg_launch_us": round(avg_s * 1e6, 2),
                 "launches_per_step": round(per_step, 1)})

    paths = {"f64": {"ms": round(sec64 * 1e3, 3), "merges": inf64.iter,
                     "stopped_by": pod.STOP_NAMES.get(inf64.stop_reason, "unknown")}}
    mixed_classes = None
    for path in [q for q in ("bf16", "f32") if q in args.paths.split(",")]:
        sec, (U, s, inf), _ = timed(path, args.other_steps)
        rel, ang = compare_modes(U, s, U64, s64)
        ok = ang <= ANGLE_TOL
        paths[path] = {"ms": round(sec * 1e3, 3), "merges": inf.iter,
                       "stopped_by": pod.STOP_NAMES.get(inf.stop_reason, "unknown"),
                       "sigma_rel_vs_f64": rel, "angle_vs_f64": ang,
                       "speedup_vs_f64": round(sec64 / sec, 3) if ok else None,
                       "speedup_note": None if ok else f"largest angle {ang:.2e} > {ANGLE_TOL:g}: unmeasured"}
        if path == "bf16" and not args.no_class_breakdown:
            mixed_classes = classes("bf16", inf.iter)

    # forward with reverse-pass checkpoints, then L = |A - U_k U_k^T A|_F^2 and
    # dL/dA through every merge, per path (one warm-up, one timed); each
    # reduced-precision gradient against the FP64 path's
    adjoint = None
    if not args.no_adjoint:
        def fwd_grad(path):
            with pod.PodContext(A, precision=precs[path], **kw) as ctx:
                ctx.enable_adjoint()
                ctx.run(chunk=RUN_CHUNK)
                L, dA = ctx.loss_grad()
                inf = ctx.info()
            return L, dA, inf

        adjoint = {}
        g64 = None
        for path in ["f64"] + [q for q in ("bf16", "f32") if q in args.paths.split(",")]:
            fwd_grad(path)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L, dA, inf = fwd_grad(path)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            e = {"ms": round(sec * 1e3, 3), "merges": inf.iter, "loss": L}
            if path == "f64":
                g64 = (sec, dA, float(torch.linalg.norm(dA)))
            else:
                d = float(torch.linalg.norm(dA.to(torch.float64) - g64[1])) / g64[2]
                e.update({"grad_rel_vs_f64": d, "speedup_vs_f64": round(g64[0] / sec, 3)})
            del dA
            adjoint[path] = e
        del g64

    out = {
        "metric": METRIC,
        "value": round(sec64 * 1e3, 3),
        "unit": "ms per time-to-k-modes (plain FP64 GPU path)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec64 * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"travelling waves {m}x{n} FP32 storage, {wl['modes']} modes a_j=j^-{wl['alpha']}, "
                               f"noise var 1e-3, rows centred; k={k}, c={c}, theta_tol={ANGLE_TOL:g}",
                   "m": m, "n": n, "k": k, "c": c, "merge_width": p},
        "roofline": roof,
        "paths": paths,
        "kernel_rooflines_f64": cls64,
        "kernel_rooflines_bf16": mixed_classes,
        "small_stage_us_per_launch": ({q: {"f64": cls64[q]["avg_launch_us"],
                                           "bf16": mixed_classes[q]["avg_launch_us"] if mixed_classes else None}
                                       for q in SMALL} if cls64 else None),
        "adjoint_included": adjoint is not None,
        "adjoint": adjoint,
        "adjoint_note": ("per path: forward with checkpoints plus loss and gradient dL/dA through every merge "
                         "(ms, outside the value's timed region)") if adjoint is not None else None,
        "gen_s": round(t_gen, 2),
    }
    if args.no_cpu_baseline:
        out["cpu_baseline"] = None
    else:
        with pod.PodContext(A, precision=pod.POD_F64, **kw) as ctx:
            ctx.run(n_iter=args.cpu_merges, chunk=RUN_CHUNK)
            draws = [ctx.indices(t)[0] for t in range(ctx.info().iter)]
        out["cpu_baseline"] = cpu_baseline(At, wl, inf64.iter, draws, min(args.cpu_rows, m), args.cpu_merges)
    print(json.dumps(out), flush=True)


def run_c5(args):
    """64 FP32 matrices (m ~ U[10k,100k], n ~ U[200,1000], k ~ U[4,16], c = 2k,
    s_i = exp(-i/tau), tau ~ U[3,12], Haar factors): batched ISMA to
    theta <= 1e-5 with reverse-pass checkpoints, then the gradient of
    sum_i |A_i - U_k U_k^T A_i|_F^2.  One step = batch set-up + forward +
    all gradients."""
    import torch

    import paper_1905_05107_amd as pod
    import snapgen

    specs = snapgen.batch_specs(args.c5_count, seed=1005)
    t_gen = time.perf_counter()
    mats = [snapgen.batch_matrix_torch(it, "cuda").T for it in specs]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    kws = [dict(k=it.k, c=it.c, seed=2005 + i, theta_tol=1e-5) for i, it in enumerate(specs)]
    nbytes = sum(A.shape[0] * A.shape[1] * 4 for A in mats)

    def step(prec):
        t0 = time.perf_counter()
        with pod.Batch(mats, [dict(kw, precision=prec) for kw in kws]) as b:
            b.enable_adjoint()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rounds = b.run()
            t2 = time.perf_counter()
            L = sum(li for li, _ in b.loss_grad_all())
            torch.cuda.synchronize()
            t3 = time.perf_counter()
        return t3 - t0, t1 - t0, t2 - t1, t3 - t2, L, rounds

    for _ in range(max(args.warmup, 1)):
        step(pod.POD_F32)
    res = [step(pod.POD_F32) for _ in range(args.steps)]
    tot = sum(r[0] for r in res) / len(res)
    f64 = [step(pod.POD_F64) for _ in range(max(1, min(args.steps, 3)))]
    tot64 = sum(r[0] for r in f64) / len(f64)
    out = {
        "metric": METRIC, "value": round(tot * 1e3, 3),
        "unit": "ms per batch of 64 (set-up + forward to theta<=1e-5 + gradient), FP32 merges",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tot * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(mats)} FP32 matrices, m~U[10k,100k], n~U[200,1000], k~U[4,16], "
                               "c=2k, s_i=exp(-i/tau), tau~U[3,12]; loss sum |A-U_kU_k^TA|_F^2 with gradient",
                   "total_bytes": nbytes},
        "breakdown_ms": {"setup": round(sum(r[1] for r in res) / len(res) * 1e3, 3),
                         "forward": round(sum(r[2] for r in res) / len(res) * 1e3, 3),
                         "gradient": round(sum(r[3] for r in res) / len(res) * 1e3, 3)},
        "rounds": res[-1][5], "loss": res[-1][4],
        "fp64_path_ms": round(tot64 * 1e3, 3), "speedup_vs_fp64_path": round(tot64 / tot, 3),
        "adjoint_included": True, "gen_s": round(t_gen, 2), "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_c4(args):
    """Alg. 3 over host blocks: travelling waves with 200 modes, a_j = j^-1.2,
    noise variance 1e-3, rows centred (generator pre-pass), m = 2M, blocks of
    512 columns (the last of 128 at n = 16,000); k = 40, c = 80, FP32 merges.

    The snapshots are generated once into device memory (untimed: 128 GB at
    the full size) and reach the library as host blocks through a ring of
    2 G pinned buffers (G = 4): a producer thread copies the next group of G
    blocks to the free half of the ring (device to host, its own stream)
    while the library copies the current group to the device (one call,
    which overlaps the copy of each block with the compute of the one
    before) and runs ISMA on it.  The timed region
    is the whole pass with the producer running.  Reported beside it: the
    host-link rate of the library's copies, the same blocks from device
    memory (compute only) and the copy/compute overlap inside the library
    (its wall time against copy + compute)."""
    import threading

    import torch

    import paper_1905_05107_amd as pod
    import snapgen

    m, w = 2_000_000, 512
    n = min(16_000, w * args.c4_blocks)
    bounds = [(j, min(j + w, n)) for j in range(0, n, w)]
    t_gen = time.perf_counter()
    gen = snapgen.WaveBlocks(m, n, 200, 1.2, 1e-3, seed=1004, device="cuda")
    Adev = torch.empty((n, m), dtype=torch.float32, device="cuda")   # row j = snapshot j
    for j0, j1 in bounds:
        Adev[j0:j1].copy_(gen.block(j0, j1))
    del gen
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    G = 4
    slots = [torch.empty((w, m), dtype=torch.float32, pin_memory=True) for _ in range(2 * G)]
    pstream = torch.cuda.Stream()
    kw = dict(k=40, c=80, seed=2004, theta_tol=1e-5, precision=pod.POD_F32)

    def fill(bs, half):
        """Blocks bs into the buffers of half `half` of the ring (producer side)."""
        with torch.cuda.stream(pstream):
            for i, b in enumerate(bs):
                j0, j1 = bounds[b]
                slots[G * half + i][:j1 - j0].copy_(Adev[j0:j1], non_blocking=True)
        pstream.synchronize()

    pairs = [list(range(b, min(b + G, len(bounds)))) for b in range(0, len(bounds), G)]

    def streamed():
        fill(pairs[0], 0)
        prod_s = 0.0
        with pod.Incremental(m, w, **kw) as inc:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i, bs in enumerate(pairs):
                th = None
                if i + 1 < len(pairs):
                    def producer(bs_next=pairs[i + 1], pair=(i + 1) & 1):
                        nonlocal prod_s
                        tp = time.perf_counter()
                        fill(bs_next, pair)
                        prod_s += time.perf_counter() - tp
                    th = threading.Thread(target=producer)
                    th.start()
                views = [slots[G * (i & 1) + q][:bounds[b][1] - bounds[b][0]] for q, b in enumerate(bs)]
                inc.add_host_blocks(views)
                if th is not None:
                    th.join()
            U, s = inc.result()
            torch.cuda.synchronize()
            return time.perf_counter() - t0, inc.info(), prod_s

    def resident():
        """The same blocks from device memory: compute only."""
        with pod.Incremental(m, w, **kw) as inc:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j0, j1 in bounds:
                inc.add_block(Adev[j0:j1].T)
            inc.result()
            torch.cuda.synchronize()
            return time.perf_counter() - t0

    for _ in range(max(args.warmup, 0)):
        streamed()
    res = [streamed() for _ in range(args.steps)]
    t_s = sum(r[0] for r in res) / len(res)
    info, prod_s = res[-1][1], res[-1][2]
    t_r = resident()
    copy_s = info.copy_ms / 1e3
    wall_s = info.wall_ms / 1e3
    link = info.host_bytes / copy_s / 1e9 if copy_s > 0 else None
    # copy/compute overlap inside the library: the share of the shorter of
    # (copy, compute) hidden behind the other
    overlap = (copy_s + t_r - wall_s) / min(copy_s, t_r) if copy_s > 0 and t_r > 0 else None
    out = {
        "metric": METRIC, "value": round(t_s * 1e3, 2),
        "unit": "ms per incremental POD over host-resident blocks (one pass), FP32 merges",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_s * 1e3, 2),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"travelling waves {m}x{n} FP32 (200 modes, a_j=j^-1.2), blocks of {w} columns from a "
                               f"ring of {2 * G} pinned host buffers filled by a producer thread, k=40, c=80, theta_tol=1e-5",
                   "blocks": len(bounds), "m": m, "n": n},
        "host_bytes": info.host_bytes, "host_link_gbs": round(link, 2) if link else None,
        "copy_ms": round(info.copy_ms, 2), "library_wall_ms": round(info.wall_ms, 2),
        "device_resident_ms": round(t_r * 1e3, 2), "producer_ms": round(prod_s * 1e3, 2),
        "copy_compute_overlap": round(overlap, 3) if overlap is not None else None,
        "gen_setup_s": round(t_gen, 2), "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "single-GPU build: the hot path runs on one GPU; "
                                   "--gpus above 1 is not supported", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "c4":
        return run_c4(args)
    return run_single(args)


if __name__ == "__main__":
    main()
