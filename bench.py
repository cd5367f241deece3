#!/usr/bin/env python3
"""Benchmark: coupled high-order Newton-Schulz / Richardson SPD solves on one MI355X.

Headline: one "step" is one whole solve (richardson_ns_solve through the C ABI)
of a seeded synthetic system already resident in HBM: N = 4096, kappa = 1e4,
A = Q diag(lam) Q^T, order-8 factorized Newton-Schulz (I+F)(I+F^2)(I+F^4) in
float64 until the ||F|| rounding floor, coupled Richardson updates and float64
refinement to a relative residual of 1e-12.

Also measured (extra keys of the same JSON line): the mixed-precision path
(bf16 powers, float32 residual / G-side, float64 Richardson) on the same
system; the N = 8192, kappa = 1e6 composite (double Newton-Schulz, order 8)
workload in mixed precision next to the same solve in float64; a batch of
2048 harmonic-regressor Gram systems of uneven size in one persistent launch;
a serving run (Poisson arrivals, sizes 32..2048) with p50/p99 latency; the
program library and the composite variants on the headline system; the
N = 64 fixed-step workload (eager, captured graph, 4096-seed batch); and a
three-frequency analogue of the paper's last comparison.

The float64 GEMM's roofline comes from per-launch HIP events recorded by the
library on its stream during the timed region; the CPU baseline is the oracle
timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# Hardware queues per process (HIP's default is 4): the serving leg runs its
# single solves on 12 streams, which would otherwise share 4 queues and
# serialise.  Read by the HIP runtime when it initialises, i.e. before torch
# touches the GPU.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

from paper_2008_11480_amd import inputs  # noqa: E402

# f32_split: float32-class products of split half-precision operands, three
# fp16 MFMA products each, so their ceiling is a third of the 2.5 PFLOP/s
# fp16 peak (frac_of_peak = fp16 matrix-core utilisation).
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f32_split": 2500.0 / 3}
GEMM_KERNEL_SRC = os.path.join(ROOT, "paper_2008_11480_amd", "csrc", "nsr_gemm_f64.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_f64_spd4096_traffic.json")
KIND = {"f64": 1, "f32": 2, "bf16": 3, "f32_split": 4}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per GEMM launch from the committed rocprofv3 PMC summary,
    or None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash(GEMM_KERNEL_SRC):
        return None
    return t.get("bytes_per_launch")


def blas_threads():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        n = [i.get("num_threads", 0) for i in info if i.get("user_api") == "blas"]
        return int(max(n)) if n else os.cpu_count()
    except Exception:
        return os.cpu_count()


def cpu_baseline(sysm, order, steps_per_solve, refine_steps):
    """Oracle (numpy float64) on a bounded sample: one order-`order` squaring
    step (its residual included) plus one Richardson update, on the same
    N = 4096 system; scaled to solves/s with the GPU solve's step count."""
    import oracle
    a, b = sysm.A, sysm.b
    alpha = oracle.alpha_frobenius(a)
    g = np.eye(a.shape[0]) / alpha
    theta = g @ b
    t0 = time.perf_counter()
    g = oracle.ns_step(a, g, order, "squaring")
    theta, _ = oracle.richardson_update(a, b, theta, g)
    f = oracle.residual(a, g)
    t_step = time.perf_counter() - t0
    t0 = time.perf_counter()
    theta, _ = oracle.richardson_update(a, b, theta, g)
    t_ref = time.perf_counter() - t0
    del f
    t_solve = steps_per_solve * t_step + (refine_steps + 1) * t_ref
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": blas_threads(),
        "kind": "oracle",
        "sample": (f"one oracle Newton-Schulz step (order {order}, squaring form, "
                   f"{oracle.form_mmm(order, 'squaring')} mmm with its residual) plus one "
                   f"Richardson update at N={a.shape[0]} took {t_step:.2f} s; scaled to the "
                   f"GPU solve's {steps_per_solve} steps + {refine_steps + 1} residual "
                   f"evaluations"),
    }


def cpu_cholesky(sysm):
    """The practitioner's CPU comparator (not the oracle): LAPACK Cholesky
    factorisation and solve (dpotrf + dpotrs through scipy) of the same
    N = 4096 system on the host's BLAS threads."""
    import scipy.linalg
    a, b = sysm.A, sysm.b
    t0 = time.perf_counter()
    c = scipy.linalg.cho_factor(a, lower=True, check_finite=False)
    x = scipy.linalg.cho_solve(c, b, check_finite=False)
    dt = time.perf_counter() - t0
    rel = float(np.linalg.norm(b - a @ x) / np.linalg.norm(b))
    return {"value": 1.0 / dt, "unit": "solves/s", "seconds": dt, "cores": blas_threads(),
            "kind": "LAPACK Cholesky (dpotrf + dpotrs), comparator, not the oracle",
            "rel_resid": rel}


def measure(torch, solver, b, theta, kw, steps, warmup, label):
    """Warm up, then time `steps` whole solves with per-launch GEMM events."""
    for i in range(warmup):
        rep = solver.solve(b, theta, **kw)
        log(f"{label} warmup {i}: ns_steps={rep.ns_steps} refine={rep.refine_steps} "
            f"rel_resid={rep.rel_resid:.2e}")
    torch.cuda.synchronize()
    solver.timing(True)
    solver.timing_reset()
    lat, reps = [], []
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    for i in range(steps):
        t0 = time.perf_counter()
        rep = solver.solve(b, theta, **kw)
        lat.append(time.perf_counter() - t0)     # solve() returns after a stream sync
        reps.append(rep)
        log(f"{label} step {i}: {lat[-1] * 1e3:.1f} ms ns_steps={rep.ns_steps} mmm={rep.mmm} "
            f"rel_resid={rep.rel_resid:.2e}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_begin
    gemm = {}
    for name, kind in KIND.items():
        cnt, ms, fl = solver.timing_read(kind)
        if cnt:
            avg = ms / cnt
            tf = fl / cnt / (avg * 1e-3) / 1e12
            gemm[name] = {"launches": cnt, "avg_launch_ms": avg, "tflops": tf,
                          "flop_per_launch": fl / cnt,
                          "frac_of_peak": tf / PEAK_TFLOPS[name],
                          "share_of_solve_time": ms / (t_total * 1e3)}
    solver.timing(False)
    lat_ms = np.array(lat) * 1e3
    return {
        "solves_per_s": steps / t_total,
        "ms_per_solve": t_total / steps * 1e3,
        "latency_ms_p50": float(np.percentile(lat_ms, 50)),
        "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "last": reps[-1],
        "gemm": gemm,
    }


def report_of(rep):
    return {"ns_steps": rep.ns_steps, "refine_steps": rep.refine_steps, "mmm": rep.mmm,
            "ns_stop": rep.ns_stop, "refine_stop": rep.refine_stop,
            "rel_resid_reported": rep.rel_resid}


def run_composite(torch, nsr, steps, warmup):
    """N = 8192, kappa = 1e6: composite (double Newton-Schulz) order 8 and the
    factorized order 8, mixed precision, next to the composite in float64."""
    w = inputs.WORKLOADS["spd8192_k1e6_dns8"]
    n = w["n"]
    log(f"generating spd8192_k1e6_dns8 on the GPU: N={n} kappa={w['kappa']:g}")
    A, b, lam, Q = inputs.spd_qlq_device(n, w["kappa"], w["seed"])
    theta_star = Q @ ((Q.T.contiguous() @ b) / lam)
    out = {"workload": "spd8192_k1e6_dns8", "n": n, "kappa": w["kappa"], "order": 8}
    theta = torch.zeros_like(b)
    for label, prec, form in (("mixed_composite", nsr.PREC_MIXED_BF16, "composite_double"),
                              ("mixed_factorized", nsr.PREC_MIXED_BF16, "squaring"),
                              ("mixed_split_composite", nsr.PREC_MIXED_SPLIT,
                               "composite_double"),
                              ("mixed_split_factorized", nsr.PREC_MIXED_SPLIT, "squaring"),
                              ("fp64_composite", nsr.PREC_FP64, "composite_double")):
        solver = nsr.Solver(n, precision=prec, composite=form == "composite_double")
        solver.bind(A)
        kw = dict(order=8, form=form, k_max=64, resid_tol=1e-10, refine_max=100)
        m = measure(torch, solver, b, theta, kw, steps if prec != nsr.PREC_FP64 else 1,
                    1 if prec != nsr.PREC_FP64 else 0, label)
        rel = float(torch.linalg.norm(b - A @ theta) / torch.linalg.norm(b))
        fwd = float(torch.linalg.norm(theta - theta_star) / torch.linalg.norm(theta_star))
        out[label] = {"solves_per_s": m["solves_per_s"], "ms_per_solve": m["ms_per_solve"],
                      "rel_resid": rel, "fwd_err_vs_closed_form": fwd,
                      "gemm": m["gemm"], **report_of(m["last"])}
        del solver
        torch.cuda.empty_cache()
    for label in ("mixed_composite", "mixed_split_composite"):
        out[f"speedup_{label}_vs_fp64_composite"] = (
            out[label]["solves_per_s"] / out["fp64_composite"]["solves_per_s"])
    return out


def run_comparisons(torch, nsr, A, b, sysm, n, resid_tol, k_max):
    """Newton-Schulz variants of Sections 5-6 and Remark 2 on the headline
    system (float64): steps, products, time and accuracy of each."""
    variants = [
        ("classical order 8 (squaring)", dict(order=8, form="squaring"), None),
        ("double NS order 8 (Section 5.1)", dict(order=8, form="composite_double"), None),
        ("double NS order 8 + accelerator q=2 (eq. ttk1)",
         dict(order=8, form="composite_double", accel_q=2), None),
        ("[sri] order 8 (Remark 2)", dict(order=8, form="sri"), None),
        ("general composite n=8, rates (2, 4) (eqs. gkgen1-ga1)",
         dict(order=8, form="composite_general"), (2, 4)),
    ]
    s = nsr.Solver(n, composite=2)
    s.bind(A)
    out = []
    for name, kw, rates in variants:
        th = torch.zeros_like(b)
        times = []
        for rep_i in range(2):
            if rates:
                s.init_scale()
                s.set_composite_rates(rates)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = s.solve(b, th, resid_tol=resid_tol, k_max=k_max, refine_max=64,
                          raise_on_error=False, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        x = th.cpu().numpy()
        rel = float(np.linalg.norm(sysm.b - sysm.A @ x) / np.linalg.norm(sysm.b))
        out.append({"variant": name, "ms_per_solve": times[-1] * 1e3, "ns_steps": rep.ns_steps,
                    "refine_steps": rep.refine_steps, "mmm": rep.mmm, "rel_resid": rel,
                    "status": rep.status})
        log(f"compare {name}: {times[-1] * 1e3:.1f} ms ns_steps={rep.ns_steps} mmm={rep.mmm} "
            f"rel_resid={rel:.2e}")
    s.close()
    return out


def run_preconditioning(torch, nsr, A, b, sysm, n, resid_tol, k_max):
    """Section 2 options at N = 4096 (float64, order 8): the diagonal
    preconditioner S = diag(A) against alpha = ||A||_F on a diagonally
    dominant system whose diagonal spans three decades (inputs.spd_jacobi),
    and the initial series of order h (eq. g01) on the headline system."""
    def timed(s, bb, **kw):
        th = torch.zeros_like(bb)
        times = []
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = s.solve(bb, th, order=8, resid_tol=resid_tol, k_max=k_max, refine_max=64,
                          raise_on_error=False, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return rep, th, times[-1]

    out = {"diagonal": {"workload": f"spd_jacobi{n}_3decades", "n": n}, "initial_series": {
        "workload": "spd4096_k1e4_o8"}}
    jac = inputs.spd_jacobi(n, seed=9)
    Aj = torch.from_numpy(jac.A).to("cuda")
    bj = torch.from_numpy(jac.b).to("cuda")
    s = nsr.Solver(n)
    s.bind(Aj)
    for name, scale in (("frobenius", nsr.SCALE_FROBENIUS), ("diag", nsr.SCALE_DIAG)):
        rep, th, dt = timed(s, bj, scale=scale)
        x = th.cpu().numpy()
        out["diagonal"][name] = {
            "ms_per_solve": dt * 1e3, "ns_steps": rep.ns_steps, "refine_steps": rep.refine_steps,
            "mmm": rep.mmm, "status": rep.status,
            "rel_resid": float(np.linalg.norm(jac.b - jac.A @ x) / np.linalg.norm(jac.b))}
        log(f"preconditioner {name}: {dt * 1e3:.1f} ms ns_steps={rep.ns_steps} mmm={rep.mmm}")
    s.bind(A)
    for h, p, w_ in ((1, 0, 0), (2, 1, 1), (4, 1, 2)):
        kw = {} if h == 1 else dict(init_order=h, init_p=p, init_w=w_)
        rep, th, dt = timed(s, b, **kw)
        x = th.cpu().numpy()
        out["initial_series"][f"h{h}"] = {
            "ms_per_solve": dt * 1e3, "ns_steps": rep.ns_steps, "refine_steps": rep.refine_steps,
            "mmm": rep.mmm, "status": rep.status,
            "rel_resid": float(np.linalg.norm(sysm.b - sysm.A @ x) / np.linalg.norm(sysm.b))}
        log(f"initial series h={h}: {dt * 1e3:.1f} ms ns_steps={rep.ns_steps} mmm={rep.mmm}")
    s.close()
    return out


def run_fig4_analogue(torch, nsr, steps=7):
    """Synthetic analogue of the paper's last comparison (Section 7): three
    close frequencies (N = 6, kappa ~ 4e3); per-step parameter error of the
    Richardson iteration with the third-order accelerator (double NS n = 3,
    q = 3, eq. ttk1) and of classical eighth-order Newton-Schulz coupled with
    Richardson, float64."""
    sysm = inputs.harmonic_three()
    theta_star = np.linalg.solve(sysm.A, sysm.b)
    A = torch.from_numpy(sysm.A).to("cuda")
    b = torch.from_numpy(sysm.b).to("cuda")
    s = nsr.Solver(6, composite=1)
    s.bind(A)
    rows = []
    for k in range(1, steps + 1):
        errs = {}
        for name, kw in (("accelerator_q3_n3", dict(order=3, form="composite_double", accel_q=3)),
                         ("classical_n8", dict(order=8, form="squaring"))):
            th = torch.zeros_like(b)
            s.solve(b, th, k_max=k, floor_detect=False, refine_max=0, resid_tol=0.0,
                    raise_on_error=False, **kw)
            x = th.cpu().numpy()
            errs[name] = float(np.linalg.norm(x - theta_star) / np.linalg.norm(theta_star))
        rows.append({"step": k, **errs})
    s.close()
    return {"workload": "harmonic_three_T30_w0.40-0.43-0.47", "n": 6,
            "kappa": float(np.linalg.cond(sysm.A)), "param_rel_error": rows}


def run_small_fixed(torch, nsr, reps=300):
    """The N = 64, kappa = 100 workload (order-4 squaring, exactly 12 coupled
    steps, refinement to 1e-13), float64: eager launches versus the captured
    graph of the 12 steps (same kernels, bit-identical results)."""
    w = inputs.WORKLOADS["spd64_k1e2_o4"]
    sysm = inputs.spd_qlq(w["n"], w["kappa"], w["seed"])
    A = torch.from_numpy(sysm.A).to("cuda")
    b = torch.from_numpy(sysm.b).to("cuda")
    s = nsr.Solver(w["n"], composite=0)
    s.bind(A)
    kw = dict(order=w["order"], form="squaring", k_max=w["k_max"], floor_detect=False,
              resid_tol=w["resid_tol"])
    out = {"workload": "spd64_k1e2_o4", "n": w["n"], "steps": w["k_max"]}
    ref = None
    for mode in ("eager", "graph"):
        th = torch.zeros_like(b)
        for _ in range(5):
            rep = s.solve(b, th, graph=(mode == "graph"), **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rep = s.solve(b, th, graph=(mode == "graph"), **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        x = th.cpu().numpy()
        if ref is None:
            ref = x
        out[mode] = {"us_per_solve": dt * 1e6, "solves_per_s": 1.0 / dt,
                     "rel_resid": float(np.linalg.norm(sysm.b - sysm.A @ x)
                                        / np.linalg.norm(sysm.b)),
                     "refine_steps": rep.refine_steps, "identical_to_eager": bool(
                         np.array_equal(x, ref))}
        log(f"N=64 fixed 12 steps, {mode}: {dt * 1e6:.0f} us/solve")
    s.close()
    # One system through the batched kernel (systems with N <= 64 solve in
    # one workgroup with every iteration matrix in LDS): the latency of a
    # single solve without host round trips between steps.
    bopts = dict(order=w["order"], k_max=w["k_max"], floor_detect=False,
                 resid_tol=w["resid_tol"], refine_max=20)
    B1 = nsr.Batch(max_n=w["n"], max_count=1, slots=1, precision=nsr.PREC_FP64)
    B1.set_launch(8, 1)
    th1 = torch.zeros_like(b)
    for _ in range(5):
        B1.poll_arrays(B1.submit([A], [b], [th1], **bopts), wait=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        t1 = B1.submit([A], [b], [th1], **bopts)
        r1 = B1.poll_arrays(t1, wait=True)
    dt1 = (time.perf_counter() - t0) / reps
    tl1, _ = B1.timeline(t1)
    x1 = th1.cpu().numpy()
    out["batch_of_one"] = {
        "us_per_solve": dt1 * 1e6,
        "device_us": float(np.nanmax(tl1[0, [1, 3]]) - np.nanmin(tl1[0, [0, 2]])),
        "rel_resid": float(np.linalg.norm(sysm.b - sysm.A @ x1) / np.linalg.norm(sysm.b)),
        "ns_steps": int(r1["ns_steps"][0]), "refine_steps": int(r1["refine_steps"][0])}
    log(f"N=64 fixed 12 steps, batch of one: {dt1 * 1e6:.0f} us/solve")
    # The same workload for 4096 independent seeds in one float64 batch
    # (persistent kernel, every solve on one workgroup, no host round trips).
    count = 4096
    systems = [inputs.spd_qlq(w["n"], w["kappa"], 1000 + i) for i in range(count)]
    P = nsr.PackedSystems.from_host([x.A for x in systems], [x.b for x in systems])
    B = nsr.Batch(max_n=w["n"], max_count=count,
                  slots=min(count, 8 * torch.cuda.get_device_properties(0).multi_processor_count),
                  precision=nsr.PREC_FP64)
    waves, groups, _ = B.autotune([P.A_of(i) for i in range(count)],
                                  [P.b_of(i) for i in range(count)],
                                  [P.theta_of(i) for i in range(count)], **bopts)
    times, dev = [], []
    for i in range(4):
        P.theta.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = B.submit_packed(P, **bopts)
        rep = B.poll_arrays(t, wait=True)
        if i:
            times.append(time.perf_counter() - t0)
            tl, _ = B.timeline(t)
            dev.append((np.nanmax(tl[:, [1, 3]]) - np.nanmin(tl[:, [0, 2]])) * 1e-6)
    mk, mk_dev = float(np.median(times)), float(np.median(dev))
    rel = max(float(np.linalg.norm(x.b - x.A @ P.theta_of(i).cpu().numpy()) / np.linalg.norm(x.b))
              for i, x in enumerate(systems[:64]))
    flop = float(rep["gemm_flop"].sum())
    out["batch4096_fp64"] = {
        "count": count, "launch": {"waves_per_group": waves, "groups": groups},
        "makespan_ms": mk * 1e3, "device_ms": mk_dev * 1e3, "solves_per_s": count / mk,
        "us_per_solve": mk / count * 1e6, "alg_tflops": flop / mk / 1e12,
        "alg_tflops_device": flop / mk_dev / 1e12,
        "ok": int((rep["status"] == nsr.NS_OK).sum()), "rel_resid_max_first64": rel,
        "ns_steps": int(rep["ns_steps"][0])}
    log(f"N=64 x 4096 float64 batch: {mk * 1e3:.1f} ms ({count / mk:.0f} solves/s), "
        f"device {mk_dev * 1e3:.2f} ms")
    return out


def release(torch):
    """Drop the finished leg's objects and return cached device memory."""
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def timeline_summary(tl, ns):
    """Critical-path view of a batch from the device timeline (ms)."""
    f32 = tl[:, 1] - tl[:, 0]
    f64 = tl[:, 3] - tl[:, 2]
    esc = ~np.isnan(tl[:, 2])
    end = np.nanmax(tl[:, [1, 3]])
    busy = np.nansum(f32) + np.nansum(f64)
    big = np.argsort(-np.nan_to_num(f32))[:3]
    return {
        "f32_pass_end": float(np.nanmax(tl[:, 1])) / 1e3,
        "f64_pass": [float(np.nanmin(tl[esc, 2])) / 1e3, float(np.nanmax(tl[esc, 3])) / 1e3]
        if esc.any() else None,
        "end": float(end) / 1e3,
        "longest_f32_solves": [{"n": int(ns[i]), "ms": float(f32[i]) / 1e3} for i in big],
        "longest_f64_solve_ms": float(np.nanmax(f64)) / 1e3 if esc.any() else None,
        # solves in flight on average (float32 and float64 attempts)
        "mean_concurrent": float(busy / end) if end > 0 else None,
    }


def run_batch(torch, nsr, reps_timed):
    """2048 harmonic-regressor Gram systems, m ~ U{8..128} (N = 16..256), in
    one persistent launch per solve of the whole batch: float32 MFMA order 4,
    float64 refinement to 1e-10, float64 re-solve where float32 cannot."""
    count = 2048
    log(f"generating {count} harmonic Gram systems (seed 4)")
    systems = inputs.harmonic_batch(count, seed=4)
    # Systems back to back in device memory (a submission's pointer arrays
    # then come from numpy, not from one call per tensor).
    P = nsr.PackedSystems.from_host([s.A for s in systems], [s.b for s in systems])
    B = nsr.Batch(max_n=256, max_count=count,
                  slots=min(count, 8 * torch.cuda.get_device_properties(0).multi_processor_count))
    opts = dict(order=4, resid_tol=1e-10, refine_max=100)
    waves, groups, tune_ms = B.autotune([P.A_of(i) for i in range(count)],
                                        [P.b_of(i) for i in range(count)],
                                        [P.theta_of(i) for i in range(count)], **opts)
    log(f"batch autotune: {waves} waves/workgroup, {groups} workgroups ({tune_ms:.1f} ms)")

    def timed(pk, o, bt=None):
        bt = bt or B
        times, dev = [], []
        for i in range(reps_timed + 1):
            pk.theta.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t = bt.submit_packed(pk, **o)
            r = bt.poll_arrays(t, wait=True)
            dt = time.perf_counter() - t0
            tl, _ = bt.timeline(t)
            if i > 0:
                times.append(dt)
                dev.append((np.nanmax(tl[:, [1, 3]]) - np.nanmin(tl[:, [0, 2]])) * 1e-6)
            log(f"batch {'warmup' if i == 0 else 'run'} {i}: {dt * 1e3:.1f} ms")
        return float(np.median(times)), float(np.median(dev)), r, tl

    def rel_resid(pk):
        return np.array([float(np.linalg.norm(s.b - s.A @ pk.theta_of(i).cpu().numpy())
                               / np.linalg.norm(s.b)) for i, s in enumerate(systems)])

    mk, mk_dev, rep, tl = timed(P, opts)
    flop = float(rep["gemm_flop"].sum())
    # Per N bucket: the float32 attempt's algorithmic rate per workgroup
    # against the two ceilings of one attempt among those in flight at once:
    # its share of the float32 MFMA peak, and its share of HBM bandwidth times the streamed
    # intensity of an n x n product (read X, Y, write D in float32: n / 6
    # flop/B).
    ns_arr = np.array([s.n for s in systems])
    dur = (tl[:, 1] - tl[:, 0]) * 1e-6          # float32 attempt, s
    # concurrency: float32 attempts running at once on average over the pass
    span32 = (np.nanmax(tl[:, 1]) - np.nanmin(tl[:, 0])) * 1e-6
    conc = max(1.0, float(np.nansum(dur)) / span32) if span32 > 0 else float(groups)
    share_mfma = 157.3e12 / conc
    share_hbm = 8.0e12 / conc
    per_bucket = []
    for lo, hi in ((16, 64), (64, 128), (128, 192), (192, 257)):
        sel = (ns_arr >= lo) & (ns_arr < hi) & np.isfinite(dur) & (dur > 0)
        if not sel.any():
            continue
        n_mid = float(np.median(ns_arr[sel]))
        f32_flop = rep["mmm"][sel] * 2.0 * ns_arr[sel].astype(float) ** 3
        rate = f32_flop / dur[sel]
        per_bucket.append({
            "n": [lo, hi - 1], "systems": int(sel.sum()),
            "f32_attempt_ms_p50": float(np.median(dur[sel]) * 1e3),
            "gflops_per_workgroup_p50": float(np.median(rate) / 1e9),
            "concurrent_attempts": conc,
            "mfma_share_gflops": share_mfma / 1e9,
            "hbm_stream_bound_gflops": share_hbm * n_mid / 6 / 1e9,
        })
    okm = rep["status"] == nsr.NS_OK
    ok, esc = int(okm.sum()), int((rep["precision"] == nsr.PREC_FP64).sum())
    rel = rel_resid(P)
    steps = rep["ns_steps"]
    # Variant: the paper's own scalar preconditioner alpha = ||A||_inf / 2 + eps
    # (Section 2), same launch shape.
    opts_inf = dict(opts, scale=nsr.SCALE_INF_HALF, eps=1e-9)
    mk_inf, mk_inf_dev, rep_inf, _ = timed(P, opts_inf)
    steps_inf = rep_inf["ns_steps"]
    ok_inf = rep_inf["status"] == nsr.NS_OK
    rel_inf = rel_resid(P)
    log(f"batch inf_half scaling: {mk_inf * 1e3:.1f} ms, ns_steps p50 "
        f"{np.median(steps_inf):.0f} (frobenius {np.median(steps):.0f})")
    # The same batch in plain float64 (every system solved in float64 from
    # the start), with its own autotuned launch: the mixed batch's speedup.
    B64 = nsr.Batch(max_n=256, max_count=count,
                    slots=min(count, 8 * torch.cuda.get_device_properties(0).multi_processor_count),
                    precision=nsr.PREC_FP64)
    w64, g64, _ = B64.autotune([P.A_of(i) for i in range(count)], [P.b_of(i) for i in range(count)],
                               [P.theta_of(i) for i in range(count)], **opts)
    mk64, mk64_dev, rep64, _ = timed(P, opts, B64)
    ok64 = rep64["status"] == nsr.NS_OK
    rel64 = rel_resid(P)
    log(f"batch float64 only: {mk64 * 1e3:.1f} ms ({w64} waves, {g64} workgroups)")
    del B64
    return {
        "workload": "harmonic_batch2048_m8-128_o4", "count": count,
        "scale": "frobenius",
        "inf_half_variant": {
            "makespan_ms": mk_inf * 1e3, "device_ms": mk_inf_dev * 1e3,
            "solves_per_s": count / mk_inf,
            "ok": int(ok_inf.sum()),
            "escalated_to_fp64": int((rep_inf["precision"] == nsr.PREC_FP64).sum()),
            "rel_resid_max_ok": float(rel_inf[ok_inf].max()),
            "ns_steps_p50": float(np.median(steps_inf)), "ns_steps_max": int(steps_inf.max()),
            "ns_steps_total": int(steps_inf.sum()), "ns_steps_total_frobenius": int(steps.sum()),
        },
        "fp64_only": {
            "makespan_ms": mk64 * 1e3, "device_ms": mk64_dev * 1e3, "solves_per_s": count / mk64,
            "launch": {"waves_per_group": w64, "groups": g64}, "ok": int(ok64.sum()),
            "rel_resid_max_ok": float(rel64[ok64].max()) if ok64.any() else None,
            "ns_steps_p50": float(np.median(rep64["ns_steps"])),
        },
        "speedup_vs_fp64_batch": mk64 / mk,
        "launch": {"waves_per_group": waves, "groups": groups},
        "makespan_ms": mk * 1e3, "device_ms": mk_dev * 1e3, "solves_per_s": count / mk,
        "alg_tflops": flop / mk / 1e12,
        "ok": ok, "escalated_to_fp64": esc, "not_converged": count - ok,
        "rel_resid_max_ok": float(rel[okm].max()),
        "rel_resid_p50": float(np.median(rel)),
        "ns_steps_p50": float(np.median(steps)), "ns_steps_max": int(steps.max()),
        "timeline_ms": timeline_summary(tl, [s.n for s in systems]),
        "per_bucket": per_bucket,
    }


def run_serving(torch, nsr, duration_s=3.0, rate=2000.0):
    """Poisson arrivals at `rate` req/s for `duration_s` s; N log-uniform in
    32..2048, kappa log-uniform in 10..1e6, mixed precision to 1e-10."""
    from paper_2008_11480_amd.serve import GpuExecutor, Server, make_requests
    trace = inputs.serving_trace(rate, duration_s, seed=5)
    log(f"generating {len(trace)} serving requests on the GPU")
    reqs = make_requests(trace)
    torch.cuda.synchronize()
    # N <= 192 requests go to the batched kernel (one workgroup per system);
    # larger ones to 12 worker threads with their own streams (and hardware
    # queues, see GPU_MAX_HW_QUEUES above).
    workers, small = 12, 192
    ex = GpuExecutor(workers=workers, precision=nsr.PREC_MIXED_BF16, small_max_n=small)
    # warm up the kernels and the allocator on a few requests of each path
    warm = make_requests(inputs.serving_trace(rate, 0.02, seed=55))
    Server(ex, budget_bytes=32 << 30, workers=workers, small_max_n=small).run(warm)
    srv = Server(ex, budget_bytes=32 << 30, workers=workers, small_max_n=small)
    log("serving")
    st = srv.run(reqs)
    torch.cuda.synchronize()
    rel = []
    for r in reqs:
        if r.status == "ok":
            A, b, th = r.payload[:3]
            rel.append(float(torch.linalg.norm(b - A @ th) / torch.linalg.norm(b)))
    st["rel_resid_max"] = max(rel) if rel else None
    st["workload"] = f"serving_poisson{int(rate)}_{duration_s:g}s_n32-2048_k10-1e6"
    st.pop("not_ok", None)
    # The same trace with every solve in float64 (batched systems too): the
    # offered load exceeds what float64 sustains, so its solves/s over the
    # span (arrival of the first request to the last completion) is the
    # float64 path's maximum sustainable rate.
    del reqs, ex, srv, warm
    release(torch)
    reqs = make_requests(trace)
    torch.cuda.synchronize()
    ex64 = GpuExecutor(workers=workers, precision=nsr.PREC_FP64, small_max_n=small)
    warm = make_requests(inputs.serving_trace(rate, 0.02, seed=55))
    Server(ex64, budget_bytes=32 << 30, workers=workers, small_max_n=small).run(warm)
    log("serving, float64")
    st64 = Server(ex64, budget_bytes=32 << 30, workers=workers, small_max_n=small).run(reqs)
    torch.cuda.synchronize()
    st["fp64"] = {k: st64[k] for k in ("served", "ok", "solves_per_s", "span_s", "latency_ms_p50",
                                       "latency_ms_p99", "latency_ms_max")}
    del reqs, ex64, warm
    return st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spd4096_k1e4_o8",
                    choices=["spd4096_k1e4_o8", "spd64_k1e2_o4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip every leg after the float64 headline (mixed, composite, batch, "
                         "serving)")
    ap.add_argument("--no-mixed4096", action="store_true",
                    help="skip the mixed-precision solve of the headline system")
    ap.add_argument("--no-composite", action="store_true", help="skip the N=8192 legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the N=64 fixed-step leg (eager versus captured graph)")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the Newton-Schulz variant comparison and the three-frequency "
                         "analogue")
    ap.add_argument("--no-programs", action="store_true",
                    help="skip timing the other evaluation programs on the headline system")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (PMC calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X "
              "(DESIGN.md describes how the path would shard); --gpus must be 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2008_11480_amd import autotune, nsr

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    w = dict(inputs.WORKLOADS[args.workload])
    n, kappa, order = w["n"], w["kappa"], w["order"]
    log(f"generating {args.workload}: N={n} kappa={kappa:g} seed={w['seed']}")
    sysm = inputs.spd_qlq(n, kappa, w["seed"])
    A = torch.from_numpy(sysm.A).to("cuda")
    b = torch.from_numpy(sysm.b).to("cuda")
    theta = torch.zeros_like(b)
    solver = nsr.Solver(n, composite=False)
    solver.bind(A)
    fixed = args.workload == "spd64_k1e2_o4"
    kw = dict(order=order, form="squaring", k_max=w["k_max"], floor_detect=not fixed,
              resid_tol=w["resid_tol"])

    if args.calibrate_copy_mib > 0:
        nel = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy_mib} MiB done")
        del src, dst

    m = measure(torch, solver, b, theta, kw, args.steps, args.warmup, "fp64")
    last = m["last"]
    th = theta.cpu().numpy()
    theta_star = sysm.Q @ ((sysm.Q.T @ sysm.b) / sysm.lam)
    fwd = float(np.linalg.norm(th - theta_star) / np.linalg.norm(theta_star))
    rel = float(np.linalg.norm(sysm.b - sysm.A @ th) / np.linalg.norm(sysm.b))
    g64 = m["gemm"]["f64"]
    flop_per_solve = last.gemm_flop + 4.0 * n * n * (last.ns_steps + last.refine_steps + 1)
    traffic = traffic_per_launch()

    out = {
        "metric": "solves/s at rel. residual <= 1e-10 (plain FP64 path; mixed in 'mixed')",
        "value": m["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "n": n, "kappa": kappa, "order": order,
            "form": "squaring (I+F)(I+F^2)(I+F^4)", "precision": "fp64",
            "stop": "||F||_F floor, then Richardson to rel. residual "
                    f"{w['resid_tol']:g}", "seed": w["seed"],
        },
        "roofline": {
            "bound": "mfma",
            "kernel": ("gemm_f64_kernel (128x128 tiles; symmetric-output power products "
                       "cut their last, partial round of tiles along K and finish it "
                       "with gemm_f64_split_fixup)"),
            "achieved": g64["tflops"],
            "peak": PEAK_TFLOPS["f64"],
            "unit": "TFLOP/s",
            "frac": g64["tflops"] / PEAK_TFLOPS["f64"],
            "traffic": traffic,
            "launches": g64["launches"],
            "avg_launch_ms": g64["avg_launch_ms"],
            "flop_per_launch": g64["flop_per_launch"],
            "note": ("float64 GEMM family: the residual and G-side products run full "
                     "(2 n^3 flop), the power products with a symmetric output "
                     "(n^2 (n+1) flop); achieved = algorithmic flop / event time, "
                     "averaged over all products of a solve; a 'launch' is one product "
                     "(the main kernel plus, for a split product, its fixup kernel)"),
        },
        "solve": {
            **report_of(last), "rel_resid": rel, "fwd_err_vs_closed_form": fwd,
            "alg_tflops_per_solve": flop_per_solve / (m["ms_per_solve"] * 1e-3) / 1e12,
            "latency_ms_p50": m["latency_ms_p50"], "latency_ms_p99": m["latency_ms_p99"],
            "fnorm_hist": last.fnorm_hist,
        },
    }
    if not args.no_programs and not fixed:
        # The same system with every candidate program (Tables 1-3, eqs.
        # ex1-ex3, ztab2), fastest first; the headline stays order-8 squaring.
        trials = autotune.time_programs(solver, b, theta, autotune.CANDIDATES, reps=1,
                                        resid_tol=w["resid_tol"], k_max=w["k_max"])
        mu = 1.0 - sysm.lam / last.alpha
        floor = min(last.fnorm_hist)
        out["programs"] = {
            "workload": args.workload, "precision": "fp64",
            "trials": [{"program": t.program.name, "ms_per_solve": t.ms,
                        "solves_per_s": 1e3 / t.ms, "ns_steps": t.ns_steps,
                        "refine_steps": t.refine_steps, "mmm": t.mmm,
                        "rel_resid": t.rel_resid, "ok": t.ok,
                        "predicted_ns_steps": autotune.predicted_steps_spectrum(
                            t.program.order, mu, floor)}
                       for t in trials],
            "chosen": trials[0].program.name,
        }
        for t in trials:
            log(f"program {t.program.name}: {t.ms:.1f} ms ns_steps={t.ns_steps} mmm={t.mmm} "
                f"rel_resid={t.rel_resid:.2e}")
    del solver
    torch.cuda.empty_cache()
    if not args.no_small and not fixed:
        out["small_fixed"] = run_small_fixed(torch, nsr)
    if not args.no_comparisons and not fixed:
        out["comparisons"] = {"workload": args.workload, "precision": "fp64",
                              "variants": run_comparisons(torch, nsr, A, b, sysm, n,
                                                          w["resid_tol"], w["k_max"])}
        out["fig4_analogue"] = run_fig4_analogue(torch, nsr)
        out["preconditioning"] = run_preconditioning(torch, nsr, A, b, sysm, n, w["resid_tol"],
                                                     w["k_max"])
        torch.cuda.empty_cache()

    if not args.no_mixed and not args.no_mixed4096 and not fixed:
        # Same N=4096 system, mixed precision, to the same 1e-12 residual.
        ms = nsr.Solver(n, precision=nsr.PREC_MIXED_BF16, composite=False)
        ms.bind(A)
        thm = torch.zeros_like(b)
        kwm = dict(kw, refine_max=100)
        mm = measure(torch, ms, b, thm, kwm, args.steps, args.warmup, "mixed")
        thc = thm.cpu().numpy()
        out["mixed"] = {
            "workload": args.workload, "precision": "mixed (bf16 powers, fp32 residual and "
                                                  "G-side, fp64 Richardson)",
            "solves_per_s": mm["solves_per_s"], "ms_per_solve": mm["ms_per_solve"],
            "speedup_vs_fp64": mm["solves_per_s"] / m["solves_per_s"],
            "rel_resid": float(np.linalg.norm(sysm.b - sysm.A @ thc) / np.linalg.norm(sysm.b)),
            "fwd_err_vs_closed_form": float(np.linalg.norm(thc - theta_star)
                                            / np.linalg.norm(theta_star)),
            "latency_ms_p50": mm["latency_ms_p50"], "latency_ms_p99": mm["latency_ms_p99"],
            "gemm": mm["gemm"], **report_of(mm["last"]),
        }
        del ms
        torch.cuda.empty_cache()
        # The same with float32-class products from split half-precision
        # operands (residual and G-side) instead of float32 MFMA.
        ss = nsr.Solver(n, precision=nsr.PREC_MIXED_SPLIT, composite=False)
        ss.bind(A)
        ths = torch.zeros_like(b)
        msp = measure(torch, ss, b, ths, kwm, args.steps, args.warmup, "mixed_split")
        # Program choice in this precision (the autotuner's trial): every
        # candidate program on the same system, fastest first.
        sp_trials = autotune.time_programs(ss, b, torch.zeros_like(b), reps=2,
                                           resid_tol=w["resid_tol"], k_max=w["k_max"],
                                           refine_max=100)
        thc = ths.cpu().numpy()
        out["mixed_split"] = {
            "workload": args.workload, "precision": "mixed (bf16 powers, residual and G-side "
                                                  "from split fp16 operands, fp64 Richardson)",
            "solves_per_s": msp["solves_per_s"], "ms_per_solve": msp["ms_per_solve"],
            "speedup_vs_fp64": msp["solves_per_s"] / m["solves_per_s"],
            "rel_resid": float(np.linalg.norm(sysm.b - sysm.A @ thc) / np.linalg.norm(sysm.b)),
            "fwd_err_vs_closed_form": float(np.linalg.norm(thc - theta_star)
                                            / np.linalg.norm(theta_star)),
            "latency_ms_p50": msp["latency_ms_p50"], "latency_ms_p99": msp["latency_ms_p99"],
            "gemm": msp["gemm"], **report_of(msp["last"]),
            "programs": [{"program": t.program.name, "ms_per_solve": t.ms,
                          "solves_per_s": 1e3 / t.ms, "ns_steps": t.ns_steps,
                          "refine_steps": t.refine_steps, "mmm": t.mmm, "ok": t.ok}
                         for t in sp_trials],
            "chosen": sp_trials[0].program.name,
        }
        # best program per precision against each other (the float64 one from
        # the programs leg, when it ran)
        if "programs" in out and sp_trials[0].ok:
            fb = out["programs"]["trials"][0]
            out["mixed_split"]["best_vs_fp64_best"] = {
                "fp64": {"program": fb["program"], "solves_per_s": fb["solves_per_s"]},
                "mixed_split": {"program": sp_trials[0].program.name,
                                "solves_per_s": 1e3 / sp_trials[0].ms},
                "speedup": (1e3 / sp_trials[0].ms) / fb["solves_per_s"]}
        del ss
        torch.cuda.empty_cache()
    if not args.no_mixed and not fixed:
        # Each leg starts from an empty allocator cache: the serving loop's
        # latencies should not depend on what earlier legs left allocated.
        if not args.no_composite:
            out["composite"] = run_composite(torch, nsr, max(2, args.steps // 2), 1)
            release(torch)
        if not args.no_batch:
            out["batch"] = run_batch(torch, nsr, 3)
            release(torch)
        if not args.no_serving:
            out["serving"] = run_serving(torch, nsr)

    if not args.no_cpu_baseline and not fixed:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(sysm, order, last.ns_steps, last.refine_steps)
        out["cpu_cholesky"] = cpu_cholesky(sysm)
        # the same oracle sample on one BLAS thread
        import threadpoolctl
        with threadpoolctl.threadpool_limits(limits=1, user_api="blas"):
            one = cpu_baseline(sysm, order, last.ns_steps, last.refine_steps)
        out["cpu_baseline_1core"] = {"value": one["value"], "unit": one["unit"],
                                     "cores": one["cores"], "kind": "oracle"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
