#!/usr/bin/env python3
"""Benchmark: coupled high-order Newton-Schulz / Richardson SPD solves on one MI355X.

Headline: one "step" is one whole solve (richardson_ns_solve through the C ABI)
of a seeded synthetic system already resident in HBM: N = 8192, kappa = 1e6,
A = Q diag(lam) Q^T, double Newton-Schulz of order 8 (Section 5.1, inner sums
in squaring form) in the mixed mode -- bf16 powers and assembly with float32
accumulation, float32 residual, G-side and merge products, float64 Richardson
refinement to a relative residual of 1e-10.  The same solve in plain float64
is timed beside it (its own warm-up and timed solves) and the ratio is
reported.

Also measured (extra keys of the same JSON line): the N = 4096, kappa = 1e4
order-8 factorized solve in float64 (with its float64 GEMM roofline), in the
mixed mode and with split-fp16 float32-class products (a separate mode: 22
significant bits in the residual and G-side operands); the factorized and
split variants of the N = 8192 system; a batch of 2048 harmonic-regressor
Gram systems of uneven size in one persistent launch; a serving run (Poisson
arrivals, sizes 32..2048) with p50/p99 latency; the program library and the
composite variants on the N = 4096 system; the N = 64 fixed-step workload
(eager, captured graph, 4096-seed batch); and a three-frequency analogue of
the paper's last comparison.

The roofline of the dominant kernel (the float32 GEMM of the headline solve)
comes from per-launch HIP events recorded by the library on its own stream
during the timed region; the CPU baseline is the oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
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
CSRC = os.path.join(ROOT, "paper_2008_11480_amd", "csrc")
# rocprofv3 PMC summaries of HBM traffic per launch, keyed by the GEMM kind
# they measure: (summary file, kernel source whose hash they were taken on)
TRAFFIC = {
    "f64": (os.path.join(ROOT, "profiles", "gemm_f64_spd4096_traffic.json"),
            os.path.join(CSRC, "nsr_gemm_f64.hip")),
    "f32": (os.path.join(ROOT, "profiles", "gemm_f32_spd8192_traffic.json"),
            os.path.join(CSRC, "nsr_gemm_lowp.hip")),
}
KIND = {"f64": 1, "f32": 2, "bf16": 3, "f32_split": 4}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_per_launch(kind):
    """HBM bytes per GEMM launch from the committed rocprofv3 PMC summary,
    or None when the kernel source changed since the counters were taken."""
    path, src = TRAFFIC[kind]
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash(src):
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


def cpu_baseline_composite(a, b, order, ns_steps, refine_steps):
    """Oracle (numpy float64) on a bounded sample of the N = 8192 workload:
    the double Newton-Schulz precalculation (L_0, Gamma_1) and one double
    Newton-Schulz step with its Richardson update on the same system, scaled
    to solves/s with the GPU solve's step counts (refinement steps priced as
    Richardson updates)."""
    import oracle
    alpha = oracle.alpha_frobenius(a)
    g0 = np.eye(a.shape[0]) / alpha
    ctr = oracle.MMCounter()
    t0 = time.perf_counter()
    st = oracle.dns_init(a, g0, order, "squaring", ctr=ctr)
    t_init = time.perf_counter() - t0
    mmm_init = ctr.n
    theta = g0 @ b
    t0 = time.perf_counter()
    st = oracle.dns_step(a, st, order, "squaring", ctr=ctr)
    theta, _ = oracle.richardson_update(a, b, theta, st.G)
    t_step = time.perf_counter() - t0
    mmm_step = ctr.n - mmm_init
    t0 = time.perf_counter()
    theta, _ = oracle.richardson_update(a, b, theta, st.G)
    t_ref = time.perf_counter() - t0
    del st
    t_solve = t_init + ns_steps * t_step + (refine_steps + 1) * t_ref
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": blas_threads(),
        "kind": "oracle",
        "sample": (f"oracle double Newton-Schulz (order {order}) at N={a.shape[0]}: the "
                   f"precalculation ({mmm_init} mmm, {t_init:.2f} s) and one step with its "
                   f"Richardson update ({mmm_step} mmm, {t_step:.2f} s); scaled to the GPU "
                   f"solve's {ns_steps} steps + {refine_steps + 1} residual evaluations "
                   f"({t_ref * 1e3:.0f} ms each)"),
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


PEAK_NOTE = ("achieved = algorithmic flop (2 N^3 per product) / the average per-launch "
             "HIP-event time recorded by the library on its stream over the timed solves")


def roofline_of(g, kind, kernel, traffic):
    return {
        "bound": "mfma", "kernel": kernel, "achieved": g["tflops"],
        "peak": PEAK_TFLOPS[kind], "unit": "TFLOP/s", "frac": g["tflops"] / PEAK_TFLOPS[kind],
        "traffic": traffic, "launches": g["launches"], "avg_launch_ms": g["avg_launch_ms"],
        "flop_per_launch": g["flop_per_launch"],
        "share_of_solve_time": g["share_of_solve_time"],
    }


def run_headline_dns8(torch, nsr, steps, warmup, host_inputs=False):
    """N = 8192, kappa = 1e6, double Newton-Schulz of order 8: the mixed
    mode (bf16 powers, float32 residual / G-side / merge, float64
    Richardson) and the same solve in float64, each with its own warm-up
    and timed solves.  host_inputs: build the system with numpy on the host
    (same recipe and draws; Q differs only by the QR's rounding) instead of
    torch on the GPU."""
    w = inputs.WORKLOADS["spd8192_k1e6_dns8"]
    n = w["n"]
    where = "host" if host_inputs else "GPU"
    log(f"generating spd8192_k1e6_dns8 on the {where}: N={n} kappa={w['kappa']:g} "
        f"seed={w['seed']}")
    if host_inputs:
        sysm = inputs.spd_qlq(n, w["kappa"], w["seed"])
        A, b = torch.from_numpy(sysm.A).cuda(), torch.from_numpy(sysm.b).cuda()
        lam, Q = torch.from_numpy(sysm.lam).cuda(), torch.from_numpy(sysm.Q).cuda()
        del sysm
    else:
        A, b, lam, Q = inputs.spd_qlq_device(n, w["kappa"], w["seed"])
    theta_star = Q @ ((Q.T.contiguous() @ b) / lam)
    del Q
    kw = dict(order=8, form="composite_double", k_max=w["k_max"], resid_tol=w["resid_tol"],
              refine_max=100)
    legs = {}
    for label, prec, st, wu in (("mixed", nsr.PREC_MIXED_BF16, steps, warmup),
                                ("fp64", nsr.PREC_FP64, max(3, steps // 2), max(1, warmup))):
        solver = nsr.Solver(n, precision=prec, composite=True)
        solver.bind(A)
        theta = torch.zeros_like(b)
        m = measure(torch, solver, b, theta, kw, st, wu, f"dns8_{label}")
        rel = float(torch.linalg.norm(b - A @ theta) / torch.linalg.norm(b))
        fwd = float(torch.linalg.norm(theta - theta_star) / torch.linalg.norm(theta_star))
        last = m["last"]
        flop = last.gemm_flop + 4.0 * n * n * (last.ns_steps + last.refine_steps + 1)
        legs[label] = {"m": m, "rel_resid": rel, "fwd_err_vs_closed_form": fwd,
                       "alg_tflops_per_solve": flop / (m["ms_per_solve"] * 1e-3) / 1e12,
                       "steps": st, "warmup": wu}
        del solver
        torch.cuda.empty_cache()
    return w, A, b, legs


def run_composite_variants(torch, nsr, steps, warmup):
    """The N = 8192, kappa = 1e6 system with the factorized order-8 program
    (mixed) and with split-fp16 float32-class products (a mode of its own)
    for the composite and factorized programs."""
    w = inputs.WORKLOADS["spd8192_k1e6_dns8"]
    n = w["n"]
    A, b, lam, Q = inputs.spd_qlq_device(n, w["kappa"], w["seed"])
    theta_star = Q @ ((Q.T.contiguous() @ b) / lam)
    del Q
    out = {"workload": "spd8192_k1e6_dns8", "n": n, "kappa": w["kappa"], "order": 8}
    theta = torch.zeros_like(b)
    for label, prec, form in (("mixed_factorized", nsr.PREC_MIXED_BF16, "squaring"),
                              ("mixed_split_composite", nsr.PREC_MIXED_SPLIT,
                               "composite_double"),
                              ("mixed_split_factorized", nsr.PREC_MIXED_SPLIT, "squaring")):
        solver = nsr.Solver(n, precision=prec, composite=form == "composite_double")
        solver.bind(A)
        kw = dict(order=8, form=form, k_max=64, resid_tol=1e-10, refine_max=100)
        m = measure(torch, solver, b, theta, kw, steps, warmup, label)
        rel = float(torch.linalg.norm(b - A @ theta) / torch.linalg.norm(b))
        fwd = float(torch.linalg.norm(theta - theta_star) / torch.linalg.norm(theta_star))
        out[label] = {"solves_per_s": m["solves_per_s"], "ms_per_solve": m["ms_per_solve"],
                      "rel_resid": rel, "fwd_err_vs_closed_form": fwd,
                      "gemm": m["gemm"], **report_of(m["last"])}
        del solver
        torch.cuda.empty_cache()
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
    # Variant: S = diag(A) (Section 2, for diagonally dominant matrices);
    # harmonic Gram matrices mostly violate 2S - A > 0, so most diverge.
    opts_diag = dict(opts, scale=nsr.SCALE_DIAG)
    mk_dg, _, rep_dg, _ = timed(P, opts_diag)
    ok_dg = rep_dg["status"] == nsr.NS_OK
    div_dg = rep_dg["status"] == nsr.NS_EDIVERGED
    log(f"batch diag(A) scaling: {mk_dg * 1e3:.1f} ms, {int(ok_dg.sum())} converged, "
        f"{int(div_dg.sum())} diverged")
    # The same submission captured into a HIP graph and replayed.
    mk_g, mk_g_dev, rep_g, _ = timed(P, dict(opts, graph=True))
    same_g = bool(np.array_equal(rep_g["ns_steps"], rep["ns_steps"]) and
                  np.array_equal(rep_g["rel_resid"], rep["rel_resid"]))
    log(f"batch graph replay: {mk_g * 1e3:.1f} ms (reports identical: {same_g})")
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
        "diag_variant": {
            "makespan_ms": mk_dg * 1e3, "ok": int(ok_dg.sum()), "diverged": int(div_dg.sum()),
            "ns_steps_p50_ok": float(np.median(rep_dg["ns_steps"][ok_dg])) if ok_dg.any() else None,
            "ns_steps_p50_ok_frobenius": float(np.median(steps[ok_dg])) if ok_dg.any() else None,
            "note": "S = diag(A) needs 2S - A > 0 (Section 2); harmonic Gram matrices are "
                    "not diagonally dominant and their diagonals are nearly equal, so the "
                    "scaling neither converges for most nor changes kappa",
        },
        "graph_replay": {"makespan_ms": mk_g * 1e3, "device_ms": mk_g_dev * 1e3,
                         "reports_identical": same_g},
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


def run_serving(torch, nsr, duration_s=60.0, rate=2000.0, fp64_seconds=5.0, program="auto"):
    """Poisson arrivals at `rate` req/s for `duration_s` s; N log-uniform in
    32..2048, kappa log-uniform in 10..1e6, mixed precision to 1e-10.  Each
    request's system is made on the device when it is admitted and freed
    when it completes; single solves use the autotuned program table."""
    from paper_2008_11480_amd.serve import GpuExecutor, Server, make_requests
    trace = inputs.serving_trace(rate, duration_s, seed=5)
    # N <= 192 requests go to the batched kernel (one workgroup per system);
    # larger ones to 12 worker threads with their own streams (and hardware
    # queues, see GPU_MAX_HW_QUEUES above).
    workers, small = 12, 192
    ex = GpuExecutor(workers=workers, precision=nsr.PREC_MIXED_BF16, small_max_n=small,
                     order=program if program == "auto" else int(program))
    t0 = time.perf_counter()
    reqs = make_requests(trace, draw=ex)     # host data now; device systems per solve
    log(f"serving trace: {len(trace)} requests over {duration_s:g} s "
        f"(host draws {time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    choices = ex.prepare([q.n for q in trace])
    log(f"program table tuned in {time.perf_counter() - t0:.1f} s: "
        + ", ".join(f"2^{c['log2_n']}/p{c['precision']}: {c['program']}" for c in choices))
    # warm up the kernels and the allocator on a few requests of each path
    warm = make_requests(inputs.serving_trace(rate, 0.02, seed=55), draw=ex)
    Server(ex, budget_bytes=32 << 30, workers=workers, small_max_n=small).run(warm)
    srv = Server(ex, budget_bytes=32 << 30, workers=workers, small_max_n=small)
    log("serving")
    st = srv.run(reqs)
    torch.cuda.synchronize()
    st["workload"] = f"serving_poisson{int(rate)}_{duration_s:g}s_n32-2048_k10-1e6"
    st["program_table"] = choices
    st["not_ok"] = st.get("not_ok", [])[:5]
    log(f"serving: {st['served']} served, {st['ok']} ok, p50 {st['latency_ms_p50']:.2f} ms, "
        f"p99 {st['latency_ms_p99']:.2f} ms, {st['solves_per_s']:.0f} solves/s; stages "
        + json.dumps(st["stages"]))
    # Capacity of the mixed path: the first fp64_seconds of the same arrivals
    # offered cap_speedup times faster, beyond what it sustains, so its
    # solves/s over the span (arrival of the first request to the last
    # completion) is its maximum sustainable rate, measured as the float64
    # one below.
    del reqs, srv
    cap_speedup = 4.0
    trace_cap = [dataclasses.replace(q, arrival_s=q.arrival_s / cap_speedup)
                 for q in trace if q.arrival_s < fp64_seconds]
    reqs = make_requests(trace_cap, draw=ex)
    log(f"serving capacity, mixed ({len(reqs)} requests over {fp64_seconds / cap_speedup:g} s)")
    stc = Server(ex, budget_bytes=32 << 30, workers=workers, small_max_n=small).run(reqs)
    torch.cuda.synchronize()
    st["capacity"] = {k: stc[k] for k in ("requests", "served", "ok", "solves_per_s", "span_s",
                                          "latency_ms_p50", "latency_ms_p99",
                                          "rel_resid_max_reported")}
    st["capacity"]["offered_per_s"] = rate * cap_speedup
    log(f"serving capacity, mixed: {stc['solves_per_s']:.0f} solves/s over {stc['span_s']:.2f} s")
    # The same arrivals with every solve in float64 (batched systems too): the
    # offered load exceeds what float64 sustains, so its solves/s over the
    # span is the float64 path's maximum sustainable rate.  A shorter trace
    # suffices.
    del reqs, ex, warm
    release(torch)
    trace64 = [q for q in trace if q.arrival_s < fp64_seconds]
    ex64 = GpuExecutor(workers=workers, precision=nsr.PREC_FP64, small_max_n=small,
                       order=program if program == "auto" else int(program))
    reqs = make_requests(trace64, draw=ex64)
    choices64 = ex64.prepare([q.n for q in trace64])
    warm = make_requests(inputs.serving_trace(rate, 0.02, seed=55), draw=ex64)
    Server(ex64, budget_bytes=32 << 30, workers=workers, small_max_n=small).run(warm)
    log(f"serving, float64 ({len(reqs)} requests over {fp64_seconds:g} s)")
    st64 = Server(ex64, budget_bytes=32 << 30, workers=workers, small_max_n=small).run(reqs)
    torch.cuda.synchronize()
    st["fp64"] = {k: st64[k] for k in ("requests", "served", "ok", "solves_per_s", "span_s",
                                       "latency_ms_p50", "latency_ms_p99", "latency_ms_max",
                                       "rel_resid_max_reported")}
    st["fp64"]["trace_seconds"] = fp64_seconds
    st["fp64"]["program_table"] = choices64
    del reqs, ex64, warm
    return st


def run_spd4096(torch, nsr, args):
    """N = 4096, kappa = 1e4, order-8 factorized Newton-Schulz in float64 to
    the ||F|| rounding floor, then refinement to 1e-12: the float64 GEMM's
    roofline, the program library, the composite variants and Section 2's
    options on this system, and the same solve in the mixed and split-fp16
    modes."""
    from paper_2008_11480_amd import autotune
    w = dict(inputs.WORKLOADS["spd4096_k1e4_o8"])
    n, kappa, order = w["n"], w["kappa"], w["order"]
    log(f"generating spd4096_k1e4_o8: N={n} kappa={kappa:g} seed={w['seed']}")
    sysm = inputs.spd_qlq(n, kappa, w["seed"])
    A = torch.from_numpy(sysm.A).to("cuda")
    b = torch.from_numpy(sysm.b).to("cuda")
    theta = torch.zeros_like(b)
    solver = nsr.Solver(n, composite=False)
    solver.bind(A)
    kw = dict(order=order, form="squaring", k_max=w["k_max"], floor_detect=True,
              resid_tol=w["resid_tol"])
    m = measure(torch, solver, b, theta, kw, args.steps, args.warmup, "spd4096_fp64")
    last = m["last"]
    th = theta.cpu().numpy()
    theta_star = sysm.Q @ ((sysm.Q.T @ sysm.b) / sysm.lam)
    fwd = float(np.linalg.norm(th - theta_star) / np.linalg.norm(theta_star))
    rel = float(np.linalg.norm(sysm.b - sysm.A @ th) / np.linalg.norm(sysm.b))
    flop_per_solve = last.gemm_flop + 4.0 * n * n * (last.ns_steps + last.refine_steps + 1)
    out = {
        "workload": "spd4096_k1e4_o8", "n": n, "kappa": kappa, "order": order,
        "form": "squaring (I+F)(I+F^2)(I+F^4)", "precision": "fp64",
        "stop": f"||F||_F floor, then Richardson to rel. residual {w['resid_tol']:g}",
        "solves_per_s": m["solves_per_s"], "ms_per_solve": m["ms_per_solve"],
        "roofline": roofline_of(m["gemm"]["f64"], "f64", (
            "gemm_f64_nn_dma_kernel (full products: 256x128 tiles fed by LDS DMA) and "
            "gemm_f64_kernel (symmetric-output power products: 128x128 tiles fed by LDS "
            "DMA, the last, partial round cut along K and finished by gemm_f64_split_fixup)"),
            traffic_per_launch("f64")),
        "solve": {
            **report_of(last), "rel_resid": rel, "fwd_err_vs_closed_form": fwd,
            "alg_tflops_per_solve": flop_per_solve / (m["ms_per_solve"] * 1e-3) / 1e12,
            "latency_ms_p50": m["latency_ms_p50"], "latency_ms_p99": m["latency_ms_p99"],
            "fnorm_hist": last.fnorm_hist,
        },
        "_m": m, "_sysm": sysm,
    }
    if not args.no_programs:
        # The same system with every candidate program (Tables 1-3, eqs.
        # ex1-ex3, ztab2), fastest first.
        trials = autotune.time_programs(solver, b, theta, autotune.CANDIDATES, reps=1,
                                        resid_tol=w["resid_tol"], k_max=w["k_max"])
        mu = 1.0 - sysm.lam / last.alpha
        floor = min(last.fnorm_hist)
        out["programs"] = {
            "precision": "fp64",
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
    if not args.no_comparisons:
        out["comparisons"] = {"precision": "fp64",
                              "variants": run_comparisons(torch, nsr, A, b, sysm, n,
                                                          w["resid_tol"], w["k_max"])}
        out["preconditioning"] = run_preconditioning(torch, nsr, A, b, sysm, n,
                                                     w["resid_tol"], w["k_max"])
        torch.cuda.empty_cache()
    if not args.no_mixed4096:
        kwm = dict(kw, refine_max=100)
        for label, prec, desc in (
                ("mixed", nsr.PREC_MIXED_BF16,
                 "mixed (bf16 powers, fp32 residual and G-side, fp64 Richardson)"),
                ("mixed_split", nsr.PREC_MIXED_SPLIT,
                 "split-fp16 mode (bf16 powers; residual and G-side from split fp16 "
                 "operands, 22 significant bits; fp64 Richardson)")):
            ms = nsr.Solver(n, precision=prec, composite=False)
            ms.bind(A)
            thm = torch.zeros_like(b)
            mm = measure(torch, ms, b, thm, kwm, args.steps, args.warmup, label)
            thc = thm.cpu().numpy()
            leg = {
                "precision": desc,
                "solves_per_s": mm["solves_per_s"], "ms_per_solve": mm["ms_per_solve"],
                "speedup_vs_fp64": mm["solves_per_s"] / m["solves_per_s"],
                "rel_resid": float(np.linalg.norm(sysm.b - sysm.A @ thc)
                                   / np.linalg.norm(sysm.b)),
                "fwd_err_vs_closed_form": float(np.linalg.norm(thc - theta_star)
                                                / np.linalg.norm(theta_star)),
                "latency_ms_p50": mm["latency_ms_p50"], "latency_ms_p99": mm["latency_ms_p99"],
                "gemm": mm["gemm"], **report_of(mm["last"]),
            }
            if label == "mixed_split" and not args.no_programs:
                sp_trials = autotune.time_programs(ms, b, torch.zeros_like(b), reps=2,
                                                   resid_tol=w["resid_tol"], k_max=w["k_max"],
                                                   refine_max=100)
                leg["programs"] = [{"program": t.program.name, "ms_per_solve": t.ms,
                                    "solves_per_s": 1e3 / t.ms, "ns_steps": t.ns_steps,
                                    "refine_steps": t.refine_steps, "mmm": t.mmm, "ok": t.ok}
                                   for t in sp_trials]
                leg["chosen"] = sp_trials[0].program.name
            out[label] = leg
            del ms
            torch.cuda.empty_cache()
    return out


def headline_line(args, metric, value, w, config, dtype, roofline, ms_per_step):
    return {
        "metric": metric, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic", "config": config, "roofline": roofline,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spd8192_k1e6_dns8",
                    choices=["spd8192_k1e6_dns8", "spd4096_k1e4_o8", "spd64_k1e2_o4"],
                    help="headline workload (default: the N=8192 mixed-vs-float64 pair)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tile-tuning", action="store_true",
                    help="keep the GEMM tile rule (skip the tile autotuner)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no other legs)")
    ap.add_argument("--no-spd4096", action="store_true", help="skip the N=4096 legs")
    ap.add_argument("--no-mixed4096", action="store_true",
                    help="skip the mixed and split solves of the N=4096 system")
    ap.add_argument("--no-composite", action="store_true",
                    help="skip the factorized / split variants of the N=8192 system")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="length of the serving trace (Poisson arrivals at 2000 req/s)")
    ap.add_argument("--serving-fp64-seconds", type=float, default=5.0,
                    help="length of the trace served in float64 (its sustainable rate)")
    ap.add_argument("--serving-program", default="auto",
                    help="single-solve program: 'auto' (autotuned table) or an order "
                         "(squaring form)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the N=64 fixed-step leg (eager versus captured graph)")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the Newton-Schulz variant comparison and the three-frequency "
                         "analogue")
    ap.add_argument("--no-programs", action="store_true",
                    help="skip timing the other evaluation programs on the N=4096 system")
    ap.add_argument("--host-inputs", action="store_true",
                    help="build the N=8192 system on the host (numpy QR) rather than on the "
                         "GPU; for profiler runs in which torch's device QR cannot run")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (PMC calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; "
              "--gpus must be 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2008_11480_amd import nsr

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)

    if args.calibrate_copy_mib > 0:
        nel = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy_mib} MiB done")
        del src, dst

    extras = not args.no_extras
    cpu_sample = None
    tiles = None
    if not args.no_tile_tuning:
        # The project's tile autotuner: every GEMM family's tiles timed per
        # size bucket, the fastest installed before anything is measured.
        from paper_2008_11480_amd import autotune
        t0 = time.perf_counter()
        tiles = autotune.tune_tiles()
        release(torch)
        log(f"tile autotune ({time.perf_counter() - t0:.1f} s): "
            + ", ".join(f"{r['family']}/{r['n']}:{r['best_tile']}" for r in tiles))
    if args.workload == "spd8192_k1e6_dns8":
        w, A8, b8, legs = run_headline_dns8(torch, nsr, args.steps, args.warmup,
                                            args.host_inputs)
        mx, f64 = legs["mixed"], legs["fp64"]
        lm, lf = mx["m"]["last"], f64["m"]["last"]
        out = headline_line(
            args, "solves/s at rel. residual <= 1e-10, mixed (bf16 powers, fp32 residual / "
                  "G-side / merge, fp64 refinement) vs plain fp64; N=8192 double "
                  "Newton-Schulz order 8",
            mx["m"]["solves_per_s"], w,
            {"workload": "spd8192_k1e6_dns8", "n": w["n"], "kappa": w["kappa"],
             "order": 8, "form": "double Newton-Schulz (Section 5.1), inner sums "
                                 "(I+F)(I+F^2)(I+F^4)",
             "precision": "mixed_bf16", "stop": "||F||_F floor, then Richardson to rel. "
                                               "residual 1e-10", "seed": w["seed"]},
            "bf16/fp32 (fp64 refinement)",
            roofline_of(mx["m"]["gemm"]["f32"], "f32",
                        "gemm_f32_nn_dma_kernel (256x256 tiles, LDS DMA, float32 MFMA "
                        "16x16x4: residual, G-side and merge products)",
                        traffic_per_launch("f32")),
            mx["m"]["ms_per_solve"])
        out["roofline"]["note"] = PEAK_NOTE
        out["fp64"] = {
            "solves_per_s": f64["m"]["solves_per_s"], "ms_per_solve": f64["m"]["ms_per_solve"],
            "steps": f64["steps"], "warmup": f64["warmup"],
            "rel_resid": f64["rel_resid"], "fwd_err_vs_closed_form": f64["fwd_err_vs_closed_form"],
            "alg_tflops_per_solve": f64["alg_tflops_per_solve"], "gemm": f64["m"]["gemm"],
            **report_of(lf)}
        out["speedup_mixed_vs_fp64"] = mx["m"]["solves_per_s"] / f64["m"]["solves_per_s"]
        out["solve"] = {**report_of(lm), "rel_resid": mx["rel_resid"],
                        "fwd_err_vs_closed_form": mx["fwd_err_vs_closed_form"],
                        "alg_tflops_per_solve": mx["alg_tflops_per_solve"],
                        "latency_ms_p50": mx["m"]["latency_ms_p50"],
                        "latency_ms_p99": mx["m"]["latency_ms_p99"],
                        "fnorm_hist": lm.fnorm_hist, "gemm": mx["m"]["gemm"]}
        log(f"headline: mixed {mx['m']['solves_per_s']:.3f} solves/s, fp64 "
            f"{f64['m']['solves_per_s']:.3f} solves/s, speedup {out['speedup_mixed_vs_fp64']:.2f}")
        if not args.no_cpu_baseline:
            cpu_sample = (A8.cpu().numpy(), b8.cpu().numpy(), lm.ns_steps, lm.refine_steps)
        del A8, b8, legs
        release(torch)
        if extras and not args.no_spd4096:
            s4 = run_spd4096(torch, nsr, args)
            s4.pop("_m"), s4.pop("_sysm")
            out["spd4096_k1e4_o8"] = s4
            release(torch)
    elif args.workload == "spd4096_k1e4_o8":
        s4 = run_spd4096(torch, nsr, args)
        m, sysm = s4.pop("_m"), s4.pop("_sysm")
        w = inputs.WORKLOADS["spd4096_k1e4_o8"]
        out = headline_line(
            args, "solves/s at rel. residual <= 1e-12, plain fp64; N=4096 order-8 "
                  "factorized Newton-Schulz", m["solves_per_s"], w,
            {"workload": "spd4096_k1e4_o8", "n": w["n"], "kappa": w["kappa"], "order": 8,
             "form": s4["form"], "precision": "fp64", "stop": s4["stop"], "seed": w["seed"]},
            "f64", s4.pop("roofline"), m["ms_per_solve"])
        out["spd4096_k1e4_o8"] = s4
        if not args.no_cpu_baseline:
            last = m["last"]
            out["cpu_baseline"] = cpu_baseline(sysm, 8, last.ns_steps, last.refine_steps)
            out["cpu_cholesky"] = cpu_cholesky(sysm)
        extras = False
        release(torch)
    else:
        out = {"small_fixed": run_small_fixed(torch, nsr)}
        print(json.dumps(out), flush=True)
        return

    if extras:
        if not args.no_small:
            out["small_fixed"] = run_small_fixed(torch, nsr)
        if not args.no_comparisons:
            out["fig4_analogue"] = run_fig4_analogue(torch, nsr)
        release(torch)
        if not args.no_composite:
            out["composite_variants"] = run_composite_variants(torch, nsr,
                                                               max(2, args.steps // 2), 1)
            release(torch)
        if not args.no_batch:
            out["batch"] = run_batch(torch, nsr, 3)
            release(torch)
        if not args.no_serving:
            out["serving"] = run_serving(torch, nsr, duration_s=args.serving_seconds,
                                         fp64_seconds=args.serving_fp64_seconds,
                                         program=args.serving_program)

    if tiles is not None:
        fam = {0: "f64", 1: "f32", 2: "bf16", 3: "f16_split"}
        out["tile_autotune"] = [{**r, "family": fam[r["family"]]} for r in tiles]
    if cpu_sample is not None:
        log("timing the CPU oracle on a bounded sample of the N=8192 workload")
        a_h, b_h, ns_steps, refine_steps = cpu_sample
        out["cpu_baseline"] = cpu_baseline_composite(a_h, b_h, 8, ns_steps, refine_steps)
        del cpu_sample, a_h, b_h
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
