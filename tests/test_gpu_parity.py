"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (each derived from the arithmetic it bounds):
* GEMM: |D - D_ref|_ij <= gamma_{k+4} (|s| |X||Y| + |diag| I + |E1| + |E2|)_ij,
  gamma_m = m u / (1 - m u), for both the kernel and the reference dot product.
* ||F_k||_F traces: |d| <= 1e-10 ||F_k|| + 10 * floor, floor = the smallest
  ||F|| either run reached (rounding differences are amplified at most ~n^k
  before the iteration contracts, and sit at the floor afterwards).
* theta: ||theta - theta_oracle|| / ||theta_oracle|| <= 10 kappa u.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2008_11480_amd import inputs, nsr

pytestmark = pytest.mark.gpu

U = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def torch():
    import torch as _torch
    if not _torch.cuda.is_available():
        pytest.skip("no GPU")
    nsr.lib()
    return _torch


def gamma(m):
    return m * U / (1 - m * U)


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


# --------------------------------------------------------------------------
# GEMM kernel
# --------------------------------------------------------------------------

GEMM_SHAPES = [(1, 1, 1), (5, 3, 7), (64, 64, 64), (100, 37, 250), (129, 130, 131),
               (257, 300, 129), (512, 512, 512), (1000, 999, 1001), (2900, 2950, 300)]


@pytest.mark.parametrize("m,n,k", GEMM_SHAPES)
@pytest.mark.parametrize("odd_ld", [False, True])
def test_gemm_f64_elementwise(torch, m, n, k, odd_ld):
    rng = np.random.default_rng(m * 7 + n * 13 + k)
    pad = 1 if odd_ld else 0
    Xb = rng.standard_normal((m, k + pad))
    Yb = rng.standard_normal((k, n + pad))
    E1 = rng.standard_normal((m, n))
    E2 = rng.standard_normal((m, n))
    X, Y = Xb[:, :k], Yb[:, :n]
    diag, scale = 0.7, -1.3
    Xd = to_dev(torch, Xb)[:, :k]
    Yd = to_dev(torch, Yb)[:, :n]
    D, ss = nsr.gemm_f64(Xd, Yd, E1=to_dev(torch, E1), E2=to_dev(torch, E2), diag=diag,
                         scale=scale, want_sumsq=True)
    torch.cuda.synchronize()
    got = D.cpu().numpy()
    ref = scale * (X @ Y) + diag * np.eye(m, n) + E1 + E2
    bound = gamma(k + 4) * (abs(scale) * (np.abs(X) @ np.abs(Y)) + abs(diag) * np.eye(m, n)
                            + np.abs(E1) + np.abs(E2))
    err = np.abs(got - ref)
    assert np.all(err <= 2 * bound + 1e-300), float(np.max(err / (bound + 1e-300)))
    ss_ref = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ss_ref) <= 1e-13 * ss_ref


@pytest.mark.parametrize("addends", [0, 2])
@pytest.mark.parametrize("m,n,k,shift", [(300, 520, 32, 0), (513, 260, 64, 0),
                                         (1000, 700, 96, 0), (2100, 1900, 1024, 0),
                                         (4100, 4000, 224, 0), (700, 520, 96, 1),
                                         (301, 259, 64, 0), (300, 256, 100, 0)])
def test_gemm_f64_dma_tiles(torch, m, n, k, shift, addends):
    """The 256 x 128 float64 tiles fed by LDS DMA (full products, K a
    multiple of 16, N even): one to many slabs (the two-stage ring's start,
    wrap and drain), ragged edge tiles, row strides above the width, every
    epilogue form.  shift = 1 starts the operand views one element in (rows
    not 16-byte aligned), N = 259 is odd and K = 100 not a multiple of 16:
    those products take the register-staged kernel instead."""
    b = int(np.ceil(np.log2(max(m, n))))
    nsr.tile_set(nsr.TILE_F64, b, 256)
    try:
        rng = np.random.default_rng(m * 3 + n * 5 + k + addends)
        Xb = rng.standard_normal((m, k + 8))
        Yb = rng.standard_normal((k, n + 6))
        E = [rng.standard_normal((m, n)) for _ in range(addends)]
        X, Y = Xb[:, shift:shift + k], Yb[:, shift:shift + n]
        diag, scale = 0.7, -1.3
        print(f"f64 dma tiles {m}x{n}x{k} shift {shift} addends {addends}", flush=True)
        D, ss = nsr.gemm_f64(to_dev(torch, Xb)[:, shift:shift + k],
                             to_dev(torch, Yb)[:, shift:shift + n],
                             E1=to_dev(torch, E[0]) if addends > 0 else None,
                             E2=to_dev(torch, E[1]) if addends > 1 else None,
                             diag=diag, scale=scale, want_sumsq=True)
        torch.cuda.synchronize()
    finally:
        nsr.tile_set(nsr.TILE_F64, b, 0)
    got = D.cpu().numpy()
    ref = scale * (X @ Y) + diag * np.eye(m, n) + sum(E, np.zeros((m, n)))
    bound = gamma(k + 4) * (abs(scale) * (np.abs(X) @ np.abs(Y)) + abs(diag) * np.eye(m, n)
                            + sum((np.abs(e) for e in E), np.zeros((m, n))))
    err = np.abs(got - ref)
    assert np.all(err <= 2 * bound + 1e-300), float(np.max(err / (bound + 1e-300)))
    ss_ref = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ss_ref) <= 1e-13 * ss_ref


@pytest.mark.parametrize("addends", [0, 2])
@pytest.mark.parametrize("m,n,k,sym", [(300, 520, 32, False), (1000, 700, 96, False),
                                       (2100, 1900, 1024, False), (130, 130, 16, True),
                                       (2064, 2064, 2064, True), (700, 522, 96, False)])
def test_gemm_f64_dma128_tiles(torch, m, n, k, sym, addends):
    """128 x 128 float64 tiles with K slabs fed by LDS DMA (K a multiple of
    16, N even, even strides, 16-byte aligned operands), forced for full and
    symmetric-output products: one to many slabs, ragged edge tiles (rows
    past M and columns past N read clamped copies that feed no stored
    output), row strides above the width, every epilogue form."""
    b = int(np.ceil(np.log2(max(m, n))))
    nsr.tile_set(nsr.TILE_F64, b, 128)
    try:
        rng = np.random.default_rng(m * 3 + n * 5 + k + addends + 11 * sym)
        if sym:
            B = rng.standard_normal((m, k))
            X = 0.5 * (B + B.T) if m == k else B
            Xb = np.concatenate([X, rng.standard_normal((m, 8))], axis=1)
            Yb = np.concatenate([X.T, rng.standard_normal((k, 6))], axis=1)
            E = [rng.standard_normal((m, n)) for _ in range(addends)]
            E = [0.5 * (e + e.T) for e in E]
        else:
            Xb = rng.standard_normal((m, k + 8))
            Yb = rng.standard_normal((k, n + 6))
            E = [rng.standard_normal((m, n)) for _ in range(addends)]
        X, Y = Xb[:, :k], Yb[:, :n]
        diag, scale = 0.7, -1.3
        print(f"f64 dma128 tiles {m}x{n}x{k} sym {sym} addends {addends}", flush=True)
        D, ss = nsr.gemm_f64(to_dev(torch, Xb)[:, :k], to_dev(torch, Yb)[:, :n],
                             E1=to_dev(torch, E[0]) if addends > 0 else None,
                             E2=to_dev(torch, E[1]) if addends > 1 else None,
                             diag=diag, scale=scale, want_sumsq=True, symmetric=sym)
        torch.cuda.synchronize()
    finally:
        nsr.tile_set(nsr.TILE_F64, b, 0)
    got = D.cpu().numpy()
    if sym:
        assert np.array_equal(got, got.T)
    ref = scale * (X @ Y) + diag * np.eye(m, n) + sum(E, np.zeros((m, n)))
    bound = gamma(k + 4) * (abs(scale) * (np.abs(X) @ np.abs(Y)) + abs(diag) * np.eye(m, n)
                            + sum((np.abs(e) for e in E), np.zeros((m, n))))
    err = np.abs(got - ref)
    if sym:
        iu = np.triu_indices(m)
        err, bound = err[iu], bound[iu]
    assert np.all(err <= 2 * bound + 1e-300), float(np.max(err / (bound + 1e-300)))
    ss_ref = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ss_ref) <= 1e-13 * ss_ref


@pytest.mark.parametrize("n", [1, 5, 64, 100, 257, 1000, 2900, 4096])
def test_gemm_f64_symmetric_output(torch, n):
    """Symmetric output: the upper triangle obeys the element-wise bound, the
    result is exactly symmetric, and the sum of squares covers both halves."""
    rng = np.random.default_rng(n + 3)
    B = rng.standard_normal((n, n))
    S = 0.5 * (B + B.T)
    E = rng.standard_normal((n, n))
    E = 0.5 * (E + E.T)
    D, ss = nsr.gemm_f64(to_dev(torch, S), to_dev(torch, S), E1=to_dev(torch, E), diag=1.0,
                         scale=-0.5, want_sumsq=True, symmetric=True)
    torch.cuda.synchronize()
    got = D.cpu().numpy()
    assert np.array_equal(got, got.T)
    ref = -0.5 * (S @ S) + np.eye(n) + E
    bound = gamma(n + 4) * (0.5 * (np.abs(S) @ np.abs(S)) + np.eye(n) + np.abs(E))
    iu = np.triu_indices(n)
    assert np.all(np.abs(got - ref)[iu] <= 2 * bound[iu])
    ssr = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ssr) <= 1e-13 * ssr


SPLIT_SHAPES = [(2944, 2944, 2944, False), (3000, 3100, 1000, False), (2944, 2944, 33, False),
                (4096, 4096, 4096, True), (4100, 4100, 4100, True), (4096, 4096, 100, True),
                (4112, 4112, 4112, True)]


@pytest.mark.parametrize("m,n,k,sym", SPLIT_SHAPES)
def test_gemm_f64_split_tail(torch, m, n, k, sym):
    """Shapes whose last round of 128 x 128 tiles is partial: with scratch,
    those tiles are cut along K and finished by the fixup kernel.  Every
    element obeys the summation error bound, the result agrees with the
    unsplit call to that bound, a symmetric output stays exactly symmetric,
    and the sum of squares (partials of whole tiles and fixup strips) is
    the sum over the written matrix."""
    rng = np.random.default_rng(m + 3 * n + 7 * k + sym)
    if sym:
        B = rng.standard_normal((m, k))
        X = 0.5 * (B + B.T) if m == k else B
        Y = X.T.copy() if m != k else X
        E1 = rng.standard_normal((m, n))
        E1 = 0.5 * (E1 + E1.T)
    else:
        X = rng.standard_normal((m, k))
        Y = rng.standard_normal((k, n))
        E1 = rng.standard_normal((m, n))
    diag, scale = 0.7, -1.3
    nbytes = nsr.gemm_f64_scratch_bytes(m, n, k, symmetric=sym)
    if torch.cuda.get_device_properties(0).multi_processor_count == 256 and k >= 100:
        assert nbytes > 0, "expected a split plan for this shape"
    scratch = torch.empty(max(nbytes, 8) // 8, dtype=torch.float64, device="cuda")
    Xd, Yd, Ed = to_dev(torch, X), to_dev(torch, Y), to_dev(torch, E1)
    D, ss = nsr.gemm_f64(Xd, Yd, E1=Ed, diag=diag, scale=scale, want_sumsq=True, symmetric=sym,
                         scratch=scratch)
    D0 = nsr.gemm_f64(Xd, Yd, E1=Ed, diag=diag, scale=scale, symmetric=sym)
    torch.cuda.synchronize()
    got, got0 = D.cpu().numpy(), D0.cpu().numpy()
    if sym:
        assert np.array_equal(got, got.T)
    ref = scale * (X @ Y) + diag * np.eye(m, n) + E1
    bound = gamma(k + 4) * (abs(scale) * (np.abs(X) @ np.abs(Y)) + abs(diag) * np.eye(m, n)
                            + np.abs(E1))
    sel = np.triu_indices(m) if sym else np.s_[:, :]
    assert np.all(np.abs(got - ref)[sel] <= 2 * bound[sel])
    assert np.all(np.abs(got - got0)[sel] <= 4 * bound[sel])
    ssr = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ssr) <= 1e-13 * ssr


def test_gemm_f64_no_addends(torch):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((200, 300))
    Y = rng.standard_normal((300, 150))
    D = nsr.gemm_f64(to_dev(torch, X), to_dev(torch, Y)).cpu().numpy()
    bound = gamma(304) * (np.abs(X) @ np.abs(Y))
    assert np.all(np.abs(D - X @ Y) <= 2 * bound)


def test_gemm_f64_full_size_sampled(torch):
    """n = 4096 (the single-solve workload's GEMM shape, same launch
    configuration): 3000 sampled entries against CPU dot products."""
    n = 4096
    g = torch.Generator(device="cuda").manual_seed(1234)
    X = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    Y = torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g)
    D = nsr.gemm_f64(X, Y, diag=1.0, scale=-1.0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    ii = rng.integers(0, n, 3000)
    jj = rng.integers(0, n, 3000)
    ii[:64] = np.arange(64)       # include diagonal entries
    jj[:64] = np.arange(64)
    Xc, Yc, Dc = X.cpu().numpy(), Y.cpu().numpy(), D.cpu().numpy()
    for i, j in zip(ii, jj):
        ref = -math.fsum(Xc[i, :] * Yc[:, j]) + (1.0 if i == j else 0.0)
        bound = gamma(n + 4) * (float(np.abs(Xc[i, :]) @ np.abs(Yc[:, j])) + (i == j))
        assert abs(Dc[i, j] - ref) <= bound, (i, j)


# --------------------------------------------------------------------------
# Solver against the oracle
# --------------------------------------------------------------------------

def compare_traces(h_gpu, h_orc, rel=1e-10, floor_mult=10.0, n_cmp=None):
    n_cmp = n_cmp if n_cmp is not None else min(len(h_gpu), len(h_orc))
    floor = max(min(h_gpu), min(h_orc))
    for k in range(n_cmp):
        d = abs(h_gpu[k] - h_orc[k])
        assert d <= rel * abs(h_orc[k]) + floor_mult * floor, (k, h_gpu[k], h_orc[k], floor)


def gpu_solve(torch, sysm, symmetric=True, **kw):
    A = to_dev(torch, sysm.A)
    b = to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(sysm.n, composite=kw.get("form") == "composite_double")
    s.set_symmetric(symmetric)
    s.bind(A)
    rep = s.solve(b, th, **kw)
    torch.cuda.synchronize()
    return th.cpu().numpy(), rep


@pytest.mark.parametrize("symmetric", [True, False])
def test_spd64_twelve_steps_matches_oracle(torch, symmetric):
    """N=64, kappa=100, order 4 (I+F)(I+F^2), 12 steps, coupled Richardson,
    target relative residual 1e-13.  All 12 steps stay at the float64 floor
    (a regression check: mirroring the residual or G-side products would let
    the non-commuting rounding error grow ~kappa per step)."""
    w = inputs.WORKLOADS["spd64_k1e2_o4"]
    sysm = inputs.spd_qlq(w["n"], w["kappa"], w["seed"])
    th, rep = gpu_solve(torch, sysm, symmetric=symmetric, order=4, form="squaring", k_max=12,
                        floor_detect=False, resid_tol=1e-13)
    assert max(rep.fnorm_hist[8:]) < 1e-12
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=4, k_max=12,
                                                           floor_detect=False,
                                                           resid_tol=1e-13))
    assert rep.ns_steps == 12 and orc.ns_steps == 12
    assert rep.alpha == pytest.approx(orc.alpha, rel=1e-14)
    compare_traces(rep.fnorm_hist, orc.fnorm_hist)
    compare_traces(rep.resid_hist, orc.resid_hist, rel=1e-8)
    assert rep.rel_resid <= 1e-13
    kappa = w["kappa"]
    assert np.linalg.norm(th - orc.theta) <= 10 * kappa * U * np.linalg.norm(orc.theta)
    # eigen closed form of ||F_k|| (eq. fk1) before the floor
    mu = 1.0 - sysm.lam / rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        ref = math.sqrt(float(np.sum(mu ** (2 * 4 ** k))))
        if ref > 1e-8:
            assert fk == pytest.approx(ref, rel=1e-9)


SOLVE_CASES = [
    # n, kappa, order, form, p, w
    (1, 1.0, 4, "squaring", 0, 0),
    (2, 10.0, 4, "squaring", 0, 0),
    (3, 10.0, 8, "squaring", 0, 0),
    (257, 1e2, 2, "squaring", 0, 0),
    (300, 1e3, 4, "squaring", 0, 0),
    (300, 1e3, 8, "squaring", 0, 0),
    (200, 1e2, 3, "horner", 0, 0),
    (200, 1e2, 6, "unified", 2, 2),
    (200, 1e2, 4, "unified", 1, 2),
    (200, 1e2, 4, "unified", 0, 4),
    (200, 1e2, 3, "unified", 2, 1),
    (200, 1e2, 5, "unified_plus1", 1, 2),
    (200, 1e2, 3, "unified_plus1", 0, 2),
    (200, 1e2, 4, "unified_plus1", 2, 1),
    (3, 10.0, 11, "table", 0, 0),
    (200, 1e3, 11, "table", 0, 0),
    (300, 1e4, 15, "table", 0, 0),
    (257, 1e4, 45, "table", 0, 0),
    (130, 1e2, 4, "composite_double", 0, 0),
    (300, 1e3, 8, "composite_double", 0, 0),
    (97, 1e2, 2, "composite_double", 0, 0),
]


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("n,kappa,order,form,p,w", SOLVE_CASES)
def test_solve_matches_oracle(torch, n, kappa, order, form, p, w, symmetric):
    sysm = inputs.spd_qlq(n, kappa, seed=100 + n)
    th, rep = gpu_solve(torch, sysm, symmetric=symmetric, order=order, form=form, p=p, w=w,
                        resid_tol=1e-13)
    oform = "squaring" if form == "composite_double" else form
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(
        order=order, form=oform, p=p if form.startswith("unified") else None,
        w=w if form.startswith("unified") else None, composite=form == "composite_double",
        resid_tol=1e-13))
    assert abs(rep.ns_steps - orc.ns_steps) <= 1, (rep.ns_steps, orc.ns_steps)
    compare_traces(rep.fnorm_hist, orc.fnorm_hist)
    assert rep.rel_resid <= max(1e-13, 2 * orc.rel_resid)
    assert np.linalg.norm(th - orc.theta) <= 10 * kappa * U * np.linalg.norm(orc.theta) + 1e-300


def test_fp64_composite_full_size_spd4096(torch):
    """Float64 double Newton-Schulz of order 8 (Section 5.1) at N = 4096, the
    size at which every product runs 128 x 128 tiles and the symmetric power
    products cut their partial last round of tiles along K: the ||F_k||
    trace, the stop step and theta against the oracle's double Newton-Schulz
    on the same system, and the trace on the closed form of eq. (ermoex1)
    while above the floor."""
    w = inputs.WORKLOADS["spd4096_k1e4_o8"]
    sysm = inputs.spd_qlq(w["n"], w["kappa"], w["seed"])
    th, rep = gpu_solve(torch, sysm, order=8, form="composite_double", k_max=64,
                        resid_tol=w["resid_tol"], refine_max=64)
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=8, composite=True,
                                                           resid_tol=w["resid_tol"]))
    print("gpu", rep.ns_steps, rep.fnorm_hist)
    print("orc", orc.ns_steps, orc.fnorm_hist)
    assert abs(rep.ns_steps - orc.ns_steps) <= 1, (rep.ns_steps, orc.ns_steps)
    compare_traces(rep.fnorm_hist, orc.fnorm_hist, rel=1e-9)
    assert rep.rel_resid <= max(w["resid_tol"], 2 * orc.rel_resid)
    kappa = w["kappa"]
    assert np.linalg.norm(th - orc.theta) <= 10 * kappa * U * np.linalg.norm(orc.theta)
    mu = 1.0 - sysm.lam / rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        e_k = k * 8 ** (k + 1) + 8 ** k
        ref = math.sqrt(float(np.sum(mu ** (2.0 * e_k))))
        if ref > 1e3 * min(rep.fnorm_hist):
            assert fk == pytest.approx(ref, rel=1e-6), (k, fk, ref)


def test_step_level_G_matches_oracle(torch):
    """ns_step / ns_get_G / ns_get_F element-wise against the oracle's G_k, F_k."""
    n = 257
    sysm = inputs.spd_qlq(n, 1e2, seed=21)
    s = nsr.Solver(n)
    s.bind(to_dev(torch, sysm.A))
    alpha, f0 = s.init_scale()
    a_orc = oracle.alpha_frobenius(sysm.A)
    assert alpha == pytest.approx(a_orc, rel=1e-14)
    g = np.eye(n) / a_orc
    for k in range(1, 3):
        fk = s.step(8, "squaring")
        g = oracle.ns_step(sysm.A, g, 8, "squaring")
        f = oracle.residual(sysm.A, g)
        G = s.get_G().cpu().numpy()
        F = s.get_F().cpu().numpy()
        assert np.linalg.norm(G - g) <= 1e-12 * np.linalg.norm(g), k
        assert np.linalg.norm(F - f) <= 1e-12 * max(1.0, np.linalg.norm(f)) * n, k
        assert fk == pytest.approx(np.linalg.norm(f), rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("order", [11, 15, 45])
def test_table_step_matches_oracle(torch, order, symmetric):
    """Nested table programs (orders 11, 15, 45): G_k and F_k element-wise
    against the oracle's step for the first two steps (the first with the
    implicit G_0), and the products per explicit step equal the program's
    mmm count (which includes the step's residual)."""
    n = 193
    sysm = inputs.spd_qlq(n, 1e4, seed=31 + order)
    s = nsr.Solver(n)
    s.set_symmetric(symmetric)
    s.bind(to_dev(torch, sysm.A))
    alpha, _ = s.init_scale()
    g = np.eye(n) / oracle.alpha_frobenius(sysm.A)
    for k in range(1, 3):
        if k == 2:
            s.timing(True)
        fk = s.step(order, "table")
        g = oracle.ns_step(sysm.A, g, order, "table")
        f = oracle.residual(sysm.A, g)
        G = s.get_G().cpu().numpy()
        F = s.get_F().cpu().numpy()
        assert np.linalg.norm(G - g) <= 1e-11 * np.linalg.norm(g), k
        assert np.linalg.norm(F - f) <= 1e-11 * max(1.0, np.linalg.norm(f)) * n, k
        assert fk == pytest.approx(np.linalg.norm(f), rel=1e-9, abs=1e-11)
    launches, _, _ = s.timing_read(0)
    assert launches == oracle.form_mmm(order, "table")


def test_table_order_rejected(torch):
    s = nsr.Solver(64)
    s.bind(torch.eye(64, dtype=torch.float64, device="cuda"))
    s.init_scale()
    with pytest.raises(nsr.NSError):
        s.step(8, "table")


def test_solve_is_deterministic(torch):
    sysm = inputs.spd_qlq(300, 1e3, seed=3)
    th1, r1 = gpu_solve(torch, sysm, order=8)
    th2, r2 = gpu_solve(torch, sysm, order=8)
    assert np.array_equal(th1, th2)
    assert r1.fnorm_hist == r2.fnorm_hist


@pytest.mark.parametrize("symmetric", [True, False])
def test_full_size_spd4096(torch, symmetric):
    """N=4096, kappa=1e4, order 8 squaring to the ||F|| floor with Richardson
    refinement: the launch configuration the benchmark times.  Checked against
    properties that hold at any size: the eigen closed form of ||F_k||
    (eq. fk1), theta* = Q diag(1/lam) Q^T b, and a LAPACK Cholesky residual."""
    import scipy.linalg
    w = inputs.WORKLOADS["spd4096_k1e4_o8"]
    sysm = inputs.spd_qlq(w["n"], w["kappa"], w["seed"])
    th, rep = gpu_solve(torch, sysm, symmetric=symmetric, order=8, form="squaring", k_max=64,
                        resid_tol=w["resid_tol"])
    assert rep.ns_stop in ("floor", "f_tol")
    mu = 1.0 - sysm.lam / rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        ref = math.sqrt(float(np.sum(mu ** (2 * 8 ** k))))
        if ref > 1e-6:
            assert fk == pytest.approx(ref, rel=1e-8), k
    theta_star = sysm.Q @ ((sysm.Q.T @ sysm.b) / sysm.lam)
    fwd = np.linalg.norm(th - theta_star) / np.linalg.norm(theta_star)
    assert fwd <= 10 * w["kappa"] * U * 4, fwd
    chol = scipy.linalg.cho_solve(scipy.linalg.cho_factor(sysm.A), sysm.b)
    rc = np.linalg.norm(sysm.b - sysm.A @ chol) / np.linalg.norm(sysm.b)
    rr = np.linalg.norm(sysm.b - sysm.A @ th) / np.linalg.norm(sysm.b)
    assert rr <= max(1e-12, 2 * rc), (rr, rc)
    assert rep.rel_resid <= max(1e-12, 2 * rc)


def test_error_paths(torch):
    n = 64
    sysm = inputs.spd_qlq(n, 10.0, seed=2)
    s = nsr.Solver(n)
    with pytest.raises(nsr.NSError) as e:
        s.step(4)
    assert e.value.status == nsr.NS_ESTATE
    s.bind(to_dev(torch, sysm.A))
    s.init_scale()
    with pytest.raises(nsr.NSError) as e:
        s.step(6, "squaring")
    assert e.value.status == nsr.NS_EINVAL
    with pytest.raises(nsr.NSError) as e:
        s.step(5, "unified", p=1, w=2)
    assert e.value.status == nsr.NS_EINVAL
    # alpha below lambda_max / 2: the splitting condition fails, diverges
    lmax = float(sysm.lam.max())
    eps = 0.4 * lmax - float(np.max(np.sum(np.abs(sysm.A), axis=1))) / 2.0
    b = to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    rep = s.solve(b, th, order=4, scale=nsr.SCALE_INF_HALF, eps=eps, raise_on_error=False)
    assert rep.ns_stop == "diverged" and rep.status == nsr.NS_EDIVERGED
    # non-finite A: alpha is not finite
    bad = sysm.A.copy()
    bad[3, 5] = np.nan
    s.bind(to_dev(torch, bad))
    with pytest.raises(nsr.NSError) as e:
        s.init_scale()
    assert e.value.status == nsr.NS_ENOTSPD
    # composite needs the composite workspace
    s2 = nsr.Solver(n, composite=False)
    s2.bind(to_dev(torch, sysm.A))
    s2.init_scale()
    with pytest.raises(nsr.NSError) as e:
        s2.step(8, "composite_double")
    assert e.value.status == nsr.NS_EINVAL


def test_timing_counts_every_gemm(torch):
    sysm = inputs.spd_qlq(256, 1e2, seed=8)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(256)
    s.bind(A)
    s.timing(True)
    rep = s.solve(b, th, order=8)
    cnt, ms, fl = s.timing_read(0)
    assert cnt == rep.mmm and ms > 0.0
    assert 256.0 ** 2 * 257 * rep.mmm < fl < 2.0 * 256 ** 3 * rep.mmm   # powers halved
    assert rep.gemm_flop == pytest.approx(fl)


# --------------------------------------------------------------------------
# Richardson with the high-order accelerator (eq. ttk1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,kappa,order,q", [(130, 1e2, 4, 4), (300, 1e3, 8, 8), (200, 1e3, 2, 1),
                                             (97, 50.0, 4, 2)])
def test_accelerated_solve_matches_oracle(torch, n, kappa, order, q):
    sysm = inputs.spd_qlq(n, kappa, seed=900 + n)
    th, rep = gpu_solve(torch, sysm, order=order, form="composite_double", accel_q=q,
                        resid_tol=1e-13)
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=order, composite=True,
                                                           accel_q=q, resid_tol=1e-13))
    assert abs(rep.ns_steps - orc.ns_steps) <= 1
    compare_traces(rep.fnorm_hist, orc.fnorm_hist)
    compare_traces(rep.resid_hist, orc.resid_hist, rel=1e-8)
    assert rep.rel_resid <= max(1e-13, 2 * orc.rel_resid)
    assert np.linalg.norm(th - orc.theta) <= 10 * kappa * U * np.linalg.norm(orc.theta)


def test_accelerated_theta_eigen_closed_form(torch):
    """theta_K = theta* - Q diag(mu^{n + gamma_K}) Q^T theta* (eqs. riem5, riem6)
    for K steps before the rounding floor."""
    sysm = inputs.spd_qlq(256, 1e3, seed=77)
    n = 2
    for K in (1, 2):
        th, rep = gpu_solve(torch, sysm, order=n, form="composite_double", accel_q=n, k_max=K,
                            floor_detect=False, refine_max=0, resid_tol=0.0)
        mu = 1.0 - sysm.lam / rep.alpha
        theta_star = sysm.Q @ ((sysm.Q.T @ sysm.b) / sysm.lam)
        ex = n + oracle.riem6_gamma(K, n)
        ref = theta_star - sysm.Q @ ((mu ** ex) * (sysm.Q.T @ theta_star))
        assert np.linalg.norm(th - ref) <= 1e-10 * np.linalg.norm(theta_star), K


def test_accelerator_needs_composite(torch):
    sysm = inputs.spd_qlq(64, 10.0, seed=1)
    with pytest.raises(nsr.NSError) as e:
        gpu_solve(torch, sysm, order=4, form="squaring", accel_q=2)
    assert e.value.status == nsr.NS_EINVAL


def test_program_trials_match_oracle_steps(torch):
    """Every candidate program solves the same system to the tolerance; its
    Newton-Schulz step count agrees with the oracle's for that program (+-1)
    and the trials come back fastest first."""
    from paper_2008_11480_amd import autotune
    sysm = inputs.spd_qlq(256, 1e3, seed=77)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(256)
    s.bind(A)
    trials = autotune.time_programs(s, b, th, resid_tol=1e-12)
    assert len(trials) == len(autotune.CANDIDATES)
    assert all(t.ok for t in trials), [(t.program.name, t.rel_resid) for t in trials]
    assert [t.ms for t in trials] == sorted(t.ms for t in trials)
    for t in trials:
        pr = t.program
        orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(
            order=pr.order, form=pr.form, p=pr.p if pr.form.startswith("unified") else None,
            w=pr.w if pr.form.startswith("unified") else None, resid_tol=1e-12))
        assert abs(t.ns_steps - orc.ns_steps) <= 1, (pr.name, t.ns_steps, orc.ns_steps)


# --------------------------------------------------------------------------
# Diagonal preconditioner and initial series (Section 2, eqs. g01-g03)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [nsr.PREC_FP64, nsr.PREC_FP32])
@pytest.mark.parametrize("order,form", [(4, "squaring"), (8, "squaring"), (6, "unified"),
                                        (11, "table")])
def test_diag_preconditioner_matches_oracle(torch, prec, order, form):
    """S = diag(A) on a Jacobi-scaled SPD matrix (kappa(A) ~ 1e3, spectrum of
    S^-1/2 A S^-1/2 in [0.85, 1.15]): ||F_k|| trace against the oracle, the
    solve converges in fewer steps than with S = ||A||_F I."""
    sysm = inputs.spd_jacobi(211, seed=order)
    p, w = (2, 2) if form == "unified" else (0, 0)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(211, precision=prec)
    s.bind(A)
    tol = 1e-13 if prec == nsr.PREC_FP64 else 1e-10
    rep = s.solve(b, th, order=order, form=form, p=p, w=w, scale=nsr.SCALE_DIAG,
                  resid_tol=tol, refine_max=100)
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(
        order=order, form=form, p=p or None, w=w or None, scale="diag", resid_tol=1e-13))
    assert rep.alpha == pytest.approx(float(np.max(np.diag(sysm.A))), rel=1e-15)
    if prec == nsr.PREC_FP64:
        assert abs(rep.ns_steps - orc.ns_steps) <= 1
        compare_traces(rep.fnorm_hist, orc.fnorm_hist)
    else:
        assert rep.fnorm_hist[0] == pytest.approx(orc.fnorm_hist[0], rel=1e-6)
    assert rep.status == nsr.NS_OK and rep.rel_resid <= tol
    th_c = th.cpu().numpy()
    assert np.linalg.norm(sysm.b - sysm.A @ th_c) / np.linalg.norm(sysm.b) <= 1.01 * tol
    th2 = torch.zeros_like(b)
    rep_f = s.solve(b, th2, order=order, form=form, p=p, w=w, resid_tol=tol, refine_max=100)
    assert rep.ns_steps < rep_f.ns_steps


@pytest.mark.parametrize("n,order", [(211, 8), (300, 4), (1100, 8), (4096, 8)])
def test_diag_scaled_mirror_matches_full_products(torch, n, order):
    """With S = diag(A) the float64 power products compute their upper tiles
    and write the lower triangle as D_ji = D_ij s_j / s_i (F = S^1/2 F_s
    S^-1/2).  Same solve with every product in full: the ||F_k|| traces and
    theta agree to rounding (n = 4096 cuts the symmetric products' last,
    partial round of tiles along K, so the mirror also runs in the fixup)."""
    sysm = inputs.spd_jacobi(n, seed=n)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    s = nsr.Solver(n)
    s.bind(A)
    ths = []
    reps = []
    for sym in (True, False):
        s.set_symmetric(sym)
        th = torch.zeros_like(b)
        reps.append(s.solve(b, th, order=order, scale=nsr.SCALE_DIAG, resid_tol=1e-13))
        ths.append(th.cpu().numpy())
    r_sym, r_full = reps
    assert r_sym.ns_steps == r_full.ns_steps
    floor = max(min(r_sym.fnorm_hist), min(r_full.fnorm_hist))
    for a_, b_ in zip(r_sym.fnorm_hist, r_full.fnorm_hist):
        assert abs(a_ - b_) <= 1e-11 * b_ + 10 * floor
    assert np.linalg.norm(ths[0] - ths[1]) <= 1e-12 * np.linalg.norm(ths[1])
    assert r_sym.gemm_flop < r_full.gemm_flop


def test_diag_preconditioner_errors(torch):
    a = np.eye(8)
    a[3, 3] = 0.0
    s = nsr.Solver(8)
    s.bind(to_dev(torch, a))
    with pytest.raises(nsr.NSError) as e:
        s.init_scale(nsr.SCALE_DIAG)
    assert e.value.status == nsr.NS_ENOTSPD
    m = nsr.Solver(8, precision=nsr.PREC_MIXED_BF16)
    m.bind(to_dev(torch, np.eye(8)))
    with pytest.raises(nsr.NSError) as e:
        m.init_scale(nsr.SCALE_DIAG)
    assert e.value.status == nsr.NS_EINVAL


@pytest.mark.parametrize("h,p,w,order", [(4, 1, 2, 4), (3, 2, 1, 8), (6, 2, 2, 4), (2, 0, 0, 8)])
def test_initial_series_matches_oracle(torch, h, p, w, order):
    """Initial series of order h (eq. g01) before order-n steps: F_0 = Y^h, the
    trace ||F_k|| against the oracle and the exponent h n^k of the eigen closed
    form."""
    sysm = inputs.spd_qlq(180, 1e3, seed=h * 10 + order)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(180)
    s.bind(A)
    rep = s.solve(b, th, order=order, init_order=h, init_p=p, init_w=w, resid_tol=1e-13)
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(
        order=order, init_order=h, init_p=p if (p or w) else None,
        init_w=w if (p or w) else None, resid_tol=1e-13))
    compare_traces(rep.fnorm_hist, orc.fnorm_hist)
    mu = 1.0 - sysm.lam / rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        ref = math.sqrt(float(np.sum(mu ** (2 * h * order ** k))))
        if ref > 1e-8:
            assert fk == pytest.approx(ref, rel=1e-9), k
    assert rep.rel_resid <= 1e-13
    assert np.linalg.norm(th.cpu().numpy() - orc.theta) <= 1e3 * 1e3 * U * np.linalg.norm(orc.theta)


def test_initial_series_mixed(torch):
    sysm = inputs.spd_qlq(300, 1e4, seed=9)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(300, precision=nsr.PREC_MIXED_BF16)
    s.bind(A)
    rep = s.solve(b, th, order=8, init_order=4, init_p=1, init_w=2, resid_tol=1e-10,
                  refine_max=100)
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10
    with pytest.raises(nsr.NSError):
        s.solve(b, th, order=8, form="composite_double", init_order=4)


# --------------------------------------------------------------------------
# General composite (eqs. gkgen1-ga1) and the [sri] algorithm of Remark 2
# --------------------------------------------------------------------------

@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("order,rates", [(2, (2,)), (4, (2, 4)), (2, (4, 2, 2)), (4, (1, 2)),
                                         (1, (1,))])
def test_composite_general_matches_oracle(torch, order, rates, symmetric):
    """||F_k|| trace against the oracle and the exponent e_k = n e_{k-1} +
    sum m_i^k of the eigen closed form."""
    n = 150
    kappa = 10.0 if order == 1 else 1e3
    sysm = inputs.spd_qlq(n, kappa, seed=len(rates) + 3 * order)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(n, composite=len(rates))
    s.set_symmetric(symmetric)
    s.bind(A)
    s.set_composite_rates(rates)
    kmax = 64 if order > 1 else 40
    rep = s.solve(b, th, order=order, form="composite_general", resid_tol=1e-13, k_max=kmax,
                  refine_max=200)
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=order, rates=tuple(rates),
                                                           resid_tol=1e-13, k_max=kmax,
                                                           refine_max=200))
    assert abs(rep.ns_steps - orc.ns_steps) <= 1
    compare_traces(rep.fnorm_hist, orc.fnorm_hist)
    mu = 1.0 - sysm.lam / rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        ref = math.sqrt(float(np.sum(mu ** (2 * oracle.gc_exponent(k, order, rates)))))
        if ref > 1e-8:
            assert fk == pytest.approx(ref, rel=1e-9), k
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-13


@pytest.mark.parametrize("order", [2, 4, 8])
def test_sri_matches_oracle(torch, order):
    sysm = inputs.spd_qlq(170, 1e3, seed=40 + order)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(170, composite=1)
    s.bind(A)
    rep = s.solve(b, th, order=order, form="sri", resid_tol=1e-13)
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=order, sri=True,
                                                           resid_tol=1e-13))
    assert abs(rep.ns_steps - orc.ns_steps) <= 1
    compare_traces(rep.fnorm_hist, orc.fnorm_hist)
    mu = 1.0 - sysm.lam / rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        ref = math.sqrt(float(np.sum(mu ** (2 * oracle.sri_exponent(k, order)))))
        if ref > 1e-8:
            assert fk == pytest.approx(ref, rel=1e-9), k
    assert rep.rel_resid <= 1e-13
    assert np.linalg.norm(th.cpu().numpy() - orc.theta) <= 1e4 * 1e3 * U * np.linalg.norm(orc.theta)


def test_composite_general_and_sri_mixed(torch):
    sysm = inputs.spd_qlq(300, 1e4, seed=17)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    s = nsr.Solver(300, precision=nsr.PREC_MIXED_BF16, composite=2)
    s.bind(A)
    s.set_composite_rates((2, 4))
    th = torch.zeros_like(b)
    rep = s.solve(b, th, order=4, form="composite_general", resid_tol=1e-10, refine_max=100)
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10
    th = torch.zeros_like(b)
    rep = s.solve(b, th, order=8, form="sri", resid_tol=1e-10, refine_max=100)
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10


def test_composite_general_errors(torch):
    s = nsr.Solver(64, composite=2)
    s.bind(torch.eye(64, dtype=torch.float64, device="cuda") * 2.0)
    with pytest.raises(nsr.NSError) as e:
        s.set_composite_rates((2, 2, 2))            # three loops, workspace for two
    assert e.value.status == nsr.NS_EINVAL
    with pytest.raises(nsr.NSError):
        s.set_composite_rates((0,))                 # below 1
    b = torch.ones(64, dtype=torch.float64, device="cuda")
    with pytest.raises(nsr.NSError) as e:
        s.solve(b, torch.zeros_like(b), order=4, form="composite_general")
    assert e.value.status == nsr.NS_ESTATE
    p = nsr.Solver(64, composite=0)
    p.bind(torch.eye(64, dtype=torch.float64, device="cuda"))
    with pytest.raises(nsr.NSError):
        p.solve(b, torch.zeros_like(b), order=4, form="sri")


@pytest.mark.parametrize("order", [3, 5])
def test_composite_horner_orders_match_oracle(torch, order):
    """Composite loops of orders that are not powers of two (Horner sums):
    double NS and [sri] against the oracle's Horner form."""
    sysm = inputs.spd_qlq(140, 1e3, seed=order)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    s = nsr.Solver(140, composite=1)
    s.bind(A)
    for form, kw in (("composite_double", dict(composite=True)), ("sri", dict(sri=True))):
        th = torch.zeros_like(b)
        rep = s.solve(b, th, order=order, form=form, resid_tol=1e-13)
        orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=order, form="horner",
                                                               resid_tol=1e-13, **kw))
        assert abs(rep.ns_steps - orc.ns_steps) <= 1, form
        compare_traces(rep.fnorm_hist, orc.fnorm_hist)
        assert rep.rel_resid <= 1e-13


def test_three_frequency_analogue_matches_oracle(torch):
    """Per-step parameters of the accelerated Richardson iteration (double NS
    n = 3, q = 3) and of classical order-8 Newton-Schulz on the three-frequency
    regressor, against the oracle (fixed step counts, no refinement)."""
    sysm = inputs.harmonic_three()
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    s = nsr.Solver(6, composite=1)
    s.bind(A)
    for k in range(1, 7):
        for kw, okw in ((dict(order=3, form="composite_double", accel_q=3),
                         dict(order=3, form="horner", composite=True, accel_q=3)),
                        (dict(order=8, form="squaring"), dict(order=8))):
            th = torch.zeros_like(b)
            s.solve(b, th, k_max=k, floor_detect=False, refine_max=0, resid_tol=0.0,
                    raise_on_error=False, **kw)
            orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(
                k_max=k, floor_detect=False, refine_max=0, resid_tol=0.0, **okw))
            x = th.cpu().numpy()
            assert np.linalg.norm(x - orc.theta) <= 1e-9 * np.linalg.norm(orc.theta), (k, kw)


# --------------------------------------------------------------------------
# Captured fixed-length iteration (HIP graph)
# --------------------------------------------------------------------------

GRAPH_CASES = [
    # precision, n, kappa, order, form, k_max
    (nsr.PREC_FP64, 64, 1e2, 4, "squaring", 12),      # the N = 64, 12-step workload
    (nsr.PREC_FP64, 300, 1e3, 8, "squaring", 6),
    (nsr.PREC_FP64, 257, 1e3, 11, "table", 5),
    (nsr.PREC_MIXED_BF16, 300, 1e3, 8, "squaring", 6),
    (nsr.PREC_FP32, 200, 1e2, 6, "unified", 5),
    (nsr.PREC_MIXED_SPLIT, 300, 1e3, 8, "squaring", 6),
    (nsr.PREC_MIXED_SPLIT, 2100, 1e3, 8, "squaring", 4),   # 128-wide split tiles
]


@pytest.mark.parametrize("prec,n,kappa,order,form,kmax", GRAPH_CASES)
def test_graph_fixed_length_matches_eager(torch, prec, n, kappa, order, form, kmax):
    """The captured Newton-Schulz phase runs the same kernels in the same order
    as the eager loop: theta and the ||F_k|| / residual histories are
    bit-identical, on the first (capturing) solve and on every replay, with
    eager work and synchronisations between the replays."""
    sysm = inputs.spd_qlq(n, kappa, seed=n + order)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    p, w = (2, 2) if form == "unified" else (0, 0)
    kw = dict(order=order, form=form, p=p, w=w, k_max=kmax, floor_detect=False,
              resid_tol=1e-13 if prec == nsr.PREC_FP64 else 1e-10, refine_max=100)
    s = nsr.Solver(n, precision=prec, composite=0)
    s.bind(A)
    th_e = torch.zeros_like(b)
    rep_e = s.solve(b, th_e, **kw)
    ref = th_e.cpu().numpy()
    th_g = torch.zeros_like(b)
    other = nsr.Solver(n, precision=prec, composite=0)
    other.bind(A)
    for rep_i in range(4):
        th_g.zero_()
        rep_g = s.solve(b, th_g, graph=True, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(th_g.cpu().numpy(), ref), rep_i
        assert rep_g.fnorm_hist == rep_e.fnorm_hist, rep_i
        assert rep_g.resid_hist == rep_e.resid_hist, rep_i
        assert rep_g.ns_steps == kmax and rep_g.ns_stop == "k_max"
        assert rep_g.mmm == rep_e.mmm and rep_g.gemm_flop == rep_e.gemm_flop
        # eager work in between (another solver on the same stream) and a sync
        other.solve(b, torch.zeros_like(b), **kw)
        torch.cuda.synchronize()
    # a different theta buffer: the graph is captured again for it
    th2 = torch.zeros_like(b)
    s.solve(b, th2, graph=True, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(th2.cpu().numpy(), ref)


def test_graph_ignored_for_adaptive_schedules(torch):
    """With the floor test on, the schedule depends on device values: the
    graph flag is ignored and the solve equals the eager one."""
    sysm = inputs.spd_qlq(128, 1e3, seed=5)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    s = nsr.Solver(128, composite=0)
    s.bind(A)
    t1, t2 = torch.zeros_like(b), torch.zeros_like(b)
    r1 = s.solve(b, t1, order=8, resid_tol=1e-13)
    r2 = s.solve(b, t2, order=8, resid_tol=1e-13, graph=True)
    assert np.array_equal(t1.cpu().numpy(), t2.cpu().numpy())
    assert r1.fnorm_hist == r2.fnorm_hist
