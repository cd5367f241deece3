"""GPU parity of the float32 / bf16 MFMA GEMMs and of the float32 and mixed
(bf16 powers, float32 residual and G-side, float64 Richardson) solver modes.

Tolerances:
* float32 / bf16 GEMMs: |D - D_ref| <= 2 gamma^(32)_{k+4} (|s||X||op(Y)| + |diag| I
  + |E1| + |E2|) with u = 2^-24 (bf16 products are exact in float32, so the
  float32 accumulation bound applies to both); the bf16 copy Db must equal
  D rounded to nearest even.
* Solves: the returned theta has relative residual <= 1e-10 after float64
  refinement, and its forward error against the float64 oracle is within
  50 kappa u64 (refinement with a float64 residual converges to the float64
  solution).  ||F_k|| traces follow the oracle while the iteration is above
  the low-precision floor: 1e-4 relative (float32) / 3e-2 relative (mixed:
  the bf16 rounding of the operands, ~4e-3, enters F_{k+1} additively).
"""
import numpy as np
import pytest

import oracle
from paper_2008_11480_amd import inputs, nsr

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def torch():
    import torch as _torch
    if not _torch.cuda.is_available():
        pytest.skip("no GPU")
    nsr.lib()
    return _torch


def g32(m):
    return m * U32 / (1 - m * U32)


SHAPES = [(1, 1, 1), (5, 3, 7), (64, 64, 64), (100, 37, 250), (129, 130, 131),
          (257, 300, 129), (1000, 999, 1001), (2100, 2000, 300)]


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_gemm_f32_elementwise(torch, m, n, k):
    g = torch.Generator(device="cpu").manual_seed(m * 31 + n * 7 + k)
    X = torch.randn(m, k, generator=g, dtype=torch.float32)
    Y = torch.randn(k, n, generator=g, dtype=torch.float32)
    E1 = torch.randn(m, n, generator=g, dtype=torch.float32)
    E2 = torch.randn(m, n, generator=g, dtype=torch.float32)
    diag, scale = 0.75, -1.25
    D, Db, ss = nsr.gemm_lp(X.cuda(), Y.cuda(), nt=False, want_bf16=True, E1=E1.cuda(),
                            E2=E2.cuda(), diag=diag, scale=scale, want_sumsq=True)
    torch.cuda.synchronize()
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    ref = scale * (Xd @ Yd) + diag * np.eye(m, n) + E1.double().numpy() + E2.double().numpy()
    bound = g32(k + 4) * (abs(scale) * (np.abs(Xd) @ np.abs(Yd)) + abs(diag) * np.eye(m, n)
                          + np.abs(E1.double().numpy()) + np.abs(E2.double().numpy()))
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))
    assert torch.equal(Db.cpu(), D.cpu().to(torch.bfloat16))
    ssr = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ssr) <= 1e-12 * ssr


@pytest.mark.parametrize("addends", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", SHAPES + [(64, 64, 40), (70, 50, 9), (4100, 4000, 200)])
def test_gemm_bf16_nt_elementwise(torch, m, n, k, addends):
    """Every epilogue form (no addend, E1, E1 + E2) on every tile family
    (64, 128 and, for the 4100 x 4000 output, 256-wide tiles with ragged
    edges)."""
    g = torch.Generator(device="cpu").manual_seed(m * 17 + n * 5 + k)
    X = torch.randn(m, k, generator=g).to(torch.bfloat16)
    Y = torch.randn(n, k, generator=g).to(torch.bfloat16)       # n x k: D = X Y^T
    E = [torch.randn(m, n, generator=g, dtype=torch.float32) for _ in range(addends)]
    diag, scale = 1.0, -0.5
    D, Db, ss = nsr.gemm_lp(X.cuda(), Y.cuda(), nt=True, want_bf16=True,
                            E1=E[0].cuda() if addends > 0 else None,
                            E2=E[1].cuda() if addends > 1 else None,
                            diag=diag, scale=scale, want_sumsq=True)
    torch.cuda.synchronize()
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    Ed = [e.double().numpy() for e in E]
    ref = scale * (Xd @ Yd.T) + diag * np.eye(m, n) + sum(Ed, np.zeros((m, n)))
    bound = g32(k + 4) * (abs(scale) * (np.abs(Xd) @ np.abs(Yd).T) + diag * np.eye(m, n)
                          + sum((np.abs(e) for e in Ed), np.zeros((m, n))))
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))
    assert torch.equal(Db.cpu(), D.cpu().to(torch.bfloat16))
    ssr = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ssr) <= 1e-12 * ssr


def test_gemm_bf16_full_size_sampled(torch):
    """N=8192 (the mixed workload's GEMM shape and launch configuration):
    2000 sampled entries against float64 dot products of the bf16 inputs."""
    n = 8192
    g = torch.Generator(device="cuda").manual_seed(7)
    X = torch.randn(n, n, device="cuda", generator=g).to(torch.bfloat16)
    Y = torch.randn(n, n, device="cuda", generator=g).to(torch.bfloat16)
    D, _, _ = nsr.gemm_lp(X, Y, nt=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    ii, jj = rng.integers(0, n, 2000), rng.integers(0, n, 2000)
    Xc, Yc, Dc = X.double().cpu().numpy(), Y.double().cpu().numpy(), D.double().cpu().numpy()
    for i, j in zip(ii, jj):
        ref = float(Xc[i] @ Yc[j])
        bound = 2 * g32(n + 4) * float(np.abs(Xc[i]) @ np.abs(Yc[j]))
        assert abs(Dc[i, j] - ref) <= bound, (i, j)


def test_gemm_f32_full_size_sampled(torch):
    n = 8192
    g = torch.Generator(device="cuda").manual_seed(8)
    X = torch.randn(n, n, device="cuda", generator=g)
    Y = torch.randn(n, n, device="cuda", generator=g)
    D, _, _ = nsr.gemm_lp(X, Y, nt=False, diag=1.0, scale=-1.0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    ii, jj = rng.integers(0, n, 2000), rng.integers(0, n, 2000)
    Xc, Yc, Dc = X.double().cpu().numpy(), Y.double().cpu().numpy(), D.double().cpu().numpy()
    for i, j in zip(ii, jj):
        ref = -float(Xc[i] @ Yc[:, j]) + (i == j)
        bound = 2 * g32(n + 4) * (float(np.abs(Xc[i]) @ np.abs(Yc[:, j])) + (i == j))
        assert abs(Dc[i, j] - ref) <= bound, (i, j)


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run(torch, sysm, precision, **kw):
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(sysm.n, precision=precision, composite=kw.get("form") == "composite_double")
    s.bind(A)
    rep = s.solve(b, th, **kw)
    torch.cuda.synchronize()
    return s, th.cpu().numpy(), rep


LOWP_CASES = [
    # precision, n, kappa, order, form
    (nsr.PREC_FP32, 300, 1e3, 4, "squaring"),
    (nsr.PREC_FP32, 257, 1e4, 8, "squaring"),
    (nsr.PREC_FP32, 200, 1e2, 3, "horner"),
    (nsr.PREC_MIXED_BF16, 300, 1e3, 8, "squaring"),
    (nsr.PREC_MIXED_BF16, 511, 1e5, 8, "squaring"),
    (nsr.PREC_MIXED_BF16, 300, 1e4, 8, "composite_double"),
    (nsr.PREC_MIXED_BF16, 130, 1e2, 4, "composite_double"),
    (nsr.PREC_MIXED_BF16, 33, 10.0, 2, "squaring"),
    (nsr.PREC_FP32, 300, 1e4, 11, "table"),
    (nsr.PREC_MIXED_BF16, 300, 1e4, 11, "table"),
    (nsr.PREC_MIXED_BF16, 257, 1e5, 15, "table"),
    (nsr.PREC_MIXED_BF16, 200, 1e4, 45, "table"),
]


@pytest.mark.parametrize("prec,n,kappa,order,form", LOWP_CASES)
def test_lowp_solve_matches_oracle(torch, prec, n, kappa, order, form):
    sysm = inputs.spd_qlq(n, kappa, seed=500 + n)
    s, th, rep = run(torch, sysm, prec, order=order, form=form, resid_tol=1e-10,
                     refine_max=100)
    assert rep.precision == prec
    assert rep.status == nsr.NS_OK, (rep.refine_stop, rep.rel_resid)
    assert rep.rel_resid <= 1e-10
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(
        order=order, form="squaring" if form == "composite_double" else form,
        composite=form == "composite_double", resid_tol=1e-13))
    fwd = np.linalg.norm(th - orc.theta) / np.linalg.norm(orc.theta)
    # The refinement stops once the residual is below the tolerance, so the
    # forward error is bounded by kappa times the attained residual (plus the
    # oracle's own float64 error), not by the float64 floor.
    rel_cpu = np.linalg.norm(sysm.b - sysm.A @ th) / np.linalg.norm(sysm.b)
    assert fwd <= 1.01 * kappa * rel_cpu + 50 * kappa * U64 + 1e-300, (fwd, rel_cpu)
    rel = 1e-4 if prec == nsr.PREC_FP32 else 3e-2
    floor = min(rep.fnorm_hist)
    for k in range(min(len(rep.fnorm_hist), len(orc.fnorm_hist))):
        ref = orc.fnorm_hist[k]
        if ref > 100 * floor:
            assert abs(rep.fnorm_hist[k] - ref) <= rel * ref + 10 * floor, (k, rep.fnorm_hist[k], ref)
    # Richardson contraction: the final G is a contraction for A (rho(I - G A) < 1/2)
    G = s.get_G().cpu().numpy()
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(n) - G @ sysm.A)))
    assert rho < 0.5, rho


def test_mixed_bind_converts_A(torch):
    """ns_bind in a low-precision mode stores float32(A); the first residual
    F_0 = I - A / alpha is formed from float64 A and rounded once."""
    sysm = inputs.spd_qlq(100, 10.0, seed=3)
    s = nsr.Solver(100, precision=nsr.PREC_MIXED_BF16)
    s.bind(to_dev(torch, sysm.A))
    alpha, f0 = s.init_scale()
    F = s.get_F().cpu().numpy()
    ref = (np.eye(100) - sysm.A / alpha).astype(np.float32).astype(np.float64)
    assert np.all(np.abs(F - ref) <= U32 * 2 * np.abs(ref) + 1e-45)     # one float32 rounding
    assert f0 == pytest.approx(np.linalg.norm(ref), rel=1e-12)


def test_mixed_accelerated_composite(torch):
    """Mixed precision with the accelerator of eq. (ttk1): reaches 1e-10 and
    agrees with the float64 oracle to the refinement's accuracy."""
    sysm = inputs.spd_qlq(300, 1e4, seed=31)
    s, th, rep = run(torch, sysm, nsr.PREC_MIXED_BF16, order=8, form="composite_double",
                     accel_q=8, resid_tol=1e-10, refine_max=100)
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10
    orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=8, composite=True, accel_q=8,
                                                           resid_tol=1e-13))
    fwd = np.linalg.norm(th - orc.theta) / np.linalg.norm(orc.theta)
    assert fwd <= 1e4 * 2e-10, fwd
