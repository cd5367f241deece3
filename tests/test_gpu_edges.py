"""Edge cases of the solver and the batch through the C ABI: degenerate and
ragged inputs, padded leading dimensions, empty batches, indefinite
matrices, a zero right-hand side."""
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


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("prec", [nsr.PREC_FP64, nsr.PREC_FP32, nsr.PREC_MIXED_BF16])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 127, 129, 255])
def test_ragged_sizes_converge(torch, prec, n):
    """Sizes around the tile edges (16, 32, 64, 128) in every precision reach
    the tolerance; float64 follows the oracle's trace."""
    sysm = inputs.spd_qlq(n, 1e2, seed=200 + n)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    th = torch.zeros_like(b)
    s = nsr.Solver(n, precision=prec, composite=0)
    s.bind(A)
    tol = 1e-13 if prec == nsr.PREC_FP64 else 1e-10
    rep = s.solve(b, th, order=8, resid_tol=tol, refine_max=100)
    assert rep.status == nsr.NS_OK, (rep.ns_stop, rep.refine_stop, rep.rel_resid)
    x = th.cpu().numpy()
    assert np.linalg.norm(sysm.b - sysm.A @ x) <= 1.01 * tol * np.linalg.norm(sysm.b)
    if prec == nsr.PREC_FP64:
        orc = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=8, resid_tol=tol))
        assert abs(rep.ns_steps - orc.ns_steps) <= 1
        for g, o in zip(rep.fnorm_hist, orc.fnorm_hist):
            assert abs(g - o) <= 1e-10 * o + 1e-12


@pytest.mark.parametrize("pad", [38, 37])
def test_padded_leading_dimension(torch, pad):
    """A is a view into a wider buffer (lda > n): the same result as a compact
    A -- bit for bit when lda is even (the residual GEMV reads rows two
    elements at a time either way), to rounding when it is odd (rows read
    one element per lane, another summation order)."""
    n = 100
    sysm = inputs.spd_qlq(n, 1e3, seed=4)
    big = np.zeros((n, n + pad))
    big[:, :n] = sysm.A
    Ad = to_dev(torch, big)[:, :n]
    assert Ad.stride(0) == n + pad
    b = to_dev(torch, sysm.b)
    s = nsr.Solver(n, composite=0)
    s.bind(Ad)
    t1 = torch.zeros_like(b)
    r1 = s.solve(b, t1, order=4, resid_tol=1e-13)
    s.bind(to_dev(torch, sysm.A))
    t2 = torch.zeros_like(b)
    r2 = s.solve(b, t2, order=4, resid_tol=1e-13)
    x1, x2 = t1.cpu().numpy(), t2.cpu().numpy()
    if pad % 2 == 0:
        assert np.array_equal(x1, x2)
        assert r1.fnorm_hist == r2.fnorm_hist
    else:
        assert np.linalg.norm(x1 - x2) <= 1e-13 * np.linalg.norm(x2)
        assert r1.ns_steps == r2.ns_steps
        for a_, b_ in zip(r1.fnorm_hist, r2.fnorm_hist):
            assert abs(a_ - b_) <= 1e-12 * b_ + 1e-15


def test_scalar_identity_and_zero_rhs(torch):
    """A = c I: F_0 = (1 - 1/sqrt(n)) I, the iteration converges like a scalar;
    n = 1: F_0 = 0 stops at once (f_tol 0).  b = 0 gives theta = 0."""
    for n in (1, 40):
        A = to_dev(torch, 3.5 * np.eye(n))
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        th = torch.zeros_like(b)
        s = nsr.Solver(n, composite=0)
        s.bind(A)
        rep = s.solve(b, th, order=4, resid_tol=1e-14)
        assert rep.status == nsr.NS_OK
        assert np.allclose(th.cpu().numpy(), 1.0 / 3.5, rtol=1e-14, atol=0)
        if n == 1:
            assert rep.ns_stop == "f_tol" and rep.fnorm_hist[0] == 0.0
    sysm = inputs.spd_qlq(30, 10.0, seed=1)
    s = nsr.Solver(30, composite=0)
    s.bind(to_dev(torch, sysm.A))
    z = torch.zeros(30, dtype=torch.float64, device="cuda")
    th = torch.full_like(z, 7.0)
    rep = s.solve(z, th, order=4, resid_tol=1e-12)
    assert rep.status == nsr.NS_OK
    assert np.array_equal(th.cpu().numpy(), np.zeros(30))


def test_indefinite_matrix_diverges(torch):
    """An indefinite A: with alpha = ||A||_F, F_0 has the eigenvalue
    1 - lambda_min / alpha > 1, so ||F_k|| grows and the solve reports
    divergence instead of a result."""
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    lam = np.linspace(1.0, 10.0, 50)
    lam[0] = -2.0
    A = (q * lam) @ q.T
    A = 0.5 * (A + A.T)
    s = nsr.Solver(50, composite=0)
    s.bind(to_dev(torch, A))
    b = torch.ones(50, dtype=torch.float64, device="cuda")
    rep = s.solve(b, torch.zeros_like(b), order=4, raise_on_error=False)
    assert rep.ns_stop == "diverged" and rep.status == nsr.NS_EDIVERGED


def test_batch_empty_and_unit_systems(torch):
    B = nsr.Batch(max_n=8, max_count=16, slots=4)
    t = B.submit([], [], [], order=4)
    assert B.poll(t, wait=True) == []
    As = [torch.full((1, 1), float(i + 1), dtype=torch.float64, device="cuda") for i in range(9)]
    bs = [torch.ones(1, dtype=torch.float64, device="cuda") for _ in range(9)]
    ths = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(9)]
    reps = B.poll(B.submit(As, bs, ths, order=4, resid_tol=1e-12), wait=True)
    assert all(r.status == nsr.NS_OK for r in reps)
    for i, t in enumerate(ths):
        assert float(t.cpu()) == pytest.approx(1.0 / (i + 1), rel=1e-12)
