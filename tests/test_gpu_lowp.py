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


def split_bound(Xd, Yd, scale, k):
    """Element-wise bound of the split half-precision product (see
    ns_gemm_f32_split): each operand keeps 22 bits (|x - x^| <= 2^-22 |x|,
    plus half a half-precision subnormal step, 2^-25 2^-e <= 2^-39 max|X|),
    the dropped lo lo term is below 2^-22 |x| |y|, and the three products are
    accumulated in float32 (3k terms)."""
    ax, ay = np.abs(Xd), np.abs(Yd)
    mx, my = ax.max(initial=0.0), ay.max(initial=0.0)
    prod = ax @ ay
    eta = 2.0 ** -38 * (mx * ay.sum(axis=0)[None, :] + my * ax.sum(axis=1)[:, None])
    return abs(scale) * ((3 * 2.0 ** -22 + g32(3 * k + 4)) * prod + eta)


@pytest.mark.parametrize("addends", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", SHAPES + [(64, 64, 40), (70, 50, 9), (4100, 4000, 200)])
def test_gemm_f32_split_elementwise(torch, m, n, k, addends):
    """Split half-precision product against float64 on every tile family
    (64, 128, 256) with ragged edges and every epilogue form."""
    g = torch.Generator(device="cpu").manual_seed(m * 13 + n * 11 + k + addends)
    X = torch.randn(m, k, generator=g, dtype=torch.float32)
    Y = torch.randn(k, n, generator=g, dtype=torch.float32)
    E = [torch.randn(m, n, generator=g, dtype=torch.float32) for _ in range(addends)]
    diag, scale = 0.75, -1.25
    D, Db, ss = nsr.gemm_f32_split(X.cuda(), Y.cuda(), want_bf16=True,
                                   E1=E[0].cuda() if addends > 0 else None,
                                   E2=E[1].cuda() if addends > 1 else None,
                                   diag=diag, scale=scale, want_sumsq=True)
    torch.cuda.synchronize()
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    Ed = [e.double().numpy() for e in E]
    ref = scale * (Xd @ Yd) + diag * np.eye(m, n) + sum(Ed, np.zeros((m, n)))
    bound = split_bound(Xd, Yd, scale, k) + g32(k + 4) * (
        abs(diag) * np.eye(m, n) + sum((np.abs(e) for e in Ed), np.zeros((m, n))))
    bound = bound + g32(4) * np.abs(ref)
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))
    assert torch.equal(Db.cpu(), D.cpu().to(torch.bfloat16))
    ssr = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ssr) <= 1e-12 * ssr


@pytest.mark.parametrize("tile", [256, 128])
@pytest.mark.parametrize("addends", [0, 2])
@pytest.mark.parametrize("m,n,k", [(300, 520, 32), (1000, 700, 96), (2100, 1900, 1024),
                                   (4100, 4000, 224), (300, 256, 100)])
def test_gemm_f32_split_dma_tiles(torch, m, n, k, addends, tile):
    """The 256 x 256 and 128 x 128 split tiles fed by LDS DMA (K a multiple
    of 32): one to many slabs, ragged edge tiles, every epilogue form; the
    last shape (K = 100) falls back to the register-staged kernel."""
    b = int(np.ceil(np.log2(max(m, n))))
    nsr.tile_set(nsr.TILE_F16S, b, tile)
    try:
        g = torch.Generator(device="cpu").manual_seed(m * 3 + n * 17 + k)
        X = torch.randn(m, k, generator=g, dtype=torch.float32)
        Y = torch.randn(k, n, generator=g, dtype=torch.float32)
        E = [torch.randn(m, n, generator=g, dtype=torch.float32) for _ in range(addends)]
        diag, scale = 0.75, -1.25
        print(f"split dma tiles {m}x{n}x{k} addends {addends}", flush=True)
        D, Db, ss = nsr.gemm_f32_split(X.cuda(), Y.cuda(), want_bf16=True,
                                       E1=E[0].cuda() if addends > 0 else None,
                                       E2=E[1].cuda() if addends > 1 else None,
                                       diag=diag, scale=scale, want_sumsq=True)
        torch.cuda.synchronize()
    finally:
        nsr.tile_set(nsr.TILE_F16S, b, 0)
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    Ed = [e.double().numpy() for e in E]
    ref = scale * (Xd @ Yd) + diag * np.eye(m, n) + sum(Ed, np.zeros((m, n)))
    bound = split_bound(Xd, Yd, scale, k) + g32(k + 4) * (
        abs(diag) * np.eye(m, n) + sum((np.abs(e) for e in Ed), np.zeros((m, n))))
    bound = bound + g32(4) * np.abs(ref)
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))
    assert torch.equal(Db.cpu(), D.cpu().to(torch.bfloat16))
    ssr = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ssr) <= 1e-12 * ssr


@pytest.mark.parametrize("sx,sy", [(1e-8, 1e6), (3e12, 2e-15), (1.0, 1e-30)])
def test_gemm_f32_split_operand_scales(torch, sx, sy):
    """Operands far outside the half-precision range are scaled into it (the
    exponents are per operand) and scaled back exactly."""
    m, n, k = 300, 200, 500
    g = torch.Generator(device="cpu").manual_seed(5)
    X = torch.randn(m, k, generator=g, dtype=torch.float32) * sx
    Y = torch.randn(k, n, generator=g, dtype=torch.float32) * sy
    D, _, _ = nsr.gemm_f32_split(X.cuda(), Y.cuda())
    torch.cuda.synchronize()
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    ref = Xd @ Yd
    bound = split_bound(Xd, Yd, 1.0, k) + g32(2) * np.abs(ref)
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))


def test_gemm_f32_split_degenerate(torch):
    """A zero operand (exponent 0), k = 0 (D = diag I + E1) and a wide
    dynamic range inside one operand."""
    m, n, k = 130, 70, 90
    g = torch.Generator(device="cpu").manual_seed(9)
    Y = torch.randn(k, n, generator=g, dtype=torch.float32)
    E1 = torch.randn(m, n, generator=g, dtype=torch.float32)
    D, _, _ = nsr.gemm_f32_split(torch.zeros(m, k).cuda(), Y.cuda(), E1=E1.cuda(), diag=2.0)
    torch.cuda.synchronize()
    assert torch.equal(D.cpu(), E1 + 2.0 * torch.eye(m, n))
    D0, _, _ = nsr.gemm_f32_split(torch.empty(m, 0).cuda(), torch.empty(0, n).cuda(),
                                  E1=E1.cuda(), diag=-1.0)
    torch.cuda.synchronize()
    assert torch.equal(D0.cpu(), E1 - torch.eye(m, n))
    # entries spread over 2^-60 .. 2^20 in one operand
    X = torch.randn(m, k, generator=g, dtype=torch.float32)
    X = X * torch.pow(2.0, torch.randint(-60, 21, (m, k), generator=g).float())
    D, _, _ = nsr.gemm_f32_split(X.cuda(), Y.cuda())
    torch.cuda.synchronize()
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    ref = Xd @ Yd
    bound = split_bound(Xd, Yd, 1.0, k) + g32(2) * np.abs(ref)
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))


def test_gemm_f32_split_full_size_sampled(torch):
    """N = 8192 (256-wide tiles, the mixed composite's size): sampled
    elements against float64 dot products."""
    n = 8192
    g = torch.Generator(device="cuda").manual_seed(21)
    X = torch.randn(n, n, generator=g, device="cuda", dtype=torch.float32)
    Y = torch.randn(n, n, generator=g, device="cuda", dtype=torch.float32)
    E1 = torch.randn(n, n, generator=g, device="cuda", dtype=torch.float32)
    D, _, _ = nsr.gemm_f32_split(X, Y, E1=E1, diag=1.0, scale=-1.0)
    torch.cuda.synchronize()
    rs = np.random.default_rng(4)
    rows = rs.integers(0, n, 64)
    cols = rs.integers(0, n, 64)
    Xs = X[torch.as_tensor(rows, device="cuda")].double().cpu().numpy()
    Ys = Y[:, torch.as_tensor(cols, device="cuda")].double().cpu().numpy()
    Es = E1.double().cpu().numpy()[rows][:, cols]
    ref = -(Xs @ Ys) + np.eye(n)[rows][:, cols] + Es
    bound = split_bound(Xs, Ys, 1.0, n) + g32(n + 4) * (np.abs(Es) + 1.0)
    got = D.double().cpu().numpy()[rows][:, cols]
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))


SYM_SKIP = pytest.mark.skip(
    reason="symmetric-output bf16 kernel disabled: its first GPU run (N=3000, K=3000, no "
           "addends) ended in a memory aperture violation whose cause has not been found")


def sym_operands(torch, n, k, addends, seed):
    """bf16 X, Y with X Y^T symmetric in exact arithmetic (Y = X) and
    symmetric float32 addends."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.randn(n, k, generator=g).to(torch.bfloat16)
    E = []
    for _ in range(addends):
        e = torch.randn(n, n, generator=g, dtype=torch.float32)
        E.append((e + e.T) / 2)
    return X, E


@SYM_SKIP
@pytest.mark.parametrize("addends", [0, 2])
@pytest.mark.parametrize("n,k", [(3000, 3000), (4096, 4096), (4100, 640), (3333, 70)])
def test_gemm_bf16_symmetric_output(torch, n, k, addends):
    """Symmetric-output bf16 product: the lower triangle is the exact mirror
    of the upper one (D and Db bitwise symmetric), the upper triangle meets
    the element-wise bound against float64, Db = bf16(D) and the sum of
    squares covers both triangles.  Shapes: one partial round (3000, 3333
    with K = 70, a ragged last K slab), a round plus a split tail (4096:
    512 whole tiles + 16 tiles in 32 K-slices), ragged tiles with a tail
    (4100 with K = 640)."""
    X, E = sym_operands(torch, n, k, addends, seed=n + k + addends)
    Xc = X.cuda()
    D, Db, ss = nsr.gemm_bf16_sym(Xc, Xc, want_bf16=True,
                                  E1=E[0].cuda() if addends > 0 else None,
                                  E2=E[1].cuda() if addends > 1 else None,
                                  diag=1.0, scale=-0.5, want_sumsq=True)
    torch.cuda.synchronize()
    assert torch.equal(D, D.T) and torch.equal(Db, Db.T)
    assert torch.equal(Db, D.to(torch.bfloat16))
    Xd = X.double().cuda()
    ref = -0.5 * (Xd @ Xd.T) + torch.eye(n, dtype=torch.float64, device="cuda")
    babs = 0.5 * (Xd.abs() @ Xd.abs().T) + torch.eye(n, dtype=torch.float64, device="cuda")
    for e in E:
        ref += e.double().cuda()
        babs += e.double().cuda().abs()
    err = (D.double() - ref).abs()
    up = torch.triu(torch.ones(n, n, dtype=torch.bool, device="cuda"))
    bound = 2 * g32(k + 4) * babs
    assert bool(torch.all(err[up] <= bound[up])), float((err / bound)[up].max())
    ssr = float((D.double() ** 2).sum())
    assert abs(float(ss.cpu()) - ssr) <= 1e-12 * ssr


@SYM_SKIP
def test_gemm_bf16_symmetric_flag_small_shape_runs_full(torch):
    """Below the size where the upper-tile kernel saves time the flag runs
    the full-output kernel: the result equals ns_gemm_bf16_nt's bitwise."""
    X, E = sym_operands(torch, 1500, 300, 1, seed=3)
    Xc, Ec = X.cuda(), E[0].cuda()
    assert nsr.lib().ns_gemm_bf16_scratch_bytes(1500, 1500, 300, nsr.GEMM_SYMMETRIC) == 0
    D1, _, _ = nsr.gemm_bf16_sym(Xc, Xc, E1=Ec, diag=1.0, scale=-1.0)
    D2, _, _ = nsr.gemm_lp(Xc, Xc, nt=True, E1=Ec, diag=1.0, scale=-1.0)
    torch.cuda.synchronize()
    assert torch.equal(D1, D2)


@SYM_SKIP
def test_gemm_bf16_symmetric_full_size(torch):
    """N = 8192 (the mixed composite's size: 4 rounds of upper tiles plus 32
    tiles in 16 K-slices): exact symmetry and sampled upper elements."""
    n = 8192
    g = torch.Generator(device="cuda").manual_seed(8)
    X = torch.randn(n, n, generator=g, device="cuda").to(torch.bfloat16)
    E1 = torch.randn(n, n, generator=g, device="cuda")
    E1 = (E1 + E1.T) / 2
    D, Db, _ = nsr.gemm_bf16_sym(X, X, want_bf16=True, E1=E1, diag=1.0, scale=-1.0)
    torch.cuda.synchronize()
    assert torch.equal(D, D.T) and torch.equal(Db, Db.T)
    rs = np.random.default_rng(5)
    ii, jj = rs.integers(0, n, 300), rs.integers(0, n, 300)
    Xc = X.double().cpu().numpy()
    Dc, Ec = D.double().cpu().numpy(), E1.double().cpu().numpy()
    for i, j in zip(ii, jj):
        i, j = min(i, j), max(i, j)
        ref = -float(Xc[i] @ Xc[j]) + (i == j) + Ec[i, j]
        bound = 2 * g32(n + 4) * (float(np.abs(Xc[i]) @ np.abs(Xc[j])) + (i == j) + abs(Ec[i, j]))
        assert abs(Dc[i, j] - ref) <= bound, (i, j)


@SYM_SKIP
def test_mixed_symmetric_powers_match_full(torch):
    """The mixed solve at N = 3072 with symmetric bf16 power products (the
    default) against ns_set_symmetric(0) (every product in full): both reach
    1e-10, with ||F_k|| traces that agree to the bf16 level while above the
    floor, and the symmetric run counts N^2 (N + 1) flop for its bf16
    products."""
    sysm = inputs.spd_qlq(3072, 1e3, seed=12)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    reps = {}
    for sym in (True, False):
        s = nsr.Solver(3072, precision=nsr.PREC_MIXED_BF16, composite=False)
        s.bind(A)
        s.set_symmetric(sym)
        s.timing(True)
        th = torch.zeros_like(b)
        rep = s.solve(b, th, order=8, resid_tol=1e-10, refine_max=50)
        assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10
        cnt, _, fl = s.timing_read(3)
        reps[sym] = (rep, cnt, fl)
    n = 3072.0
    (ra, ca, fa), (rb, cb, fb) = reps[True], reps[False]
    assert fa == pytest.approx(ca * n * n * (n + 1)) and fb == pytest.approx(cb * 2 * n ** 3)
    for k in range(min(len(ra.fnorm_hist), len(rb.fnorm_hist))):
        x, y = ra.fnorm_hist[k], rb.fnorm_hist[k]
        if y > 100 * 1e-3:
            assert abs(x - y) <= 3e-2 * y, (k, x, y)


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


@pytest.mark.parametrize("tile", [256, 128])
@pytest.mark.parametrize("addends", [0, 2])
@pytest.mark.parametrize("m,n,k", [(300, 520, 32), (513, 260, 64), (1000, 700, 96),
                                   (2100, 1900, 1024), (4100, 4000, 224),
                                   (257, 259, 64), (300, 256, 100)])
def test_gemm_f32_dma_tiles(torch, m, n, k, addends, tile):
    """The 256 x 256 and 128 x 128 float32 tiles fed by LDS DMA (K a
    multiple of 32, N of 4): one to many slabs (the two-stage ring's start,
    wrap and drain), ragged edge tiles, every epilogue form, within the
    element-wise bound.  The last two shapes miss the DMA requirements
    (N = 259, K = 100) and take the register-staged 128 x 128 kernel."""
    b = int(np.ceil(np.log2(max(m, n))))
    nsr.tile_set(nsr.TILE_F32, b, tile)
    try:
        g = torch.Generator(device="cpu").manual_seed(m * 5 + n * 11 + k)
        X = torch.randn(m, k, generator=g, dtype=torch.float32)
        Y = torch.randn(k, n, generator=g, dtype=torch.float32)
        E = [torch.randn(m, n, generator=g, dtype=torch.float32) for _ in range(addends)]
        diag, scale = 0.75, -1.25
        print(f"f32 dma tiles {tile}: {m}x{n}x{k} addends {addends}", flush=True)
        D, Db, ss = nsr.gemm_lp(X.cuda(), Y.cuda(), nt=False, want_bf16=True,
                                E1=E[0].cuda() if addends > 0 else None,
                                E2=E[1].cuda() if addends > 1 else None,
                                diag=diag, scale=scale, want_sumsq=True)
        torch.cuda.synchronize()
    finally:
        nsr.tile_set(nsr.TILE_F32, b, 0)
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    Ed = [e.double().numpy() for e in E]
    ref = scale * (Xd @ Yd) + diag * np.eye(m, n) + sum(Ed, np.zeros((m, n)))
    bound = g32(k + 4) * (abs(scale) * (np.abs(Xd) @ np.abs(Yd)) + diag * np.eye(m, n)
                          + sum((np.abs(e) for e in Ed), np.zeros((m, n))))
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))
    assert torch.equal(Db.cpu(), D.cpu().to(torch.bfloat16))
    ssr = float(np.sum(got * got))
    assert abs(float(ss.cpu()) - ssr) <= 1e-12 * ssr


@pytest.mark.parametrize("nt", [False, True])
@pytest.mark.parametrize("shift", [0, 1])
def test_gemm_dma_strided_operands(torch, nt, shift):
    """256-tile products on strided views: row strides larger than the
    operand (the DMA sources step by the stride, not the width); with shift
    = 1 the views start one element in, so the rows are not 16-byte aligned
    and the products take the register-staged kernels instead."""
    m, n, k = 700, 520, 96
    fam = nsr.TILE_BF16 if nt else nsr.TILE_F32
    b = int(np.ceil(np.log2(max(m, n))))
    nsr.tile_set(fam, b, 256)
    try:
        g = torch.Generator(device="cpu").manual_seed(91 + shift + 2 * nt)
        dt = torch.bfloat16 if nt else torch.float32
        bigx = torch.randn(m, k + 40, generator=g).to(dt)
        bigy = torch.randn(n, k + 24, generator=g).to(dt) if nt else \
            torch.randn(k, n + 24, generator=g).to(dt)
        X = bigx.cuda()[:, shift:shift + k]
        Y = bigy.cuda()[:, shift:shift + k] if nt else bigy.cuda()[:, shift:shift + n]
        E = torch.randn(m, n, generator=g, dtype=torch.float32)
        print(f"dma strided nt={nt} shift={shift}", flush=True)
        D, _, _ = nsr.gemm_lp(X, Y, nt=nt, E1=E.cuda(), diag=1.0, scale=-0.5)
        torch.cuda.synchronize()
    finally:
        nsr.tile_set(fam, b, 0)
    Xd = X.cpu().double().numpy()
    Yd = Y.cpu().double().numpy()
    P = Xd @ (Yd.T if nt else Yd)
    Pa = np.abs(Xd) @ (np.abs(Yd).T if nt else np.abs(Yd))
    Ed = E.double().numpy()
    ref = -0.5 * P + np.eye(m, n) + Ed
    bound = g32(k + 4) * (0.5 * Pa + np.eye(m, n) + np.abs(Ed))
    got = D.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2 * bound), float(np.max(np.abs(got - ref) / bound))


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
    (nsr.PREC_MIXED_SPLIT, 300, 1e3, 8, "squaring"),
    (nsr.PREC_MIXED_SPLIT, 511, 1e5, 8, "squaring"),
    (nsr.PREC_MIXED_SPLIT, 300, 1e4, 8, "composite_double"),
    (nsr.PREC_MIXED_SPLIT, 33, 10.0, 2, "squaring"),
    (nsr.PREC_MIXED_SPLIT, 257, 1e5, 15, "table"),
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


def test_split_mode_tracks_float32_mixed(torch):
    """The split mode runs the same iteration as the float32 mixed mode with
    float32-class residual and G-side products: its ||F_k|| trace follows the
    float32 mixed trace down to the float32 floor, at N = 1000 (128-wide
    tiles), and its timed products are of kind 4."""
    sysm = inputs.spd_qlq(1000, 1e4, seed=77)
    reps = {}
    for prec in (nsr.PREC_MIXED_BF16, nsr.PREC_MIXED_SPLIT):
        s, th, rep = run(torch, sysm, prec, order=8, form="squaring", resid_tol=1e-10,
                         refine_max=100)
        assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10
        reps[prec] = rep
    a, b = reps[nsr.PREC_MIXED_BF16].fnorm_hist, reps[nsr.PREC_MIXED_SPLIT].fnorm_hist
    floor = 1e4 * 1000 * U32
    for k in range(min(len(a), len(b))):
        if a[k] > 100 * floor:
            assert abs(a[k] - b[k]) <= 1e-3 * a[k], (k, a[k], b[k])
    assert abs(len(a) - len(b)) <= 1


def test_split_mode_timing_kind(torch):
    sysm = inputs.spd_qlq(200, 1e3, seed=8)
    A, b = to_dev(torch, sysm.A), to_dev(torch, sysm.b)
    s = nsr.Solver(200, precision=nsr.PREC_MIXED_SPLIT, composite=False)
    s.bind(A)
    s.timing(True)
    s.init_scale()
    s.step(8, "squaring")
    s.step(8, "squaring")
    cnt = {k: s.timing_read(k)[0] for k in (0, 2, 3, 4)}
    # powers and assembly in bf16 (4 per step), residual and G-side split
    assert cnt[2] == 0 and cnt[3] == 8 and cnt[4] >= 2, cnt
    assert cnt[0] == cnt[3] + cnt[4], cnt


@pytest.mark.parametrize("prec", [nsr.PREC_FP64, nsr.PREC_MIXED_BF16])
def test_ragged_tiles_solve_n2112(torch, prec):
    """N = 2112 = 16.5 x 128 (K a multiple of 64, ragged last tile row and
    column): every product of the solve takes a 128 x 128 tile fed by LDS DMA
    (float64 full and symmetric, float32, bf16), with clamped edge reads.
    Order 8 to the floor, kappa = 1e4: the ||F_k|| trace follows the eigen
    closed form of eq. (fk1) above the precision's floor, and theta matches
    theta* = Q diag(1/lam) Q^T b within kappa times the attained residual."""
    n, kappa = 2112, 1e4
    sysm = inputs.spd_qlq(n, kappa, seed=21)
    print(f"ragged tiles solve n={n} precision {prec}", flush=True)
    s, th, rep = run(torch, sysm, prec, order=8, form="squaring", k_max=64, resid_tol=1e-12,
                     refine_max=100)
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-12
    mu = 1.0 - sysm.lam / rep.alpha
    floor = min(rep.fnorm_hist)
    tol = 1e-8 if prec == nsr.PREC_FP64 else 3e-2
    for k, fk in enumerate(rep.fnorm_hist):
        ref = float(np.sqrt(np.sum(mu ** (2 * 8 ** k))))
        if ref > 1e3 * floor:
            assert abs(fk - ref) <= tol * ref, (k, fk, ref)
    theta_star = sysm.Q @ ((sysm.Q.T @ sysm.b) / sysm.lam)
    rel_cpu = np.linalg.norm(sysm.b - sysm.A @ th) / np.linalg.norm(sysm.b)
    fwd = np.linalg.norm(th - theta_star) / np.linalg.norm(theta_star)
    assert rel_cpu <= 2e-12
    assert fwd <= 1.01 * kappa * rel_cpu + 50 * kappa * U64, (fwd, rel_cpu)


@pytest.mark.parametrize("prec", [nsr.PREC_MIXED_BF16, nsr.PREC_MIXED_SPLIT])
def test_mixed_full_size_spd4096(torch, prec):
    """N = 4096, kappa = 1e4, order 8 (the mixed legs the benchmark times, in
    the same launch configuration): refinement reaches the workload's 1e-12,
    the ||F_k|| trace follows the eigen closed form of eq. (fk1) to the bf16
    level while above the low-precision floor, and theta matches
    theta* = Q diag(1/lam) Q^T b within kappa times the attained residual."""
    w = inputs.WORKLOADS["spd4096_k1e4_o8"]
    sysm = inputs.spd_qlq(w["n"], w["kappa"], w["seed"])
    s, th, rep = run(torch, sysm, prec, order=8, form="squaring", k_max=64,
                     resid_tol=w["resid_tol"], refine_max=100)
    assert rep.status == nsr.NS_OK and rep.rel_resid <= w["resid_tol"]
    mu = 1.0 - sysm.lam / rep.alpha
    floor = min(rep.fnorm_hist)
    for k, fk in enumerate(rep.fnorm_hist):
        ref = float(np.sqrt(np.sum(mu ** (2 * 8 ** k))))
        if ref > 1e3 * floor:
            assert abs(fk - ref) <= 3e-2 * ref, (k, fk, ref)
    theta_star = sysm.Q @ ((sysm.Q.T @ sysm.b) / sysm.lam)
    rel_cpu = np.linalg.norm(sysm.b - sysm.A @ th) / np.linalg.norm(sysm.b)
    fwd = np.linalg.norm(th - theta_star) / np.linalg.norm(theta_star)
    assert rel_cpu <= 2 * w["resid_tol"]
    assert fwd <= 1.01 * w["kappa"] * rel_cpu + 50 * w["kappa"] * U64, (fwd, rel_cpu)


def test_split_composite_full_size_spd8192(torch):
    """N = 8192, kappa = 1e6, double Newton-Schulz order 8 in the split mode
    (the composite leg the benchmark times): relative residual <= 1e-10 and
    the forward error against theta* within kappa times the residual."""
    w = inputs.WORKLOADS["spd8192_k1e6_dns8"]
    A, b, lam, Q = inputs.spd_qlq_device(w["n"], w["kappa"], w["seed"])
    s = nsr.Solver(w["n"], precision=nsr.PREC_MIXED_SPLIT, composite=True)
    s.bind(A)
    th = torch.zeros_like(b)
    rep = s.solve(b, th, order=8, form="composite_double", k_max=64, resid_tol=1e-10,
                  refine_max=100)
    torch.cuda.synchronize()
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10
    rel = float(torch.linalg.norm(b - A @ th) / torch.linalg.norm(b))
    theta_star = Q @ ((Q.T.contiguous() @ b) / lam)
    fwd = float(torch.linalg.norm(th - theta_star) / torch.linalg.norm(theta_star))
    assert rel <= 2e-10
    assert fwd <= 1.01 * w["kappa"] * rel + 50 * w["kappa"] * U64, (fwd, rel)


def double_ns_exponent(n, k):
    """Exponent of F_0 in the double Newton-Schulz residual after k steps,
    eq. (ermoex1) with h = 1: k n^(k+1) + n^k."""
    return k * n ** (k + 1) + n ** k


def test_mixed_bf16_composite_full_size_spd8192(torch):
    """N = 8192, kappa = 1e6, double Newton-Schulz of order 8 (Section 5.1) in
    the mixed mode the benchmark's headline times (bf16 powers and assembly,
    float32 residual, G-side and merge, float64 Richardson), with the same
    solver set-up: relative residual <= 1e-10 after refinement, the forward
    error against theta* = Q diag(1/lam) Q^T b within kappa times the
    attained residual, and the ||F_k|| trace on the eigen closed form of
    eq. (ermoex1), ||F_k||_F = sqrt(sum mu_i^(2 e_k)), e_k = k n^(k+1) + n^k,
    while the iteration is above its float32 floor."""
    w = inputs.WORKLOADS["spd8192_k1e6_dns8"]
    A, b, lam, Q = inputs.spd_qlq_device(w["n"], w["kappa"], w["seed"])
    s = nsr.Solver(w["n"], precision=nsr.PREC_MIXED_BF16, composite=True)
    s.bind(A)
    th = torch.zeros_like(b)
    rep = s.solve(b, th, order=8, form="composite_double", k_max=64, resid_tol=1e-10,
                  refine_max=100)
    torch.cuda.synchronize()
    assert rep.precision == nsr.PREC_MIXED_BF16
    assert rep.status == nsr.NS_OK and rep.rel_resid <= 1e-10, (rep.refine_stop, rep.rel_resid)
    rel = float(torch.linalg.norm(b - A @ th) / torch.linalg.norm(b))
    theta_star = Q @ ((Q.T.contiguous() @ b) / lam)
    fwd = float(torch.linalg.norm(th - theta_star) / torch.linalg.norm(theta_star))
    assert rel <= 2e-10
    assert fwd <= 1.01 * w["kappa"] * rel + 50 * w["kappa"] * U64, (fwd, rel)
    mu = 1.0 - lam.cpu().numpy() / rep.alpha
    floor = min(rep.fnorm_hist)
    checked = 0
    for k, fk in enumerate(rep.fnorm_hist):
        ref = float(np.sqrt(np.sum(mu ** (2.0 * double_ns_exponent(8, k)))))
        print(f"k={k} gpu={fk:.6e} closed_form={ref:.6e} rel={abs(fk - ref) / ref:.2e}")
        if ref > 10 * floor:
            assert abs(fk - ref) <= 3e-2 * ref, (k, fk, ref)
            checked += 1
    assert checked >= 3, (checked, rep.fnorm_hist)


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


@pytest.mark.parametrize("tile", [256, 128])
@pytest.mark.parametrize("addends", [0, 2])
@pytest.mark.parametrize("m,n,k", [(300, 520, 32), (513, 260, 64), (1000, 700, 96),
                                   (2100, 1900, 1024), (4100, 4000, 224)])
def test_gemm_bf16_dma_tiles(torch, m, n, k, addends, tile):
    """The 256 x 256 and 128 x 128 bf16 tiles fed by LDS DMA (K a multiple
    of 32): one to many slabs (the ring's start, wrap and drain; two stages
    of 64-deep slabs when K is a multiple of 64, else four of 32), ragged
    edge tiles, every epilogue form, within the element-wise bound."""
    b = int(np.ceil(np.log2(max(m, n))))
    nsr.tile_set(nsr.TILE_BF16, b, tile)
    try:
        g = torch.Generator(device="cpu").manual_seed(m * 7 + n * 3 + k)
        X = torch.randn(m, k, generator=g).to(torch.bfloat16)
        Y = torch.randn(n, k, generator=g).to(torch.bfloat16)
        E = [torch.randn(m, n, generator=g, dtype=torch.float32) for _ in range(addends)]
        diag, scale = 1.0, -0.5
        print(f"bf16 dma tiles {tile}: {m}x{n}x{k} addends {addends}", flush=True)
        D, Db, ss = nsr.gemm_lp(X.cuda(), Y.cuda(), nt=True, want_bf16=True,
                                E1=E[0].cuda() if addends > 0 else None,
                                E2=E[1].cuda() if addends > 1 else None,
                                diag=diag, scale=scale, want_sumsq=True)
        torch.cuda.synchronize()
    finally:
        nsr.tile_set(nsr.TILE_BF16, b, 0)
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
