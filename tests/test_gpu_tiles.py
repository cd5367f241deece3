"""The tile table (ns_tile_set) and the tile autotuner: every tile of every
GEMM family, forced on ragged and large shapes, gives the product within the
element-wise bound against a float64 CPU reference, and its sum of squares;
the autotuner installs the fastest tile per bucket.

Bound: |D - D_ref| <= 2 gamma_{k+4} |X||Y| with the precision's unit roundoff
(float64: 2^-53; float32 accumulation of float32 / bf16 operands: 2^-24,
bf16 products being exact in float32); split half-precision operands carry
22 bits (2^-22 per operand, three products: 3 2^-22 added)."""
import numpy as np
import pytest

from paper_2008_11480_amd import autotune, nsr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _torch
    if not _torch.cuda.is_available():
        pytest.skip("no GPU")
    nsr.lib()
    return _torch


@pytest.fixture(autouse=True)
def reset_tiles():
    yield
    for fam in nsr.TILE_OPTIONS:
        for b in range(24):
            nsr.tile_set(fam, b, 0)


def gamma(m, u):
    return m * u / (1 - m * u)


SHAPES = [(300, 257, 129), (2100, 2100, 64), (65, 1000, 333)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("family", [nsr.TILE_F64, nsr.TILE_F32, nsr.TILE_BF16, nsr.TILE_F16S])
def test_every_tile_matches_reference(torch, family, m, n, k):
    g = torch.Generator(device="cpu").manual_seed(m + 7 * n + k)
    b = int(np.ceil(np.log2(max(m, n))))
    if family == nsr.TILE_F64:
        X = torch.randn(m, k, generator=g, dtype=torch.float64)
        Y = torch.randn(k, n, generator=g, dtype=torch.float64)
        ref = X.numpy() @ Y.numpy()
        absref = np.abs(X.numpy()) @ np.abs(Y.numpy())
        bound = 2 * gamma(k + 4, 2.0 ** -53) * absref
    else:
        X = torch.randn(m, k, generator=g, dtype=torch.float32)
        Y = torch.randn(k, n, generator=g, dtype=torch.float32)
        if family == nsr.TILE_BF16:
            Xr, Yr = X.to(torch.bfloat16), Y.t().contiguous().to(torch.bfloat16)
            Xn, Yn = Xr.double().numpy(), Yr.double().numpy().T
        else:
            Xn, Yn = X.double().numpy(), Y.double().numpy()
        ref = Xn @ Yn
        absref = np.abs(Xn) @ np.abs(Yn)
        u = 2.0 ** -24
        bound = 2 * gamma(k + 4, u) * absref
        if family == nsr.TILE_F16S:
            bound = bound + 3 * 2.0 ** -22 * absref
    for tile in nsr.TILE_OPTIONS[family]:
        nsr.tile_set(family, b, tile)
        assert nsr.tile_get(family, b) == tile
        print(f"family {family} tile {tile} shape {m}x{n}x{k}", flush=True)
        if family == nsr.TILE_F64:
            D, ss = nsr.gemm_f64(X.cuda(), Y.cuda(), want_sumsq=True)
        elif family == nsr.TILE_F32:
            D, _, ss = nsr.gemm_lp(X.cuda(), Y.cuda(), nt=False, want_sumsq=True)
        elif family == nsr.TILE_BF16:
            D, _, ss = nsr.gemm_lp(Xr.cuda(), Yr.cuda(), nt=True, want_sumsq=True)
        else:
            D, _, ss = nsr.gemm_f32_split(X.cuda(), Y.cuda(), want_sumsq=True)
        torch.cuda.synchronize()
        d = D.double().cpu().numpy()
        err = np.abs(d - ref)
        assert (err <= bound).all(), (tile, float((err / (bound + 1e-300)).max()))
        assert float(ss) == pytest.approx(float((d ** 2).sum()), rel=1e-9)


def test_tile_set_rejects_unknown(torch):
    for bad in ((4, 10, 64), (0, 24, 64), (nsr.TILE_F64, 10, 512), (nsr.TILE_F32, 10, 32)):
        with pytest.raises(nsr.NSError):
            nsr.tile_set(*bad)
    assert nsr.tile_get(9, 0) == -1


def test_autotuner_installs_the_fastest(torch):
    rec = autotune.tune_tiles(families=(nsr.TILE_F32, nsr.TILE_BF16), sizes=(512, 2048), reps=2)
    assert len(rec) == 4
    for r in rec:
        timed = {int(t): ms for t, ms in r["ms"].items() if int(t)}
        assert r["best_tile"] == min(timed, key=timed.get)
        assert nsr.tile_get(r["family"], r["log2_dim"]) == r["best_tile"]
        assert r["speedup_vs_rule"] >= 0.9        # the rule's tile is among the candidates
