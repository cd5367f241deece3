"""The allocation-free split product (ns_gemm_f32_split_noalloc) against the
split product with a caller workspace (ns_gemm_f32_split), through the C ABI.

Both run the same kernels on the same operands, so their outputs (the float32
product, its bf16 copy and the sum of squares) must be identical bit for bit.
Two calls in a row, the second on a smaller shape, check that the built-in
scratch carries nothing from one call into the next; a shape beyond the
built-in scratch must be rejected before anything is launched.
"""
import pytest

from paper_2008_11480_amd import nsr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _torch
    if not _torch.cuda.is_available():
        pytest.skip("no GPU")
    nsr.lib()
    return _torch


def operands(torch, m, n, k, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.randn(m, k, generator=g, dtype=torch.float32).cuda()
    Y = torch.randn(k, n, generator=g, dtype=torch.float32).cuda()
    E1 = torch.randn(m, n, generator=g, dtype=torch.float32).cuda()
    return X, Y, E1


def both(torch, m, n, k, seed):
    X, Y, E1 = operands(torch, m, n, k, seed)
    D0, Db0, ss0 = nsr.gemm_f32_split(X, Y, want_bf16=True, E1=E1, diag=1.0, scale=-0.5,
                                      want_sumsq=True)
    ss1 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    D1, Db1 = nsr.gemm_f32_split_noalloc(X, Y, want_bf16=True, E1=E1, diag=1.0, scale=-0.5,
                                         sumsq=ss1)
    torch.cuda.synchronize()
    return (D0, Db0, ss0), (D1, Db1, ss1[0])


@pytest.mark.parametrize("first,second", [((700, 650, 900), (130, 129, 77)),
                                          ((2048, 2048, 2048), (257, 300, 5))])
def test_noalloc_matches_workspace_entry_point(torch, first, second):
    for seed, (m, n, k) in enumerate((first, second)):
        print(f"noalloc split product m={m} n={n} k={k}", flush=True)
        (D0, Db0, ss0), (D1, Db1, ss1) = both(torch, m, n, k, seed + 11)
        assert torch.equal(D0, D1), (m, n, k)
        assert torch.equal(Db0.view(torch.int16), Db1.view(torch.int16)), (m, n, k)
        assert float(ss0) == float(ss1), (float(ss0), float(ss1))
        assert float(ss1) == pytest.approx(float((D1.double() ** 2).sum()), rel=1e-6)


def test_noalloc_without_sumsq_and_degenerate(torch):
    X, Y, _ = operands(torch, 96, 80, 64, 3)
    D0, _, _ = nsr.gemm_f32_split(X, Y)
    D1, _ = nsr.gemm_f32_split_noalloc(X, Y)
    torch.cuda.synchronize()
    assert torch.equal(D0, D1)
    # k = 0: D = diag I
    Xe = torch.empty(5, 0, dtype=torch.float32, device="cuda")
    Ye = torch.empty(0, 5, dtype=torch.float32, device="cuda")
    De, _ = nsr.gemm_f32_split_noalloc(Xe, Ye, diag=2.0)
    torch.cuda.synchronize()
    assert torch.equal(De.cpu(), 2.0 * torch.eye(5))


def test_noalloc_rejects_shapes_beyond_its_scratch(torch):
    n = 4096
    need = int(nsr.lib().ns_gemm_f32_split_scratch_bytes(n, n, n))
    assert need > nsr.SPLIT_NOALLOC_MAX_BYTES
    X = torch.zeros(n, n, dtype=torch.float32, device="cuda")
    with pytest.raises(nsr.NSError) as ei:
        nsr.gemm_f32_split_noalloc(X, X)
    assert ei.value.status == nsr.NS_ENOMEM
    assert "built-in" in str(ei.value)
