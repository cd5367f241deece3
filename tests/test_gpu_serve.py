"""GPU serving loop: every served request is checked against the closed-form
solution of its Householder-product system and, for a sample of small ones,
against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2008_11480_amd import inputs, nsr
from paper_2008_11480_amd.serve import GpuExecutor, Server, make_requests

pytestmark = pytest.mark.gpu
U64 = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def torch():
    import torch as _torch
    if not _torch.cuda.is_available():
        pytest.skip("no GPU")
    nsr.lib()
    return _torch


def test_serving_short_trace(torch):
    trace = inputs.serving_trace(2000.0, 0.12, seed=7)
    reqs = make_requests(trace)
    ex = GpuExecutor(workers=4, precision=nsr.PREC_MIXED_BF16)
    ex.keep_results = True                 # keep each request's system to check it
    choices = ex.prepare([r.n for r in reqs])
    assert choices and all(c["program"] for c in choices)
    srv = Server(ex, budget_bytes=8 << 30, workers=4)
    st = srv.run(reqs)
    torch.cuda.synchronize()
    assert st["served"] == len(reqs) and st["rejected"] == 0
    assert st["ok"] == len(reqs), st["not_ok"]
    assert st["hbm_peak_in_service_bytes"] <= 8 << 30
    checked = 0
    for r, q in zip(reqs, trace):
        A, b, th, lam, V = r.payload
        rel = float(torch.linalg.norm(b - A @ th) / torch.linalg.norm(b))
        assert rel <= 1.01e-10, (r.rid, r.n, rel)
        xs = inputs.householder_solve_device(lam, V, b)
        fwd = float(torch.linalg.norm(th - xs) / torch.linalg.norm(xs))
        assert fwd <= q.kappa * 2e-10 + 50 * q.kappa * U64, (r.rid, r.n, fwd)
        if r.n <= 200 and checked < 6:
            orc = oracle.solve(A.cpu().numpy(), b.cpu().numpy(),
                               oracle.SolveOptions(order=8, resid_tol=1e-13))
            d = np.linalg.norm(th.cpu().numpy() - orc.theta) / np.linalg.norm(orc.theta)
            assert d <= q.kappa * 2e-10 + 50 * q.kappa * U64, (r.rid, d)
            checked += 1
    assert checked > 0
    assert st["batched"] > 0 and st["single"] > 0
    # single solves from split_min_n on run the split mode (checked above
    # like every other request)
    big = [r for r in reqs if r.path == "single" and r.n >= ex.split_min_n]
    assert big and all(r.precision == nsr.PREC_MIXED_SPLIT for r in big)
    assert st["single_split"] == len(big)


def test_serving_admission_rejects_oversize(torch):
    """A budget below the footprint of the largest request: it is rejected,
    the rest are served."""
    trace = [inputs.Request(arrival_s=0.001 * i, n=n, kappa=100.0, seed=i)
             for i, n in enumerate([64, 700, 1500, 96])]
    reqs = make_requests(trace)
    ex = GpuExecutor(workers=2, precision=nsr.PREC_MIXED_BF16)
    fp = [ex.footprint(r) for r in reqs]
    srv = Server(ex, budget_bytes=fp[1] + fp[0] + fp[3], workers=2)
    st = srv.run(reqs)
    assert reqs[2].status == "rejected"
    assert st["rejected"] == 1 and st["ok"] == 3
