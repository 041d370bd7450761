"""The allocation-free error statistics (static device scratch) give the same
float64 results, bit for bit, as the workspace entry point, on two calls in a
row with the second smaller than the first (the scratch keeps the first
call's partial rows; the second must not read them)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import paper_2407_06107_amd as sf
    sf.lib()
    return sf


def _pair(n, seed):
    g = np.random.default_rng(seed)
    ref = g.standard_normal(n)
    est = (ref + 1e-3 * g.standard_normal(n)).astype(np.float32)
    est[:: 997] = np.nan   # non-finite entries are counted, not summed
    return torch.from_numpy(est).cuda(), torch.from_numpy(ref).cuda()


def test_noalloc_matches_workspace_entry_point(sf):
    assert torch.cuda.is_available()
    # 3,000,000 entries use all 1024 partial rows, 70,001 use 69 of them, and
    # the last pair holds one finite entry and one NaN
    for n, seed in ((3_000_000, 1), (70_001, 2), (2, 3)):
        print(f"error stats, n = {n}, seed = {seed}", flush=True)
        est, ref = _pair(n, seed)
        out_ws = sf.sf_error_stats(est, ref)
        out_na = torch.full((8,), -1.0, dtype=torch.float64, device="cuda")
        sf.sf_error_stats_noalloc(est, ref, out_na)
        torch.cuda.synchronize()
        a, b = out_ws.cpu().numpy(), out_na.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (n, a, b)
        # and the statistics are the ones numpy computes on the finite entries
        e, r = est.cpu().numpy().astype(np.float64), ref.cpu().numpy()
        fin = np.isfinite(e)
        d = e[fin] - r[fin]
        assert b[4] == fin.sum() and b[6] == (~fin).sum()
        assert np.isclose(b[0], (d * d).sum(), rtol=1e-12)
        assert b[2] == (np.abs(d).max() if d.size else 0.0)


def test_noalloc_empty_input(sf):
    out = torch.full((8,), -1.0, dtype=torch.float64, device="cuda")
    est = torch.empty(0, dtype=torch.float32, device="cuda")
    ref = torch.empty(0, dtype=torch.float64, device="cuda")
    sf.sf_error_stats_noalloc(est, ref, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.zeros(8))
