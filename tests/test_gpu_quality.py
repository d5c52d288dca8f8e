"""Quality measures of Section 4.1 on the GPU: the Procrustes statistic
against the oracle's SVD form, the normalized stress against the oracle's
full stress, and the full-stress reference layout (k = n) that both compare
with."""
import numpy as np
import pytest

import oracle
from paper_1608_08909_amd import graphs as G
from tests import brute

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1608_08909_amd import ssm


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ssm.load()
    yield


@pytest.mark.parametrize("n", [2, 7, 300, 5000, 200003])
def test_procrustes_matches_oracle(n):
    rng = np.random.Generator(np.random.PCG64(n))
    for trial in range(3):
        x = rng.normal(size=(n, 2)) * np.array([3.0, 0.5]) + 7.0
        y = x @ np.array([[0.3, -0.9], [0.9, 0.3]]) * 2.0 + rng.normal(size=(n, 2)) * (0.1 * trial)
        ref = oracle.procrustes(x, y)
        for xd, yd in ((torch.float64, torch.float64), (torch.float32, torch.float64), (torch.float32, torch.float32)):
            xt = torch.from_numpy(x).to(xd).cuda()
            yt = torch.from_numpy(y).to(yd).cuda()
            got = ssm.procrustes(xt, yt)
            want = oracle.procrustes(xt.double().cpu().numpy(), yt.double().cpu().numpy())
            assert abs(got - want) <= 1e-12 + 1e-9 * abs(want), (n, trial, xd, yd, got, want)
        assert -1e-12 <= ref <= 1.0 + 1e-12  # a perfect match rounds to within eps of 0


def test_procrustes_reflection_and_errors():
    c = torch.tensor([[1.0, 0.0], [-1.0, 0.0], [0.0, 2.0], [0.0, -2.0]], dtype=torch.float64, device="cuda")
    m = c * torch.tensor([1.0, -1.0], dtype=torch.float64, device="cuda")
    assert abs(ssm.procrustes(m, c) - 0.64) < 1e-15
    with pytest.raises(ssm.SSMError) as ei:
        ssm.procrustes(torch.ones(5, 2, dtype=torch.float64, device="cuda"), c.new_ones(5, 2) * torch.arange(
            5, dtype=torch.float64, device="cuda")[:, None])
    assert ei.value.status == ssm.E_INVAL


def test_full_stress_reference_and_quality():
    """k = n reproduces the full-stress majorization (weights 1/d^2 for every
    pair); the sparse layouts are then scored against it."""
    g = G.grid(12, 15)
    dg = ssm.DeviceGraph.from_csr(g)
    xr, _ = ssm.full_stress_layout(dg, 500)   # n = 180: PivotMDS on all n pivots, as the oracle
    xo, _, _, _ = oracle.layout(g.n, g.row_ptr, g.col_idx, g.n, 500)
    assert brute.coord_error(xr.cpu().numpy(), xo, align=True) < 1e-9
    ns_ref = ssm.normalized_stress(dg, xr)  # SSM_STRESS_NORMALIZED, divided in the library
    assert abs(ns_ref - oracle.normalized_stress(g.row_ptr, g.col_idx, xr.cpu().numpy())) <= 1e-12 * ns_ref
    assert ns_ref == ssm.stress(dg, None, xr, ssm.STRESS_FULL) / (g.n * (g.n - 1) / 2)
    for sampling in ("maxmin", "kmeans"):
        for k in (6, 20):
            x, *_ = ssm.layout(dg, k, 200, ssm.FP64, sampling=sampling)
            ns = ssm.normalized_stress(dg, x)
            xh = x.cpu().numpy()
            assert abs(ns - oracle.normalized_stress(g.row_ptr, g.col_idx, xh)) <= 1e-12 * ns
            pr = ssm.procrustes(x, xr)
            assert abs(pr - oracle.procrustes(xh, xr.cpu().numpy())) <= 1e-12
            assert -1e-12 <= pr <= 1.0 + 1e-12
            assert ns >= ns_ref * (1 - 1e-9)  # the reference minimizes the full stress
