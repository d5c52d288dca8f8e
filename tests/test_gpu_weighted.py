"""Graphs with edge lengths (Algorithm 1's general input) on the GPU against
the oracle: pivots, distance rows, deltas, regions, per-term weights and
denominators bit for bit; PivotMDS within 1e-9 of the RMS radius; the FP64
sweep bit for bit; FP32 final stress within 1e-4 of FP64; unit lengths give
the unweighted path's results."""
import numpy as np
import pytest

import oracle
from paper_1608_08909_amd import graphs as G
from tests import brute

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1608_08909_amd import ssm


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ssm.load()
    yield


def _cases():
    return [
        (G.grid(9, 11), 7, dict(seed=1)),
        (G.tree_plus(300, 2), 17, dict(seed=2, lo=1, hi=3, integer=True)),
        (G.grid(20, 20), 20, dict(seed=3, lo=1, hi=3, integer=True)),
        (G.rgg(1500, 4), 33, dict(seed=4)),
        (G.holed_mesh(60, 70, 4, 3, 8, 5), 40, dict(seed=5, lo=0.25, hi=4.0)),
        (G.barabasi_albert(2000, 5, 7), 50, dict(seed=6)),
        (G.cycle(17), 4, dict(seed=7, lo=1, hi=1, integer=True)),
    ]


CASES = _cases()
IDS = [f"{g.name}-k{k}-{'int' if o.get('integer') else 'real'}" for g, k, o in CASES]


def _lengths(g, o):
    return G.edge_lengths(g, o["seed"], o.get("lo", 0.5), o.get("hi", 2.0), o.get("integer", False))


@pytest.mark.parametrize("g,k,o", CASES, ids=IDS)
def test_weighted_preprocessing_bit_exact(g, k, o):
    say("case", g.name, k, o)
    ln = _lengths(g, o)
    ref = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, ln, k)
    dg = ssm.DeviceGraph.from_csr(g)
    lt = torch.from_numpy(ln).cuda()
    piv, dist_sel = ssm.select_pivots_w(dg, lt, k, 0, with_dist=True)
    assert np.array_equal(piv.cpu().numpy(), ref.pivots)
    assert np.array_equal(dist_sel.cpu().numpy(), ref.dist)
    dist = ssm.sssp_pivots(dg, lt, piv)
    assert np.array_equal(dist.cpu().numpy(), ref.dist)
    T = ssm.build_terms_w(dg, lt, piv, dist)
    ex = T.export()
    assert np.array_equal(ex["delta"], ref.delta)
    assert np.array_equal(ex["region"], ref.region)
    assert np.array_equal(ex["w"], ref.w)
    assert np.array_equal(ex["den"], ref.den)


@pytest.mark.parametrize("g,k,o", CASES, ids=IDS)
def test_weighted_layout(g, k, o):
    say("case", g.name, k, o)
    ln = _lengths(g, o)
    ref = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, ln, k)
    dg = ssm.DeviceGraph.from_csr(g)
    lt = torch.from_numpy(ln).cuda()
    piv = torch.from_numpy(ref.pivots).cuda()
    dist = torch.from_numpy(ref.dist).cuda()
    T = ssm.build_terms_w(dg, lt, piv, dist)
    x0 = ssm.pivotmds_init_w(dg, lt, T)
    xo, _, _ = oracle.pivotmds_w(ref.dist)
    xr = oracle.rescale_w(g.row_ptr, g.col_idx, ln, xo)
    w = np.linalg.eigvalsh(_gram_w(ref.dist))[::-1]
    if not (w[1] > 1e-8 * w[0] and (w[1] - w[2]) / w[0] < 1e-6):
        well = (w[0] - w[1]) / w[0] > 1e-3 and w[1] > 1e-8 * w[0]
        assert brute.coord_error(x0.cpu().numpy(), xr, align=not well) < 1e-9
    # FP64 sweeps bit for bit from the GPU's own start
    x1 = x0.clone()
    ssm.majorize_w(dg, lt, T, x1, 5)
    x1r = oracle.majorize_w(g.row_ptr, g.col_idx, ln, ref.pivots, ref.dist, ref.w, ref.den, x0.cpu().numpy(), 5)
    assert np.array_equal(x1.cpu().numpy(), x1r)
    s64 = ssm.stress_w(dg, lt, T, x1)
    s_or = oracle.stress_w(g.row_ptr, g.col_idx, ln, ref.pivots, ref.dist, ref.w, x1r)
    assert abs(s64 - s_or) <= 1e-12 * s_or
    # FP32 (first sweep FP64) against the FP64 path after 100 sweeps
    xa = x0.clone()
    ssm.majorize_w(dg, lt, T, xa, 100)
    xb = ssm.majorize_mixed_w(dg, lt, T, x0.clone(), 100)
    sa, sb = ssm.stress_w(dg, lt, T, xa), ssm.stress_w(dg, lt, T, xb)
    say("stress", sa, sb, abs(sa - sb) / sa)
    assert abs(sa - sb) <= 1e-4 * sa


def _gram_w(dist):
    d2 = dist.astype(np.float64) ** 2
    C = -0.5 * (d2 - d2.mean(axis=1, keepdims=True) - d2.mean(axis=0, keepdims=True) + d2.mean())
    return C @ C.T


def test_unit_lengths_match_the_unweighted_path():
    g = G.grid(30, 30)
    k = 30
    dg = ssm.DeviceGraph.from_csr(g)
    lt = torch.ones(g.col_idx.size, dtype=torch.float64, device="cuda")
    pw, dw = ssm.select_pivots_w(dg, lt, k, 0, with_dist=True)
    pu, du = ssm.select_pivots(dg, k, 0, with_dist=True)
    assert torch.equal(pw, pu)
    assert torch.equal(dw, du.double())
    Tw = ssm.build_terms_w(dg, lt, pw, dw)
    dist, delta, region = ssm.bfs_pivots(dg, pu)
    assert torch.equal(torch.from_numpy(Tw.export()["region"]).cuda(), region)
    Tu = ssm.build_terms(dg, pu, dist, delta, region)
    x0 = ssm.pivotmds_init(dg, Tu, ssm.FP64)
    xa, xb = x0.clone(), x0.clone()
    ssm.majorize(dg, Tu, xa, 7)
    ssm.majorize_w(dg, lt, Tw, xb, 7)
    assert torch.equal(xa, xb)


def test_weighted_large_rows_and_errors():
    g = G.rgg(50000, 9, 8.0)
    ln = G.edge_lengths(g, 11)
    dg = ssm.DeviceGraph.from_csr(g)
    lt = torch.from_numpy(ln).cuda()
    piv = ssm.select_pivots_w(dg, lt, 12, 0)
    pr, dr = oracle.select_pivots_w(g.n, g.row_ptr, g.col_idx, ln, 12, 0)
    assert np.array_equal(piv.cpu().numpy(), pr)
    dist = ssm.sssp_pivots(dg, lt, piv).cpu().numpy()
    assert np.array_equal(dist, dr)
    d = G.csr_from_edges(6, np.array([[0, 1], [1, 2], [3, 4], [4, 5]]))
    dd = ssm.DeviceGraph.from_csr(d)
    ld = torch.ones(d.col_idx.size, dtype=torch.float64, device="cuda")
    with pytest.raises(ssm.SSMError) as ei:
        ssm.select_pivots_w(dd, ld, 2, 0)
    assert ei.value.status == ssm.E_DISCONNECTED
    with pytest.raises(ssm.SSMError) as ei:
        ssm.sssp_pivots(dd, ld, torch.tensor([0, 3], dtype=torch.int32, device="cuda"))
    assert ei.value.status == ssm.E_DISCONNECTED


@pytest.mark.parametrize("order", ["nearfar", "band3", "plain"])
def test_weighted_search_orders(order, forced):
    """Both search orders (near-far bands, the default, also three lengths
    wide; plain label-correcting rounds) reach the oracle's Dijkstra
    distances and max/min pivots bit for bit, also on a graph whose searches
    run through many far passes."""
    if order == "plain":
        forced("sssp_nearfar", -1)
    if order == "band3":
        forced("sssp_band", 3)
    for g, k, o in [(G.rgg(20000, 9, 8.0), 24, dict(seed=11)), (G.grid(40, 45), 12, dict(seed=12, lo=1, hi=4, integer=True)),
                    (G.holed_mesh(90, 80, 5, 3, 10, 6), 16, dict(seed=13, lo=0.01, hi=5.0))]:
        say("order", order, "case", g.name, k, o)
        ln = _lengths(g, o)
        ref = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, ln, k)
        dg = ssm.DeviceGraph.from_csr(g)
        lt = torch.from_numpy(ln).cuda()
        piv = ssm.select_pivots_w(dg, lt, k, 0)
        assert np.array_equal(piv.cpu().numpy(), ref.pivots)
        dist = ssm.sssp_pivots(dg, lt, piv)
        assert np.array_equal(dist.cpu().numpy(), ref.dist)


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf")], ids=["zero", "negative", "nan", "inf"])
def test_weighted_invalid_lengths(bad):
    """A length that is not positive and finite is refused (SSM_E_INVAL) by
    the searches before any of them runs."""
    g = G.grid(6, 7)
    ln = G.edge_lengths(g, 3, 0.5, 2.0, False)
    ln[5] = bad
    dg = ssm.DeviceGraph.from_csr(g)
    lt = torch.from_numpy(ln).cuda()
    with pytest.raises(ssm.SSMError) as ei:
        ssm.select_pivots_w(dg, lt, 4, 0)
    assert ei.value.status == ssm.E_INVAL
    with pytest.raises(ssm.SSMError) as ei:
        ssm.sssp_pivots(dg, lt, torch.tensor([0, 9], dtype=torch.int32).cuda())
    assert ei.value.status == ssm.E_INVAL
