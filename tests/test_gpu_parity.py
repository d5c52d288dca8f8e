"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer outputs (pivots, distances, nearest-pivot distances, regions,
histograms) and the FP64 weight tables and denominators must match bit for
bit; the FP64 sweeps mirror the oracle's operation order and must match bit
for bit too; PivotMDS (a different eigen solver and summation order) within
1e-9 of the layout's RMS radius; FP32 sweeps within 1e-4 relative stress.
"""
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
    torch.cuda.synchronize()


def _cases():
    return [
        (G.path(30), 5), (G.cycle(17), 4), (G.star(12), 3), (G.complete(9), 4),
        (G.grid(7, 9), 63), (G.tri_grid(9, 11), 10), (G.random_connected(40, 0.1, 3), 7),
        (G.tree_plus(300, 2), 17), (G.rgg(1500, 4), 33), (G.barabasi_albert(2000, 5, 7), 50),
        (G.grid(50, 50), 50), (G.holed_mesh(120, 130, 6, 4, 12, 5), 40),
    ]


CASES = _cases()
IDS = [f"{g.name}-k{k}" for g, k in CASES]


def _device_pipeline(g, k):
    dg = ssm.DeviceGraph.from_csr(g)
    piv, dist_sel = ssm.select_pivots(dg, k, 0, with_dist=True)
    dist, delta, region = ssm.bfs_pivots(dg, piv)
    terms = ssm.build_terms(dg, piv, dist, delta, region)
    return dg, piv, dist_sel, dist, delta, region, terms


@pytest.mark.parametrize("g,k", CASES, ids=IDS)
def test_preprocessing_bit_exact(g, k):
    say("case", g.name, "k", k)
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    dg, piv, dist_sel, dist, delta, region, terms = _device_pipeline(g, k)
    assert np.array_equal(piv.cpu().numpy(), ref.pivots)
    assert np.array_equal(dist_sel.cpu().numpy(), ref.dist)
    assert np.array_equal(dist.cpu().numpy(), ref.dist)
    assert np.array_equal(delta.cpu().numpy(), ref.delta)
    assert np.array_equal(region.cpu().numpy(), ref.region)
    ex = terms.export()
    assert ex["delta_max"] == ref.delta_max and ex["dmax"] == ref.dmax
    assert np.array_equal(ex["H"], ref.H)
    assert np.array_equal(ex["wtab64"], ref.wtab)
    assert np.array_equal(ex["wtab32"], ref.wtab.astype(np.float32))
    assert np.array_equal(ex["den64"], ref.den)
    assert np.array_equal(ex["den32"], ref.den.astype(np.float32))


def test_regions_with_given_pivots():
    g = G.tri_grid(30, 31)
    piv_h = np.array([0, 929, 15, 465, 900, 30, 300, 777], dtype=np.int32)
    dref = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, piv_h)
    delta_r, region_r, _, _ = oracle.regions(dref)
    d = torch.from_numpy(dref).cuda()
    delta, region = ssm.regions(d)
    assert np.array_equal(delta.cpu().numpy(), delta_r)
    assert np.array_equal(region.cpu().numpy(), region_r)


# Launch-variant overrides (ssm_set_variant): each selects
# another kernel variant (cooperative-grid selection over CSR or padded rows,
# per-pivot selection, selection
# without the LDS byte copy or over the plain CSR with node-id queues or
# another precheck, the CSR per-workgroup BFS, the bit-parallel BFS, one- or
# many-workgroup region tie resolution, other lanes per node).
VARIANTS = [
    {"select_mode": 2}, {"select_mode": 2, "select_blocks": 3}, {"select_mode": 3},
    {"select_mode": 4}, {"select_mode": 4, "select_blocks": 3}, {"select_mode": 4, "select_hyb": 1},
    {"select_mode": 4, "select_hyb": 1, "select_blocks": 2},
    {"select_mode": 4, "ell_width": 8}, {"select_mode": 4, "ell_width": 32},
    {"select_m8": 2}, {"select_ell": 2}, {"select_mode": 1},
    {"select_ell": 2, "select_rowq": 2},
    {"select_ell": 2, "select_rowq": 2, "select_pre": 3},
    {"select_ell": 2, "select_pre": 1},
    {"msbfs": -1}, {"bfs_rowq": 2, "bfs_ell": 2, "bfs_grp": -1, "msbfs": -1}, {"bfs_ell": 2, "msbfs": -1},
    {"bfs_ell": 2, "bfs_grp": -1, "msbfs": -1},
    {"bfs_ell": 2, "bfs_loads": 3, "bfs_grp": -1, "msbfs": -1}, {"bfs_ell": 2, "bfs_loads": 2, "bfs_grp": -1, "msbfs": -1},
    {"bfs_ell": 3, "msbfs": -1}, {"bfs_ell": 4, "msbfs": -1}, {"msbfs": 1},
    {"msbfs": 1, "msbfs_budget": 3},
    {"region_mode": 1}, {"region_mode": 2}, {"bfs_lanes": 2, "msbfs": -1}, {"bfs_lanes": 64, "msbfs": -1},
    {"select_wave": -1}, {"select_wave": 2},
]
# (the star's first level overflows the LDS part of the frontier queue; the
# path's levels pass the state byte's saturation)
VARIANT_CASES = [(G.barabasi_albert(2000, 5, 7), 50), (G.rgg(1500, 4), 33), (G.holed_mesh(120, 130, 6, 4, 12, 5), 40),
                 (G.tree_plus(300, 2), 17), (G.star(12), 3), (G.path(600), 6), (G.star(3000), 3)]


@pytest.mark.parametrize("env", VARIANTS, ids=["-".join(f"{a}={b}" for a, b in v.items()) for v in VARIANTS])
def test_kernel_variants_bit_exact(env, forced):
    for name, val in env.items():
        forced(name, val)
    for g, k in VARIANT_CASES:
        say("variant", env, "case", g.name, "k", k)
        ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
        dg, piv, dist_sel, dist, delta, region, terms = _device_pipeline(g, k)
        assert np.array_equal(piv.cpu().numpy(), ref.pivots)
        assert np.array_equal(dist_sel.cpu().numpy(), ref.dist)
        assert np.array_equal(dist.cpu().numpy(), ref.dist)
        assert np.array_equal(delta.cpu().numpy(), ref.delta)
        assert np.array_equal(region.cpu().numpy(), ref.region)


@pytest.mark.parametrize("g,k", [(G.rgg(150000, 21, 8.0), 24), (G.grid(400, 400), 8), (G.barabasi_albert(120000, 2, 5), 30)],
                         ids=["rgg150000-k24", "grid400x400-k8", "ba120000-k30"])
@pytest.mark.parametrize("mode", ["0", "2", "4"], ids=["auto", "grid", "grid-ell"])
def test_select_beyond_byte_copy(g, k, mode, forced):
    """Graphs too large for the LDS byte copy of m but within one workgroup's
    visited bits, and the cooperative grid form; the grid graph has
    eccentricities far above 255; the BA graph has frontiers wider than one
    pass."""
    forced("select_mode", int(mode))
    say("case", g.name, "k", k, "mode", mode)
    piv_r, _ = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
    dg = ssm.DeviceGraph.from_csr(g)
    assert np.array_equal(ssm.select_pivots(dg, k, 0).cpu().numpy(), piv_r)


@pytest.mark.parametrize("env", [{}, {"msbfs": 1}, {"msbfs": -1}, {"bfs_ell": 2, "msbfs": -1},
                                 {"bfs_ell": 2, "bfs_grp": -1, "msbfs": -1},
                                 {"bfs_ell": 2, "bfs_loads": 3, "bfs_grp": -1, "msbfs": -1},
                                 {"bfs_ell": 2, "bfs_loads": 2, "bfs_grp": -1, "msbfs": -1}, {"bfs_ell": 3, "msbfs": -1},
                                 {"bfs_ell": 4, "msbfs": -1}],
                         ids=["default", "bitparallel", "per-pivot", "csr", "csr-one-block", "csr-agent", "csr-plain-checks",
                              "ell-global", "ell-global-noread"])
def test_bfs_large_frontiers(env, forced):
    """Frontiers beyond the LDS queue and more long rows per level than the
    LDS list holds: the global overflow areas of the per-pivot BFS (and the
    bit-parallel BFS, which the library picks on this graph by default)."""
    for name, val in env.items():
        forced(name, val)
    g = G.barabasi_albert(60000, 5, 3)
    piv = np.array([0, 17, 999, 30000, 59999, 12345, 4242, 777], dtype=np.int32)
    say("case", g.name, "pivots", piv.tolist(), "env", env)
    dref = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, piv)
    dg = ssm.DeviceGraph.from_csr(g)
    dist, delta, region = ssm.bfs_pivots(dg, torch.from_numpy(piv).cuda())
    assert np.array_equal(dist.cpu().numpy(), dref)
    delta_r, region_r, _, _ = oracle.regions(dref)
    assert np.array_equal(delta.cpu().numpy(), delta_r)
    assert np.array_equal(region.cpu().numpy(), region_r)


@pytest.mark.parametrize("env", [{}, {"msbfs": -1}], ids=["default", "per-pivot"])
def test_bfs_hub_graph_with_long_tail(env, forced):
    """A hub-dominated graph (the bit-parallel rows go first) with a 2000-node
    path hanging off one hub and most pivots on the path: the settled pairs
    stop doubling once the graph's own pivots are done, long before the path
    pivots are, so the rows hand over to the per-pivot BFS part way."""
    for name, val in env.items():
        forced(name, val)
    ba = G.barabasi_albert(60000, 5, 3)
    src = np.repeat(np.arange(ba.n), np.diff(ba.row_ptr))
    tail = np.arange(ba.n, ba.n + 2000)
    edges = np.concatenate([np.stack([src, ba.col_idx], 1), np.stack([np.r_[0, tail[:-1]], tail], 1)])
    g = G.csr_from_edges(ba.n + 2000, edges, "ba60000+path2000")
    piv = np.array([g.n - 1, g.n - 500, g.n - 1000, g.n - 1500, g.n - 1800, 0, 17, 30000], dtype=np.int32)
    say("case", g.name, "pivots", piv.tolist(), "env", env)
    dref = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, piv)
    dg = ssm.DeviceGraph.from_csr(g)
    dist, delta, region = ssm.bfs_pivots(dg, torch.from_numpy(piv).cuda())
    assert np.array_equal(dist.cpu().numpy(), dref)
    delta_r, region_r, _, _ = oracle.regions(dref)
    assert np.array_equal(delta.cpu().numpy(), delta_r)
    assert np.array_equal(region.cpu().numpy(), region_r)


def test_regions_many_ties_per_level_path():
    """Enough tied nodes that the default takes the multi-workgroup per-level
    resolution, on levels both sparse (tied-node list) and dense (full scan)."""
    g = G.barabasi_albert(60000, 3, 11)
    k = 64
    say("case", g.name, "k", k)
    _, dref = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
    delta_r, region_r, _, _ = oracle.regions(dref)
    assert int((np.sum(dref == delta_r[None, :], axis=0) > 1).sum()) > 16384
    delta, region = ssm.regions(torch.from_numpy(dref).cuda())
    assert np.array_equal(delta.cpu().numpy(), delta_r)
    assert np.array_equal(region.cpu().numpy(), region_r)


@pytest.mark.parametrize("g,k", [c for c in CASES if c[1] >= 3], ids=[i for c, i in zip(CASES, IDS) if c[1] >= 3])
def test_pivotmds_parity(g, k):
    say("case", g.name, "k", k)
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    xo, Vo, lamo = oracle.pivotmds(ref.dist)
    x0 = oracle.rescale(g.row_ptr, g.col_idx, xo)
    dg, piv, _, dist, delta, region, terms = _device_pipeline(g, k)
    x = ssm.pivotmds_init(dg, terms, ssm.FP64).cpu().numpy()
    M = ssm.pivotmds_gram(terms)
    Mo = oracle.gram(oracle.pmds_center(ref.dist))
    assert np.abs(M - Mo).max() <= 1e-12 * np.abs(Mo).max()
    V, lam, iters = ssm.pivotmds_eig(terms)
    assert np.allclose(lam, lamo, rtol=1e-10, atol=1e-12 * abs(lamo[0]))
    w = np.linalg.eigvalsh(oracle.gram(oracle.pmds_center(ref.dist)))[::-1]
    gap12 = (w[0] - w[1]) / w[0]
    gap23 = (w[1] - w[2]) / w[0]
    if w[1] > 1e-8 * w[0] and gap23 < 1e-6:
        # the dominant plane itself is not unique (the complete graph): the
        # eigenvalues are fixed, and any orthonormal pair of eigenvectors of
        # those eigenvalues is a valid answer; the layout must be that pair's
        # projection C V, rescaled to the summed edge lengths
        assert np.abs(V.T @ V - np.eye(2)).max() < 1e-12
        assert np.abs(Mo @ V - V * lam[None, :]).max() < 1e-9 * abs(lamo[0])
        C = oracle.pmds_center(ref.dist)
        xw = oracle.rescale(g.row_ptr, g.col_idx, C @ V)
        assert brute.coord_error(x, xw) < 1e-9
        assert iters < 20000
        return
    if gap12 > 1e-3 and w[1] > 1e-8 * w[0]:
        # well separated: eigenvectors and layout match directly
        assert np.abs(V - Vo).max() < 1e-9
        assert brute.coord_error(x, x0) < 1e-9
    else:
        # near-degenerate pair (the plane is fixed, its axes are not) or a
        # negligible second axis: compare after a rigid alignment
        assert brute.coord_error(x, x0, align=True) < 1e-9
    assert iters < 20000


@pytest.mark.parametrize("k", [240, 256, 1000])
def test_pivotmds_gram_round_sizes(k):
    """The Gram product stages 32 nodes per LDS round while the staged block
    fits 64 KB (k <= 240) and 8 above it, past 64 KB of LDS at k = 1000; every
    form matches the oracle's C^T C."""
    g = G.rgg(3000, 5)
    say("case", g.name, "k", k)
    _, dref = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
    dg, piv, _, dist, delta, region, terms = _device_pipeline(g, k)
    assert np.array_equal(dist.cpu().numpy(), dref)
    ssm.pivotmds_init(dg, terms, ssm.FP64)
    M = ssm.pivotmds_gram(terms)
    Mo = oracle.gram(oracle.pmds_center(dref))
    assert np.abs(M - Mo).max() <= 1e-12 * np.abs(Mo).max()


@pytest.mark.parametrize("form", ["default", "thread-per-node"])
@pytest.mark.parametrize("g,k", CASES, ids=IDS)
def test_sweeps_f64_bit_exact(g, k, form, forced):
    """Both FP64 sweep kernels (a lane group per node for small graphs, the
    default here; a thread per node) against the oracle, bit for bit."""
    if form == "thread-per-node":
        forced("sweep_f64_terms", -1)
    say("case", g.name, "k", k, form)
    iters = 25
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    rng = np.random.default_rng(11)
    x0 = rng.normal(size=(g.n, 2)) * np.sqrt(g.n)
    dg, *_, terms = _device_pipeline(g, k)
    xg = torch.from_numpy(x0).cuda()
    ssm.majorize(dg, terms, xg, iters, sync=True)
    xr, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, iters)
    assert np.array_equal(xg.cpu().numpy(), xr)
    s = ssm.stress(dg, terms, xg)
    sr = oracle.stress_sparse(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, xr)
    assert abs(s - sr) <= 1e-9 * sr


@pytest.mark.parametrize("g,k", [c for c in CASES if c[0].n >= 60], ids=[i for c, i in zip(CASES, IDS) if c[0].n >= 60])
def test_sweeps_f32_stress(g, k):
    say("case", g.name, "k", k)
    iters = 60
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, ref) if k >= 3 else \
        np.random.default_rng(1).normal(size=(g.n, 2)) * 10
    x0 = x0.astype(np.float32).astype(np.float64)
    dg, *_, terms = _device_pipeline(g, k)
    xg = torch.from_numpy(x0.astype(np.float32)).cuda()
    ssm.majorize(dg, terms, xg, iters, sync=True)
    xr, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, iters)
    s32 = ssm.stress(dg, terms, xg)
    sr = oracle.stress_sparse(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, xr)
    assert abs(s32 - sr) <= 1e-4 * sr, (s32, sr)


SWEEP_VARIANTS = [{"sweep_split": 1}, {"sweep_split": 2}, {"sweep_split": 4},
                  {"sweep_mode": 1}, {"sweep_mode": 2}, {"sweep_mode": 2, "sweep_split": 4},
                  {"sweep_blocks_per_cu": 1}]


@pytest.mark.parametrize("env", SWEEP_VARIANTS, ids=["-".join(f"{a[6:]}={b}" for a, b in v.items()) for v in SWEEP_VARIANTS])
def test_sweep_f32_variants(env, forced):
    """Every FP32 sweep form (waves per chunk, LDS table, LDS histograms,
    global table, one block per CU) against the FP64 oracle's stress, on a
    graph with rows of more than one segment (their neighbour sums) and on a
    low-degree one."""
    for name, val in env.items():
        forced(name, val)
    for g, k in [(G.barabasi_albert(60000, 5, 3), 32), (G.rgg(3000, 5), 48)]:
        say("sweep variant", env, "case", g.name, "k", k)
        ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
        x0 = oracle.initial_layout(g.row_ptr, g.col_idx, ref).astype(np.float32).astype(np.float64)
        dg, *_, terms = _device_pipeline(g, k)
        xg = torch.from_numpy(x0.astype(np.float32)).cuda()
        ssm.majorize(dg, terms, xg, 40, sync=True)
        xr, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, 40)
        s32 = ssm.stress(dg, terms, xg)
        sr = oracle.stress_sparse(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, xr)
        assert abs(s32 - sr) <= 1e-4 * sr, (s32, sr)


TWIN_EDGES = [[0, 1], [1, 2], [2, 0], [3, 9], [3, 1], [9, 1], [3, 4], [9, 4], [3, 8], [9, 8],
              [4, 6], [6, 10], [10, 11], [8, 11], [5, 6], [7, 6], [2, 11], [4, 2]]


def test_twins_stay_together():
    """Adjacent nodes with one closed neighbourhood (3, 9) and nodes with one
    open neighbourhood (5, 7) start on one point and stay there in both
    precisions, as in exact arithmetic."""
    g = G.csr_from_edges(12, np.array(TWIN_EDGES))
    dg = ssm.DeviceGraph.from_csr(g)
    for k in (3, 5):
        piv = ssm.select_pivots(dg, k, 6)
        dist, delta, region = ssm.bfs_pivots(dg, piv)
        terms = ssm.build_terms(dg, piv, dist, delta, region)
        for prec in (ssm.FP64, ssm.FP32):
            x = ssm.pivotmds_init(dg, terms, prec)
            ssm.majorize(dg, terms, x, 300, sync=True)
            xa = x.cpu().numpy()
            assert np.array_equal(xa[3], xa[9]) and np.array_equal(xa[5], xa[7])
            assert np.abs(xa[3] - xa[1]).max() > 1e-3


def test_sweeps_f32_coordinates_rgg():
    """Random geometric graph (many twins): FP32 sweeps track the FP64 oracle
    in coordinates, not only in stress."""
    g, k, iters = G.rgg(4000, 21), 60, 200
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, ref).astype(np.float32).astype(np.float64)
    dg, *_, terms = _device_pipeline(g, k)
    xg = torch.from_numpy(x0.astype(np.float32)).cuda()
    ssm.majorize(dg, terms, xg, iters, sync=True)
    xr, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, iters)
    err = brute.coord_error(xg.cpu().numpy().astype(np.float64), xr)
    say("rgg fp32 coordinate error", err)
    assert err < 1e-4


@pytest.mark.parametrize("g,k,iters", [(G.rgg(20000, 7, 8.0), 100, 300), (G.tree_plus(5000, 4), 60, 200),
                                        (G.holed_mesh(150, 160, 8, 4, 12, 3), 80, 200)],
                         ids=["rgg20000", "tree5000", "holedmesh150"])
def test_mixed_precision_end_to_end(g, k, iters):
    """FP32 form (PivotMDS and the first sweep in FP64, then FP32) against the
    oracle's FP64 run from the same start: final stress within 1e-6 relative
    and coordinates within 1e-4 of the layout radius."""
    say("case", g.name, "k", k)
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, ref)
    xr, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, iters, threads=8)
    sr = oracle.stress_sparse(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, xr)
    dg, *_, terms = _device_pipeline(g, k)
    x64 = torch.from_numpy(x0).cuda()
    x32 = ssm.majorize_mixed(dg, terms, x64, iters, warm=1)
    s32 = ssm.stress(dg, terms, x32)
    say("rel stress", abs(s32 - sr) / sr)
    assert abs(s32 - sr) <= 1e-6 * sr
    assert brute.coord_error(x32.cpu().numpy().astype(np.float64), xr) < 1e-4
    # one sweep: the FP32 result is the rounded oracle sweep, bit for bit
    x64 = torch.from_numpy(x0).cuda()
    x1 = ssm.majorize_mixed(dg, terms, x64, 1, warm=1)
    xr1, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, 1)
    assert np.array_equal(x1.cpu().numpy(), xr1.astype(np.float32))


def test_sweeps_f32_coordinates_on_grid():
    """A grid is bipartite, so no two adjacent nodes share a position in the
    start layout and the FP32 trajectory tracks the FP64 one."""
    g, k, iters = G.grid(50, 50), 50, 200
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, ref).astype(np.float32).astype(np.float64)
    dg, *_, terms = _device_pipeline(g, k)
    xg = torch.from_numpy(x0.astype(np.float32)).cuda()
    ssm.majorize(dg, terms, xg, iters, sync=True)
    xr, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, iters)
    assert brute.coord_error(xg.cpu().numpy().astype(np.float64), xr) < 1e-4


def test_end_to_end_grid50_fp64():
    """50 x 50 grid, k = 50, maxmin from node 0, PivotMDS, 200 sweeps, FP64."""
    g, k, iters = G.grid(50, 50), 50, 200
    xr, ref, x0r, _ = oracle.layout(g.n, g.row_ptr, g.col_idx, k, iters)
    dg = ssm.DeviceGraph.from_csr(g)
    x, terms, piv, dist, delta, region = ssm.layout(dg, k, iters, ssm.FP64)
    assert np.array_equal(piv.cpu().numpy(), ref.pivots)
    assert np.array_equal(region.cpu().numpy(), ref.region)
    xa = x.cpu().numpy()
    assert brute.coord_error(xa, xr, align=True) < 1e-9
    s = ssm.stress(dg, terms, x)
    sr = oracle.stress_sparse(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, xr)
    assert abs(s - sr) <= 1e-9 * sr
    full = ssm.stress(dg, None, x, ssm.STRESS_FULL)
    full_r = oracle.stress_full(g.row_ptr, g.col_idx, xr)
    assert abs(full - full_r) <= 1e-9 * full_r


def test_full_stress_matches_oracle():
    for g in [G.cycle(12), G.grid(9, 11), G.rgg(700, 9)]:
        x = np.random.default_rng(2).normal(size=(g.n, 2))
        dg = ssm.DeviceGraph.from_csr(g)
        s = ssm.stress(dg, None, torch.from_numpy(x).cuda(), ssm.STRESS_FULL)
        sr = oracle.stress_full(g.row_ptr, g.col_idx, x)
        assert abs(s - sr) <= 1e-9 * sr
        s32 = ssm.stress(dg, None, torch.from_numpy(x.astype(np.float32)).cuda(), ssm.STRESS_FULL)
        sr32 = oracle.stress_full(g.row_ptr, g.col_idx, x.astype(np.float32).astype(np.float64))
        assert abs(s32 - sr32) <= 1e-9 * sr32


def test_resume_and_determinism():
    g, k = G.rgg(3000, 5), 40
    dg, *_, terms = _device_pipeline(g, k)
    for dt in (torch.float64, torch.float32):
        x0 = torch.from_numpy(np.random.default_rng(3).normal(size=(g.n, 2)) * 30).to(dt).cuda()
        a = x0.clone()
        ssm.majorize(dg, terms, a, 40)
        b = x0.clone()
        ssm.majorize(dg, terms, b, 15)
        ssm.majorize(dg, terms, b, 25)
        c = x0.clone()
        ssm.majorize(dg, terms, c, 40)
        torch.cuda.synchronize()
        assert torch.equal(a, b) and torch.equal(a, c)


def test_tolerance_stop_matches_oracle():
    g = G.grid(8, 8)
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, g.n)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, ref)
    xr, done_r = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, 1000, tol=1e-4)
    dg, *_, terms = _device_pipeline(g, g.n)
    xg = torch.from_numpy(x0).cuda()
    done = ssm.majorize(dg, terms, xg, 1000, tol=1e-4)
    assert done == done_r
    assert np.array_equal(xg.cpu().numpy(), xr)


def test_edge_cases():
    # k = 1 and k = n
    g = G.path(6)
    dg = ssm.DeviceGraph.from_csr(g)
    for k in (1, g.n):
        piv = ssm.select_pivots(dg, k, 2)
        pr, _ = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 2)
        assert np.array_equal(piv.cpu().numpy(), pr)
    # PivotMDS needs k >= 3
    piv = ssm.select_pivots(dg, 2, 0)
    dist, delta, region = ssm.bfs_pivots(dg, piv)
    terms = ssm.build_terms(dg, piv, dist, delta, region)
    with pytest.raises(ssm.SSMError) as ei:
        ssm.pivotmds_init(dg, terms)
    assert ei.value.status == ssm.E_INVAL
    # zero sweeps leave x alone
    x = torch.arange(12, dtype=torch.float64, device="cuda").reshape(6, 2)
    y = x.clone()
    ssm.majorize(dg, terms, y, 0, sync=True)
    assert torch.equal(x, y)
    # disconnected input
    d = G.csr_from_edges(6, np.array([[0, 1], [1, 2], [3, 4], [4, 5]]))
    dd = ssm.DeviceGraph.from_csr(d)
    with pytest.raises(ssm.SSMError) as ei:
        ssm.select_pivots(dd, 2, 0)
    assert ei.value.status == ssm.E_DISCONNECTED
    with pytest.raises(ssm.SSMError) as ei:
        ssm.bfs_pivots(dd, torch.tensor([0, 3], dtype=torch.int32, device="cuda"))
    assert ei.value.status == ssm.E_DISCONNECTED


def test_largest_distance():
    """Distances are stored in 16 bits: a path of 65,536 nodes (largest
    distance 65,535) runs end to end, bit for bit against the oracle in FP64;
    one node more is refused with SSM_E_RANGE."""
    g = G.path(65536)
    k, iters = 3, 2
    say("case", g.name, "k", k)
    dg = ssm.DeviceGraph.from_csr(g)
    piv = ssm.select_pivots(dg, k, 0)
    dist, delta, region = ssm.bfs_pivots(dg, piv)
    ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    assert np.array_equal(piv.cpu().numpy(), ref.pivots)
    assert np.array_equal(dist.cpu().numpy(), ref.dist)
    assert int(dist.max()) == 65535
    terms = ssm.build_terms(dg, piv, dist, delta, region)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, ref)
    xg = torch.from_numpy(x0).cuda()
    ssm.majorize(dg, terms, xg, iters, sync=True)
    xr, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, iters)
    assert np.array_equal(xg.cpu().numpy(), xr)
    # FP32 sweeps over 16-bit distances whose tables do not fit LDS, from a
    # perturbed start (PivotMDS lays a path out exactly)
    x32 = (x0 + np.random.default_rng(5).normal(size=x0.shape) * 3.0).astype(np.float32).astype(np.float64)
    xf = torch.from_numpy(x32.astype(np.float32)).cuda()
    ssm.majorize(dg, terms, xf, 20, sync=True)
    xr32, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x32, 20)
    s32 = ssm.stress(dg, terms, xf)
    sr = oracle.stress_sparse(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, xr32)
    assert abs(s32 - sr) <= 1e-4 * sr, (s32, sr)
    del terms
    g2 = G.path(65537)
    say("case", g2.name, "k", k)
    dg2 = ssm.DeviceGraph.from_csr(g2)
    piv2 = ssm.select_pivots(dg2, k, 0)
    dist2, delta2, region2 = ssm.bfs_pivots(dg2, piv2)
    with pytest.raises(ssm.SSMError) as ei:
        ssm.build_terms(dg2, piv2, dist2, delta2, region2)
    assert ei.value.status == ssm.E_RANGE


KM_CASES = [(G.path(9), 2), (G.cycle(17), 4), (G.star(12), 3), (G.complete(9), 9), (G.grid(9, 11), 6),
            (G.tri_grid(20, 23), 12), (G.rgg(300, 3), 7), (G.tree_plus(300, 2), 17),
            (G.barabasi_albert(2000, 3, 7), 50), (G.holed_mesh(120, 130, 6, 4, 12, 5), 40), (G.rgg(20000, 7, 8.0), 60)]


@pytest.mark.parametrize("g,k", KM_CASES, ids=[f"{g.name}-k{k}" for g, k in KM_CASES])
def test_kmeans_sp_bit_exact(g, k):
    """k-means sp: refined pivots, final clusters and pass count equal the oracle's."""
    say("case", g.name, "k", k)
    dg = ssm.DeviceGraph.from_csr(g)
    piv, dist = ssm.select_pivots(dg, k, 0, with_dist=True)
    ph, dh = piv.cpu().numpy(), dist.cpu().numpy()
    for iters in (50, 1, 2):
        newp, assign, it = ssm.kmeans_pivots(piv, dist, iters)
        rp, ra, rit = oracle.kmeans_sp(dh, ph, iters)
        assert it == rit, iters
        assert np.array_equal(assign.cpu().numpy(), ra), iters
        assert np.array_equal(newp.cpu().numpy(), rp), iters
    # then the BFS from the refined pivots, as in the layout pipeline
    d2, delta2, region2 = ssm.bfs_pivots(dg, newp)
    d2r = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, rp)
    assert np.array_equal(d2.cpu().numpy(), d2r)
    delta_r, region_r, _, _ = oracle.regions(d2r)
    assert np.array_equal(delta2.cpu().numpy(), delta_r)
    assert np.array_equal(region2.cpu().numpy(), region_r)


@pytest.mark.parametrize("chunk", ["32", "40", "48", "56", "64"])
def test_kmeans_sp_chunk_variants(chunk, forced):
    """Every cluster-chunk width of the assignment kernel, k not a multiple of it."""
    forced("km_chunk", int(chunk))
    g = G.rgg(5000, 11, 8.0)
    dg = ssm.DeviceGraph.from_csr(g)
    piv, dist = ssm.select_pivots(dg, 77, 0, with_dist=True)
    newp, assign, it = ssm.kmeans_pivots(piv, dist)
    rp, ra, rit = oracle.kmeans_sp(dist.cpu().numpy(), piv.cpu().numpy())
    assert it == rit
    assert np.array_equal(assign.cpu().numpy(), ra)
    assert np.array_equal(newp.cpu().numpy(), rp)


def test_kmeans_sp_given_pivots():
    """Arbitrary start pivots, repeated ones included (the duplicate's cluster
    stays empty and keeps its centroid)."""
    g = G.tri_grid(30, 31)
    dg = ssm.DeviceGraph.from_csr(g)
    for ph in ([0, 929, 15, 465, 900, 30, 300, 777], [5, 5, 600, 5, 12]):
        ph = np.array(ph, dtype=np.int32)
        dh = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, ph)
        newp, assign, it = ssm.kmeans_pivots(torch.from_numpy(ph).cuda(), torch.from_numpy(dh).cuda())
        rp, ra, rit = oracle.kmeans_sp(dh, ph)
        assert it == rit
        assert np.array_equal(assign.cpu().numpy(), ra)
        assert np.array_equal(newp.cpu().numpy(), rp)
    with pytest.raises(ssm.SSMError) as ei:
        ssm.kmeans_pivots(torch.tensor([0, g.n], dtype=torch.int32, device="cuda"),
                          torch.zeros(2, g.n, dtype=torch.int32, device="cuda"))
    assert ei.value.status == ssm.E_INVAL
    with pytest.raises(ssm.SSMError) as ei:
        ssm.kmeans_pivots(torch.tensor([0, 1], dtype=torch.int32, device="cuda"),
                          torch.zeros(2, g.n, dtype=torch.int32, device="cuda"), 0)
    assert ei.value.status == ssm.E_INVAL


def test_kmeans_sp_layout_end_to_end():
    """layout(sampling="kmeans") runs the oracle's pipeline on the refined pivots."""
    g = G.grid(30, 30)
    dg = ssm.DeviceGraph.from_csr(g)
    x, terms, piv, dist, delta, region = ssm.layout(dg, 20, 30, ssm.FP64, sampling="kmeans")
    p0, d0 = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, 20, 0)
    rp, _, _ = oracle.kmeans_sp(d0, p0)
    assert np.array_equal(piv.cpu().numpy(), rp)
    T = oracle.build_terms(g.row_ptr, g.col_idx, rp, oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, rp))
    assert np.array_equal(region.cpu().numpy(), T.region)
    xr = ssm.pivotmds_init(dg, terms, ssm.FP64)
    ssm.majorize(dg, terms, xr, 30)
    assert torch.equal(x, xr)


def test_validate_csr():
    g = G.grid(5, 6)
    ssm.validate_csr(ssm.DeviceGraph.from_csr(g))
    bad = []
    ci = g.col_idx.copy(); ci[0] = 0
    bad.append(ci)                                    # self-loop
    ci = g.col_idx.copy(); ci[1] = ci[0]
    bad.append(ci)                                    # duplicate arc
    ci = g.col_idx.copy(); ci[3] = g.n + 5
    bad.append(ci)                                    # out of range
    ci = g.col_idx.copy(); ci[2] = (ci[2] + 7) % g.n
    bad.append(ci)                                    # asymmetric
    for c in bad:
        dg = ssm.DeviceGraph(g.n, torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(c).cuda())
        with pytest.raises(ssm.SSMError) as ei:
            ssm.validate_csr(dg)
        assert ei.value.status == ssm.E_INVAL


def test_build_terms_unaligned_table():
    """A distance table that starts 4 bytes past a 16-byte boundary (a view
    into a larger buffer) gives the same terms as an aligned one."""
    g, k = G.rgg(3000, 5), 48
    dg, piv, _, dist, delta, region, terms = _device_pipeline(g, k)
    buf = torch.empty(dist.numel() + 1, dtype=torch.int32, device="cuda")
    buf[1:].copy_(dist.reshape(-1))
    view = buf[1:].view(dist.shape)
    assert view.data_ptr() % 16 != 0
    t2 = ssm.build_terms(dg, piv, view, delta, region)
    a, b = terms.export(), t2.export()
    assert a.keys() == b.keys()
    for key in a:
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("g,k", [(G.barabasi_albert(20000, 5, 3), 37), (G.rgg(3000, 5), 48), (G.grid(13, 17), 10),
                                 (G.holed_mesh(120, 130, 6, 4, 12, 5), 40)],
                         ids=["ba20000", "rgg3000", "grid13x17", "holedmesh120"])
def test_sweep_order_bit_identical(g, k, forced):
    """The FP32 sweep renumbers the nodes (by region, then delta) for
    locality; every node's arithmetic is unchanged, so the coordinates equal
    those of sweeps in the caller's order bit for bit (rows above the heavy
    degree, padded ranks, a ragged last chunk)."""
    outs = []
    for flag in (2, -1):  # reordered (forced: the library may skip graphs it would not gain on) / not
        forced("sweep_perm", flag)
        dg, *_, terms = _device_pipeline(g, k)
        x0 = ssm.pivotmds_init(dg, terms, ssm.FP32)
        x = x0.clone()
        ssm.majorize(dg, terms, x, 25, sync=True)
        outs.append((x0.cpu().numpy(), x.cpu().numpy(), ssm.stress(dg, terms, x)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.isfinite(outs[0][1]).all()
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


SHAPES = [dict(sweep_split=sp, sweep_waves=wv, sweep_blocks_per_cu=bpc)
          for sp in (1, 2, 4) for wv in (4, 16) for bpc in (1, 3, 8)]


@pytest.mark.parametrize("g,k", [(G.barabasi_albert(20000, 5, 3), 37), (G.rgg(3000, 5), 48),
                                 (G.holed_mesh(120, 130, 6, 4, 12, 5), 40), (G.grid(13, 17), 10)],
                         ids=["ba20000", "rgg3000", "holedmesh120", "grid13x17"])
def test_sweep_f32_launch_shapes_bit_identical(g, k, forced):
    """The FP32 sweep sums each node's terms in four fixed classes, whatever
    the waves per chunk, waves per block or grid: every launch shape gives
    the same coordinates bit for bit (so the autotuner may pick any), and
    the tuned loop equals the rule shape's."""
    say("case", g.name, "k", k)
    dg, *_, terms = _device_pipeline(g, k)
    x0 = ssm.pivotmds_init(dg, terms, ssm.FP32)
    forced("sweep_tune", -1)
    ref = x0.clone()
    ssm.majorize(dg, terms, ref, 30, sync=True)
    ref = ref.cpu().numpy()
    assert np.isfinite(ref).all()
    for shape in SHAPES:
        for name, val in shape.items():
            forced(name, val)
        x = x0.clone()
        ssm.majorize(dg, terms, x, 30, sync=True)
        assert np.array_equal(x.cpu().numpy(), ref), shape
    ssm.set_variant(None)
    x = x0.clone()
    ssm.majorize(dg, terms, x, 30, sync=True)  # tuned (30 >= 24 sweeps)
    assert np.array_equal(x.cpu().numpy(), ref)


def test_sweep_tuning_follows_the_weight_form(forced):
    """A loop run with a forced weight form must not leave its launch plan
    for later loops of the same graph shape: after it, the default loop
    (tuned) equals the rule shape's loop bit for bit."""
    g, k = G.rgg(3000, 5), 40
    dg, *_, terms = _device_pipeline(g, k)
    x0 = ssm.pivotmds_init(dg, terms, ssm.FP32)
    forced("sweep_mode", 2)
    x = x0.clone()
    ssm.majorize(dg, terms, x, 30, sync=True)
    ssm.set_variant(None)
    tuned = x0.clone()
    ssm.majorize(dg, terms, tuned, 30, sync=True)
    forced("sweep_tune", -1)
    rule = x0.clone()
    ssm.majorize(dg, terms, rule, 30, sync=True)
    assert torch.equal(tuned, rule)
