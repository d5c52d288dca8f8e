"""The layout pool (ssm_pool_*): many graphs per launch must give every graph
exactly what the oracle gives it alone.

- preprocessing of each graph in a mixed batch: pivots, distances, delta,
  regions, H, the FP64 weight table and denominators bit-exact;
- PivotMDS start within 1e-9 of the RMS radius (rigid alignment where the
  dominant plane's axes are not unique);
- the FP64 warm-up sweep bit-exact against the oracle's sweep from the same
  start;
- the FP32 sweeps: final stress within 1e-4 of the plain FP64 path;
- a graph's result is identical alone and in a mix (added at another time,
  swept in other quanta next to other graphs);
- admission: a full arena refuses a graph until a slot is removed.
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


MIX = [
    (G.grid(7, 9), 6), (G.path(30), 5), (G.cycle(17), 4), (G.tri_grid(9, 11), 10),
    (G.random_connected(40, 0.1, 3), 7), (G.tree_plus(300, 2), 17), (G.rgg(1500, 4), 33),
    (G.barabasi_albert(2000, 5, 7), 50), (G.grid(50, 50), 50), (G.holed_mesh(120, 130, 6, 4, 12, 5), 40),
    (G.star(12), 3), (G.complete(9), 4),
]


def _pool_with(graphs, warm, cap=1 << 30):
    pool = ssm.Pool(cap)
    slots = [pool.add(g, k) for g, k in graphs]
    assert all(s is not None for s in slots)
    pool.prepare(slots, warm=warm)
    return pool, slots


def test_pool_preprocessing_bit_exact():
    pool, slots = _pool_with(MIX, warm=0)
    for (g, k), s in zip(MIX, slots):
        say("case", g.name, "k", k)
        info = pool.info(s)
        assert info["state"] == ssm.POOL_READY
        ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
        assert np.array_equal(pool.export(s, ssm.POOL_PIVOTS), ref.pivots)
        assert np.array_equal(pool.export(s, ssm.POOL_DIST), ref.dist)
        assert np.array_equal(pool.export(s, ssm.POOL_DELTA), ref.delta)
        assert np.array_equal(pool.export(s, ssm.POOL_REGION), ref.region)
        assert info["dmax"] == ref.dmax and info["delta_max"] == ref.delta_max
        assert np.array_equal(pool.export(s, ssm.POOL_H), ref.H)
        assert np.array_equal(pool.export(s, ssm.POOL_WTAB64), ref.wtab)
        assert np.array_equal(pool.export(s, ssm.POOL_DEN64), ref.den)
    pool.close()


def test_pool_pivotmds_and_warm_sweep():
    graphs = [c for c in MIX if c[1] >= 3]
    p0, s0 = _pool_with(graphs, warm=0)
    p1, s1 = _pool_with(graphs, warm=1)
    for (g, k), a, b in zip(graphs, s0, s1):
        say("case", g.name, "k", k)
        ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
        x0 = p0.export(a, ssm.POOL_X64)
        xo, _, _ = oracle.pivotmds(ref.dist)
        xr = oracle.rescale(g.row_ptr, g.col_idx, xo)
        w = np.linalg.eigvalsh(oracle.gram(oracle.pmds_center(ref.dist)))[::-1]
        if not (w[1] > 1e-8 * w[0] and (w[1] - w[2]) / w[0] < 1e-6):  # the plane itself is unique
            well = (w[0] - w[1]) / w[0] > 1e-3 and w[1] > 1e-8 * w[0]
            assert brute.coord_error(x0, xr, align=not well) < 1e-9
        # the warm-up sweep: the oracle's FP64 sweep from the pool's own start
        x1 = p1.export(b, ssm.POOL_X64)
        x1r, _ = oracle.majorize(g.row_ptr, g.col_idx, ref.pivots, ref.dist, ref.wtab, ref.den, x0, 1)
        assert np.array_equal(x1, x1r)
        assert np.array_equal(p1.export(b, ssm.POOL_X32), x1r.astype(np.float32))
    p0.close()
    p1.close()


LARGE_K = [(G.rgg(3000, 5), 150), (G.tri_grid(30, 40), 200), (G.tree_plus(2000, 3), 250), (G.grid(20, 25), 60)]


def test_pool_pivotmds_large_k():
    """A batch whose largest k lies in (128, 256]: the pooled eigen step's
    larger register form, rows from 128 on read from memory."""
    pool, slots = _pool_with(LARGE_K, warm=0)
    for (g, k), s in zip(LARGE_K, slots):
        say("case", g.name, "k", k)
        ref = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
        x0 = pool.export(s, ssm.POOL_X64)
        xo, _, _ = oracle.pivotmds(ref.dist)
        xr = oracle.rescale(g.row_ptr, g.col_idx, xo)
        w = np.linalg.eigvalsh(oracle.gram(oracle.pmds_center(ref.dist)))[::-1]
        assert w[1] > 1e-8 * w[0] and (w[1] - w[2]) / w[0] > 1e-6  # the plane is unique on these graphs
        well = (w[0] - w[1]) / w[0] > 1e-3
        assert brute.coord_error(x0, xr, align=not well) < 1e-9
    pool.close()


def test_pool_fp32_final_stress_vs_plain_fp64():
    graphs = [(G.grid(50, 50), 50), (G.rgg(3000, 9, 8.0), 100), (G.tree_plus(2000, 6), 100),
              (G.grid(23, 71), 100), (G.rgg(800, 2, 7.0), 80)]
    iters = 200
    pool, slots = _pool_with(graphs, warm=1)
    pool.sweep(slots, 37)
    pool.sweep(slots, 1000)  # capped at each graph's sweep count
    s32 = pool.stress(slots)
    for (g, k), s, st in zip(graphs, slots, s32):
        assert pool.info(s)["done"] == iters
        dg = ssm.DeviceGraph.from_csr(g)
        x, terms, *_ = ssm.layout(dg, k, iters, ssm.FP64)
        s64 = ssm.stress(dg, terms, x)
        say("case", g.name, "k", k, "stress", st, s64, abs(st - s64) / s64)
        assert abs(st - s64) <= 1e-4 * s64
    pool.close()


def test_pool_alone_equals_mixed():
    g, k = G.rgg(2500, 17, 8.0), 60
    alone, (sa,) = _pool_with([(g, k)], warm=1)
    alone.sweep([sa], 200)
    xa = alone.export(sa, ssm.POOL_X32)
    # the same graph added later, next to others, swept in other quanta
    mix = ssm.Pool(1 << 30)
    others = [mix.add(G.grid(30, 40), 40), mix.add(G.tree_plus(900, 3), 30)]
    mix.prepare(others, warm=1)
    mix.sweep(others, 13)
    sm = mix.add(g, k)
    extra = mix.add(G.rgg(1200, 5, 8.0), 50)
    mix.prepare([extra, sm], warm=1)
    mix.sweep(others + [sm, extra], 7)
    mix.sweep([sm], 50)
    mix.sweep([extra, sm] + others, 500)
    xm = mix.export(sm, ssm.POOL_X32)
    assert np.array_equal(xa, xm)
    assert mix.stress([sm])[0] == alone.stress([sa])[0]
    alone.close()
    mix.close()


def test_pool_captured_quanta_match_direct_launches():
    """Sweep quanta replayed from captured HIP graphs (the default) equal the
    same quanta launched kernel by kernel, bit for bit, after every replay:
    the same shapes again and again (replays of one graph), another shape in
    between, a graph with the stop test, exports (synchronizing reads)
    between the replays.  The same holds for either sweep schedule (a block
    per chunk, a persistent grid), captured or not."""
    specs = [(G.grid(30, 40), 40), (G.tree_plus(900, 3), 30), (G.rgg(1200, 5, 8.0), 50), (G.rgg(2500, 17, 8.0), 60)]

    def run():
        pool, slots = _pool_with(specs, warm=1)
        pool.set_tol(slots[2], 1e-3)
        outs = []
        for rep in range(4):
            pool.sweep(slots, 9)
            outs.append([pool.export(s, ssm.POOL_X32).copy() for s in slots])
            pool.sweep(slots[:2], 5)
            torch.cuda.synchronize()
            outs.append([pool.export(s, ssm.POOL_X32).copy() for s in slots])
        outs.append([np.array(pool.stress(slots)), np.array(pool.stopped(slots[2:3]))])
        pool.close()
        return outs

    captured = run()
    for v in ({"pool_graph": -1}, {"pool_persist": 1}, {"pool_persist": -1}, {"pool_persist": 1, "pool_graph": -1}):
        say("variant", v)
        with ssm.variants(**v):
            other = run()
        for step, (a, b) in enumerate(zip(captured, other)):
            for q, (x, y) in enumerate(zip(a, b)):
                assert np.array_equal(x, y), (v, step, q)


def test_pool_admission_and_failures():
    pool = ssm.Pool(4 << 20)
    used0, cap = pool.usage()
    assert used0 == 0 and cap >= 4 << 20
    slots = []
    while True:
        s = pool.add(G.grid(40, 40), 50)
        if s is None:
            break
        slots.append(s)
        assert len(slots) < 100
    assert len(slots) >= 1
    pool.remove(slots.pop())
    s = pool.add(G.grid(40, 40), 50)
    assert s is not None
    slots.append(s)
    for s in slots:
        pool.remove(s)
    assert pool.usage()[0] == 0
    # a disconnected graph fails in preparation; the others in the batch do not
    d = G.csr_from_edges(6, np.array([[0, 1], [1, 2], [3, 4], [4, 5]]))
    good = pool.add(G.grid(6, 7), 5)
    bad = pool.add(d, 3)
    pool.prepare([bad, good])
    assert pool.info(bad)["state"] == ssm.POOL_FAILED and pool.info(bad)["fail"] == ssm.E_DISCONNECTED
    assert pool.info(good)["state"] == ssm.POOL_READY
    with pytest.raises(ssm.SSMError):
        pool.sweep([bad], 1)
    with pytest.raises(ssm.SSMError) as ei:
        pool.add(G.grid(3, 3), 10)        # k > n
    assert ei.value.status == ssm.E_RANGE
    # ids out of range are refused at admission; a one-way arc, a self-loop
    # or a repeated neighbour fail the graph in preparation
    g4 = G.grid(4, 4)
    ci = g4.col_idx.copy()
    ci[3] = g4.n + 2
    with pytest.raises(ssm.SSMError) as ei:
        pool.add(G.CSR(g4.n, g4.row_ptr, ci, "bad"), 3)
    assert ei.value.status == ssm.E_INVAL
    bads = []
    for mutate in (lambda c: (c.__setitem__(2, (c[2] + 5) % g4.n), c)[1],   # one-way arc
                   lambda c: (c.__setitem__(0, 0), c)[1],                    # self-loop at node 0
                   lambda c: (c.__setitem__(1, c[0]), c)[1]):                # repeated neighbour
        bads.append(pool.add(G.CSR(g4.n, g4.row_ptr, mutate(g4.col_idx.copy()), "bad"), 3))
    ok = pool.add(G.grid(5, 5), 4)
    pool.prepare(bads + [ok])
    for b in bads:
        assert pool.info(b)["state"] == ssm.POOL_FAILED and pool.info(b)["fail"] == ssm.E_INVAL
    assert pool.info(ok)["state"] == ssm.POOL_READY
    pool.close()


def _oracle_changes(g, k, x0, count):
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    out, x = [], x0
    for _ in range(count):
        xn, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x, 1)
        out.append(oracle.rigid_change(x, xn))
        x = xn
    return np.array(out)


STOP_MIX = [(G.rgg(3000, 3), 40), (G.grid(20, 30), 25), (G.tree_plus(800, 5), 30), (G.grid(12, 15), 18),
            (G.barabasi_albert(3000, 4, 2), 60)]


def test_pool_stop_test_per_graph():
    """Algorithm 1's stop test per graph in a mixed batch: each graph stops
    on a sweep where the oracle's change sequence (FP64, from the pool's own
    FP64 start) is within rounding of tol, and takes no sweep after it; a
    graph that keeps moving runs its sweep count; the same graph alone stops
    on the same sweep with the same layout."""
    tol, cap = 1e-4, 600
    pool = ssm.Pool(1 << 30)
    slots = [pool.add(g, k, 0, cap) for g, k in STOP_MIX]
    for s in slots:
        pool.set_tol(s, tol)
    pool.prepare(slots, warm=1)
    starts = [pool.export(s, ssm.POOL_X64) for s in slots]  # after the FP64 warm-up sweep
    ran = np.full(len(slots), -1)
    for _ in range(cap // 25 + 1):
        pool.sweep(slots, 25)
        r = pool.stopped(slots)
        ran = np.where(ran < 0, r, ran)
    for (g, k), s, x1, n_run in zip(STOP_MIX, slots, starts, ran):
        say("case", g.name, "k", k, "stopped after", n_run)
        ch = _oracle_changes(g, k, x1, cap - 1)  # FP64 continuation of the warm-up sweep
        if n_run < 0:
            assert pool.info(s)["done"] == cap
            assert np.all(ch > 0.95 * tol)
            continue
        j = n_run - 2  # the change of FP32 sweep n_run - 1 (sweep 1 is the FP64 warm-up)
        assert 0 <= j and ch[j] <= 1.05 * tol and np.all(ch[:j] > 0.95 * tol)
        # alone: same stop, same layout
        alone = ssm.Pool(1 << 28)
        sa = alone.add(g, k, 0, cap)
        alone.set_tol(sa, tol)
        alone.prepare([sa], warm=1)
        alone.sweep([sa], cap)
        assert alone.stopped([sa])[0] == n_run
        assert np.array_equal(alone.export(sa, ssm.POOL_X32), pool.export(s, ssm.POOL_X32))
        alone.close()
    pool.close()
