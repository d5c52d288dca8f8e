"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
closed forms, brute force over all pairs on tiny graphs, invariants, special
cases and hand-derived values (tests/golden/hand_derived.json)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1608_08909_amd import graphs as G
from tests import brute

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_derived.json")))


def _graph(spec):
    if spec["family"] == "path":
        return G.path(spec["n"])
    if spec["family"] == "grid":
        return G.grid(spec["rows"], spec["cols"])
    if spec["family"] == "edges":
        return G.csr_from_edges(spec["n"], np.array(spec["edges"]))
    raise ValueError(spec)


def _tiny_graphs():
    out = [G.path(9), G.cycle(10), G.cycle(7), G.star(8), G.complete(6), G.grid(4, 5),
           G.tri_grid(4, 4)]
    for s in range(4):
        out.append(G.random_connected(14 + s, 0.15, seed=s))
        out.append(G.tree_plus(16 + s, seed=s))
    out.append(G.rgg(60, seed=3, mean_degree=7.0))
    out.append(G.barabasi_albert(40, 2, seed=5))
    return out


# ------------------------------------------------------------------ BFS

def _closed_form_rows(g, kind, shape=None):
    n = g.n
    i = np.arange(n)
    if kind == "path":
        return np.abs(i[:, None] - i[None, :])
    if kind == "cycle":
        a = np.abs(i[:, None] - i[None, :])
        return np.minimum(a, n - a)
    if kind == "star":
        d = np.where((i[:, None] == 0) | (i[None, :] == 0), 1, 2)
        d[i, i] = 0
        return d
    if kind == "complete":
        return (i[:, None] != i[None, :]).astype(int)
    R, C = shape
    r, c = i // C, i % C
    dr = r[None, :] - r[:, None]
    dc = c[None, :] - c[:, None]
    if kind == "grid":
        return np.abs(dr) + np.abs(dc)
    if kind == "tri":
        same = dr * dc >= 0
        return np.where(same, np.maximum(np.abs(dr), np.abs(dc)), np.abs(dr) + np.abs(dc))
    raise ValueError(kind)


@pytest.mark.parametrize("g,kind,shape", [
    (G.path(23), "path", None), (G.cycle(17), "cycle", None), (G.cycle(18), "cycle", None),
    (G.star(9), "star", None), (G.complete(7), "complete", None),
    (G.grid(6, 9), "grid", (6, 9)), (G.tri_grid(7, 5), "tri", (7, 5)),
])
def test_bfs_closed_forms(g, kind, shape):
    want = _closed_form_rows(g, kind, shape)
    for s in range(g.n):
        assert np.array_equal(oracle.bfs(g.n, g.row_ptr, g.col_idx, s), want[s])


def test_bfs_matches_all_pairs():
    for g in _tiny_graphs():
        D = brute.apsp(g)
        for s in range(g.n):
            assert np.array_equal(oracle.bfs(g.n, g.row_ptr, g.col_idx, s), D[s]), g.name


def test_bfs_invariants():
    for g in _tiny_graphs():
        k = min(6, g.n)
        piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
        e = g.edges()
        assert np.all(np.abs(dist[:, e[:, 0]] - dist[:, e[:, 1]]) <= 1)
        assert np.array_equal(dist[:, piv], dist[:, piv].T)
        assert np.all(dist[np.arange(k), piv] == 0)


# --------------------------------------------------------------- pivots

@pytest.mark.parametrize("key", ["maxmin_path30_k5", "maxmin_grid50_first4"])
def test_maxmin_golden(key):
    gd = GOLDEN[key]
    g = _graph(gd["graph"])
    piv, _ = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, gd["k"], gd["first"])
    assert piv.tolist() == gd["pivots"]


def test_maxmin_brute():
    for g in _tiny_graphs():
        D = brute.apsp(g)
        for k in sorted({1, 2, 3, g.n // 2, g.n}):
            for first in (0, g.n - 1):
                piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, first)
                assert piv.tolist() == brute.maxmin_brute(D, k, first), (g.name, k, first)
                assert np.array_equal(dist, D[piv])
                assert len(set(piv.tolist())) == k


# -------------------------------------------------------------- regions

@pytest.mark.parametrize("key", ["regions_path5_equal_sizes", "regions_tie_to_smaller"])
def test_regions_golden(key):
    gd = GOLDEN[key]
    g = _graph(gd["graph"])
    dist = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, gd["pivots"])
    _, region, _, _ = oracle.regions(dist)
    assert region.tolist() == gd["region"]
    if "pivots_swapped" in gd:
        dist = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, gd["pivots_swapped"])
        _, region, _, _ = oracle.regions(dist)
        assert region.tolist() == gd["region_swapped"]


def _check_region_rule(dist, delta, region, size):
    """A-posteriori check of the tie rule: every tied node at level l sits in a
    candidate region whose size (all members below l plus the single-candidate
    members at l) is minimal, lowest rank among equals."""
    k, n = dist.shape
    ncand = (dist == delta[None, :]).sum(0)
    for lvl in np.unique(delta):
        at = np.flatnonzero(delta == lvl)
        below = np.bincount(region[delta < lvl], minlength=k)
        single = at[ncand[at] == 1]
        snap = below + np.bincount(region[single], minlength=k)
        for i in at[ncand[at] > 1]:
            cands = np.flatnonzero(dist[:, i] == lvl)
            best = min(cands, key=lambda t: (snap[t], t))
            assert region[i] == best


def test_regions_invariants():
    for g in _tiny_graphs() + [G.grid(50, 50)]:
        for k in sorted({1, 2, min(5, g.n), g.n // 3 or 1}):
            piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
            delta, region, size, dm = oracle.regions(dist)
            assert np.array_equal(delta, dist.min(0))
            assert dm == delta.max()
            assert region.min() >= 0 and region.max() < k
            assert np.array_equal(np.bincount(region, minlength=k), size)   # partition
            assert np.all(region[piv] == np.arange(k))                       # p in R(p)
            assert np.all(dist[region, np.arange(g.n)] == delta)             # nearest pivot
            _check_region_rule(dist, delta, region, size)


def test_regions_k_equals_n():
    for g in _tiny_graphs():
        piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, g.n, 0)
        _, region, size, dm = oracle.regions(dist)
        assert dm == 0 and np.all(size == 1)
        assert np.array_equal(piv[region], np.arange(g.n))


def test_regions_grid50_k50():
    g = G.grid(50, 50)
    piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, 50, 0)
    delta, region, size, dm = oracle.regions(dist)
    assert dm == 6 and size.min() == 21 and size.max() == 78
    assert int(((dist == delta[None, :]).sum(0) > 1).sum()) == 277


# -------------------------------------------------------------- weights

def test_weights_golden():
    gd = GOLDEN["regions_tie_to_smaller"]
    g = _graph(gd["graph"])
    dist = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, gd["pivots"])
    T = oracle.build_terms(g.row_ptr, g.col_idx, gd["pivots"], dist)
    for i, t, w in gd["weights"]["node_pivotrank_weight"]:
        assert T.wtab[t, dist[t, i]] == w


def test_weights_brute():
    for g in _tiny_graphs() + [G.grid(12, 13)]:
        D = brute.apsp(g)
        for k in sorted({2, min(5, g.n), g.n // 2, g.n}):
            piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
            T = oracle.build_terms(g.row_ptr, g.col_idx, piv, dist)
            Wb = brute.weights_brute(D, piv, T.region)
            Wo = T.wtab[np.arange(k)[None, :], dist.T]
            assert np.array_equal(Wo, Wb), (g.name, k)
            # s >= 1 wherever a pivot term exists
            s = np.rint(Wo * dist.T.astype(float) ** 2)
            assert np.all(s[dist.T >= 2] >= 1)
            assert np.all(Wo[dist.T < 2] == 0)
            deg = np.diff(g.row_ptr)
            assert np.array_equal(T.den, deg + Wb.sum(1)) or np.allclose(T.den, deg + Wb.sum(1), rtol=1e-15)


def test_weights_k_equals_n_full_model():
    for g in _tiny_graphs():
        piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, g.n, 0)
        T = oracle.build_terms(g.row_ptr, g.col_idx, piv, dist)
        W = T.wtab[np.arange(g.n)[None, :], dist.T]
        d = dist.T.astype(float)
        want = np.where(d >= 2, 1.0 / np.where(d > 0, d, 1) ** 2, 0.0)
        assert np.array_equal(W, want)


def test_weights_path_two_pivots_closed_form():
    for n in (9, 10, 31, 32):
        g = G.path(n)
        piv = [0, n - 1]
        dist = oracle.bfs_pivots(g.n, g.row_ptr, g.col_idx, piv)
        T = oracle.build_terms(g.row_ptr, g.col_idx, piv, dist)
        sizes = [(n + 1) // 2, n // 2]   # odd n: the middle node joins rank 0
        assert T.size.tolist() == sizes
        for t in range(2):
            for i in range(n):
                d = int(dist[t, i])
                if d < 2:
                    continue
                s = min(d // 2 + 1, sizes[t])
                assert T.wtab[t, d] == s / (d * d)


# ------------------------------------------------------------- PivotMDS

def test_pmds_centering_and_gram():
    for g in [G.grid(20, 30), G.rgg(400, seed=2), G.barabasi_albert(300, 3, seed=1)]:
        piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, 20, 0)
        C = oracle.pmds_center(dist)
        scale = np.abs(C).max()
        assert np.abs(C.sum(0)).max() <= 1e-12 * scale * g.n
        assert np.abs(C.sum(1)).max() <= 1e-12 * scale * 20
        M = oracle.gram(C)
        assert np.allclose(M, C.T @ C, rtol=1e-12, atol=1e-12 * np.abs(M).max())
        ev, E = oracle.sym_eig(M)
        wn, vn = np.linalg.eigh(M)
        assert np.allclose(np.sort(ev), wn, rtol=0, atol=1e-12 * wn.max())
        x, V, lam = oracle.pivotmds(dist)
        assert np.allclose(lam, wn[::-1][:2], rtol=1e-12)
        for a in range(2):
            v = vn[:, -1 - a]
            big = np.flatnonzero(np.abs(v) >= np.abs(v).max() * (1 - 1e-9))[0]
            v = v * np.sign(v[big])
            assert np.allclose(V[:, a], v, atol=1e-10)
            assert V[np.argmax(np.abs(V[:, a])), a] > 0
        assert np.allclose(x, C @ V, rtol=1e-12, atol=1e-12 * np.abs(x).max())


def test_pmds_sign_rule_on_symmetric_star():
    """Star with pivots [centre, leaf, leaf]: the dominant eigenvector has two
    entries of equal magnitude in exact arithmetic; the lower index decides."""
    g = G.star(12)
    piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, 3, 0)
    x, V, lam = oracle.pivotmds(dist)
    assert abs(abs(V[1, 0]) - abs(V[2, 0])) < 1e-12 and V[1, 0] > 0
    assert lam[0] == pytest.approx(4.0) and lam[1] == pytest.approx(1.5)


def test_pmds_path_is_exact():
    """A path's pivot distances are Euclidean on a line: PivotMDS is exact and
    after the rescale every edge has length 1 (zero full stress)."""
    for n, k in [(30, 5), (57, 8)]:
        g = G.path(n)
        piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
        x0 = oracle.rescale(g.row_ptr, g.col_idx, oracle.pivotmds(dist)[0])
        assert oracle.stress_full(g.row_ptr, g.col_idx, x0) < 1e-20
        assert brute.full_stress(brute.apsp(g), x0) < 1e-20


def test_rescale_closed_form():
    g = G.rgg(300, seed=5)
    x = np.random.default_rng(0).normal(size=(g.n, 2))
    y = oracle.rescale(g.row_ptr, g.col_idx, x)
    e = g.edges()
    assert abs(np.linalg.norm(y[e[:, 0]] - y[e[:, 1]], axis=1).sum() - g.m) < 1e-9 * g.m
    c = y / x
    assert np.allclose(c, c[0, 0])


# ---------------------------------------------------------- majorization

def _terms_full(g):
    piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, g.n, 0)
    return oracle.build_terms(g.row_ptr, g.col_idx, piv, dist)


def test_k_equals_n_update_is_localized_full_stress():
    rng = np.random.default_rng(1)
    for g in _tiny_graphs():
        T = _terms_full(g)
        D = brute.apsp(g)
        x = rng.normal(size=(g.n, 2)) * 3
        x1, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x, 1)
        assert np.allclose(x1, brute.localized_full_step(D, x), rtol=1e-12, atol=1e-12), g.name


def test_monotone_full_stress_k_equals_n():
    rng = np.random.default_rng(2)
    for g in _tiny_graphs():
        T = _terms_full(g)
        D = brute.apsp(g)
        x = rng.normal(size=(g.n, 2)) * 2
        s_prev = brute.full_stress(D, x)
        for _ in range(15):
            x, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x, 1)
            s = brute.full_stress(D, x)
            assert s <= s_prev * (1 + 1e-12) + 1e-12, g.name
            s_prev = s


def test_twins_stay_together():
    """Two adjacent nodes with the same closed neighbourhood have the same
    pivot distances, so PivotMDS puts them on one point; in exact arithmetic
    Eq. 5 then moves them identically forever (their vote to each other is at
    distance zero).  The oracle must reproduce that exactly, whatever the CSR
    order puts between them."""
    # twins 3 and 9 (ids far apart, other neighbours in between), plus a
    # false twin pair 5, 7 (same open neighbourhood, not adjacent)
    e = [[0, 1], [1, 2], [2, 0], [3, 9], [3, 1], [9, 1], [3, 4], [9, 4], [3, 8], [9, 8],
         [4, 6], [6, 10], [10, 11], [8, 11], [5, 6], [7, 6], [2, 11], [4, 2]]
    g = G.csr_from_edges(12, np.array(e))
    N = [set(g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]].tolist()) for i in range(g.n)]
    assert N[3] | {3} == N[9] | {9} and N[5] == N[7]
    for k in (3, 4, 5):   # from node 6 no twin becomes a pivot (a pivot breaks the symmetry)
        T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k, first=6)
        assert not set(T.pivots.tolist()) & {3, 9, 5, 7}
        x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
        assert np.array_equal(x0[3], x0[9]) and np.array_equal(x0[5], x0[7])
        x, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, 300)
        assert np.array_equal(x[3], x[9]) and np.array_equal(x[5], x[7])
        assert np.abs(x[3] - x[1]).max() > 1e-3


def test_zero_stress_path_is_fixed():
    for n, k in [(20, 3), (20, 7), (31, 31)]:
        g = G.path(n)
        piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
        T = oracle.build_terms(g.row_ptr, g.col_idx, piv, dist)
        ang = 0.3
        x = np.stack([np.arange(n) * math.cos(ang), np.arange(n) * math.sin(ang)], 1) + [2.0, -1.0]
        x1, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x, 3)
        assert np.abs(x1 - x).max() < 1e-12


def _ngon_radius(n):
    h = np.arange(1, n)
    d = np.minimum(h, n - h).astype(float)
    c = 2 * np.sin(np.pi * h / n)
    w = 1 / d ** 2
    return (w * d * c).sum() / (w * c * c).sum()


def test_regular_polygon_fixed_point():
    n = 12
    g = G.cycle(n)
    T = _terms_full(g)
    r = _ngon_radius(n)
    assert abs(r - 2.1854946005562663) < 1e-14
    a = 2 * np.pi * np.arange(n) / n
    x = r * np.stack([np.cos(a), np.sin(a)], 1)
    x1, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x, 1)
    assert np.abs(x1 - x).max() < 1e-13


def test_stress_closed_forms():
    g = G.path(25)
    x = np.stack([np.arange(25.0), np.zeros(25)], 1)
    assert oracle.stress_full(g.row_ptr, g.col_idx, x) == 0.0
    n, r = 12, 1.7
    g = G.cycle(n)
    a = 2 * np.pi * np.arange(n) / n
    x = r * np.stack([np.cos(a), np.sin(a)], 1)
    h = np.arange(1, n)
    d = np.minimum(h, n - h)
    want = n / 2 * ((2 * r * np.sin(np.pi * h / n) - d) ** 2 / d ** 2).sum()
    assert abs(oracle.stress_full(g.row_ptr, g.col_idx, x) - want) < 1e-12 * want
    R, C = 7, 9
    g = G.grid(R, C)
    rr, cc = np.divmod(np.arange(R * C), C)
    x = np.stack([cc, rr], 1).astype(float)
    want = 0.0
    for aa in range(R):
        for bb in range(C):
            if aa == 0 and bb == 0:
                continue
            mult = (R - aa) * (C - bb) * (2 if aa > 0 and bb > 0 else 1)
            want += mult * (math.hypot(aa, bb) - (aa + bb)) ** 2 / (aa + bb) ** 2
    assert abs(oracle.stress_full(g.row_ptr, g.col_idx, x) - want) < 1e-12 * want


def test_sparse_stress_brute_and_full_identity():
    rng = np.random.default_rng(3)
    for g in _tiny_graphs():
        D = brute.apsp(g)
        x = rng.normal(size=(g.n, 2)) * 2
        for k in sorted({2, min(5, g.n), g.n}):
            piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
            T = oracle.build_terms(g.row_ptr, g.col_idx, piv, dist)
            s, se, sp = oracle.stress_sparse(g.row_ptr, g.col_idx, piv, dist, T.wtab, x, parts=True)
            W = brute.weights_brute(D, piv, T.region)
            r = np.linalg.norm(x[:, None, :] - x[None, piv, :], axis=-1)
            want_p = (W * (r - D[:, piv]) ** 2).sum()
            e = g.edges()
            want_e = ((np.linalg.norm(x[e[:, 0]] - x[e[:, 1]], axis=1) - 1) ** 2).sum()
            assert abs(sp - want_p) <= 1e-12 * max(1, want_p)
            assert abs(se - want_e) <= 1e-12 * max(1, want_e)
            if k == g.n:   # each non-edge pair appears once from each side
                full = brute.full_stress(D, x)
                assert abs(s - (se + 2 * (full - se))) <= 1e-11 * full


def test_rigid_motion_equivariance():
    """Eq. 5 commutes with rotations, reflections and translations.  The start
    layout is random: PivotMDS puts nodes with equal pivot-distance vectors on
    one point, where the update's direction term is discontinuous (r = 0), so
    rounding alone would decide how such twins separate."""
    g = G.rgg(200, seed=8)
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, 12)
    x0 = np.random.default_rng(4).normal(size=(g.n, 2)) * 5
    th = 0.77
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    F = np.diag([1.0, -1.0])
    args = (g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den)
    x1, _ = oracle.majorize(*args, x0, 20)
    y1, _ = oracle.majorize(*args, x0 @ R.T @ F + [5.0, -3.0], 20)
    assert np.abs(y1 - (x1 @ R.T @ F + [5.0, -3.0])).max() < 1e-9 * np.abs(x1).max()


def test_resume_and_thread_independence():
    g = G.grid(20, 20)
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, 10)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
    args = (g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den)
    a, _ = oracle.majorize(*args, x0, 30)
    b, _ = oracle.majorize(*args, x0, 12)
    b, _ = oracle.majorize(*args, b, 18)
    c, _ = oracle.majorize(*args, x0, 30, threads=4)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_tolerance_stop():
    """The early stop fires at the first sweep whose relative change is within
    tol.  k = n (symmetric weights) converges to a fixed point; with k < n the
    asymmetric w' leave a steady rigid drift, so a raw change never vanishes."""
    g = G.grid(8, 8)
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, g.n)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
    args = (g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den)
    x, done = oracle.majorize(*args, x0, 1000, tol=1e-4)
    assert 0 < done < 1000
    prev, _ = oracle.majorize(*args, x0, done - 1)
    assert np.linalg.norm(x - prev) / np.linalg.norm(prev) <= 1e-4
    prev2, _ = oracle.majorize(*args, x0, done - 2)
    assert np.linalg.norm(prev - prev2) / np.linalg.norm(prev2) > 1e-4


def test_sparse_layout_tracks_full_stress():
    """Soft check of the paper's trend (Table 2): more pivots, full stress
    closer to the full-stress (k = n) layout."""
    g = G.grid(20, 20)
    D = brute.apsp(g)
    out = {}
    for k in (10, 40, g.n):
        x, T, x0, _ = oracle.layout(g.n, g.row_ptr, g.col_idx, k, 200)
        x = x * ((D[np.triu_indices(g.n, 1)] ** -1.0 * np.linalg.norm(
            x[:, None] - x[None], axis=-1)[np.triu_indices(g.n, 1)]).sum()
            / (np.linalg.norm(x[:, None] - x[None], axis=-1)[np.triu_indices(g.n, 1)] ** 2
               * D[np.triu_indices(g.n, 1)] ** -2.0).sum())
        out[k] = brute.full_stress(D, x)
    assert out[g.n] <= out[40] * 1.01 and out[40] <= out[10] * 1.05


# ------------------------------------------------------------- contract

def test_validate_rejects_bad_input():
    g = G.grid(3, 3)
    assert oracle.validate(g.n, g.row_ptr, g.col_idx) == oracle.OK
    ci = g.col_idx.copy(); ci[0] = 0                       # self loop at node 0
    assert oracle.validate(g.n, g.row_ptr, ci) == oracle.INVAL
    ci = g.col_idx.copy(); ci[1] = ci[0]                   # duplicate in row 0
    assert oracle.validate(g.n, g.row_ptr, ci) == oracle.INVAL
    e = np.array([[0, 1], [1, 2]])
    h = G.csr_from_edges(3, e)
    rp = np.array([0, 1, 2, 3], dtype=np.int32)            # 0->1, 1->2, 2->1: asymmetric
    assert oracle.validate(3, rp, np.array([1, 2, 1], dtype=np.int32)) == oracle.INVAL
    d = G.csr_from_edges(4, np.array([[0, 1], [2, 3]]))
    with pytest.raises(oracle.OracleError) as ei:
        oracle.select_pivots(d.n, d.row_ptr, d.col_idx, 2, 0)
    assert ei.value.status == oracle.DISCONNECTED
    assert oracle.validate(h.n, h.row_ptr, h.col_idx) == oracle.OK


# ----------------------------------------------------------------- k-means sp

@pytest.mark.parametrize("key,n", [("kmeans_sp_path5_k2", 5), ("kmeans_sp_path9_k2", 9)])
def test_kmeans_sp_golden(key, n):
    gd = GOLDEN[key]
    g = G.path(n)
    piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, 2, 0)
    assert piv.tolist() == [0, n - 1]
    newp, assign, it = oracle.kmeans_sp(dist, piv)
    assert newp.tolist() == gd["pivots"]
    assert assign.tolist() == gd["assign"]
    assert it == gd["iterations"]


def test_kmeans_sp_k_equals_n_keeps_maxmin_pivots():
    """With k = n every node is a cluster of its own vector (rows of the full
    distance matrix are distinct), so the pivots come back unchanged."""
    g = G.random_connected(25, 0.15, 4)
    piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, g.n, 0)
    newp, assign, it = oracle.kmeans_sp(dist, piv)
    assert newp.tolist() == piv.tolist()
    assert np.array_equal(assign[piv], np.arange(g.n))
    assert it == 2


def _sqdist_exact(y, S, N):
    """||y - S/N||^2 as an exact rational."""
    from fractions import Fraction
    return sum((Fraction(int(a)) - Fraction(int(b), int(N))) ** 2 for a, b in zip(y, S))


@pytest.mark.parametrize("g,k", [(G.grid(9, 11), 6), (G.tree_plus(150, 3), 8), (G.rgg(300, 9), 7)],
                         ids=["grid9x11", "tree150", "rgg300"])
def test_kmeans_sp_fixed_point(g, k):
    """At termination before the cap: every node sits in a cluster whose
    centroid (the exact mean of its members) is nearest to it, and every new
    pivot is the nearest free node to its centroid (exact rational
    arithmetic, checked against the definitions, not the implementation)."""
    from fractions import Fraction
    piv, dist = oracle.select_pivots(g.n, g.row_ptr, g.col_idx, k, 0)
    newp, assign, it = oracle.kmeans_sp(dist, piv, 50)
    assert it < 50
    Y = dist.T.astype(np.int64)  # n x k feature vectors
    S = np.zeros((k, k), dtype=np.int64)
    N = np.zeros(k, dtype=np.int64)
    for i in range(g.n):
        S[assign[i]] += Y[i]
        N[assign[i]] += 1
    assert N.min() >= 1  # no cluster emptied on these graphs
    for i in range(g.n):
        d = [_sqdist_exact(Y[i], S[t], N[t]) for t in range(k)]
        best = min(d)
        assert d[assign[i]] == best
        assert assign[i] == d.index(best)  # lowest rank on ties
    taken = set()
    for t in range(k):
        cand = [(_sqdist_exact(Y[i], S[t], N[t]), i) for i in range(g.n) if i not in taken]
        assert newp[t] == min(cand)[1]
        taken.add(int(newp[t]))
    assert len(set(newp.tolist())) == k


# ----------------------------------------------------------- quality measures

def test_procrustes_closed_forms():
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.normal(size=(40, 2))
    assert abs(oracle.procrustes(x, x)) < 1e-14
    # a translated, rotated and dilated copy matches perfectly
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    y = 3.5 * x @ R.T + np.array([10.0, -4.0])
    assert abs(oracle.procrustes(y, x)) < 1e-12
    assert abs(oracle.procrustes(x, y)) < 1e-12
    # a reflection is not an allowed operation: for centred axis-aligned
    # spreads a = sum x^2, b = sum y^2 with sum xy = 0, the mirror image leaves
    # 1 - ((b - a) / (a + b))^2 = 4ab / (a + b)^2 unmatched
    c = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 2.0], [0.0, -2.0]])
    m = c * np.array([1.0, -1.0])
    a, b = 2.0, 8.0
    assert abs(oracle.procrustes(m, c) - 4 * a * b / (a + b) ** 2) < 1e-15
    # a layout squeezed onto a line against a round one
    ring = np.array([[np.cos(2 * np.pi * q / 12), np.sin(2 * np.pi * q / 12)] for q in range(12)])
    line = ring * np.array([1.0, 0.0])
    # best match explains sigma_1 = sum cos^2 = 6 of the ring's spread 12 and
    # the line's spread 6: 1 - 36 / (6 * 12) = 1/2
    assert abs(oracle.procrustes(line, ring) - 0.5) < 1e-12


def test_procrustes_range_and_symmetry():
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(50):
        x = rng.normal(size=(25, 2))
        y = rng.normal(size=(25, 2))
        p = oracle.procrustes(x, y)
        assert 0.0 <= p <= 1.0
        assert abs(p - oracle.procrustes(y, x)) < 1e-12


def test_normalized_stress_of_a_path():
    # a path drawn on a line with unit spacing has zero stress; doubling the
    # spacing gives sum over pairs (2d - d)^2 / d^2 = C(n, 2) pairs of 1
    g = G.path(9)
    x = np.stack([np.arange(9, dtype=np.float64), np.zeros(9)], axis=1)
    assert oracle.normalized_stress(g.row_ptr, g.col_idx, x) == 0.0
    assert abs(oracle.normalized_stress(g.row_ptr, g.col_idx, 2 * x) - 1.0) < 1e-15


# ---------------------------------------------------------- weighted graphs

def _bellman_ford(n, rp, ci, ln, src):
    """Value iteration to the least fixed point of d(v) = min_u d(u) + len."""
    d = np.full(n, np.inf)
    d[src] = 0.0
    srcs = np.repeat(np.arange(n), np.diff(rp))
    while True:
        cand = d[srcs] + ln
        nd = d.copy()
        np.minimum.at(nd, ci, cand)
        if np.array_equal(nd, d):
            return d
        d = nd


@pytest.mark.parametrize("g,seed,integer", [(G.grid(9, 11), 1, False), (G.rgg(400, 3), 2, False),
                                            (G.tree_plus(300, 4), 3, True), (G.grid(7, 7), 5, True)])
def test_sssp_is_the_least_fixed_point(g, seed, integer):
    ln = G.edge_lengths(g, seed, 1 if integer else 0.5, 4 if integer else 2.0, integer)
    for src in (0, g.n // 2, g.n - 1):
        assert np.array_equal(oracle.sssp(g.n, g.row_ptr, g.col_idx, ln, src),
                              _bellman_ford(g.n, g.row_ptr, g.col_idx, ln, src))


def test_weighted_path_closed_form():
    g = G.path(6)
    steps = np.array([0.5, 1.25, 2.0, 0.75, 3.5])  # dyadic: every prefix sum is exact
    ln = np.empty(g.col_idx.size)
    for i in range(g.n):
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            ln[e] = steps[min(i, g.col_idx[e])]
    pref = np.concatenate([[0.0], np.cumsum(steps)])
    assert np.array_equal(oracle.sssp(g.n, g.row_ptr, g.col_idx, ln, 0), pref)
    piv, dist = oracle.select_pivots_w(g.n, g.row_ptr, g.col_idx, ln, 3, 0)
    # farthest from 0 is node 5 (8.0); then the node maximizing min(d0, d5):
    # node 3 (min(3.75, 4.25)) against node 2 (min(1.75, 6.25))
    assert list(piv) == [0, 5, 3]


def test_weighted_regions_tie_rule():
    # path 0 - 1 - 2 with lengths 1.5: node 1 is tied between pivots 0 and 2;
    # both regions hold one node at its level, so the lower rank wins
    g = G.path(3)
    ln = np.full(g.col_idx.size, 1.5)
    piv, dist = oracle.select_pivots_w(g.n, g.row_ptr, g.col_idx, ln, 2, 0)
    assert list(piv) == [0, 2]
    delta, region, size = oracle.regions_w(dist)
    assert list(region) == [0, 0, 1] and list(size) == [2, 1] and list(delta) == [0.0, 1.5, 0.0]


@pytest.mark.parametrize("g,k", [(G.grid(9, 11), 7), (G.tree_plus(300, 2), 17), (G.rgg(500, 4), 25),
                                 (G.cycle(17), 4)])
def test_unit_lengths_reproduce_the_unweighted_model(g, k):
    ln = np.ones(g.col_idx.size)
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    W = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, ln, k)
    assert np.array_equal(W.pivots, T.pivots)
    assert np.array_equal(W.dist, T.dist.astype(np.float64))
    assert np.array_equal(W.region, T.region)
    assert np.array_equal(W.delta, T.delta.astype(np.float64))
    wref = np.take_along_axis(T.wtab, T.dist, axis=1)  # w'(t, d_ti) from the table
    assert np.array_equal(W.w, wref)
    assert np.array_equal(W.den, T.den)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
    xa, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, 5)
    xb = oracle.majorize_w(g.row_ptr, g.col_idx, ln, W.pivots, W.dist, W.w, W.den, x0, 5)
    assert np.array_equal(xa, xb)
    sa = oracle.stress_sparse(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, xa)
    sb = oracle.stress_w(g.row_ptr, g.col_idx, ln, W.pivots, W.dist, W.w, xb)
    assert abs(sa - sb) <= 1e-12 * sa


def test_weights_by_definition_and_power_of_two_scaling():
    g = G.rgg(300, 6)
    ln = G.edge_lengths(g, 7)
    k = 12
    W = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, ln, k)
    # w' and den straight from the definitions (all pairs, numpy)
    adj = np.zeros((g.n, g.n), dtype=bool)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    adj[src, g.col_idx] = True
    for t in range(k):
        p = W.pivots[t]
        d = W.dist[t]
        s = ((W.region[None, :] == t) & (W.delta[None, :] <= d[:, None] / 2)).sum(axis=1)
        with np.errstate(divide="ignore"):  # d = 0 at the pivot itself, masked out
            want = np.where((np.arange(g.n) != p) & ~adj[:, p], s / (d * d), 0.0)
        assert np.array_equal(W.w[t], want)
    # den: the arcs' len^-2 in CSR order, then the ranks in order
    den = np.array([sum(1.0 / (ln[e] * ln[e]) for e in range(g.row_ptr[i], g.row_ptr[i + 1])) for i in range(g.n)])
    for i in range(g.n):
        s = den[i]
        for t in range(k):
            s += W.w[t, i]
        assert s == W.den[i]
    # lengths times 4: distances times 4, same pivots and regions, weights
    # and denominators divided by 16, layouts times 4 -- all exact
    W4 = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, 4 * ln, k)
    assert np.array_equal(W4.pivots, W.pivots) and np.array_equal(W4.region, W.region)
    assert np.array_equal(W4.dist, 4 * W.dist)
    assert np.array_equal(W4.w, W.w / 16) and np.array_equal(W4.den, W.den / 16)
    x0, _, _ = oracle.pivotmds_w(W.dist)
    x0 = oracle.rescale_w(g.row_ptr, g.col_idx, ln, x0)
    x = oracle.majorize_w(g.row_ptr, g.col_idx, ln, W.pivots, W.dist, W.w, W.den, x0, 10)
    x4 = oracle.majorize_w(g.row_ptr, g.col_idx, 4 * ln, W4.pivots, W4.dist, W4.w, W4.den, 4 * x0, 10)
    assert np.array_equal(x4, 4 * x)


@pytest.mark.parametrize("g,k", [(G.grid(9, 11), 7), (G.tree_plus(300, 2), 17), (G.rgg(500, 4), 25)])
def test_weighted_pivotmds_and_rescale_at_unit_lengths(g, k):
    # Algorithm 1's initialisation with every length 1 is the unweighted one:
    # the real-valued distance table holds the same integers, so PivotMDS and
    # the rescale to the summed edge lengths (m) agree bit for bit
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    xa, Va, la = oracle.pivotmds(T.dist)
    xb, Vb, lb = oracle.pivotmds_w(T.dist.astype(np.float64))
    assert np.array_equal(xa, xb) and np.array_equal(Va, Vb) and np.array_equal(la, lb)
    ln = np.ones(g.col_idx.size)
    assert np.array_equal(oracle.rescale(g.row_ptr, g.col_idx, xa), oracle.rescale_w(g.row_ptr, g.col_idx, ln, xb))


def _edge_length_sum(g, x):
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    up = g.col_idx > src
    return np.linalg.norm(x[src[up]] - x[g.col_idx[up]], axis=1).sum()


def test_weighted_rescale_matches_summed_lengths_and_scales_exactly():
    g = G.rgg(400, 11)
    ln = G.edge_lengths(g, 12)
    k = 16
    W = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, ln, k)
    x0, V, lam = oracle.pivotmds_w(W.dist)
    x = oracle.rescale_w(g.row_ptr, g.col_idx, ln, x0)
    # after the rescale the drawn edges sum to the summed edge lengths (Algorithm 1)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    want = ln[g.col_idx > src].sum()
    assert abs(_edge_length_sum(g, x) - want) <= 1e-12 * want
    # lengths x 4: the centred squared distances scale by 16, the Gram by 256,
    # the eigenvectors are unchanged and the projection scales by 16; the
    # rescale then brings the layout to exactly 4 times the unit-scale one
    W4 = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, 4 * ln, k)
    x40, V4, lam4 = oracle.pivotmds_w(W4.dist)
    assert np.array_equal(V4, V) and np.array_equal(lam4, 256 * lam) and np.array_equal(x40, 16 * x0)
    assert np.array_equal(oracle.rescale_w(g.row_ptr, g.col_idx, 4 * ln, x40), 4 * x)


def _stress_w_by_definition(g, ln, pivots, dist, w, x):
    """Eq. 3 with edge lengths, summed by numpy: every edge once with weight
    len^-2, every (node, pivot) term with its adapted weight."""
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    up = g.col_idx > src
    r = np.linalg.norm(x[src[up]] - x[g.col_idx[up]], axis=1)
    le = ln[up]
    s_edges = np.sum((r - le) ** 2 / le ** 2)
    s_piv = 0.0
    for t, p in enumerate(pivots):
        rp = np.linalg.norm(x - x[p], axis=1)
        s_piv += np.sum(w[t] * (rp - dist[t]) ** 2)
    return s_edges + s_piv


def test_weighted_stress_by_definition_and_exact_scaling():
    g = G.grid(13, 17)
    ln = G.edge_lengths(g, 5)
    k = 9
    W = oracle.preprocess_w(g.n, g.row_ptr, g.col_idx, ln, k)
    x = oracle.layout_w(g.n, g.row_ptr, g.col_idx, ln, k, 7)[0]
    s = oracle.stress_w(g.row_ptr, g.col_idx, ln, W.pivots, W.dist, W.w, x)
    ref = _stress_w_by_definition(g, ln, W.pivots, W.dist, W.w, x)
    assert abs(s - ref) <= 1e-12 * ref
    # a perturbed layout: the length terms are not near zero there
    rng = np.random.default_rng(3)
    xp = x + rng.normal(scale=0.3, size=x.shape)
    s = oracle.stress_w(g.row_ptr, g.col_idx, ln, W.pivots, W.dist, W.w, xp)
    ref = _stress_w_by_definition(g, ln, W.pivots, W.dist, W.w, xp)
    assert abs(s - ref) <= 1e-12 * ref
    # lengths, distances and layout x 4, weights / 16: every term is unchanged
    s4 = oracle.stress_w(g.row_ptr, g.col_idx, 4 * ln, W.pivots, 4 * W.dist, W.w / 16, 4 * xp)
    assert s4 == s


# ------------------------------------------ Algorithm 1's stop test (reading 5)

def _rot(th):
    return np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])


def _kabsch_change(x, y):
    """min over proper rotations R and translations t of ||y - (R x + t)|| /
    ||x - mean x||, by the SVD of the cross-covariance (Kabsch, with the
    determinant correction that excludes reflections)."""
    a, b = x - x.mean(0), y - y.mean(0)
    U, _, Vt = np.linalg.svd(a.T @ b)
    D = np.diag([1.0, np.sign(np.linalg.det(U @ Vt))])
    R = U @ D @ Vt          # a @ R best matches b
    return np.linalg.norm(b - a @ R) / np.linalg.norm(a)


def test_rigid_change_is_zero_for_a_rigid_motion_and_not_for_a_mirror():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(300, 2)) * 7
    for th in (0.0, 0.4, 2.5, -1.2):
        y = x @ _rot(th).T + np.array([3.0, -11.0])
        assert oracle.rigid_change(x, y) < 1e-14
    # a reflection is not a proper rigid motion: an anisotropic cloud keeps
    # a large change after the best rotation
    x[:, 0] *= 3
    y = x * np.array([-1.0, 1.0])
    assert oracle.rigid_change(x, y) > 0.5


def test_rigid_change_matches_the_kabsch_solution():
    rng = np.random.default_rng(6)
    for trial in range(20):
        n = int(rng.integers(3, 400))
        x = rng.normal(size=(n, 2)) * rng.uniform(0.1, 100)
        y = x @ _rot(rng.uniform(-3, 3)).T + rng.normal(size=2) * 10 + rng.normal(size=(n, 2)) * rng.uniform(1e-6, 1)
        want = _kabsch_change(x, y)
        assert abs(oracle.rigid_change(x, y) - want) <= 1e-9 * want
        # unchanged by scaling both layouts by a power of two (exact)
        assert oracle.rigid_change(4 * x, 4 * y) == oracle.rigid_change(x, y)
    # zero spread: never counts as converged
    assert oracle.rigid_change(np.ones((5, 2)), np.ones((5, 2))) == np.inf


def _stepwise(g, T, x, iters, centred=False):
    """Per-sweep (raw change, rigid change) by running one sweep at a time;
    with centred=True also the change after removing the translation only."""
    out = []
    for _ in range(iters):
        xn, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x, 1)
        a, b = x - x.mean(0), xn - xn.mean(0)
        row = (np.linalg.norm(xn - x) / np.linalg.norm(x), _kabsch_change(x, xn))
        out.append(row + (np.linalg.norm(b - a) / np.linalg.norm(a),) if centred else row)
        x = xn
    return out


@pytest.mark.parametrize("g", [G.grid(12, 15), G.cycle(40), G.tree_plus(150, 9)])
def test_stop_agrees_with_the_raw_rule_at_k_equal_n(g):
    # k = n: the weights are symmetric and the PivotMDS start is centred, so
    # there is no steady rigid drift: the change after the best rigid motion
    # stays within a few per cent of the raw change (until both reach the
    # rounding floor), so the two readings stop within one sweep of each
    # other
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, g.n)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
    assert np.abs(x0.mean(0)).max() < 1e-12 * np.abs(x0).max()
    tol = 1e-4
    steps = _stepwise(g, T, x0, 300, centred=True)
    for raw, rig, trans in steps:
        if raw > 1e-8:
            # no rotation (identity) is one candidate motion
            assert rig <= trans * (1 + 1e-9)
            assert rig >= 0.97 * raw
    first_raw = next(q + 1 for q, (raw, _, _) in enumerate(steps) if raw <= tol)
    first_rigid = next(q + 1 for q, (_, rig, _) in enumerate(steps) if rig <= tol)
    assert first_raw - 1 <= first_rigid <= first_raw
    _, done = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, 300, tol=tol)
    assert done == first_rigid


def test_stop_fires_for_k_below_n_where_the_raw_rule_does_not():
    g = G.rgg(3000, 3)
    k = 40
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
    tol = 1e-4
    steps = _stepwise(g, T, x0, 400)
    assert min(raw for raw, _ in steps[50:]) > 2 * tol   # the steady drift keeps the raw change up
    first = next(q + 1 for q, (_, rig) in enumerate(steps) if rig <= tol * (1 - 1e-6))
    assert all(rig > tol * (1 + 1e-6) for _, rig in steps[:first - 1])
    x, done = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, 400, tol=tol)
    assert done == first
    xr, _ = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, first)
    assert np.array_equal(x, xr)


def test_stop_is_unchanged_by_a_rigid_motion_of_the_start():
    g = G.grid(20, 30)
    k = 25
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
    R, t = _rot(0.9), np.array([250.0, -40.0])
    xa, da = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, 400, tol=1e-4)
    xb, db = oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0 @ R.T + t, 400, tol=1e-4)
    assert da == db and da < 400
    assert np.abs(xb - (xa @ R.T + t)).max() < 1e-9 * np.abs(xa).max()
