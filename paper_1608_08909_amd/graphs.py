"""Seeded synthetic graph generators.

This module only builds input graphs (symmetric CSR, int32, unit edge lengths);
it holds none of the layout method's arithmetic.  Both the CPU oracle's tests
and the GPU path's tests and benchmark draw their inputs from here, so the two
sides always consume byte-identical graphs.

The paper's evaluation graphs (Section 4, Table 1) are not available; the
families below stand in for its graph classes: finite-element meshes (grid,
holed triangulated mesh), geometric graphs (random geometric graph), hub-heavy
low-diameter graphs (Barabasi-Albert) and near-trees (random tree plus a few
extra edges).  The paper keeps only the largest connected component of a
disconnected input (Section 4, "Data"); every generator here does the same and
relabels the kept nodes in ascending order of their generation id.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "csr_from_edges", "largest_component", "path", "cycle", "star",
    "complete", "grid", "tri_grid", "rgg", "barabasi_albert", "tree_plus",
    "holed_mesh", "random_connected", "serving_requests", "make_request_graph",
]


@dataclass(frozen=True)
class CSR:
    """Symmetric CSR adjacency of a simple undirected graph (rows sorted)."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [2m]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def edges(self) -> np.ndarray:
        """Each undirected edge once as (u, v) with u < v, in CSR order."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        cols = self.col_idx.astype(np.int64)
        keep = rows < cols
        return np.stack([rows[keep], cols[keep]], axis=1)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(self.row_ptr.astype(np.int32).tobytes())
        h.update(self.col_idx.astype(np.int32).tobytes())
        return h.hexdigest()


def csr_from_edges(n: int, edges: np.ndarray, name: str = "") -> CSR:
    """Build a sorted symmetric CSR from an undirected edge list.

    Self-loops and duplicate edges are dropped so the result is a simple graph.
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n
    hi = key % n
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSR(n, row_ptr.astype(np.int32), cols.astype(np.int32), name)


def largest_component(g: CSR) -> CSR:
    """Keep the largest connected component; relabel by ascending old id.

    Ties between equally large components go to the one holding the smallest id.
    """
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.csr_matrix(
        (np.ones(g.nnz, dtype=np.int8), g.col_idx, g.row_ptr), shape=(g.n, g.n)
    )
    ncomp, label = connected_components(a, directed=False)
    if ncomp == 1:
        return g
    sizes = np.bincount(label, minlength=ncomp)
    first = np.full(ncomp, g.n, dtype=np.int64)
    np.minimum.at(first, label, np.arange(g.n))
    best = max(range(ncomp), key=lambda c: (sizes[c], -first[c]))
    keep = label == best
    newid = np.full(g.n, -1, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    e = g.edges()
    e = e[keep[e[:, 0]] & keep[e[:, 1]]]
    return csr_from_edges(int(keep.sum()), newid[e], g.name)


# ---------------------------------------------------------------- small shapes

def path(n: int) -> CSR:
    i = np.arange(n - 1)
    return csr_from_edges(n, np.stack([i, i + 1], 1), f"path{n}")


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return csr_from_edges(n, np.stack([i, (i + 1) % n], 1), f"cycle{n}")


def star(n: int) -> CSR:
    i = np.arange(1, n)
    return csr_from_edges(n, np.stack([np.zeros_like(i), i], 1), f"star{n}")


def complete(n: int) -> CSR:
    a, b = np.triu_indices(n, 1)
    return csr_from_edges(n, np.stack([a, b], 1), f"K{n}")


def grid(rows: int, cols: int) -> CSR:
    """rows x cols lattice, node id = cols*r + c, edges right and down."""
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    ids = (r * cols + c).ravel()
    right = np.stack([ids[(c < cols - 1).ravel()], ids[(c < cols - 1).ravel()] + 1], 1)
    down = np.stack([ids[(r < rows - 1).ravel()], ids[(r < rows - 1).ravel()] + cols], 1)
    return csr_from_edges(rows * cols, np.concatenate([right, down]), f"grid{rows}x{cols}")


def _tri_edges(rows: int, cols: int) -> np.ndarray:
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    ids = (r * cols + c).ravel()
    mr = (c < cols - 1).ravel()
    md = (r < rows - 1).ravel()
    mg = mr & md
    return np.concatenate([
        np.stack([ids[mr], ids[mr] + 1], 1),
        np.stack([ids[md], ids[md] + cols], 1),
        np.stack([ids[mg], ids[mg] + cols + 1], 1),
    ])


def tri_grid(rows: int, cols: int) -> CSR:
    """Lattice triangulated by the diagonal (r,c)-(r+1,c+1) in every cell."""
    return csr_from_edges(rows * cols, _tri_edges(rows, cols), f"trigrid{rows}x{cols}")


# ------------------------------------------------------------ random families

def rgg(n: int, seed: int, mean_degree: float = 8.0) -> CSR:
    """Random geometric graph: n points uniform in the unit square (PCG64),
    an edge between points at distance <= r with (n-1)*pi*r^2 = mean_degree;
    largest component kept."""
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    r = float(np.sqrt(mean_degree / (np.pi * (n - 1))))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    g = csr_from_edges(n, pairs, f"rgg{n}_s{seed}")
    return largest_component(g)


def barabasi_albert(n: int, m0: int, seed: int) -> CSR:
    """Preferential attachment: seed graph K_{m0+1}; each new node draws m0
    distinct targets with probability proportional to degree (uniform draws
    from the list of edge endpoints, duplicates redrawn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = m0 + 1
    a, b = np.triu_indices(s, 1)
    m_total = len(a) + (n - s) * m0
    src = np.empty(m_total, dtype=np.int32)
    dst = np.empty(m_total, dtype=np.int32)
    src[: len(a)] = a
    dst[: len(a)] = b
    ends = np.empty(2 * m_total, dtype=np.int32)
    ends[0: 2 * len(a): 2] = a
    ends[1: 2 * len(a): 2] = b
    ne = 2 * len(a)
    ecount = len(a)
    batch = 1 << 16
    u = rng.random(batch)
    ui = 0
    for v in range(s, n):
        chosen: list[int] = []
        while len(chosen) < m0:
            if ui == batch:
                u = rng.random(batch)
                ui = 0
            t = int(ends[int(u[ui] * ne)])
            ui += 1
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            src[ecount] = v
            dst[ecount] = t
            ends[ne] = v
            ends[ne + 1] = t
            ne += 2
            ecount += 1
    g = csr_from_edges(n, np.stack([src, dst], 1), f"ba{n}_m{m0}_s{seed}")
    return largest_component(g)


def _pruefer_tree(n: int, rng: np.random.Generator) -> np.ndarray:
    import heapq

    if n == 1:
        return np.zeros((0, 2), dtype=np.int64)
    if n == 2:
        return np.array([[0, 1]], dtype=np.int64)
    seq = rng.integers(0, n, size=n - 2)
    degree = np.ones(n, dtype=np.int64)
    np.add.at(degree, seq, 1)
    leaves = [i for i in range(n) if degree[i] == 1]
    heapq.heapify(leaves)
    edges = []
    for x in seq:
        leaf = heapq.heappop(leaves)
        edges.append((leaf, int(x)))
        degree[x] -= 1
        if degree[x] == 1:
            heapq.heappush(leaves, int(x))
    u = heapq.heappop(leaves)
    w = heapq.heappop(leaves)
    edges.append((u, w))
    return np.array(edges, dtype=np.int64)


def tree_plus(n: int, seed: int, extra_frac: float = 0.05) -> CSR:
    """Uniform random labelled tree (Pruefer code) plus floor(extra_frac*n)
    extra uniformly drawn non-edges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = _pruefer_tree(n, rng)
    have = set(map(tuple, np.sort(t, axis=1).tolist()))
    want = int(np.floor(extra_frac * n))
    extra = []
    while len(extra) < want:
        a, b = (int(v) for v in rng.integers(0, n, size=2))
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key in have:
            continue
        have.add(key)
        extra.append(key)
    e = np.concatenate([t, np.array(extra, dtype=np.int64).reshape(-1, 2)])
    return csr_from_edges(n, e, f"tree{n}_s{seed}")


def holed_mesh(rows: int, cols: int, holes: int, rmin: float, rmax: float,
               seed: int) -> CSR:
    """Triangulated lattice with circular holes removed, largest component kept.

    Hole centres are uniform in [0,rows) x [0,cols), radii uniform in
    [rmin, rmax]; a node (r, c) is removed when it lies inside or on a hole's
    circle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cy = rng.random(holes) * rows
    cx = rng.random(holes) * cols
    rad = rmin + rng.random(holes) * (rmax - rmin)
    alive = np.ones((rows, cols), dtype=bool)
    for y, x, q in zip(cy, cx, rad):
        r0, r1 = max(0, int(np.floor(y - q))), min(rows, int(np.ceil(y + q)) + 1)
        c0, c1 = max(0, int(np.floor(x - q))), min(cols, int(np.ceil(x + q)) + 1)
        rr, cc = np.meshgrid(np.arange(r0, r1), np.arange(c0, c1), indexing="ij")
        alive[r0:r1, c0:c1] &= (rr - y) ** 2 + (cc - x) ** 2 > q * q
    e = _tri_edges(rows, cols)
    flat = alive.ravel()
    e = e[flat[e[:, 0]] & flat[e[:, 1]]]
    newid = np.cumsum(flat) - 1
    n = int(flat.sum())
    g = csr_from_edges(n, newid[e], f"holedmesh{rows}x{cols}_h{holes}_s{seed}")
    return largest_component(g)


def random_connected(n: int, p: float, seed: int) -> CSR:
    """G(n, p) plus a random spanning path, so that it is connected."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a, b = np.triu_indices(n, 1)
    keep = rng.random(len(a)) < p
    perm = rng.permutation(n)
    chain = np.stack([perm[:-1], perm[1:]], 1)
    e = np.concatenate([np.stack([a[keep], b[keep]], 1), chain])
    return csr_from_edges(n, e, f"gnp{n}_s{seed}")


# ------------------------------------------------------------ serving stream

def serving_requests(count: int, seed: int) -> list[dict]:
    """Request specs of the mixed serving stream: each draws one of three
    families uniformly (grid a x b with a, b in [10,150]; random geometric
    graph with n in [200,20000] and mean degree in [6,10]; random tree plus 5%
    extra edges with n in [200,20000]) and k = min(100, floor(n/10))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        fam = int(rng.integers(0, 3))
        gseed = int(rng.integers(0, 2**31 - 1))
        if fam == 0:
            a, b = (int(v) for v in rng.integers(10, 151, size=2))
            out.append({"family": "grid", "a": a, "b": b, "seed": gseed})
        elif fam == 1:
            n = int(rng.integers(200, 20001))
            deg = float(6.0 + 4.0 * rng.random())
            out.append({"family": "rgg", "n": n, "deg": deg, "seed": gseed})
        else:
            n = int(rng.integers(200, 20001))
            out.append({"family": "tree", "n": n, "seed": gseed})
    return out


def make_request_graph(spec: dict) -> CSR:
    if spec["family"] == "grid":
        return grid(spec["a"], spec["b"])
    if spec["family"] == "rgg":
        return rgg(spec["n"], spec["seed"], spec["deg"])
    if spec["family"] == "tree":
        return tree_plus(spec["n"], spec["seed"])
    raise ValueError(spec)


def edge_lengths(g: CSR, seed: int, lo: float = 0.5, hi: float = 2.0, integer: bool = False) -> np.ndarray:
    """Positive edge lengths per arc (float64 [2m]), the same on both arcs of
    an edge: uniform in [lo, hi) (PCG64), or uniform integers in
    [lo, hi] when `integer` (many equal distances, hence region ties)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col_idx.astype(np.int64)
    a, b = np.minimum(src, dst), np.maximum(src, dst)
    key = a * g.n + b
    uniq, inv = np.unique(key, return_inverse=True)
    if integer:
        vals = rng.integers(int(lo), int(hi) + 1, size=uniq.size).astype(np.float64)
    else:
        vals = lo + (hi - lo) * rng.random(uniq.size)
    return vals[inv]
