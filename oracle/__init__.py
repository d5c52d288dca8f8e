"""Plain FP64 CPU oracle of the sparse stress model (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It wraps ``ssm_oracle.c`` (serial C, FP64, correctly rounded sqrt and
division, no fast-math, no contraction) through ctypes and returns numpy
arrays.  It imports nothing from the GPU package and shares no code with it.

Each function follows a passage of Ortmann, Klimenta, Brandes, "A Sparse
Stress Model": Section 3 (regions, adapted weights, Eqs. 3 and 5), Algorithm 1
(pipeline, rescale), Section 4.1 (max/min sp sampling), Eq. 1 (full stress).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssm_oracle.c")
_LIB = os.path.join(_HERE, "_ssm_oracle.so")
_lock = threading.Lock()
_lib = None

OK, INVAL, RANGE, DISCONNECTED, NOMEM = 0, 1, 2, 3, 4


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what}: status {status}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
             "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            I, D, P = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
            sig = {
                "orc_validate": (I, [I, P, P]),
                "orc_bfs": (I, [I, P, P, I, P]),
                "orc_select_pivots": (I, [I, P, P, I, I, P, P]),
                "orc_bfs_pivots": (I, [I, P, P, I, P, P]),
                "orc_regions": (I, [I, I, P, P, P, P, P]),
                "orc_histogram": (None, [I, I, P, P, I, P]),
                "orc_weight_table": (None, [I, I, P, I, P]),
                "orc_denominator": (None, [I, P, I, P, P, I, P]),
                "orc_pmds_center": (None, [I, I, P, P]),
                "orc_gram": (None, [I, I, P, P]),
                "orc_sym_eig": (I, [I, P, P, P]),
                "orc_pivotmds": (I, [I, I, P, P, P, P]),
                "orc_rescale": (I, [I, P, P, P]),
                "orc_majorize": (I, [I, P, P, I, P, P, P, I, P, P, I, D, I, I, P]),
                "orc_rigid_change": (D, [I, P, P]),
                "orc_stress_sparse": (D, [I, P, P, I, P, P, P, I, P, P]),
                "orc_stress_full": (D, [I, P, P, P]),
                "orc_kmeans_sp": (I, [I, I, P, P, I, P, P, P]),
                "orc_sssp": (I, [I, P, P, P, I, P]),
                "orc_select_pivots_w": (I, [I, P, P, P, I, I, P, P]),
                "orc_regions_w": (I, [I, I, P, P, P, P]),
                "orc_terms_w": (I, [I, P, P, P, I, P, P, P, P, P, P]),
                "orc_majorize_w": (I, [I, P, P, P, I, P, P, P, P, P, I]),
                "orc_stress_w": (D, [I, P, P, P, I, P, P, P, P]),
                "orc_pivotmds_w": (I, [I, I, P, P, P, P]),
                "orc_rescale_w": (I, [I, P, P, P, P]),
            }
            for name, (res, args) in sig.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ wrappers

def validate(n, row_ptr, col_idx) -> int:
    rp, ci = _i32(row_ptr), _i32(col_idx)
    return _load().orc_validate(n, _p(rp), _p(ci))


def bfs(n, row_ptr, col_idx, src: int) -> np.ndarray:
    rp, ci = _i32(row_ptr), _i32(col_idx)
    d = np.empty(n, dtype=np.int32)
    _load().orc_bfs(n, _p(rp), _p(ci), int(src), _p(d))
    return d


def select_pivots(n, row_ptr, col_idx, k: int, first: int = 0):
    """Max/min sp sampling; returns (pivots[k], dist[k][n])."""
    rp, ci = _i32(row_ptr), _i32(col_idx)
    piv = np.empty(k, dtype=np.int32)
    dist = np.empty((k, n), dtype=np.int32)
    st = _load().orc_select_pivots(n, _p(rp), _p(ci), int(k), int(first), _p(piv), _p(dist))
    if st != OK:
        raise OracleError(st, "select_pivots")
    return piv, dist


def bfs_pivots(n, row_ptr, col_idx, pivots) -> np.ndarray:
    rp, ci, pv = _i32(row_ptr), _i32(col_idx), _i32(pivots)
    dist = np.empty((len(pv), n), dtype=np.int32)
    st = _load().orc_bfs_pivots(n, _p(rp), _p(ci), len(pv), _p(pv), _p(dist))
    if st != OK:
        raise OracleError(st, "bfs_pivots")
    return dist


def regions(dist: np.ndarray):
    """Returns (delta[n], region[n], size[k], delta_max)."""
    dist = _i32(dist)
    k, n = dist.shape
    delta = np.empty(n, dtype=np.int32)
    region = np.empty(n, dtype=np.int32)
    size = np.empty(k, dtype=np.int32)
    dm = ctypes.c_int(0)
    _load().orc_regions(n, k, _p(dist), _p(delta), _p(region), _p(size), ctypes.byref(dm))
    return delta, region, size, int(dm.value)


def histogram(delta, region, k: int, delta_max: int) -> np.ndarray:
    delta, region = _i32(delta), _i32(region)
    H = np.empty((k, delta_max + 1), dtype=np.int32)
    _load().orc_histogram(len(delta), k, _p(delta), _p(region), int(delta_max), _p(H))
    return H


def weight_table(H: np.ndarray, dmax: int) -> np.ndarray:
    H = _i32(H)
    k, w = H.shape
    wt = np.empty((k, dmax + 1), dtype=np.float64)
    _load().orc_weight_table(k, w - 1, _p(H), int(dmax), _p(wt))
    return wt


def denominator(row_ptr, dist, wtab) -> np.ndarray:
    rp, dist, wtab = _i32(row_ptr), _i32(dist), _f64(wtab)
    k, n = dist.shape
    den = np.empty(n, dtype=np.float64)
    _load().orc_denominator(n, _p(rp), k, _p(dist), _p(wtab), wtab.shape[1] - 1, _p(den))
    return den


def pmds_center(dist) -> np.ndarray:
    dist = _i32(dist)
    k, n = dist.shape
    C = np.empty((n, k), dtype=np.float64)
    _load().orc_pmds_center(n, k, _p(dist), _p(C))
    return C


def gram(C) -> np.ndarray:
    C = _f64(C)
    n, k = C.shape
    M = np.empty((k, k), dtype=np.float64)
    _load().orc_gram(n, k, _p(C), _p(M))
    return M


def sym_eig(M):
    """Cyclic Jacobi eigen-decomposition; returns (evals, evecs), unsorted."""
    M = _f64(M)
    k = M.shape[0]
    ev = np.empty(k, dtype=np.float64)
    E = np.empty((k, k), dtype=np.float64)
    _load().orc_sym_eig(k, _p(M), _p(ev), _p(E))
    return ev, E


def pivotmds(dist):
    """Returns (x[n][2], V[k][2], lambda[2])."""
    dist = _i32(dist)
    k, n = dist.shape
    x = np.empty((n, 2), dtype=np.float64)
    V = np.empty((k, 2), dtype=np.float64)
    lam = np.empty(2, dtype=np.float64)
    st = _load().orc_pivotmds(n, k, _p(dist), _p(x), _p(V), _p(lam))
    if st != OK:
        raise OracleError(st, "pivotmds")
    return x, V, lam


def rescale(row_ptr, col_idx, x) -> np.ndarray:
    rp, ci = _i32(row_ptr), _i32(col_idx)
    x = _f64(x).copy()
    st = _load().orc_rescale(x.shape[0], _p(rp), _p(ci), _p(x))
    if st != OK:
        raise OracleError(st, "rescale")
    return x


def majorize(row_ptr, col_idx, pivots, dist, wtab, den, x, iters: int, tol: float = 0.0,
             gauss_seidel: bool = False, threads: int = 1):
    """Runs the Eq. 5 sweeps; returns (x_new, iterations_done)."""
    rp, ci, pv, dist = _i32(row_ptr), _i32(col_idx), _i32(pivots), _i32(dist)
    wtab, den = _f64(wtab), _f64(den)
    x = _f64(x).copy()
    k, n = dist.shape
    done = ctypes.c_int(0)
    st = _load().orc_majorize(n, _p(rp), _p(ci), k, _p(pv), _p(dist), _p(wtab),
                              wtab.shape[1] - 1, _p(den), _p(x), int(iters), float(tol),
                              int(bool(gauss_seidel)), int(threads), ctypes.byref(done))
    if st != OK:
        raise OracleError(st, "majorize")
    return x, int(done.value)


def rigid_change(x_old, x_new) -> float:
    """Algorithm 1's relative positional change of one sweep, after the best
    proper rigid motion (rotation and translation) of x_old onto x_new,
    relative to the spread of x_old about its centroid."""
    a, b = _f64(x_old), _f64(x_new)
    return _load().orc_rigid_change(a.shape[0], _p(a), _p(b))


def stress_sparse(row_ptr, col_idx, pivots, dist, wtab, x, parts: bool = False):
    rp, ci, pv, dist = _i32(row_ptr), _i32(col_idx), _i32(pivots), _i32(dist)
    wtab, x = _f64(wtab), _f64(x)
    k, n = dist.shape
    pr = np.zeros(2, dtype=np.float64)
    s = _load().orc_stress_sparse(n, _p(rp), _p(ci), k, _p(pv), _p(dist), _p(wtab),
                                  wtab.shape[1] - 1, _p(x), _p(pr))
    return (s, pr[0], pr[1]) if parts else s


def stress_full(row_ptr, col_idx, x) -> float:
    rp, ci, x = _i32(row_ptr), _i32(col_idx), _f64(x)
    return _load().orc_stress_full(x.shape[0], _p(rp), _p(ci), _p(x))


def normalized_stress(row_ptr, col_idx, x) -> float:
    """Section 4.1's normalized stress: the full stress of Eq. 1 divided by the
    number of node pairs n (n - 1) / 2."""
    n = np.asarray(x).shape[0]
    return stress_full(row_ptr, col_idx, x) / (n * (n - 1) / 2)


def procrustes(x, y) -> float:
    """Section 4.1's Procrustes statistic of layout x against reference y:
    after the best translation, dilation and rotation (reflections are not
    among the allowed operations), the share of the spread left unmatched,
    in [0, 1].  Computed the textbook way: centre both layouts, take the SVD
    of X^T Y; the best proper rotation achieves sigma_1 + s sigma_2 with s the
    sign of det(U V^T) (Kabsch); the statistic is 1 - that squared over
    tr(X^T X) tr(Y^T Y)."""
    X = np.asarray(x, dtype=np.float64)
    Y = np.asarray(y, dtype=np.float64)
    X = X - X.mean(axis=0)
    Y = Y - Y.mean(axis=0)
    U, S, Vt = np.linalg.svd(X.T @ Y)
    sgn = 1.0 if np.linalg.det(U @ Vt) >= 0 else -1.0
    t = S[0] + sgn * S[1]
    return float(1.0 - t * t / ((X * X).sum() * (Y * Y).sum()))


def kmeans_sp(dist, pivots, max_iters: int = 50):
    """k-means sp refinement of max/min pivots (Section 4.1): returns
    (new_pivots[k], assign[n], iterations)."""
    dist, pv = _i32(dist), _i32(pivots)
    k, n = dist.shape
    newp = np.empty(k, dtype=np.int32)
    assign = np.empty(n, dtype=np.int32)
    it = ctypes.c_int(0)
    st = _load().orc_kmeans_sp(n, k, _p(dist), _p(pv), int(max_iters), _p(newp), _p(assign), ctypes.byref(it))
    if st != OK:
        raise OracleError(st, "kmeans_sp")
    return newp, assign, int(it.value)


# ----------------------------------------------------------------- pipeline

@dataclass
class Terms:
    pivots: np.ndarray
    dist: np.ndarray
    delta: np.ndarray
    region: np.ndarray
    size: np.ndarray
    delta_max: int
    dmax: int
    H: np.ndarray
    wtab: np.ndarray
    den: np.ndarray


def build_terms(row_ptr, col_idx, pivots, dist) -> Terms:
    """Regions, histograms, adapted weights and denominators (Section 3)."""
    delta, region, size, dm = regions(dist)
    k = dist.shape[0]
    dmax = int(dist.max())
    H = histogram(delta, region, k, dm)
    wt = weight_table(H, dmax)
    den = denominator(row_ptr, dist, wt)
    return Terms(_i32(pivots), _i32(dist), delta, region, size, dm, dmax, H, wt, den)


def preprocess(n, row_ptr, col_idx, k: int, first: int = 0) -> Terms:
    piv, dist = select_pivots(n, row_ptr, col_idx, k, first)
    return build_terms(row_ptr, col_idx, piv, dist)


def initial_layout(row_ptr, col_idx, terms: Terms) -> np.ndarray:
    """PivotMDS on the selected pivots, then Algorithm 1's rescale."""
    x, _, _ = pivotmds(terms.dist)
    return rescale(row_ptr, col_idx, x)


def layout(n, row_ptr, col_idx, k: int, iters: int, first: int = 0, tol: float = 0.0,
           threads: int = 1):
    """Algorithm 1 end to end (Jacobi order).  Returns (x, terms, x0, iters_done)."""
    t = preprocess(n, row_ptr, col_idx, k, first)
    x0 = initial_layout(row_ptr, col_idx, t)
    x, done = majorize(row_ptr, col_idx, t.pivots, t.dist, t.wtab, t.den, x0, iters, tol,
                       threads=threads)
    return x, t, x0, done


# ------------------------------------------------------- weighted graphs
# Algorithm 1's general input: positive edge lengths len[e] per arc (equal in
# both directions).  Distances are shortest-path lengths summed from the
# source outwards in FP64; edge terms carry len^-2; pivot terms are Section
# 3's with real distances.

def sssp(n, row_ptr, col_idx, length, src: int) -> np.ndarray:
    """Dijkstra's algorithm: FP64 distances from src (inf where unreached)."""
    rp, ci, ln = _i32(row_ptr), _i32(col_idx), _f64(length)
    d = np.empty(n, dtype=np.float64)
    st = _load().orc_sssp(n, _p(rp), _p(ci), _p(ln), int(src), _p(d))
    if st != OK:
        raise OracleError(st, "sssp")
    return d


def select_pivots_w(n, row_ptr, col_idx, length, k: int, first: int = 0):
    """max/min sp on weighted distances; returns (pivots[k], dist[k][n] FP64)."""
    rp, ci, ln = _i32(row_ptr), _i32(col_idx), _f64(length)
    piv = np.empty(k, dtype=np.int32)
    dist = np.empty((k, n), dtype=np.float64)
    st = _load().orc_select_pivots_w(n, _p(rp), _p(ci), _p(ln), int(k), int(first), _p(piv), _p(dist))
    if st != OK:
        raise OracleError(st, "select_pivots_w")
    return piv, dist


def regions_w(dist):
    """Rule R1 regions on real distances; returns (delta[n], region[n], size[k])."""
    dist = _f64(dist)
    k, n = dist.shape
    delta = np.empty(n, dtype=np.float64)
    region = np.empty(n, dtype=np.int32)
    size = np.empty(k, dtype=np.int32)
    st = _load().orc_regions_w(n, k, _p(dist), _p(delta), _p(region), _p(size))
    if st != OK:
        raise OracleError(st, "regions_w")
    return delta, region, size


def terms_w(row_ptr, col_idx, length, pivots, dist, delta, region):
    """Per-term adapted weights w[k][n] (0 where no term) and denominators."""
    rp, ci, ln, pv = _i32(row_ptr), _i32(col_idx), _f64(length), _i32(pivots)
    dist, delta, region = _f64(dist), _f64(delta), _i32(region)
    k, n = dist.shape
    w = np.empty((k, n), dtype=np.float64)
    den = np.empty(n, dtype=np.float64)
    st = _load().orc_terms_w(n, _p(rp), _p(ci), _p(ln), k, _p(pv), _p(dist), _p(delta), _p(region), _p(w),
                             _p(den))
    if st != OK:
        raise OracleError(st, "terms_w")
    return w, den


def majorize_w(row_ptr, col_idx, length, pivots, dist, w, den, x, iters: int) -> np.ndarray:
    rp, ci, ln, pv = _i32(row_ptr), _i32(col_idx), _f64(length), _i32(pivots)
    dist, w, den = _f64(dist), _f64(w), _f64(den)
    x = _f64(x).copy()
    k, n = dist.shape
    st = _load().orc_majorize_w(n, _p(rp), _p(ci), _p(ln), k, _p(pv), _p(dist), _p(w), _p(den), _p(x), int(iters))
    if st != OK:
        raise OracleError(st, "majorize_w")
    return x


def stress_w(row_ptr, col_idx, length, pivots, dist, w, x) -> float:
    rp, ci, ln, pv = _i32(row_ptr), _i32(col_idx), _f64(length), _i32(pivots)
    dist, w, x = _f64(dist), _f64(w), _f64(x)
    k, n = dist.shape
    return _load().orc_stress_w(n, _p(rp), _p(ci), _p(ln), k, _p(pv), _p(dist), _p(w), _p(x))


def pivotmds_w(dist):
    """PivotMDS on real distances; returns (x[n][2], V[k][2], lambda[2])."""
    dist = _f64(dist)
    k, n = dist.shape
    x = np.empty((n, 2), dtype=np.float64)
    V = np.empty((k, 2), dtype=np.float64)
    lam = np.empty(2, dtype=np.float64)
    st = _load().orc_pivotmds_w(n, k, _p(dist), _p(x), _p(V), _p(lam))
    if st != OK:
        raise OracleError(st, "pivotmds_w")
    return x, V, lam


def rescale_w(row_ptr, col_idx, length, x) -> np.ndarray:
    rp, ci, ln = _i32(row_ptr), _i32(col_idx), _f64(length)
    x = _f64(x).copy()
    st = _load().orc_rescale_w(x.shape[0], _p(rp), _p(ci), _p(ln), _p(x))
    if st != OK:
        raise OracleError(st, "rescale_w")
    return x


@dataclass
class WTerms:
    pivots: np.ndarray
    dist: np.ndarray
    delta: np.ndarray
    region: np.ndarray
    size: np.ndarray
    w: np.ndarray
    den: np.ndarray


def preprocess_w(n, row_ptr, col_idx, length, k: int, first: int = 0) -> WTerms:
    piv, dist = select_pivots_w(n, row_ptr, col_idx, length, k, first)
    delta, region, size = regions_w(dist)
    w, den = terms_w(row_ptr, col_idx, length, piv, dist, delta, region)
    return WTerms(piv, dist, delta, region, size, w, den)


def layout_w(n, row_ptr, col_idx, length, k: int, iters: int, first: int = 0):
    """Algorithm 1 with edge lengths (Jacobi order); returns (x, terms, x0)."""
    t = preprocess_w(n, row_ptr, col_idx, length, k, first)
    x0, _, _ = pivotmds_w(t.dist)
    x0 = rescale_w(row_ptr, col_idx, length, x0)
    x = majorize_w(row_ptr, col_idx, length, t.pivots, t.dist, t.w, t.den, x0, iters)
    return x, t, x0
