"""Thin ctypes binding of libssm (the HIP library).  Argument marshalling only:
every step runs in the library's kernels.  Device buffers are torch tensors
(used for device memory and streams only); the current torch stream is passed
to every call.

Raises RuntimeError at first use if libssm.so is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import threading
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssm.so")

OK, E_INVAL, E_RANGE, E_DISCONNECTED, E_NOMEM, E_DEVICE = range(6)
FP64, FP32 = 0, 1
STRESS_SPARSE, STRESS_FULL, STRESS_NORMALIZED = 0, 1, 2

_lock = threading.Lock()
_lib = None
_live = weakref.WeakSet()   # objects that own a library handle


def shutdown():
    """Frees every live handle (terms, pools) and the library's cached
    scratch, after the device work queued so far has finished.  Registered
    with atexit when the library is loaded, so that no HIP call is left for
    the interpreter's own teardown; the handles are unusable afterwards."""
    if _lib is None:
        return
    try:
        torch.cuda.synchronize()
    except Exception:
        pass
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass
    _lib.ssm_release_cache()


class SSMError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: status {status}: {msg}")
        self.status = status


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


EXPORTS = [
    "ssm_validate_csr", "ssm_select_pivots", "ssm_bfs_pivots", "ssm_regions", "ssm_kmeans_pivots", "ssm_build_terms",
    "ssm_terms_free", "ssm_terms_dims", "ssm_terms_export", "ssm_pivotmds_init",
    "ssm_pivotmds_eig", "ssm_pivotmds_gram", "ssm_majorize", "ssm_majorize_mixed", "ssm_stress", "ssm_last_error",
    "ssm_pool_create", "ssm_pool_destroy", "ssm_pool_usage", "ssm_pool_add", "ssm_pool_prepare", "ssm_pool_sweep",
    "ssm_pool_stress", "ssm_pool_layout", "ssm_pool_export", "ssm_pool_info", "ssm_pool_remove", "ssm_procrustes",
    "ssm_select_pivots_w", "ssm_sssp_pivots", "ssm_build_terms_w", "ssm_wterms_free", "ssm_wterms_export",
    "ssm_pivotmds_init_w", "ssm_majorize_w", "ssm_majorize_mixed_w", "ssm_stress_w", "ssm_release_cache",
    "ssm_set_variant", "ssm_pool_set_tol", "ssm_pool_stopped", "ssm_procrustes_noalloc",
]


def load(path: str | None = None):
    """Load libssm.so (once) and declare its signatures."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"libssm.so not built ({p}); run __graft_entry__.build()")
        lib = ctypes.CDLL(p)
        V, I, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        S = ctypes.c_int
        P = ctypes.POINTER(_CSR)
        sig = {
            "ssm_validate_csr": (S, [P, V]),
            "ssm_select_pivots": (S, [P, I, I, V, V, V]),
            "ssm_bfs_pivots": (S, [P, I, V, V, V, V, V]),
            "ssm_regions": (S, [I, I, V, V, V, V]),
            "ssm_kmeans_pivots": (S, [I, I, V, V, I, V, V, V, V]),
            "ssm_build_terms": (S, [P, I, V, V, V, V, ctypes.POINTER(V), V]),
            "ssm_terms_free": (None, [V]),
            "ssm_terms_dims": (S, [V, V, V, V]),
            "ssm_terms_export": (S, [V, V, V, V, V, V]),
            "ssm_pivotmds_init": (S, [P, V, I, V, V]),
            "ssm_pivotmds_eig": (S, [V, V, V, V]),
            "ssm_pivotmds_gram": (S, [V, V]),
            "ssm_majorize": (S, [P, V, I, V, I, D, V, V]),
            "ssm_majorize_mixed": (S, [P, V, V, V, I, I, V]),
            "ssm_stress": (S, [P, V, I, V, I, V, V]),
            "ssm_last_error": (ctypes.c_char_p, []),
            "ssm_pool_create": (S, [ctypes.c_int64, ctypes.POINTER(V)]),
            "ssm_pool_destroy": (None, [V]),
            "ssm_pool_usage": (S, [V, V, V]),
            "ssm_pool_add": (S, [V, I, I, V, V, I, I, I, V, V]),
            "ssm_pool_prepare": (S, [V, I, V, I, V]),
            "ssm_pool_sweep": (S, [V, I, V, I, V]),
            "ssm_pool_stress": (S, [V, I, V, V, V]),
            "ssm_pool_layout": (S, [V, I, V, V]),
            "ssm_pool_export": (S, [V, I, I, V, V]),
            "ssm_pool_info": (S, [V, I, V]),
            "ssm_pool_remove": (S, [V, I]),
            "ssm_procrustes": (S, [I, I, V, I, V, V, V]),
            "ssm_procrustes_noalloc": (S, [I, I, V, I, V, V, V]),
            "ssm_select_pivots_w": (S, [P, V, I, I, V, V, V]),
            "ssm_sssp_pivots": (S, [P, V, I, V, V, V]),
            "ssm_build_terms_w": (S, [P, V, I, V, V, ctypes.POINTER(V), V]),
            "ssm_wterms_free": (None, [V]),
            "ssm_wterms_export": (S, [V, V, V, V, V]),
            "ssm_pivotmds_init_w": (S, [P, V, V, I, V, V]),
            "ssm_majorize_w": (S, [P, V, V, I, V, I, V]),
            "ssm_majorize_mixed_w": (S, [P, V, V, V, V, I, I, V]),
            "ssm_stress_w": (S, [P, V, V, I, V, V, V]),
            "ssm_release_cache": (None, []),
            "ssm_set_variant": (S, [ctypes.c_char_p, I]),
            "ssm_pool_set_tol": (S, [V, I, D]),
            "ssm_pool_stopped": (S, [V, I, V, V, V]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        if path is None:
            _lib = lib
            atexit.register(shutdown)
        return lib


def set_variant(name: str | None, value: int = 0):
    """Forces a launch variant (ssm_set_variant); value 0 restores the
    library's choice, name None clears every override."""
    _check(load().ssm_set_variant(name.encode() if name is not None else None, int(value)), "ssm_set_variant")


class variants:
    """Context manager: `with ssm.variants(sweep_split=4): ...` forces the
    given launch variants and clears them on exit."""

    def __init__(self, **kw):
        self.kw = kw

    def __enter__(self):
        for name, value in self.kw.items():
            set_variant(name, int(value))
        return self

    def __exit__(self, *exc):
        for name in self.kw:
            set_variant(name, 0)
        return False


def _check(st: int, func: str):
    if st != OK:
        msg = load().ssm_last_error()
        raise SSMError(st, func, msg.decode() if msg else "")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class DeviceGraph:
    """A CSR graph resident in device memory (int32 row_ptr and col_idx)."""

    def __init__(self, n: int, row_ptr: torch.Tensor, col_idx: torch.Tensor):
        assert row_ptr.dtype == torch.int32 and col_idx.dtype == torch.int32
        self.n = int(n)
        self.row_ptr = row_ptr.contiguous()
        self.col_idx = col_idx.contiguous()
        self.nnz = int(self.col_idx.numel())
        self._c = _CSR(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr())

    @classmethod
    def from_csr(cls, g, device="cuda"):
        rp = torch.from_numpy(g.row_ptr).to(device)
        ci = torch.from_numpy(g.col_idx).to(device) if g.nnz else torch.zeros(1, dtype=torch.int32, device=device)
        return cls(g.n, rp, ci)

    @property
    def cref(self):
        return ctypes.byref(self._c)


class Terms:
    """Owner of an ssm_terms handle (freed with the object)."""

    def __init__(self, handle: int, graph: DeviceGraph, k: int):
        self.handle = ctypes.c_void_p(handle)
        self.graph = graph
        self.k = k
        _live.add(self)

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.ssm_terms_free(h)
        self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the atexit hook has already freed the handle (the
        # check is bound here: module globals may be gone by then)
        if getattr(self, "handle", None) is None or _finalizing():
            return
        self.close()

    def dims(self):
        k, dm, dx = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().ssm_terms_dims(self.handle, ctypes.byref(k), ctypes.byref(dm), ctypes.byref(dx)),
               "ssm_terms_dims")
        return k.value, dm.value, dx.value

    def export(self):
        import numpy as np
        k, dm, dx = self.dims()
        n = self.graph.n
        H = np.empty((k, dm + 1), dtype=np.int32)
        w64 = np.empty((k, dx + 1), dtype=np.float64)
        w32 = np.empty((k, dx + 1), dtype=np.float32)
        d64 = np.empty(n, dtype=np.float64)
        d32 = np.empty(n, dtype=np.float32)
        _check(load().ssm_terms_export(self.handle, _hptr(H), _hptr(w64), _hptr(w32), _hptr(d64), _hptr(d32)),
               "ssm_terms_export")
        return {"H": H, "wtab64": w64, "wtab32": w32, "den64": d64, "den32": d32,
                "delta_max": dm, "dmax": dx}


# ------------------------------------------------------------------- calls

def validate_csr(g: DeviceGraph):
    _check(load().ssm_validate_csr(g.cref, _stream()), "ssm_validate_csr")


def select_pivots(g: DeviceGraph, k: int, first: int = 0, with_dist: bool = False):
    piv = torch.empty(k, dtype=torch.int32, device="cuda")
    dist = torch.empty((k, g.n), dtype=torch.int32, device="cuda") if with_dist else None
    _check(load().ssm_select_pivots(g.cref, k, first, _ptr(piv), _ptr(dist), _stream()), "ssm_select_pivots")
    return (piv, dist) if with_dist else piv


def bfs_pivots(g: DeviceGraph, pivots: torch.Tensor):
    k = int(pivots.numel())
    dist = torch.empty((k, g.n), dtype=torch.int32, device="cuda")
    delta = torch.empty(g.n, dtype=torch.int32, device="cuda")
    region = torch.empty(g.n, dtype=torch.int32, device="cuda")
    _check(load().ssm_bfs_pivots(g.cref, k, _ptr(pivots), _ptr(dist), _ptr(delta), _ptr(region), _stream()),
           "ssm_bfs_pivots")
    return dist, delta, region


def regions(dist: torch.Tensor):
    k, n = dist.shape
    delta = torch.empty(n, dtype=torch.int32, device="cuda")
    region = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(load().ssm_regions(n, k, _ptr(dist), _ptr(delta), _ptr(region), _stream()), "ssm_regions")
    return delta, region


def kmeans_pivots(pivots: torch.Tensor, dist: torch.Tensor, max_iters: int = 50):
    """k-means sp refinement of max/min pivots; returns (new_pivots, assign, passes)."""
    k, n = dist.shape
    newp = torch.empty(k, dtype=torch.int32, device="cuda")
    assign = torch.empty(n, dtype=torch.int32, device="cuda")
    it = ctypes.c_int32()
    _check(load().ssm_kmeans_pivots(n, k, _ptr(pivots), _ptr(dist), int(max_iters), _ptr(newp), _ptr(assign),
                                    ctypes.byref(it), _stream()), "ssm_kmeans_pivots")
    return newp, assign, it.value


def build_terms(g: DeviceGraph, pivots, dist, delta, region) -> Terms:
    k = int(pivots.numel())
    h = ctypes.c_void_p()
    _check(load().ssm_build_terms(g.cref, k, _ptr(pivots), _ptr(dist), _ptr(delta), _ptr(region),
                                  ctypes.byref(h), _stream()), "ssm_build_terms")
    return Terms(h.value, g, k)


def _xtensor(n: int, prec: int):
    return torch.empty((n, 2), dtype=torch.float64 if prec == FP64 else torch.float32, device="cuda")


def _prec_of(x: torch.Tensor) -> int:
    if x.dtype == torch.float64:
        return FP64
    if x.dtype == torch.float32:
        return FP32
    raise ValueError("layout must be float64 or float32")


def pivotmds_init(g: DeviceGraph, terms: Terms, prec: int = FP64, out: torch.Tensor | None = None):
    x = out if out is not None else _xtensor(g.n, prec)
    _check(load().ssm_pivotmds_init(g.cref, terms.handle, _prec_of(x), _ptr(x), _stream()), "ssm_pivotmds_init")
    return x


def pivotmds_eig(terms: Terms):
    import numpy as np
    V = np.empty((terms.k, 2), dtype=np.float64)
    lam = np.empty(2, dtype=np.float64)
    it = ctypes.c_int32()
    _check(load().ssm_pivotmds_eig(terms.handle, _hptr(V), _hptr(lam), ctypes.byref(it)), "ssm_pivotmds_eig")
    return V, lam, it.value


def pivotmds_gram(terms: Terms):
    import numpy as np
    M = np.empty((terms.k, terms.k), dtype=np.float64)
    _check(load().ssm_pivotmds_gram(terms.handle, _hptr(M)), "ssm_pivotmds_gram")
    return M


def majorize(g: DeviceGraph, terms: Terms, x: torch.Tensor, iters: int, tol: float = 0.0,
             sync: bool = False):
    """Runs the sweeps in place on x; returns the sweep count if sync or tol > 0."""
    done = ctypes.c_int32(-1)
    want = sync or tol > 0
    _check(load().ssm_majorize(g.cref, terms.handle, _prec_of(x), _ptr(x), int(iters), float(tol),
                               ctypes.byref(done) if want else None, _stream()), "ssm_majorize")
    return done.value if want else None


def majorize_mixed(g: DeviceGraph, terms: Terms, x64: torch.Tensor, iters: int, warm: int = 1,
                   out: torch.Tensor | None = None) -> torch.Tensor:
    """`warm` FP64 sweeps on x64 (in place), then FP32 sweeps on the rounded
    layout; returns the FP32 layout."""
    if x64.dtype != torch.float64:
        raise ValueError("x64 must be float64")
    x32 = out if out is not None else torch.empty(x64.shape, dtype=torch.float32, device=x64.device)
    _check(load().ssm_majorize_mixed(g.cref, terms.handle, _ptr(x64), _ptr(x32), int(iters), int(warm),
                                     _stream()), "ssm_majorize_mixed")
    return x32


def stress(g: DeviceGraph, terms: Terms | None, x: torch.Tensor, kind: int = STRESS_SPARSE) -> float:
    out = ctypes.c_double()
    h = terms.handle if terms is not None else None
    _check(load().ssm_stress(g.cref, h, _prec_of(x), _ptr(x), int(kind), ctypes.byref(out), _stream()),
           "ssm_stress")
    return out.value


def procrustes(x: torch.Tensor, y: torch.Tensor) -> float:
    """Procrustes statistic of layout x against reference y (0 = perfect match)."""
    if x.shape != y.shape or x.dim() != 2 or x.shape[1] != 2:
        raise ValueError("expected two n x 2 layouts")
    out = ctypes.c_double()
    _check(load().ssm_procrustes(int(x.shape[0]), _prec_of(x), _ptr(x), _prec_of(y), _ptr(y), ctypes.byref(out),
                                 _stream()), "ssm_procrustes")
    return out.value


def normalized_stress(g: DeviceGraph, x: torch.Tensor) -> float:
    """Full stress s(x) (Eq. 1) divided by the number of node pairs."""
    return stress(g, None, x, STRESS_NORMALIZED)


def full_stress_layout(g: DeviceGraph, iters: int, first: int = 0, start_k: int | None = None):
    """The full-stress reference of Section 4.1: the sparse model with k = n
    (every node a pivot, so every pair carries weight 1/d^2) swept `iters`
    times in FP64.  Start: PivotMDS on the first start_k max/min pivots
    (default min(n, 1024); a prefix of the k = n selection).  Returns (x, terms)."""
    n = g.n
    k0 = min(n, 1024) if start_k is None else start_k
    piv = select_pivots(g, n, first)
    dist, delta, region = bfs_pivots(g, piv)
    terms = build_terms(g, piv, dist, delta, region)
    if k0 == n:
        x = pivotmds_init(g, terms, FP64)
    else:
        p0 = piv[:k0].contiguous()
        d0, de0, r0 = bfs_pivots(g, p0)
        t0 = build_terms(g, p0, d0, de0, r0)
        x = pivotmds_init(g, t0, FP64)
        del t0, d0
    majorize(g, terms, x, iters)
    return x, terms


def layout(g: DeviceGraph, k: int, iters: int, prec: int = FP64, first: int = 0, warm: int = 1,
           sampling: str = "maxmin"):
    """Algorithm 1 end to end on the device; returns (x, terms, pivots, dist, delta, region).
    FP32 runs PivotMDS and the first `warm` sweeps in FP64, the rest in FP32.
    sampling "kmeans" refines the max/min pivots by k-means sp before the BFS."""
    if sampling not in ("maxmin", "kmeans"):
        raise ValueError(f"unknown pivot sampling {sampling!r}")
    if sampling == "kmeans":
        piv0, dist0 = select_pivots(g, k, first, with_dist=True)
        piv, _, _ = kmeans_pivots(piv0, dist0)
        del dist0
    else:
        piv = select_pivots(g, k, first)
    dist, delta, region = bfs_pivots(g, piv)
    terms = build_terms(g, piv, dist, delta, region)
    x = pivotmds_init(g, terms, FP64)
    if prec == FP32:
        x = majorize_mixed(g, terms, x, iters, warm)
    else:
        majorize(g, terms, x, iters)
    return x, terms, piv, dist, delta, region


# ------------------------------------------------------------------ layout pool

POOL_FREE, POOL_ADDED, POOL_READY, POOL_FAILED = range(4)
POOL_PIVOTS, POOL_DIST, POOL_DELTA, POOL_REGION, POOL_H, POOL_WTAB64, POOL_DEN64, POOL_X32, POOL_X64 = range(9)


class Pool:
    """Many small graphs laid out together in one device arena (the ssm_pool_*
    calls): add graphs, prepare them in batches, sweep any set of ready slots
    per call, read stress and layouts, remove finished slots."""

    def __init__(self, capacity_bytes: int):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.ssm_pool_create(int(capacity_bytes), ctypes.byref(h)), "ssm_pool_create")
        self.handle = h.value
        _live.add(self)

    def close(self):
        if getattr(self, "handle", None):
            self._lib.ssm_pool_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def usage(self):
        used, cap = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.ssm_pool_usage(self.handle, ctypes.byref(used), ctypes.byref(cap)), "ssm_pool_usage")
        return used.value, cap.value

    def add(self, g, k: int, first: int = 0, sweeps: int = 200):
        """Admit CSR graph g (host arrays); returns the slot, or None when the
        arena has no room (status E_NOMEM)."""
        import numpy as np
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
        slot = ctypes.c_int32()
        st = self._lib.ssm_pool_add(self.handle, int(g.n), int(ci.size), _hptr(rp), _hptr(ci), int(k), int(first),
                                    int(sweeps), ctypes.byref(slot), _stream())
        if st == E_NOMEM:
            return None
        _check(st, "ssm_pool_add")
        return slot.value

    @staticmethod
    def _slots(slots):
        import numpy as np
        return np.ascontiguousarray(slots, dtype=np.int32)

    def prepare(self, slots, warm: int = 1):
        a = self._slots(slots)
        _check(self._lib.ssm_pool_prepare(self.handle, a.size, _hptr(a), int(warm), _stream()), "ssm_pool_prepare")

    def sweep(self, slots, iters: int):
        a = self._slots(slots)
        _check(self._lib.ssm_pool_sweep(self.handle, a.size, _hptr(a), int(iters), _stream()), "ssm_pool_sweep")

    def stress(self, slots):
        import numpy as np
        a = self._slots(slots)
        out = np.empty(a.size, dtype=np.float64)
        _check(self._lib.ssm_pool_stress(self.handle, a.size, _hptr(a), _hptr(out), _stream()), "ssm_pool_stress")
        return out

    def layout(self, slot: int, n: int) -> torch.Tensor:
        x = torch.empty(n, 2, dtype=torch.float32, device="cuda")
        _check(self._lib.ssm_pool_layout(self.handle, int(slot), _ptr(x), _stream()), "ssm_pool_layout")
        return x

    def info(self, slot: int) -> dict:
        import numpy as np
        v = np.empty(8, dtype=np.int32)
        _check(self._lib.ssm_pool_info(self.handle, int(slot), _hptr(v)), "ssm_pool_info")
        keys = ["state", "fail", "n", "k", "done", "sweeps", "dmax", "delta_max"]
        return dict(zip(keys, (int(q) for q in v)))

    def export(self, slot: int, what: int):
        import numpy as np
        inf = self.info(slot)
        n, k, W, L = inf["n"], inf["k"], inf["dmax"] + 1, inf["delta_max"] + 1
        shape, dt = {
            POOL_PIVOTS: ((k,), np.int32), POOL_DIST: ((k, n), np.int32), POOL_DELTA: ((n,), np.int32),
            POOL_REGION: ((n,), np.int32), POOL_H: ((k, L), np.int32), POOL_WTAB64: ((k, W), np.float64),
            POOL_DEN64: ((n,), np.float64), POOL_X32: ((n, 2), np.float32), POOL_X64: ((n, 2), np.float64),
        }[what]
        out = np.empty(shape, dtype=dt)
        _check(self._lib.ssm_pool_export(self.handle, int(slot), int(what), _hptr(out), _stream()), "ssm_pool_export")
        return out

    def remove(self, slot: int):
        _check(self._lib.ssm_pool_remove(self.handle, int(slot)), "ssm_pool_remove")

    def set_tol(self, slot: int, tol: float):
        """Stop test of the slot's FP32 sweeps (0: its fixed sweep count)."""
        _check(self._lib.ssm_pool_set_tol(self.handle, int(slot), float(tol)), "ssm_pool_set_tol")

    def stopped(self, slots):
        """Per slot: the sweeps its layout took if its stop test fired, else -1."""
        import numpy as np
        a = self._slots(slots)
        out = np.empty(a.size, dtype=np.int32)
        _check(self._lib.ssm_pool_stopped(self.handle, a.size, _hptr(a), _hptr(out), _stream()), "ssm_pool_stopped")
        return out


# ------------------------------------------------------- graphs with edge lengths

class WTerms:
    """Handle of ssm_build_terms_w (regions, per-term weights, denominators)."""

    def __init__(self, handle: int, graph: DeviceGraph, k: int):
        self.handle, self.graph, self.k = handle, graph, k
        _live.add(self)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ssm_wterms_free(self.handle)
        self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def export(self):
        import numpy as np
        n, k = self.graph.n, self.k
        delta = np.empty(n, dtype=np.float64)
        region = np.empty(n, dtype=np.int32)
        w = np.empty((k, n), dtype=np.float64)
        den = np.empty(n, dtype=np.float64)
        _check(load().ssm_wterms_export(self.handle, _hptr(delta), _hptr(region), _hptr(w), _hptr(den)),
               "ssm_wterms_export")
        return {"delta": delta, "region": region, "w": w, "den": den}


def select_pivots_w(g: DeviceGraph, length: torch.Tensor, k: int, first: int = 0, with_dist: bool = False):
    piv = torch.empty(k, dtype=torch.int32, device="cuda")
    dist = torch.empty(k, g.n, dtype=torch.float64, device="cuda") if with_dist else None
    _check(load().ssm_select_pivots_w(g.cref, _ptr(length), k, first, _ptr(piv), _ptr(dist), _stream()),
           "ssm_select_pivots_w")
    return (piv, dist) if with_dist else piv


def sssp_pivots(g: DeviceGraph, length: torch.Tensor, pivots: torch.Tensor) -> torch.Tensor:
    k = pivots.numel()
    dist = torch.empty(k, g.n, dtype=torch.float64, device="cuda")
    _check(load().ssm_sssp_pivots(g.cref, _ptr(length), k, _ptr(pivots), _ptr(dist), _stream()), "ssm_sssp_pivots")
    return dist


def build_terms_w(g: DeviceGraph, length: torch.Tensor, pivots: torch.Tensor, dist: torch.Tensor) -> WTerms:
    k = pivots.numel()
    h = ctypes.c_void_p()
    _check(load().ssm_build_terms_w(g.cref, _ptr(length), k, _ptr(pivots), _ptr(dist), ctypes.byref(h), _stream()),
           "ssm_build_terms_w")
    return WTerms(h.value, g, k)


def pivotmds_init_w(g: DeviceGraph, length: torch.Tensor, terms: WTerms, prec: int = FP64) -> torch.Tensor:
    x = _xtensor(g.n, prec)
    _check(load().ssm_pivotmds_init_w(g.cref, _ptr(length), terms.handle, prec, _ptr(x), _stream()),
           "ssm_pivotmds_init_w")
    return x


def majorize_w(g: DeviceGraph, length: torch.Tensor, terms: WTerms, x: torch.Tensor, iters: int):
    _check(load().ssm_majorize_w(g.cref, _ptr(length), terms.handle, _prec_of(x), _ptr(x), int(iters), _stream()),
           "ssm_majorize_w")
    return x


def majorize_mixed_w(g: DeviceGraph, length: torch.Tensor, terms: WTerms, x64: torch.Tensor, iters: int,
                     warm: int = 1) -> torch.Tensor:
    x32 = _xtensor(g.n, FP32)
    _check(load().ssm_majorize_mixed_w(g.cref, _ptr(length), terms.handle, _ptr(x64), _ptr(x32), int(iters),
                                       int(warm), _stream()), "ssm_majorize_mixed_w")
    return x32


def stress_w(g: DeviceGraph, length: torch.Tensor, terms: WTerms, x: torch.Tensor) -> float:
    out = ctypes.c_double()
    _check(load().ssm_stress_w(g.cref, _ptr(length), terms.handle, _prec_of(x), _ptr(x), ctypes.byref(out),
                               _stream()), "ssm_stress_w")
    return out.value


def layout_w(g: DeviceGraph, length: torch.Tensor, k: int, iters: int, prec: int = FP64, first: int = 0,
             warm: int = 1):
    """Algorithm 1 with edge lengths on the device; returns (x, terms, pivots, dist)."""
    piv = select_pivots_w(g, length, k, first)
    dist = sssp_pivots(g, length, piv)
    terms = build_terms_w(g, length, piv, dist)
    x = pivotmds_init_w(g, length, terms, FP64)
    if prec == FP32:
        x = majorize_mixed_w(g, length, terms, x, iters, warm)
    else:
        majorize_w(g, length, terms, x, iters)
    return x, terms, piv, dist
