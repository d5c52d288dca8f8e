"""The allocation-free Procrustes entry point (ssm_procrustes_noalloc, its
partial sums in the library's static device array) gives what
ssm_procrustes gives, bit for bit, on two calls in a row (the second with a
smaller input, so stale partials of the first would show) and after it."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1608_08909_amd import ssm


def _call(fn, x, y):
    out = ctypes.c_double()
    st = fn(int(x.shape[0]), ssm._prec_of(x), ssm._ptr(x), ssm._prec_of(y), ssm._ptr(y), ctypes.byref(out),
            ssm._stream())
    return st, out.value


def test_noalloc_procrustes_matches_allocating_call():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = ssm.load()
    rng = np.random.default_rng(7)
    # two calls in a row, the second smaller (fewer blocks: the first call's
    # later partials stay in the array), then mixed precisions
    for n, dx, dy in ((300000, torch.float64, torch.float64), (1000, torch.float64, torch.float64),
                      (70001, torch.float32, torch.float64), (2, torch.float32, torch.float32)):
        y = rng.normal(size=(n, 2)) * 50
        th = rng.uniform(-3, 3)
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        x = 1.7 * y @ R.T + rng.normal(size=2) * 9 + rng.normal(size=(n, 2))
        xt = torch.from_numpy(x).to(dx).cuda()
        yt = torch.from_numpy(y).to(dy).cuda()
        print("case n", n, dx, dy, flush=True)
        st0, v0 = _call(lib.ssm_procrustes_noalloc, xt, yt)
        st1, v1 = _call(lib.ssm_procrustes, xt, yt)
        assert st0 == ssm.OK and st1 == ssm.OK
        assert v0 == v1
        assert 0.0 <= v0 <= 1.0
    # argument errors before any device work
    d = ctypes.c_void_p(0x3000)
    out = ctypes.c_double()
    assert lib.ssm_procrustes_noalloc(1, 0, d, 0, d, ctypes.byref(out), None) == ssm.E_INVAL
    assert lib.ssm_procrustes_noalloc((1 << 30) + 1, 0, d, 0, d, ctypes.byref(out), None) == ssm.E_RANGE
    assert lib.ssm_procrustes_noalloc(10, 0, None, 0, d, ctypes.byref(out), None) == ssm.E_INVAL
    # a layout with no spread is refused, as by the allocating call
    z = torch.zeros(50, 2, dtype=torch.float64, device="cuda")
    w = torch.from_numpy(rng.normal(size=(50, 2))).cuda()
    assert _call(lib.ssm_procrustes_noalloc, z, w)[0] == ssm.E_INVAL
