"""The serving loop (continuous batching over the layout pool): every request
of a mixed stream completes, and its result is the one the same graph gets
alone (bit for bit: the pool's per-graph arithmetic does not depend on which
graphs share a launch or when the graph was admitted)."""
import numpy as np
import pytest

from paper_1608_08909_amd import graphs as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1608_08909_amd import serve, ssm


def test_serve_mixed_stream_matches_alone():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    specs = G.serving_requests(24, 11)
    rng = np.random.Generator(np.random.PCG64(5))
    graphs = []
    for sp in specs:  # small members of the three families
        if sp["family"] == "grid":
            sp = dict(sp, a=10 + sp["a"] % 30, b=10 + sp["b"] % 30)
        else:
            sp = dict(sp, n=200 + sp["n"] % 1800)
        graphs.append(G.make_request_graph(sp))
    arrivals = serve.poisson_arrivals(len(graphs), 400.0, 3)
    reqs = [serve.Request(i, g, min(100, g.n // 10), float(a), sweeps=int(rng.integers(20, 120)))
            for i, (g, a) in enumerate(zip(graphs, arrivals))]
    cap = 24 << 20  # room for a few graphs at a time: admission waits for retirements
    rep = serve.serve(reqs, cap, quantum=9, keep_layouts=True)
    print("rounds", rep.rounds, "prepares", rep.prepares, "peak active", rep.peak_active, "peak bytes",
          rep.peak_bytes, flush=True)
    assert all(r.status == "done" for r in reqs), [r.status for r in reqs]
    assert rep.peak_bytes <= cap
    assert rep.peak_active < len(reqs)  # the budget really held requests back
    for r in reqs:
        alone = ssm.Pool(1 << 28)
        s = alone.add(r.graph, r.k, 0, r.sweeps)
        alone.prepare([s], 1)
        alone.sweep([s], r.sweeps)
        assert alone.stress([s])[0] == r.stress
        assert torch.equal(alone.layout(s, r.graph.n), r.layout)
        alone.close()
    lat = rep.latencies_ms()
    assert (lat > 0).all()


def test_serve_stream_with_stop_test_matches_alone():
    """Requests with Algorithm 1's stop test: each retires after the sweep on
    which its test fired, with the layout and sweep count the same graph
    gets alone."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    specs = G.serving_requests(16, 23)
    graphs = []
    for sp in specs:
        if sp["family"] == "grid":
            sp = dict(sp, a=10 + sp["a"] % 30, b=10 + sp["b"] % 30)
        else:
            sp = dict(sp, n=200 + sp["n"] % 1800)
        graphs.append(G.make_request_graph(sp))
    arrivals = serve.poisson_arrivals(len(graphs), 400.0, 4)
    reqs = [serve.Request(i, g, min(100, g.n // 10), float(a), sweeps=400, tol=1e-4)
            for i, (g, a) in enumerate(zip(graphs, arrivals))]
    rep = serve.serve(reqs, 24 << 20, quantum=9, keep_layouts=True)
    assert all(r.status == "done" for r in reqs), [r.status for r in reqs]
    assert any(r.sweeps_run < r.sweeps for r in reqs)
    for r in reqs:
        alone = ssm.Pool(1 << 28)
        s = alone.add(r.graph, r.k, 0, r.sweeps)
        alone.set_tol(s, r.tol)
        alone.prepare([s], 1)
        alone.sweep([s], r.sweeps)
        got = alone.stopped([s])[0]
        assert (got if got >= 0 else r.sweeps) == r.sweeps_run
        assert alone.stress([s])[0] == r.stress
        assert torch.equal(alone.layout(s, r.graph.n), r.layout)
        alone.close()
