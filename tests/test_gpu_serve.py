"""Serving loop on the GPU: continuous batching of TGV and Poisson requests of
mixed size, order and Reynolds number; results identical alone and in the mix;
HBM-budget admission (queueing, rejection) never fails a request."""
import numpy as np
import pytest

from paper_2608_24348_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_24348_amd import serve as s
    yield s
    # the servers' workspace arena outlives them; give it back to later tests
    s.release_arena()


def _stream(n=12, qps=200.0, seed=7):
    return inputs.request_stream(n_requests=n, qps=qps, seed=seed, nmin=2, nmax=5, orders=(3, 5), tgv_steps=4)


def _same(a, b):
    if a.kind == "tgv":
        return np.array_equal(a.result["u"], b.result["u"]) and np.array_equal(a.result["p"], b.result["p"])
    return np.array_equal(a.result["p"], b.result["p"]) and a.result["stats"]["iters"] == b.result["stats"]["iters"]


def test_stream_completes_and_mix_equals_alone(serve):
    specs = _stream()
    srv = serve.Server(max_batch=8, gmres_chunk=10, keep_fields=True, streams=4, graph=True)
    done, makespan = srv.run(specs)
    assert len(done) == len(specs) and all(r.status == "ok" for r in done)
    summ = serve.summarize(done, makespan)
    assert summ["p99_s"] >= summ["p50_s"] > 0 and summ["gdof_per_s"] > 0
    assert srv.used == 0
    kinds = {r.kind for r in done}
    assert kinds == {"tgv", "poisson"}
    # every request again, alone (arrival 0, batch of one), on one stream with
    # host-driven steps: the mix ran batched, on up to four streams from
    # concurrent host threads, with its steps replayed as graphs
    for r in done:
        spec = dict(r.spec, arrival=0.0)
        alone, _ = serve.Server(max_batch=1, gmres_chunk=10, keep_fields=True, streams=1, graph=False).run([spec])
        assert alone[0].status == "ok"
        assert _same(alone[0], r), r.spec


def test_admission_queues_under_small_budget_and_rejects_oversize(serve):
    specs = _stream(n=6, seed=11)
    probe = serve.Server()
    sizes = []
    for s in specs:
        r = serve.Request(s, probe.hsmg)
        probe._setup(r)
        sizes.append(r.bytes)
        r.ctx.close()
    # room for the largest request only: requests run (almost) one at a time
    srv = serve.Server(budget_bytes=max(sizes), max_batch=8, gmres_chunk=10)
    done, _ = srv.run(specs)
    assert all(r.status == "ok" for r in done) and srv.used == 0
    # a budget below every request rejects all of them without deadlock
    srv = serve.Server(budget_bytes=min(sizes) - 1, max_batch=8)
    done, _ = srv.run(specs)
    assert all(r.status == "rejected" for r in done)
