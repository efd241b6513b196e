"""GPU tests of the serving loop (continuous batching over a resident forest): every
request's result in a mix of concurrent requests of uneven sizes and K equals the result
of the same request run alone, and equals the oracle's."""

import numpy as np
import pytest
import torch

import oracle
from paper_1812_11689_amd import workloads as W
from tests.helpers import problem

pytestmark = pytest.mark.gpu


def _forest(x, R, T, n0, prec):
    from paper_1812_11689_amd import rpf
    return rpf.build(torch.from_numpy(x).cuda(), T, n0, torch.from_numpy(np.ascontiguousarray(R[:T])).cuda(),
                     dist_prec=prec)


def _requests(seed, x, count, n_clusters, m_max):
    _, sizes, ks = W.serving_requests(seed, count, 1000.0, b_median=48, b_sigma=1.2, b_max=m_max)
    qs = [torch.from_numpy(W.mixture_queries(seed * 7 + i, x, int(m), n_clusters, mean_seed=seed)).cuda()
          for i, m in enumerate(sizes)]
    return qs, [int(k) for k in ks]


@pytest.mark.parametrize("prec,slots", [("fp16", 3), ("fp32", 2), ("bf16", 4)])
def test_mix_equals_alone(prec, slots):
    from paper_1812_11689_amd import rpf
    n, d, T, n0 = 30_000, 48, 6, 64
    print(f"[serving] mix vs alone n={n} d={d} T={T} n0={n0} {prec} slots={slots}", flush=True)
    x, R = problem(n, d, T, n0, seed=501, clusters=20)
    f = _forest(x, R, T, n0, prec)
    qs, ks = _requests(502, x, 48, 20, 700)
    srv = rpf.Server(f, slots=slots, max_batch_rows=1024)
    tickets = [srv.submit(q, k) for q, k in zip(qs, ks)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    print(f"    stats {st}", flush=True)
    assert st["failed_requests"] == 0 and st["bad_index_rows"] == 0
    assert st["requests"] == len(qs)
    assert st["rows"] == sum(q.shape[0] for q in qs)
    assert st["batches"] < len(qs), "no request was batched with another"
    assert st["p99_s"] >= st["p50_s"] > 0
    for (gi, gd, lat), q, k in zip(res, qs, ks):
        ai, ad = f.query(q, k)
        torch.cuda.synchronize()
        assert torch.equal(gi, ai) and torch.equal(gd, ad)
        assert lat > 0
    # a few requests against the oracle as well
    ref = oracle.build_forest(x, R, T, n0)
    for j in (0, 1, len(qs) - 1):
        ri, rd = oracle.query_knn(ref, qs[j].cpu().numpy(), ks[j])
        np.testing.assert_array_equal(res[j][0].cpu().numpy(), ri)
        np.testing.assert_allclose(res[j][1].cpu().numpy(), rd, rtol=1e-5)
    srv.close()
    f.free()


def test_memory_budget_serialises_batches_and_poll():
    from paper_1812_11689_amd import rpf
    n, d, T, n0 = 8000, 16, 4, 40
    print(f"[serving] budget n={n} d={d} T={T} n0={n0}", flush=True)
    x, R = problem(n, d, T, n0, seed=511)
    f = _forest(x, R, T, n0, "fp32")
    qs, ks = _requests(512, x, 20, 5, 300)
    srv = rpf.Server(f, slots=4, max_batch_rows=64, mem_budget_bytes=1)  # one batch at a time
    tickets = [srv.submit(q, k) for q, k in zip(qs, ks)]
    out = {}
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
    for t, q, k in zip(tickets, qs, ks):
        ai, ad = f.query(q, k)
        torch.cuda.synchronize()
        assert torch.equal(out[t][0], ai) and torch.equal(out[t][1], ad)
    st = srv.stats()
    assert st["requests"] == len(qs) and st["failed_requests"] == 0 and st["bad_index_rows"] == 0
    # one batch at a time: no two device spans intersect
    spans = sorted((b["start_ms"], b["end_ms"]) for b in srv.batch_log())
    assert len(spans) == st["batches"] and all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
    srv.close()
    f.free()


def test_destroy_serves_waiting_requests():
    from paper_1812_11689_amd import rpf
    x, R = problem(5000, 12, 3, 30, seed=521)
    print("[serving] destroy drains", flush=True)
    f = _forest(x, R, 3, 30, "fp32")
    q = torch.from_numpy(W.mixture_queries(523, x, 200, 5, mean_seed=521)).cuda()
    srv = rpf.Server(f, slots=1)
    outs = [(torch.full((200, 5), -7, dtype=torch.int32, device="cuda"),
             torch.zeros((200, 5), dtype=torch.float32, device="cuda")) for _ in range(6)]
    for o in outs:
        srv.submit(q, 5, out=o)
    srv.close()  # serves all six before stopping
    torch.cuda.synchronize()
    ai, ad = f.query(q, 5)
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o[0], ai) and torch.equal(o[1], ad)
    f.free()
