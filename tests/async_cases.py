"""Parity cases run with the library's per-launch synchronisation off (RPF_SYNC_CHECK unset),
the way the benchmark and a serving process run it: every launch of a call is queued on the
stream at once, workspace blocks of the library's cache are reused across streams behind
events, and the serving slots' batches run side by side on the device.

Run as a child process by tests/test_gpu_async.py (the flag is read once per process, and
the test suite's own process sets it).  Prints one line per step; exits non-zero on a
mismatch."""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
from paper_1812_11689_amd import rpf  # noqa: E402
from paper_1812_11689_amd import workloads as W  # noqa: E402
from tests.helpers import problem  # noqa: E402


def say(msg):
    print(msg, flush=True)


def compare(gi, gd, ri, rd, what):
    np.testing.assert_array_equal(gi, ri, err_msg=what)
    fin = np.isfinite(rd)
    assert np.array_equal(np.isfinite(gd), fin), what
    np.testing.assert_allclose(gd[fin], rd[fin], rtol=1e-5, atol=0, err_msg=what)


def all_points():
    # several forests in flight on two streams at once: the cache hands workspace blocks
    # from one stream's freed call to the other's next call behind events
    cases = [(20_000, 128, 8, 256, 20, "fp32", "aniso"), (7800, 128, 8, 256, 20, "bf16", "aniso"),
             (12_000, 16, 12, 200, 100, "fp32", "mixture"), (8000, 8, 40, 200, 40, "bf16", "mixture")]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for j, (n, d, T, n0, K, prec, kind) in enumerate(cases):
        say(f"[async all_knn] n={n} d={d} T={T} n0={n0} K={K} {prec}")
        x, R = problem(n, d, T, n0, seed=900 + j, kind=kind)
        s = streams[j % 2]
        with torch.cuda.stream(s):
            X = torch.from_numpy(x).cuda()
            Rd = torch.from_numpy(np.ascontiguousarray(R[:T])).cuda()
            f = rpf.build(X, T, n0, Rd, dist_prec=prec, stream=s)
            gi, gd = f.all_knn(K, stream=s)
            gi2, gd2 = f.all_knn(K, stream=s)  # a second call on the warm cache
        outs.append((x, R, T, n0, K, f, gi, gd, gi2, gd2, s))
    torch.cuda.synchronize()
    for x, R, T, n0, K, f, gi, gd, gi2, gd2, s in outs:
        ref = oracle.build_forest(x, R, T, n0)
        ri, rd = oracle.all_knn(ref, K)
        compare(gi.cpu().numpy(), gd.cpu().numpy(), ri, rd, f"all_knn n={x.shape[0]}")
        assert torch.equal(gi, gi2) and torch.equal(gd, gd2)
        f.knn_stats(stream=s)
        f.free()
    say("[async all_knn] ok")


def serving():
    n, d, T, n0 = 30_000, 48, 6, 64
    say(f"[async serving] n={n} d={d} T={T} n0={n0} fp16 slots=4")
    x, R = problem(n, d, T, n0, seed=951, clusters=20)
    f = rpf.build(torch.from_numpy(x).cuda(), T, n0, torch.from_numpy(np.ascontiguousarray(R[:T])).cuda(),
                  dist_prec="fp16")
    _, sizes, ks = W.serving_requests(952, 64, 1000.0, b_median=200, b_sigma=1.0, b_max=2000)
    qs = [torch.from_numpy(W.mixture_queries(952 * 7 + i, x, int(m), 20, mean_seed=951)).cuda()
          for i, m in enumerate(sizes)]
    ks = [int(k) for k in ks]
    torch.cuda.synchronize()
    srv = rpf.Server(f, slots=4, max_batch_rows=2048)
    tickets = [srv.submit(q, k) for q, k in zip(qs, ks)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    spans = srv.batch_log()
    say(f"    stats {st}")
    assert st["failed_requests"] == 0 and st["bad_index_rows"] == 0
    assert st["requests"] == len(qs)
    # batches of different slots in flight on the device at the same time
    over = 0
    for i, a in enumerate(spans):
        for b in spans[i + 1:]:
            if a["slot"] != b["slot"] and a["start_ms"] < b["end_ms"] and b["start_ms"] < a["end_ms"]:
                over += 1
    say(f"    {len(spans)} batches, {over} pairs on different slots overlap on the device")
    assert over > 0, "no two batches of different slots were in flight together"
    srv.close()
    for (gi, gd, _), q, k in zip(res, qs, ks):
        ai, ad = f.query(q, k)
        torch.cuda.synchronize()
        assert torch.equal(gi, ai) and torch.equal(gd, ad)
    ref = oracle.build_forest(x, R, T, n0)
    for j in (0, len(qs) // 2, len(qs) - 1):
        ri, rd = oracle.query_knn(ref, qs[j].cpu().numpy(), ks[j])
        compare(res[j][0].cpu().numpy(), res[j][1].cpu().numpy(), ri, rd, f"request {j}")
    f.free()
    say("[async serving] ok")


if __name__ == "__main__":
    assert os.environ.get("RPF_SYNC_CHECK", "0") != "1", "run with the per-launch synchronisation off"
    all_points()
    serving()
    say("async cases ok")
