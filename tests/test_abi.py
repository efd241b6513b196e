"""The C ABI library: it loads, exports every entry point declared in include/rpf.h, and
rejects invalid arguments before touching the device.  CPU only (no GPU calls)."""

import ctypes
import os
import re

import pytest

import oracle
from paper_1812_11689_amd import rpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rpf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rpf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = rpf.load()
    names = _declared()
    assert "rpf_build" in names and "rpf_all_knn" in names and "rpf_query" in names
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(rpf.EXPORTS) <= set(names)


@pytest.mark.parametrize("n,n0", [(1, 1), (10, 1), (10_000, 50), (1_000_000, 256), (4_000_000, 256),
                                  (1_000_000, 512), (7, 7), (8, 7), (2**31 - 1, 1000)])
def test_depth_matches_oracle(n, n0):
    assert rpf.depth(n, n0) == oracle.depth(n, n0)


def test_invalid_arguments_rejected_without_device():
    lib = rpf.load()
    p = rpf.Params(n_trees=4, leaf_size=10, n_try=1, split_rule=0, dist_prec=0, build_flags=0,
                   directions_dev=None, mem_budget_bytes=0)
    h = ctypes.c_void_p(1234)
    fake = ctypes.c_void_p(0x1000)
    assert lib.rpf_build(None, 100, 4, ctypes.byref(p), None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert h.value is None  # *out cleared on error
    assert b"NULL" in lib.rpf_last_error()
    assert lib.rpf_build(fake, 0, 4, ctypes.byref(p), None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert lib.rpf_build(fake, 100, 0, ctypes.byref(p), None, ctypes.byref(h)) == rpf.RPF_EINVAL
    for rule in (0, 1):
        for field, bad in [("n_trees", 0), ("leaf_size", 0), ("n_try", 0), ("split_rule", 2), ("dist_prec", 7),
                           ("build_flags", 2)]:
            q = rpf.Params(n_trees=4, leaf_size=10, n_try=1, split_rule=rule, dist_prec=0, build_flags=0,
                           directions_dev=0x2000, mem_budget_bytes=0)
            setattr(q, field, bad)
            assert lib.rpf_build(fake, 100, 4, ctypes.byref(q), None, ctypes.byref(h)) == rpf.RPF_EINVAL, field
    # the uniform rule grows one data set per forest: no batches
    q = rpf.Params(n_trees=4, leaf_size=10, n_try=1, split_rule=1, dist_prec=0, build_flags=0,
                   directions_dev=None, mem_budget_bytes=0, seed=5)
    sizes = (ctypes.c_int64 * 2)(50, 50)
    assert lib.rpf_build_batched(fake, sizes, 2, 4, ctypes.byref(q), None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert b"uniform" in lib.rpf_last_error()
    # a uniform forest over budget is refused before any device work
    q.mem_budget_bytes = 1000
    assert lib.rpf_build(fake, 100, 4, ctypes.byref(q), None, ctypes.byref(h)) == rpf.RPF_ENOMEM
    cnt64 = ctypes.c_int64(0)
    assert lib.rpf_tree_nodes(None, 0, None, 0, ctypes.byref(cnt64)) == rpf.RPF_EINVAL
    # a tree with splits needs directions
    assert lib.rpf_build(fake, 100, 4, ctypes.byref(p), None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert b"directions" in lib.rpf_last_error()
    # budget below the plan
    q = rpf.Params(n_trees=4, leaf_size=10, n_try=1, split_rule=0, dist_prec=0, build_flags=0,
                   directions_dev=0x2000, mem_budget_bytes=1000)
    assert lib.rpf_build(fake, 100, 4, ctypes.byref(q), None, ctypes.byref(h)) == rpf.RPF_ENOMEM
    assert lib.rpf_free(None) == rpf.RPF_OK
    assert lib.rpf_all_knn(None, 5, 1, fake, fake, None) == rpf.RPF_EINVAL
    assert lib.rpf_query(None, fake, 10, 5, fake, fake, None) == rpf.RPF_EINVAL
    assert lib.rpf_route(None, fake, 10, fake, None) == rpf.RPF_EINVAL
    assert lib.rpf_tree_dump(None, 0, None, None, None, None, None, None) == rpf.RPF_EINVAL
    assert lib.rpf_forest_info(None, None) == rpf.RPF_EINVAL
    cnt = ctypes.c_int32(-1)
    assert lib.rpf_profile_read(None, 0, ctypes.byref(cnt)) == rpf.RPF_OK and cnt.value >= 0


def test_server_and_workspace_arguments_rejected_without_device():
    lib = rpf.load()
    fake = ctypes.c_void_p(0x1000)
    cfg = rpf.ServerConfig(slots=2, reserved=0, max_batch_rows=1024, max_queue=16, mem_budget_bytes=0)
    h = ctypes.c_void_p(1234)
    assert lib.rpf_server_create(None, ctypes.byref(cfg), ctypes.byref(h)) == rpf.RPF_EINVAL
    assert h.value is None
    for field, bad in [("slots", 0), ("slots", 17), ("max_batch_rows", 0), ("max_queue", 0)]:
        c = rpf.ServerConfig(slots=2, reserved=0, max_batch_rows=1024, max_queue=16, mem_budget_bytes=0)
        setattr(c, field, bad)
        assert lib.rpf_server_create(fake, ctypes.byref(c), ctypes.byref(h)) == rpf.RPF_EINVAL, field
    t = ctypes.c_uint64(5)
    assert lib.rpf_server_submit(None, fake, 10, 5, fake, fake, None, ctypes.byref(t)) == rpf.RPF_EINVAL
    assert t.value == 0
    done = ctypes.c_int32(3)
    assert lib.rpf_server_poll(None, 1, ctypes.byref(done), None) == rpf.RPF_EINVAL and done.value == 0
    assert lib.rpf_server_wait(None, 1, None) == rpf.RPF_EINVAL
    assert lib.rpf_server_stats(None, None) == rpf.RPF_EINVAL
    assert lib.rpf_server_reset_stats(None) == rpf.RPF_EINVAL
    assert lib.rpf_server_destroy(None) == rpf.RPF_OK
    b = ctypes.c_uint64(0)
    assert lib.rpf_query_workspace_bytes(None, 10, 5, ctypes.byref(b)) == rpf.RPF_EINVAL


def test_plan_arguments_rejected_without_device():
    lib = rpf.load()
    p = rpf.Params(n_trees=2, leaf_size=10, n_try=1, split_rule=0, dist_prec=0, build_flags=0,
                   directions_dev=None, mem_budget_bytes=0)
    h = ctypes.c_void_p(1234)
    ns = (ctypes.c_int64 * 2)(100, 200)
    ds = (ctypes.c_int32 * 2)(4, 4)
    assert lib.rpf_plan_create(None, ds, 2, ctypes.byref(p), 5, 1, 0, None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert h.value is None
    assert lib.rpf_plan_create(ns, None, 2, ctypes.byref(p), 5, 1, 0, None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert lib.rpf_plan_create(ns, ds, 0, ctypes.byref(p), 5, 1, 0, None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert lib.rpf_plan_create(ns, ds, 2, ctypes.byref(p), 0, 1, 0, None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert lib.rpf_plan_create(ns, ds, 2, ctypes.byref(p), 5, 2, 0, None, ctypes.byref(h)) == rpf.RPF_EINVAL
    bad = (ctypes.c_int32 * 2)(4, 0)
    assert lib.rpf_plan_create(ns, bad, 2, ctypes.byref(p), 5, 1, 0, None, ctypes.byref(h)) == rpf.RPF_EINVAL
    assert lib.rpf_plan_launch(None, None) == rpf.RPF_EINVAL
    assert lib.rpf_plan_check(None, None) == rpf.RPF_EINVAL
    assert lib.rpf_plan_tune(None, None, None) == rpf.RPF_EINVAL
    assert lib.rpf_plan_info(None, None, None) == rpf.RPF_EINVAL
    assert lib.rpf_plan_part(None, 0, None) == rpf.RPF_EINVAL
    assert lib.rpf_plan_entry_of(None, 0, None) == rpf.RPF_EINVAL
    assert lib.rpf_plan_destroy(None) == rpf.RPF_OK
    assert lib.rpf_build_batched(ctypes.c_void_p(0x1000), None, 2, 4, ctypes.byref(p), None,
                                 ctypes.byref(h)) == rpf.RPF_EINVAL


def test_tuning_table_round_trip(tmp_path):
    # host only: the tuner's table is read from and written to a text file, one JSON object
    # per line; a malformed file is refused and leaves the table as it was
    import json
    lib = rpf.load()
    assert lib.rpf_tune_clear() == rpf.RPF_OK
    rows = [dict(d=64, max_leaf=64, prec=2, K=16, T=16, n_log2=17, first_trees=4, tile_shape=3, bucket_size=8,
                 subtrees=1),
            dict(d=128, max_leaf=245, prec=3, K=20, T=80, n_log2=19, first_trees=4, tile_shape=4, bucket_size=16,
                 subtrees=0)]
    src = tmp_path / "tune.jsonl"
    src.write_text("".join(json.dumps(r) + "\n" for r in rows) + "\n")
    assert rpf.tune_load(str(src)) == 2
    out = tmp_path / "again.jsonl"
    rpf.tune_save(str(out))
    got = sorted((json.loads(ln) for ln in out.read_text().splitlines() if ln.strip()), key=lambda r: r["d"])
    assert got == rows
    bad = tmp_path / "bad.jsonl"
    bad.write_text(json.dumps(rows[0]) + "\n" + '{"d": 8, "max_leaf": 9}\n')
    n = ctypes.c_int32(-1)
    assert lib.rpf_tune_load(os.fsencode(str(bad)), ctypes.byref(n)) == rpf.RPF_EINVAL
    assert b"line 2" in lib.rpf_last_error()
    assert n.value == -1
    assert lib.rpf_tune_load(os.fsencode(str(tmp_path / "missing.jsonl")), None) == rpf.RPF_EINVAL
    rpf.tune_save(str(out))
    assert len([ln for ln in out.read_text().splitlines() if ln.strip()]) == 2
    assert lib.rpf_tune_clear() == rpf.RPF_OK
    rpf.tune_save(str(out))
    assert out.read_text() == ""
