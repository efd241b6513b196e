"""ctypes binding of the rpForests HIP library (include/rpf.h).

Argument marshalling only: every step of the path runs in the library's kernels.  Torch
tensors provide device memory and the current HIP stream.  The library must be built
(`python -m paper_1812_11689_amd.build`); loading fails loudly when it is missing.
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpf.so")

RPF_OK, RPF_EINVAL, RPF_ENOMEM, RPF_EDEVICE, RPF_EBUSY, RPF_ENOTREADY, RPF_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
_STATUS = {0: "RPF_OK", -1: "RPF_EINVAL", -2: "RPF_ENOMEM", -3: "RPF_EDEVICE", -4: "RPF_EBUSY",
           -5: "RPF_ENOTREADY", -6: "RPF_EINTERNAL"}
PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16x3": 3, "u8grid": 4}

EXPORTS = ["rpf_depth", "rpf_build", "rpf_all_knn", "rpf_query", "rpf_route", "rpf_free", "rpf_tree_dump",
           "rpf_forest_info", "rpf_last_knn_stats", "rpf_profile_enable", "rpf_profile_reset",
           "rpf_profile_read", "rpf_release_cached_memory", "rpf_query_workspace_bytes", "rpf_server_create",
           "rpf_server_submit", "rpf_server_poll", "rpf_server_wait", "rpf_server_stats", "rpf_server_reset_stats",
           "rpf_server_batch_log", "rpf_server_destroy", "rpf_query_noalloc", "rpf_exact_knn", "rpf_build_batched", "rpf_batch_info", "rpf_plan_create", "rpf_plan_info",
           "rpf_plan_part", "rpf_plan_entry_of", "rpf_plan_launch", "rpf_plan_check", "rpf_plan_tune",
           "rpf_plan_destroy", "rpf_last_error", "rpf_tree_nodes", "rpf_tune_save", "rpf_tune_load",
           "rpf_tune_clear"]


class RpfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("n_trees", ctypes.c_int32), ("leaf_size", ctypes.c_int32), ("n_try", ctypes.c_int32),
                ("split_rule", ctypes.c_int32), ("dist_prec", ctypes.c_int32), ("build_flags", ctypes.c_int32),
                ("directions_dev", ctypes.c_void_p), ("mem_budget_bytes", ctypes.c_uint64),
                ("seed", ctypes.c_uint64)]


class Node(ctypes.Structure):
    _fields_ = [("heap", ctypes.c_int64), ("split", ctypes.c_double), ("size", ctypes.c_int32),
                ("left", ctypes.c_int32), ("chosen", ctypes.c_int32), ("depth", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("n_trees", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("n_try", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("dist_prec", ctypes.c_int32), ("n_leaves", ctypes.c_int64), ("device_bytes", ctypes.c_uint64),
                ("batch_count", ctypes.c_int32), ("split_rule", ctypes.c_int32)]


class BatchEntry(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("n", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("heap_base", ctypes.c_int64), ("leaf_heap_base", ctypes.c_int64)]


class KnnStats(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("fallback_rows", ctypes.c_int64), ("reranked32", ctypes.c_int64),
                ("reranked64", ctypes.c_int64), ("first_phase_kept", ctypes.c_int64),
                ("second_phase_emitted", ctypes.c_int64), ("block_merged_rows", ctypes.c_int64)]


class ProfileRecord(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("algo_bytes", ctypes.c_double), ("algo_flops", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("reserved", ctypes.c_int32), ("max_batch_rows", ctypes.c_int64),
                ("max_queue", ctypes.c_int64), ("mem_budget_bytes", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("rows", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("mean_batch_rows", ctypes.c_double), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("rows_per_s", ctypes.c_double),
                ("failed_requests", ctypes.c_int64), ("bad_index_rows", ctypes.c_int64)]


class ServerBatch(ctypes.Structure):
    _fields_ = [("slot", ctypes.c_int32), ("requests", ctypes.c_int32), ("rows", ctypes.c_int64),
                ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double)]


class PlanEntry(ctypes.Structure):
    _fields_ = [("part", ctypes.c_int32), ("index_in_part", ctypes.c_int32), ("d", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n", ctypes.c_int64), ("row", ctypes.c_int64),
                ("heap_base", ctypes.c_int64), ("n_nodes", ctypes.c_int64)]


class PlanPartInfo(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("d", ctypes.c_int32), ("n_sets", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("X_dev", ctypes.c_void_p), ("directions_dev", ctypes.c_void_p),
                ("out_idx_dev", ctypes.c_void_p), ("out_dist_dev", ctypes.c_void_p), ("forest", ctypes.c_void_p),
                ("first_trees", ctypes.c_int32), ("tile_shape", ctypes.c_int32), ("bucket_size", ctypes.c_int32),
                ("subtrees", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"rpForests HIP library not built: {path} is missing "
                           "(run `python -m paper_1812_11689_amd.build`)")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.rpf_depth.restype = i32
    lib.rpf_depth.argtypes = [i64, i32]
    lib.rpf_build.restype = i32
    lib.rpf_build.argtypes = [vp, i64, i32, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    lib.rpf_all_knn.restype = i32
    lib.rpf_all_knn.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.rpf_query.restype = i32
    lib.rpf_query.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    lib.rpf_route.restype = i32
    lib.rpf_route.argtypes = [vp, vp, i64, vp, vp]
    lib.rpf_free.restype = i32
    lib.rpf_free.argtypes = [vp]
    lib.rpf_tree_dump.restype = i32
    lib.rpf_tree_dump.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.rpf_tree_nodes.restype = i32
    lib.rpf_tree_nodes.argtypes = [vp, i32, ctypes.POINTER(Node), i64, ctypes.POINTER(i64)]
    lib.rpf_forest_info.restype = i32
    lib.rpf_forest_info.argtypes = [vp, ctypes.POINTER(Info)]
    lib.rpf_last_knn_stats.restype = i32
    lib.rpf_last_knn_stats.argtypes = [vp, ctypes.POINTER(KnnStats), vp]
    lib.rpf_profile_enable.restype = i32
    lib.rpf_profile_enable.argtypes = [i32]
    lib.rpf_profile_reset.restype = i32
    lib.rpf_profile_reset.argtypes = []
    lib.rpf_profile_read.restype = i32
    lib.rpf_profile_read.argtypes = [ctypes.POINTER(ProfileRecord), i32, ctypes.POINTER(i32)]
    u64 = ctypes.c_uint64
    lib.rpf_query_workspace_bytes.restype = i32
    lib.rpf_query_workspace_bytes.argtypes = [vp, i64, i32, ctypes.POINTER(u64)]
    lib.rpf_server_create.restype = i32
    lib.rpf_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.rpf_server_submit.restype = i32
    lib.rpf_server_submit.argtypes = [vp, vp, i64, i32, vp, vp, vp, ctypes.POINTER(u64)]
    lib.rpf_server_poll.restype = i32
    lib.rpf_server_poll.argtypes = [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    lib.rpf_server_wait.restype = i32
    lib.rpf_server_wait.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double)]
    lib.rpf_server_stats.restype = i32
    lib.rpf_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.rpf_server_reset_stats.restype = i32
    lib.rpf_server_reset_stats.argtypes = [vp]
    lib.rpf_exact_knn.restype = i32
    lib.rpf_exact_knn.argtypes = [vp, i64, i32, vp, i64, vp, i32, vp, vp, vp]
    lib.rpf_query_noalloc.restype = i32
    lib.rpf_query_noalloc.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    lib.rpf_server_batch_log.restype = i32
    lib.rpf_server_batch_log.argtypes = [vp, ctypes.POINTER(ServerBatch), i32, ctypes.POINTER(i32)]
    lib.rpf_server_destroy.restype = i32
    lib.rpf_server_destroy.argtypes = [vp]
    lib.rpf_build_batched.restype = i32
    lib.rpf_build_batched.argtypes = [vp, ctypes.POINTER(i64), i32, i32, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    lib.rpf_batch_info.restype = i32
    lib.rpf_batch_info.argtypes = [vp, i32, ctypes.POINTER(BatchEntry)]
    lib.rpf_plan_create.restype = i32
    lib.rpf_plan_create.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i32), i32, ctypes.POINTER(Params), i32, i32,
                                    i64, vp, ctypes.POINTER(vp)]
    lib.rpf_plan_info.restype = i32
    lib.rpf_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.rpf_plan_part.restype = i32
    lib.rpf_plan_part.argtypes = [vp, i32, ctypes.POINTER(PlanPartInfo)]
    lib.rpf_plan_entry_of.restype = i32
    lib.rpf_plan_entry_of.argtypes = [vp, i32, ctypes.POINTER(PlanEntry)]
    lib.rpf_plan_launch.restype = i32
    lib.rpf_plan_launch.argtypes = [vp, vp]
    lib.rpf_plan_check.restype = i32
    lib.rpf_plan_check.argtypes = [vp, vp]
    lib.rpf_plan_tune.restype = i32
    lib.rpf_plan_tune.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.rpf_tune_save.restype = i32
    lib.rpf_tune_save.argtypes = [ctypes.c_char_p]
    lib.rpf_tune_load.restype = i32
    lib.rpf_tune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32)]
    lib.rpf_tune_clear.restype = i32
    lib.rpf_tune_clear.argtypes = []
    lib.rpf_plan_destroy.restype = i32
    lib.rpf_plan_destroy.argtypes = [vp]
    lib.rpf_release_cached_memory.restype = i32
    lib.rpf_release_cached_memory.argtypes = [i32]
    lib.rpf_last_error.restype = ctypes.c_char_p
    lib.rpf_last_error.argtypes = []
    _lib = lib
    return lib


def _check(st: int):
    if st != RPF_OK:
        raise RpfError(st, load().rpf_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, dtype) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("expected a device (cuda) tensor")
    if t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    return t.contiguous()


def depth(n: int, leaf_size: int) -> int:
    return load().rpf_depth(n, leaf_size)


class Forest:
    """A forest resident in device memory; owns its library handle."""

    def __init__(self, handle, n, d, n_trees, leaf_size, n_try, L):
        self._h = handle
        self.n, self.d, self.n_trees, self.leaf_size, self.n_try, self.depth = n, d, n_trees, leaf_size, n_try, L

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("forest was freed")
        return self._h

    def all_knn(self, K: int, exclude_self: bool = True, stream=None):
        idx = torch.empty((self.n, K), dtype=torch.int32, device="cuda")
        dist = torch.empty((self.n, K), dtype=torch.float32, device="cuda")
        _check(load().rpf_all_knn(self.handle, K, int(exclude_self), idx.data_ptr(), dist.data_ptr(),
                                  _stream(stream)))
        return idx, dist

    def query(self, Q: torch.Tensor, K: int, stream=None, out=None):
        Q = _dev(Q, torch.float32)
        m = Q.shape[0]
        if out is None:
            idx = torch.empty((m, K), dtype=torch.int32, device="cuda")
            dist = torch.empty((m, K), dtype=torch.float32, device="cuda")
        else:
            idx, dist = out
        _check(load().rpf_query(self.handle, Q.data_ptr(), m, K, idx.data_ptr(), dist.data_ptr(), _stream(stream)))
        return idx, dist

    def query_noalloc(self, Q: torch.Tensor, K: int, out, stream=None):
        """rpf_query_noalloc: like query(), into the caller's outputs `out` = (idx int32 [m][K],
        dist float32 [m][K]); the library allocates nothing."""
        Q = _dev(Q, torch.float32)
        idx, dist = out
        m = Q.shape[0]
        if tuple(idx.shape) != (m, K) or tuple(dist.shape) != (m, K):
            raise ValueError("out must be ([m][K] int32, [m][K] float32)")
        for t, dt in ((idx, torch.int32), (dist, torch.float32)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError("out tensors must be contiguous device tensors of int32 / float32")
        _check(load().rpf_query_noalloc(self.handle, Q.data_ptr(), m, K, idx.data_ptr(), dist.data_ptr(),
                                        _stream(stream)))
        return idx, dist

    def route(self, Q: torch.Tensor, stream=None):
        Q = _dev(Q, torch.float32)
        out = torch.empty((self.n_trees, Q.shape[0]), dtype=torch.int32, device="cuda")
        _check(load().rpf_route(self.handle, Q.data_ptr(), Q.shape[0], out.data_ptr(), _stream(stream)))
        return out

    def _nodes(self) -> int:
        return (1 << self.depth) - 1

    def tree_dump(self, t: int, stream=None):
        if getattr(self, "split_rule", "median") == "uniform":  # leaves only: perm and leaf ordinals
            perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
            leaf_of = torch.empty(self.n, dtype=torch.int32, device="cuda")
            _check(load().rpf_tree_dump(self.handle, t, None, None, None, perm.data_ptr(), leaf_of.data_ptr(),
                                        _stream(stream)))
            return dict(perm=perm, leaf_of=leaf_of)
        H = self._nodes()
        split = torch.empty(max(H, 1), dtype=torch.float64, device="cuda")
        sidx = torch.empty(max(H, 1), dtype=torch.int32, device="cuda")
        chosen = torch.empty(max(H, 1), dtype=torch.int32, device="cuda")
        perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
        leaf_of = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(load().rpf_tree_dump(self.handle, t, split.data_ptr(), sidx.data_ptr(), chosen.data_ptr(),
                                    perm.data_ptr(), leaf_of.data_ptr(), _stream(stream)))
        return dict(split=split[:H], split_idx=sidx[:H], chosen=chosen[:H], perm=perm, leaf_of=leaf_of)

    def tree_nodes(self, t: int) -> list:
        """rpf_tree_nodes (uniform rule): the nodes of tree t where a split was attempted, as
        dicts (heap, split, size, left, chosen, depth)."""
        cnt = ctypes.c_int64(0)
        _check(load().rpf_tree_nodes(self.handle, t, None, 0, ctypes.byref(cnt)))
        buf = (Node * max(cnt.value, 1))()
        _check(load().rpf_tree_nodes(self.handle, t, buf, cnt.value, ctypes.byref(cnt)))
        return [{k: getattr(buf[i], k) for k, _ in Node._fields_} for i in range(cnt.value)]

    def query_workspace_bytes(self, m: int, K: int) -> int:
        b = ctypes.c_uint64(0)
        _check(load().rpf_query_workspace_bytes(self.handle, m, K, ctypes.byref(b)))
        return b.value

    def info(self) -> dict:
        inf = Info()
        _check(load().rpf_forest_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    def knn_stats(self, stream=None) -> dict:
        st = KnnStats()
        _check(load().rpf_last_knn_stats(self.handle, ctypes.byref(st), _stream(stream)))
        return {k: getattr(st, k) for k, _ in KnnStats._fields_}

    def free(self):
        if self._h is not None:
            _check(load().rpf_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def exact_knn(X: torch.Tensor, Q: torch.Tensor, K: int, self_idx: torch.Tensor | None = None, stream=None):
    """rpf_exact_knn: the exact K nearest points of X to each row of Q by (binary64 distance,
    index); self_idx (int64 [m], optional) leaves out one point per query."""
    X = _dev(X, torch.float32)
    Q = _dev(Q, torch.float32)
    n, d = X.shape
    m = Q.shape[0]
    if Q.shape[1] != d:
        raise ValueError("X and Q need the same number of columns")
    sp = None
    if self_idx is not None:
        self_idx = _dev(self_idx, torch.int64)
        if self_idx.shape != (m,):
            raise ValueError("self_idx must be int64 [m]")
        sp = self_idx.data_ptr()
    idx = torch.empty((m, K), dtype=torch.int32, device="cuda")
    dist = torch.empty((m, K), dtype=torch.float32, device="cuda")
    _check(load().rpf_exact_knn(X.data_ptr(), n, d, Q.data_ptr(), m, sp, K, idx.data_ptr(), dist.data_ptr(),
                                _stream(stream)))
    return idx, dist


SPLIT = {"median": 0, "uniform": 1}


BUILD_SUBTREES = 1  # RPF_BUILD_SUBTREES: the small levels in one persistent launch


def build(X: torch.Tensor, n_trees: int, leaf_size: int, directions: torch.Tensor | None, n_try: int = 1,
          dist_prec: str = "fp32", mem_budget_bytes: int = 0, stream=None, split_rule: str = "median",
          seed: int = 0, subtrees: bool = False) -> Forest:
    """Grow a forest over X (float32 [n][d] on the device).  Median rule: with the given
    directions (float32 [n_trees][2^L-1][n_try][d] on the device, L = depth(n, leaf_size)).
    Uniform rule (split_rule="uniform"): directions None, the random numbers come from the
    library's counter-based generator keyed by `seed`.  subtrees: RPF_BUILD_SUBTREES."""
    X = _dev(X, torch.float32)
    n, d = X.shape
    rule = SPLIT[split_rule]
    L = depth(n, leaf_size) if n >= 1 and leaf_size >= 1 and rule == 0 else 0
    dptr = None
    if directions is not None:
        directions = _dev(directions, torch.float32)
        dptr = directions.data_ptr()
    p = Params(n_trees=n_trees, leaf_size=leaf_size, n_try=n_try, split_rule=rule,
               dist_prec=PREC[dist_prec] if isinstance(dist_prec, str) else int(dist_prec),
               build_flags=BUILD_SUBTREES if subtrees else 0,
               directions_dev=dptr, mem_budget_bytes=mem_budget_bytes, seed=seed & (2**64 - 1))
    h = ctypes.c_void_p()
    _check(load().rpf_build(X.data_ptr(), n, d, ctypes.byref(p), _stream(stream), ctypes.byref(h)))
    f = Forest(h, n, d, n_trees, leaf_size, n_try, L)
    f.split_rule = split_rule
    if rule:
        f.depth = f.info()["depth"]
    return f


class BatchedForest(Forest):
    """A forest over several data sets of the same d, grown together (rpf_build_batched)."""

    def _nodes(self) -> int:
        return sum((1 << depth(n, self.leaf_size)) - 1 for n in self.sizes)

    def entries(self):
        out = []
        for i in range(self.count):
            e = BatchEntry()
            _check(load().rpf_batch_info(self.handle, i, ctypes.byref(e)))
            out.append({k: getattr(e, k) for k, _ in BatchEntry._fields_})
        return out

    def all_knn_split(self, K: int, exclude_self: bool = True, stream=None):
        """all_knn, split into one (idx, dist) pair per data set (indices within the set)."""
        idx, dist = self.all_knn(K, exclude_self, stream)
        return [(idx[e["offset"]:e["offset"] + e["n"]], dist[e["offset"]:e["offset"] + e["n"]])
                for e in self.entries()]


def batched_directions_rows(sizes, leaf_size: int):
    """Heap-node count H_i of every data set and the row offset hbase_i of its directions."""
    Hs = [(1 << depth(int(n), leaf_size)) - 1 for n in sizes]
    base = [0]
    for h in Hs[:-1]:
        base.append(base[-1] + h)
    return Hs, base


def build_batched(Xs, n_trees: int, leaf_size: int, directions: torch.Tensor | None, n_try: int = 1,
                  dist_prec: str = "fp32", mem_budget_bytes: int = 0, stream=None,
                  subtrees: bool = False) -> BatchedForest:
    """Grow one forest per data set (same d) in shared launches.  Xs: list of float32 [n_i][d]
    device tensors (or one concatenated tensor with `sizes` given as a list of (X, n) pairs);
    directions: float32 [n_trees][sum H_i][n_try][d] on the device (see batched_directions_rows)."""
    sizes = [int(x.shape[0]) for x in Xs]
    d = int(Xs[0].shape[1])
    if any(int(x.shape[1]) != d for x in Xs):
        raise ValueError("every data set of one batched forest needs the same d")
    X = torch.cat([_dev(x, torch.float32) for x in Xs]) if len(Xs) > 1 else _dev(Xs[0], torch.float32)
    dptr = None
    if directions is not None:
        directions = _dev(directions, torch.float32)
        dptr = directions.data_ptr()
    p = Params(n_trees=n_trees, leaf_size=leaf_size, n_try=n_try, split_rule=0,
               dist_prec=PREC[dist_prec] if isinstance(dist_prec, str) else int(dist_prec),
               build_flags=BUILD_SUBTREES if subtrees else 0,
               directions_dev=dptr, mem_budget_bytes=mem_budget_bytes)
    ns = (ctypes.c_int64 * len(sizes))(*sizes)
    h = ctypes.c_void_p()
    _check(load().rpf_build_batched(X.data_ptr(), ns, len(sizes), d, ctypes.byref(p), _stream(stream),
                                    ctypes.byref(h)))
    f = BatchedForest(h, sum(sizes), d, n_trees, leaf_size, n_try, max(depth(n, leaf_size) for n in sizes))
    f.count = len(sizes)
    f.sizes = sizes
    return f


class _DeviceArray:
    """A device buffer of the library seen by torch without a copy (CUDA array interface)."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(int(x) for x in shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 3, "strides": None}


def _view(ptr: int, shape, dtype) -> torch.Tensor:
    typestr = {torch.float32: "<f4", torch.int32: "<i4"}[dtype]
    return torch.as_tensor(_DeviceArray(ptr, shape, typestr), device="cuda")


def tune_save(path: str):
    """Write the process's tuning table (rpf_tune_save)."""
    _check(load().rpf_tune_save(os.fsencode(path)))


def tune_load(path: str) -> int:
    """Merge a tuning table file into the process's table (rpf_tune_load); its entry count."""
    n = ctypes.c_int32(0)
    _check(load().rpf_tune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tune_clear():
    _check(load().rpf_tune_clear())


class Plan:
    """Build + all-points search of many data sets recorded as one HIP graph (rpf_plan_*).
    set_inputs() writes the points and directions into the plan's buffers, launch() runs the
    graph, result(i) views data set i's (idx, dist)."""

    def __init__(self, sizes, dims, n_trees: int, leaf_size: int, K: int, exclude_self: bool = True,
                 n_try: int = 1, dist_prec: str = "fp32", max_part_points: int = 0, stream=None):
        self.sizes = [int(n) for n in sizes]
        self.dims = [int(d) for d in dims] if not isinstance(dims, int) else [int(dims)] * len(self.sizes)
        self.n_trees, self.leaf_size, self.n_try, self.K = n_trees, leaf_size, n_try, K
        p = Params(n_trees=n_trees, leaf_size=leaf_size, n_try=n_try, split_rule=0,
                   dist_prec=PREC[dist_prec] if isinstance(dist_prec, str) else int(dist_prec), build_flags=0,
                   directions_dev=None, mem_budget_bytes=0)
        c = len(self.sizes)
        ns = (ctypes.c_int64 * c)(*self.sizes)
        ds = (ctypes.c_int32 * c)(*self.dims)
        h = ctypes.c_void_p()
        _check(load().rpf_plan_create(ns, ds, c, ctypes.byref(p), K, int(exclude_self), max_part_points,
                                      _stream(stream), ctypes.byref(h)))
        self._h = h
        npart = ctypes.c_int32(0)
        _check(load().rpf_plan_info(h, ctypes.byref(npart), None))
        self.parts = []
        for k in range(npart.value):
            pi = PlanPartInfo()
            _check(load().rpf_plan_part(h, k, ctypes.byref(pi)))
            self.parts.append({
                "rows": pi.rows, "d": pi.d, "n_sets": pi.n_sets, "n_nodes": pi.n_nodes,
                "X": _view(pi.X_dev, (pi.rows, pi.d), torch.float32),
                "directions": _view(pi.directions_dev, (n_trees, pi.n_nodes, n_try, pi.d), torch.float32)
                if pi.n_nodes else None,
                "idx": _view(pi.out_idx_dev, (pi.rows, K), torch.int32),
                "dist": _view(pi.out_dist_dev, (pi.rows, K), torch.float32),
                "forest": pi.forest})
        self.entries = []
        for i in range(c):
            e = PlanEntry()
            _check(load().rpf_plan_entry_of(h, i, ctypes.byref(e)))
            self.entries.append({k: getattr(e, k) for k, _ in PlanEntry._fields_})

    def set_inputs(self, xs, directions):
        """xs[i]: [n_i][d_i] points of data set i, directions[i]: [n_trees][H_i][n_try][d_i]
        (numpy arrays or tensors); copied into the plan's buffers."""
        for e, x, r in zip(self.entries, xs, directions):
            pt = self.parts[e["part"]]
            pt["X"][e["row"]:e["row"] + e["n"]].copy_(torch.as_tensor(x))
            if e["n_nodes"]:
                pt["directions"][:, e["heap_base"]:e["heap_base"] + e["n_nodes"]].copy_(torch.as_tensor(r))

    def launch(self, stream=None):
        _check(load().rpf_plan_launch(self._h, _stream(stream)))

    def check(self, stream=None):
        _check(load().rpf_plan_check(self._h, _stream(stream)))

    def choices(self):
        """The tuned choices of every part (first-phase trees, Phase II tile shape, bucket
        size, persistent subtree build)."""
        out = []
        for k, pt in enumerate(self.parts):
            pi = PlanPartInfo()
            _check(load().rpf_plan_part(self._h, k, ctypes.byref(pi)))
            pt.update(first_trees=pi.first_trees, tile_shape=pi.tile_shape, bucket_size=pi.bucket_size,
                      subtrees=pi.subtrees)
            out.append({"first_trees": pi.first_trees, "tile_shape": pi.tile_shape, "bucket_size": pi.bucket_size,
                        "subtrees": pi.subtrees})
        return out

    def tune(self, stream=None) -> float:
        ms = ctypes.c_double(0.0)
        _check(load().rpf_plan_tune(self._h, _stream(stream), ctypes.byref(ms)))
        self.choices()
        return ms.value

    def result(self, i: int):
        e = self.entries[i]
        pt = self.parts[e["part"]]
        return pt["idx"][e["row"]:e["row"] + e["n"]], pt["dist"][e["row"]:e["row"] + e["n"]]

    def close(self):
        if self._h is not None:
            _check(load().rpf_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True):
    _check(load().rpf_profile_enable(int(on)))


def profile_reset():
    _check(load().rpf_profile_reset())


def profile_read() -> dict:
    cap = 64
    recs = (ProfileRecord * cap)()
    cnt = ctypes.c_int32(0)
    _check(load().rpf_profile_read(recs, cap, ctypes.byref(cnt)))
    out = {}
    for r in recs[: min(cnt.value, cap)]:
        out[r.name.decode()] = dict(launches=r.launches, total_ms=r.total_ms, algo_bytes=r.algo_bytes,
                                    algo_flops=r.algo_flops)
    return out


def release_cached_memory(device: int = -1):
    """Return the library's idle cached device blocks to the runtime."""
    _check(load().rpf_release_cached_memory(device))


class Server:
    """Continuous-batching query server over a resident forest (the library's serving loop).
    submit() is non-blocking and returns a ticket; the caller keeps Q and the outputs alive
    until the request is collected by poll() or wait()."""

    def __init__(self, forest: Forest, slots: int = 4, max_batch_rows: int = 8192, max_queue: int = 1 << 16,
                 mem_budget_bytes: int = 0):
        self.forest = forest
        cfg = ServerConfig(slots=slots, reserved=0, max_batch_rows=max_batch_rows, max_queue=max_queue,
                           mem_budget_bytes=mem_budget_bytes)
        h = ctypes.c_void_p()
        _check(load().rpf_server_create(forest.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, Q: torch.Tensor, K: int, out=None, stream=None) -> int:
        Q = _dev(Q, torch.float32)
        m = Q.shape[0]
        if out is None:
            out = (torch.empty((m, K), dtype=torch.int32, device=Q.device),
                   torch.empty((m, K), dtype=torch.float32, device=Q.device))
        t = ctypes.c_uint64(0)
        _check(load().rpf_server_submit(self._h, Q.data_ptr(), m, K, out[0].data_ptr(), out[1].data_ptr(),
                                        _stream(stream), ctypes.byref(t)))
        self._keep[t.value] = (Q, out)
        return t.value

    def poll(self, ticket: int):
        """(idx, dist, latency_s) once done, else None."""
        done = ctypes.c_int32(0)
        lat = ctypes.c_double(0.0)
        st = load().rpf_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(lat))
        if st == RPF_ENOTREADY:
            return None
        _, out = self._keep.pop(ticket)
        _check(st)
        return out[0], out[1], lat.value

    def wait(self, ticket: int):
        lat = ctypes.c_double(0.0)
        st = load().rpf_server_wait(self._h, ticket, ctypes.byref(lat))
        _, out = self._keep.pop(ticket)
        _check(st)
        return out[0], out[1], lat.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(load().rpf_server_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def batch_log(self) -> list:
        """Device-side spans of the batches: dicts of slot, requests, rows, start_ms, end_ms."""
        cnt = ctypes.c_int32(0)
        _check(load().rpf_server_batch_log(self._h, None, 0, ctypes.byref(cnt)))
        buf = (ServerBatch * max(cnt.value, 1))()
        _check(load().rpf_server_batch_log(self._h, buf, cnt.value, ctypes.byref(cnt)))
        return [{k: getattr(buf[i], k) for k, _ in ServerBatch._fields_} for i in range(cnt.value)]

    def reset_stats(self):
        _check(load().rpf_server_reset_stats(self._h))

    def close(self):
        if self._h is not None:
            _check(load().rpf_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
