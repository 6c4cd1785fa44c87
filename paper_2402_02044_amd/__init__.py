"""MI355X (gfx950) LVQ library: Python binding of the C ABI in include/lvq.h.

Locally-adaptive Vector Quantization after arXiv 2402.02044: encoding
(Sec. 2.3, Eq. 1-3; two-level LVQ-B1xB2; multi-means Def. 1; Turbo layout
Sec. 3.1) and similarities between float queries and LVQ codes (Sec. 3.2)
over candidate lists and as an exhaustive top-k (Sec. 2.1).

This module only marshals arguments: every step runs in the HIP kernels of
``liblvq.so``.  Functions named ``lvq_*`` mirror the C entry points one to one
(raw device pointers as ints, ``stream`` a hipStream_t as int, 0 = default).
``Index`` is a convenience wrapper over torch tensors (PyTorch supplies device
memory and streams).  There is no CPU fallback: importing fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblvq.so")
TILE_CACHE = os.path.join(HERE, "tile_cache.json")

LVQ_L2, LVQ_IP = 0, 1
LVQ_SEQUENTIAL, LVQ_TURBO = 0, 1
LVQ_PRIMARY, LVQ_FULL = 1, 2
LVQ_FP32, LVQ_BF16, LVQ_FP16, LVQ_FP32_VALU = 0, 1, 2, 3

LVQ_OK = 0
LVQ_ERR_INVALID_ARG = -1
LVQ_ERR_UNSUPPORTED = -2
LVQ_ERR_OOM = -3
LVQ_ERR_CAPACITY = -4
LVQ_ERR_DEVICE = -5
LVQ_ERR_NONFINITE = -6
LVQ_ERR_BAD_SLOT = -7
LVQ_ERR_SCRATCH = -8
LVQ_NOALLOC_SCRATCH_BYTES = 32 << 20

EXPORTS = ["lvq_row_format", "lvq_create", "lvq_destroy", "lvq_set_means", "lvq_encode", "lvq_insert",
           "lvq_delete", "lvq_consolidate", "lvq_distances", "lvq_distances_noalloc", "lvq_topk",
           "lvq_probe_topk", "lvq_retire_means",
           "lvq_add_means", "lvq_mean_members", "lvq_graph_search", "lvq_graph_prune", "lvq_graph_build",
           "lvq_graph_insert", "lvq_graph_delete", "lvq_bw_stream", "lvq_bw_gather", "lvq_read_rows",
           "lvq_get_stats", "lvq_sync", "lvq_mean", "lvq_kmeans", "lvq_strerror", "lvq_set_timing",
           "lvq_kernel_time", "lvq_autotune", "lvq_set_tile", "lvq_server_create", "lvq_server_submit",
           "lvq_server_wait", "lvq_server_drain", "lvq_server_get_stats", "lvq_server_destroy",
           "lvq_num_tile_shapes", "lvq_tile_shape"]


class lvq_config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("bits1", ctypes.c_int32), ("bits2", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("layout", ctypes.c_int32), ("align", ctypes.c_int32),
                ("capacity", ctypes.c_int64), ("mem_budget_bytes", ctypes.c_int64)]


class lvq_stats(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("free_slots", ctypes.c_int64),
                ("live_estimate", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("n_means", ctypes.c_int32), ("row_bytes", ctypes.c_int32),
                ("resid_bytes", ctypes.c_int32), ("code_positions", ctypes.c_int32),
                ("epoch", ctypes.c_uint32), ("last_workgroups", ctypes.c_int64),
                ("last_lists", ctypes.c_int64), ("last_parts", ctypes.c_int32)]


class lvq_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("k", ctypes.c_int32),
                ("k_first", ctypes.c_int32), ("precision", ctypes.c_int32), ("scan_level", ctypes.c_int32),
                ("rerank_level", ctypes.c_int32), ("pool_bytes", ctypes.c_int64)]


class lvq_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nq", ctypes.c_int32), ("epoch", ctypes.c_uint32),
                ("slot", ctypes.c_int32), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class lvq_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("pool_bytes", ctypes.c_int64),
                ("pool_peak", ctypes.c_int64), ("batch_bytes_max", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("peak_in_flight", ctypes.c_int32), ("peak_queue", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("in_flight", ctypes.c_int32)]


class LVQError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__("%s: %s (%d)" % (where, lvq_strerror(code), code))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblvq.so is not built (run __graft_entry__.build() or "
                          "python paper_2402_02044_amd/build_lib.py); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "lvq_row_format": [ctypes.POINTER(lvq_config), P, P, P],
        "lvq_create": [ctypes.POINTER(lvq_config), P, i32, ctypes.POINTER(P)],
        "lvq_destroy": [P],
        "lvq_set_means": [P, P, i32, P, P],
        "lvq_encode": [P, P, i64, P, P, P],
        "lvq_insert": [P, P, i64, P, P, P],
        "lvq_delete": [P, P, i64, P],
        "lvq_consolidate": [P, P, P],
        "lvq_distances": [P, P, i64, P, P, i64, i32, P, i32, P, P, P],
        "lvq_distances_noalloc": [P, P, i64, P, P, i64, i32, P, i32, P, P, P],
        "lvq_topk": [P, P, i32, i64, i32, i32, P, P, P],
        "lvq_probe_topk": [P, P, i64, i32, i32, i32, P, P, P, P],
        "lvq_retire_means": [P, P, i32, P],
        "lvq_add_means": [P, P, i32, P, P],
        "lvq_mean_members": [P, P, i32, P, P, i64, P],
        "lvq_graph_search": [P, P, i64, P, i32, P, i32, i32, i32, P, P, P, P],
        "lvq_graph_prune": [P, i64, i32, i32, P, i64, P, P, i32, ctypes.c_float, P, P],
        "lvq_graph_build": [P, i64, i32, i32, i64, i32, i32, ctypes.c_float, i32, i32, i32, P, P],
        "lvq_graph_insert": [P, i64, i32, i32, P, i64, i32, i32, ctypes.c_float, i32, i32, P, P],
        "lvq_graph_delete": [P, i64, i32, i32, P, i32, ctypes.c_float, P, P],
        "lvq_read_rows": [P, P, i64, P, P, P],
        "lvq_bw_stream": [P, i64, P, P],
        "lvq_bw_gather": [P, P, i64, i32, P, P],
        "lvq_get_stats": [P, ctypes.POINTER(lvq_stats)],
        "lvq_sync": [P, P],
        "lvq_mean": [P, i64, i32, P, P],
        "lvq_kmeans": [P, i64, i32, i32, P, i32, P, P],
        "lvq_strerror": [ctypes.c_int],
        "lvq_set_timing": [P, i32],
        "lvq_autotune": [P, P, i64, P, P, i64, i32, i32, P, P, P],
        "lvq_set_tile": [P, i32, i32, i32],
        "lvq_kernel_time": [P, P, P],
        "lvq_server_create": [P, ctypes.POINTER(lvq_server_config), ctypes.POINTER(P)],
        "lvq_server_submit": [P, P, i32, P],
        "lvq_server_wait": [P, i64, P, P, ctypes.POINTER(lvq_request_info)],
        "lvq_server_drain": [P],
        "lvq_server_get_stats": [P, ctypes.POINTER(lvq_server_stats)],
        "lvq_server_destroy": [P],
        "lvq_num_tile_shapes": [],
        "lvq_tile_shape": [i32, P, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "lvq_strerror" else ctypes.c_int
    return lib


_lib = _load()


def lvq_strerror(code: int) -> str:
    return _lib.lvq_strerror(code).decode()


def _chk(rc, where):
    if rc != LVQ_OK:
        raise LVQError(rc, where)
    return rc


# ---- one-to-one wrappers of the C entry points (raw pointers) -------------

def lvq_row_format(cfg: lvq_config):
    rb, rs, npos = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _chk(_lib.lvq_row_format(ctypes.byref(cfg), ctypes.byref(rb), ctypes.byref(rs), ctypes.byref(npos)),
         "lvq_row_format")
    return rb.value, rs.value, npos.value


def lvq_create(cfg: lvq_config, means_host_ptr: int, n_means: int) -> int:
    out = ctypes.c_void_p()
    _chk(_lib.lvq_create(ctypes.byref(cfg), means_host_ptr, n_means, ctypes.byref(out)), "lvq_create")
    return out.value


def lvq_destroy(ix: int):
    return _chk(_lib.lvq_destroy(ix), "lvq_destroy")


def lvq_set_means(ix, means_host_ptr, n_means, stream=0) -> int:
    first = ctypes.c_int32()
    _chk(_lib.lvq_set_means(ix, means_host_ptr, n_means, ctypes.byref(first), stream), "lvq_set_means")
    return first.value


def lvq_encode(ix, x, n, rows, resid, stream=0):
    return _chk(_lib.lvq_encode(ix, x, n, rows, resid, stream), "lvq_encode")


def lvq_insert(ix, x, n, ext_ids, slots_out, stream=0):
    return _chk(_lib.lvq_insert(ix, x, n, ext_ids, slots_out, stream), "lvq_insert")


def lvq_delete(ix, slots, n, stream=0):
    return _chk(_lib.lvq_delete(ix, slots, n, stream), "lvq_delete")


def lvq_consolidate(ix, stream=0) -> int:
    freed = ctypes.c_int64()
    _chk(_lib.lvq_consolidate(ix, stream, ctypes.byref(freed)), "lvq_consolidate")
    return freed.value


def lvq_distances(ix, q, nq, offsets, ids, total, level, dist, k, topk_ids, topk_dist, stream=0):
    return _chk(_lib.lvq_distances(ix, q, nq, offsets, ids, total, level, dist, k, topk_ids, topk_dist,
                                   stream), "lvq_distances")


def lvq_distances_noalloc(ix, q, nq, offsets, ids, total, level, dist, k, topk_ids, topk_dist, stream=0):
    return _chk(_lib.lvq_distances_noalloc(ix, q, nq, offsets, ids, total, level, dist, k, topk_ids, topk_dist,
                                           stream), "lvq_distances_noalloc")


def lvq_topk(ix, q, prec, nq, k, level, ids, dist, stream=0):
    return _chk(_lib.lvq_topk(ix, q, prec, nq, k, level, ids, dist, stream), "lvq_topk")


def lvq_probe_topk(ix, q, nq, nprobe, k, level, probe, ids, dist, stream=0):
    return _chk(_lib.lvq_probe_topk(ix, q, nq, nprobe, k, level, probe, ids, dist, stream), "lvq_probe_topk")


def lvq_retire_means(ix, ids_host, n, stream=0):
    return _chk(_lib.lvq_retire_means(ix, ids_host, n, stream), "lvq_retire_means")


def lvq_add_means(ix, means_host, n, ids_out_host, stream=0):
    return _chk(_lib.lvq_add_means(ix, means_host, n, ids_out_host, stream), "lvq_add_means")


def lvq_graph_search(ix, q, nq, graph, degree, entries, n_entries, window, k, ids, dist, explored, stream=0):
    return _chk(_lib.lvq_graph_search(ix, q, nq, graph, degree, entries, n_entries, window, k, ids, dist, explored,
                                      stream), "lvq_graph_search")


def lvq_graph_prune(x, n, dim, metric, nodes, m, cand_offsets, cand_ids, degree, alpha, graph, stream=0):
    return _chk(_lib.lvq_graph_prune(x, n, dim, metric, nodes, m, cand_offsets, cand_ids, degree, alpha, graph,
                                     stream), "lvq_graph_prune")


def lvq_graph_build(x, n, dim, metric, first, degree, window, alpha, passes, entry, max_batch, graph, stream=0):
    return _chk(_lib.lvq_graph_build(x, n, dim, metric, first, degree, window, alpha, passes, entry, max_batch,
                                     graph, stream), "lvq_graph_build")


def lvq_bw_stream(src, nbytes, sink, stream=0):
    return _chk(_lib.lvq_bw_stream(src, nbytes, sink, stream), "lvq_bw_stream")


def lvq_bw_gather(ix, ids, n, level, sink, stream=0):
    return _chk(_lib.lvq_bw_gather(ix, ids, n, level, sink, stream), "lvq_bw_gather")


def lvq_graph_insert(x, n, dim, metric, nodes_host, m, degree, window, alpha, entry, max_batch, graph, stream=0):
    return _chk(_lib.lvq_graph_insert(x, n, dim, metric, nodes_host, m, degree, window, alpha, entry, max_batch,
                                      graph, stream), "lvq_graph_insert")


def lvq_graph_delete(x, n, dim, metric, deleted, degree, alpha, graph, stream=0):
    return _chk(_lib.lvq_graph_delete(x, n, dim, metric, deleted, degree, alpha, graph, stream), "lvq_graph_delete")


def _graph_args(x, graph):
    import torch
    if x.dtype != torch.float32 or x.dim() != 2 or not x.is_contiguous():
        raise LVQError(LVQ_ERR_INVALID_ARG, "x must be a contiguous float32 matrix")
    if graph.dim() != 2 or graph.shape[0] != x.shape[0] or graph.dtype != torch.int32 or not graph.is_contiguous():
        raise LVQError(LVQ_ERR_INVALID_ARG, "graph must be a contiguous int32 (n x degree) tensor")


def graph_insert(x, graph, nodes, window, alpha, metric, entry, max_batch=16384, stream=None):
    """Insert the listed nodes (host sequence) into graph (App. A, one pass)."""
    import numpy as np
    _graph_args(x, graph)
    nodes = np.ascontiguousarray(nodes, np.int32)
    lvq_graph_insert(_ptr(x), x.shape[0], x.shape[1], metric, nodes.ctypes.data, nodes.shape[0], graph.shape[1],
                     window, alpha, entry, max_batch, _ptr(graph), _stream(stream))
    return graph


def graph_delete(x, graph, deleted, alpha, metric, stream=None):
    """Delete consolidation (App. A); deleted: n uint8/bool device flags."""
    import torch
    _graph_args(x, graph)
    deleted = deleted.to(torch.uint8).contiguous()
    if deleted.shape != (x.shape[0],):
        raise LVQError(LVQ_ERR_INVALID_ARG, "deleted must hold one flag per node")
    lvq_graph_delete(_ptr(x), x.shape[0], x.shape[1], metric, _ptr(deleted), graph.shape[1], alpha, _ptr(graph),
                     _stream(stream))
    return graph


def graph_prune(x, nodes, cand_offsets, cand_ids, graph, alpha, metric, stream=None):
    """Alg. 2 on torch tensors: x (n x dim float32), nodes (m int32),
    cand_offsets (m + 1 int64), cand_ids (int32), graph (n x degree int32,
    rewritten in place)."""
    import torch
    for t, dt in ((x, torch.float32), (nodes, torch.int32), (cand_offsets, torch.int64), (cand_ids, torch.int32),
                  (graph, torch.int32)):
        if t.dtype != dt or not t.is_contiguous():
            raise LVQError(LVQ_ERR_INVALID_ARG, "graph_prune: contiguous tensors of the documented types")
    if graph.shape[0] != x.shape[0] or cand_offsets.shape[0] != nodes.shape[0] + 1:
        raise LVQError(LVQ_ERR_INVALID_ARG, "graph_prune: shapes")
    lvq_graph_prune(_ptr(x), x.shape[0], x.shape[1], metric, _ptr(nodes), nodes.shape[0], _ptr(cand_offsets),
                    _ptr(cand_ids) if cand_ids.numel() else _ptr(cand_offsets), graph.shape[1], alpha, _ptr(graph),
                    _stream(stream))


def graph_build(x, degree, window, alpha, metric, entry, passes=2, first=0, graph=None, max_batch=16384,
                stream=None):
    """Graph construction (App. A) over x (n x dim float32 on the device);
    returns graph (n x degree int32).  With first > 0, graph holds the rows
    of nodes [0, first) and nodes [first, n) are inserted."""
    import torch
    if x.dtype != torch.float32 or x.dim() != 2 or not x.is_contiguous():
        raise LVQError(LVQ_ERR_INVALID_ARG, "graph_build: x must be a contiguous float32 matrix")
    n = x.shape[0]
    if graph is None:
        graph = torch.empty((n, degree), dtype=torch.int32, device=x.device)
    if graph.shape != (n, degree) or graph.dtype != torch.int32 or not graph.is_contiguous():
        raise LVQError(LVQ_ERR_INVALID_ARG, "graph_build: graph must be a contiguous int32 (n x degree) tensor")
    lvq_graph_build(_ptr(x), n, x.shape[1], metric, first, degree, window, alpha, passes, entry, max_batch,
                    _ptr(graph), _stream(stream))
    return graph


def lvq_mean_members(ix, ids_host, n, offsets_host, slots, cap, stream=0):
    return _chk(_lib.lvq_mean_members(ix, ids_host, n, offsets_host, slots, cap, stream), "lvq_mean_members")


def lvq_read_rows(ix, slots, n, rows, resid, stream=0):
    return _chk(_lib.lvq_read_rows(ix, slots, n, rows, resid, stream), "lvq_read_rows")


def lvq_get_stats(ix) -> lvq_stats:
    st = lvq_stats()
    _chk(_lib.lvq_get_stats(ix, ctypes.byref(st)), "lvq_get_stats")
    return st


def lvq_sync(ix, stream=0) -> int:
    """Returns the sticky kernel error code (0 when none); raises nothing."""
    return _lib.lvq_sync(ix, stream)


def lvq_autotune(ix, q, nq, offsets, ids, total, level, k, stream=0):
    """(chosen shape, milliseconds per call)."""
    shape, ms = ctypes.c_int32(), ctypes.c_float()
    _chk(_lib.lvq_autotune(ix, q, nq, offsets, ids, total, level, k, ctypes.byref(shape), ctypes.byref(ms),
                           stream), "lvq_autotune")
    return shape.value, ms.value


def lvq_set_tile(ix, level, topk, shape):
    return _chk(_lib.lvq_set_tile(ix, level, topk, shape), "lvq_set_tile")


def lvq_num_tile_shapes() -> int:
    return _lib.lvq_num_tile_shapes()


def lvq_tile_shape(shape):
    """(lanes per candidate, bytes per load, loads per lane, pipeline flags)."""
    v = [ctypes.c_int32() for _ in range(4)]
    _chk(_lib.lvq_tile_shape(shape, *[ctypes.byref(x) for x in v]), "lvq_tile_shape")
    return tuple(x.value for x in v)


def lvq_set_timing(ix, enable):
    return _chk(_lib.lvq_set_timing(ix, int(enable)), "lvq_set_timing")


def lvq_kernel_time(ix):
    """(summed kernel milliseconds, launches) since the previous read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _chk(_lib.lvq_kernel_time(ix, ctypes.byref(ms), ctypes.byref(n)), "lvq_kernel_time")
    return ms.value, n.value


def lvq_server_create(ix, cfg: lvq_server_config) -> int:
    out = ctypes.c_void_p()
    _chk(_lib.lvq_server_create(ix, ctypes.byref(cfg), ctypes.byref(out)), "lvq_server_create")
    return out.value


def lvq_server_submit(sv, q_host_ptr, nq) -> int:
    t = ctypes.c_int64()
    _chk(_lib.lvq_server_submit(sv, q_host_ptr, nq, ctypes.byref(t)), "lvq_server_submit")
    return t.value


def lvq_server_wait(sv, ticket, ids_host_ptr, dist_host_ptr) -> lvq_request_info:
    """Blocks until the batch is done; returns its record (status included)."""
    info = lvq_request_info()
    _lib.lvq_server_wait(sv, ticket, ids_host_ptr, dist_host_ptr, ctypes.byref(info))
    return info


def lvq_server_drain(sv):
    return _chk(_lib.lvq_server_drain(sv), "lvq_server_drain")


def lvq_server_get_stats(sv) -> lvq_server_stats:
    st = lvq_server_stats()
    _chk(_lib.lvq_server_get_stats(sv, ctypes.byref(st)), "lvq_server_get_stats")
    return st


def lvq_server_destroy(sv):
    return _chk(_lib.lvq_server_destroy(sv), "lvq_server_destroy")


def lvq_mean(x, n, dim, out, stream=0):
    return _chk(_lib.lvq_mean(x, n, dim, out, stream), "lvq_mean")


def lvq_kmeans(x, n, dim, k, init_idx_host_ptr, iters, out, stream=0):
    return _chk(_lib.lvq_kmeans(x, n, dim, k, init_idx_host_ptr, iters, out, stream), "lvq_kmeans")


# ---- torch convenience layer ------------------------------------------------

def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t):
    return 0 if t is None else int(t.data_ptr())


class Index:
    """An LVQ store on the current GPU.  Tensors are torch CUDA tensors."""

    def __init__(self, dim, bits1, bits2=0, metric=LVQ_IP, layout=LVQ_TURBO, align=32, capacity=0,
                 means=None, mem_budget_bytes=0):
        import numpy as np
        self.cfg = lvq_config(dim, bits1, bits2, metric, layout, align, capacity, mem_budget_bytes)
        self.row_bytes, self.resid_bytes, self.code_positions = lvq_row_format(self.cfg)
        m = np.zeros((1, dim), np.float32) if means is None else np.ascontiguousarray(means, np.float32)
        if m.ndim == 1:
            m = m[None]
        self._means = m
        self.handle = lvq_create(self.cfg, m.ctypes.data, m.shape[0])
        self.dim, self.bits1, self.bits2, self.metric = dim, bits1, bits2, metric

    def close(self):
        if getattr(self, "handle", None):
            lvq_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_means(self, means, stream=None) -> int:
        import numpy as np
        m = np.ascontiguousarray(means, np.float32).reshape(-1, self.dim)
        return lvq_set_means(self.handle, m.ctypes.data, m.shape[0], _stream(stream))

    def encode(self, x, stream=None):
        import torch
        n = x.shape[0]
        rows = torch.empty((n, self.row_bytes), dtype=torch.uint8, device=x.device)
        resid = torch.empty((n, self.resid_bytes), dtype=torch.uint8, device=x.device) if self.bits2 else None
        lvq_encode(self.handle, _ptr(x), n, _ptr(rows), _ptr(resid), _stream(stream))
        return rows, resid

    def insert(self, x, ext_ids=None, stream=None):
        import torch
        n = x.shape[0]
        slots = torch.empty(n, dtype=torch.int32, device=x.device)
        lvq_insert(self.handle, _ptr(x), n, _ptr(ext_ids), _ptr(slots), _stream(stream))
        return slots

    def delete(self, slots, stream=None):
        lvq_delete(self.handle, _ptr(slots), slots.shape[0], _stream(stream))

    def consolidate(self, stream=None) -> int:
        return lvq_consolidate(self.handle, _stream(stream))

    def distances(self, q, offsets, ids, level=LVQ_PRIMARY, k=0, want_dist=True, stream=None):
        import torch
        nq = q.shape[0]
        total = ids.shape[0]
        dist = torch.empty(total, dtype=torch.float32, device=q.device) if want_dist or k == 0 else None
        ti = td = None
        if k > 0:
            ti = torch.empty((nq, k), dtype=torch.int32, device=q.device)
            td = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        lvq_distances(self.handle, _ptr(q), nq, _ptr(offsets), _ptr(ids), total, level, _ptr(dist), k,
                      _ptr(ti), _ptr(td), _stream(stream))
        return dist, ti, td

    def topk(self, q, k, level=LVQ_PRIMARY, stream=None, plain=False):
        """Exhaustive top-k; the query dtype picks the precision (plain: FP32
        on the vector ALUs only)."""
        import torch
        prec = {torch.float32: LVQ_FP32, torch.bfloat16: LVQ_BF16, torch.float16: LVQ_FP16}[q.dtype]
        if plain:
            if prec != LVQ_FP32:
                raise ValueError("plain takes float32 queries")
            prec = LVQ_FP32_VALU
        nq = q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        lvq_topk(self.handle, _ptr(q), prec, nq, k, level, _ptr(ids), _ptr(dist), _stream(stream))
        return ids, dist

    def probe_topk(self, q, nprobe, k, level=LVQ_PRIMARY, stream=None):
        """Soft inverted index: (probed means nq x nprobe, ids nq x k, values nq x k)."""
        import torch
        nq = q.shape[0]
        probe = torch.empty((nq, nprobe), dtype=torch.int32, device=q.device)
        ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        lvq_probe_topk(self.handle, _ptr(q), nq, nprobe, k, level, _ptr(probe), _ptr(ids), _ptr(dist),
                       _stream(stream))
        return probe, ids, dist

    def graph_search(self, q, graph, entries, window, k, stream=None):
        """Greedy graph search: (ids nq x k, values nq x k, counts nq x 2 --
        nodes explored, nodes scored).

        graph: (capacity x degree) contiguous int32 on the device -- the
        kernel reads the row of every slot a walk reaches."""
        import torch
        if (graph.dim() != 2 or graph.dtype != torch.int32 or not graph.is_contiguous()
                or graph.shape[0] < self.stats().capacity):
            raise LVQError(LVQ_ERR_INVALID_ARG, "graph must be a contiguous int32 (capacity x degree) tensor")
        if entries.dtype != torch.int32 or entries.dim() != 1 or not entries.is_contiguous():
            raise LVQError(LVQ_ERR_INVALID_ARG, "entries must be a contiguous int32 vector")
        nq = q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        explored = torch.empty((nq, 2), dtype=torch.int32, device=q.device)
        lvq_graph_search(self.handle, _ptr(q), nq, _ptr(graph), graph.shape[1], _ptr(entries), entries.shape[0],
                         window, k, _ptr(ids), _ptr(dist), _ptr(explored), _stream(stream))
        return ids, dist, explored

    def retire_means(self, ids, stream=None):
        import numpy as np
        ids = np.ascontiguousarray(ids, np.int32)
        lvq_retire_means(self.handle, ids.ctypes.data, ids.shape[0], _stream(stream))

    def add_means(self, means, stream=None):
        """New centres; returns their ids (freed retired ids first)."""
        import numpy as np
        means = np.ascontiguousarray(np.atleast_2d(means), np.float32)
        ids = np.zeros(means.shape[0], np.int32)
        lvq_add_means(self.handle, means.ctypes.data, means.shape[0], ids.ctypes.data, _stream(stream))
        return ids

    def mean_members(self, ids, cap, device="cuda", stream=None):
        """Live slots of the given means: (offsets n+1 host int64, slots tensor)."""
        import numpy as np
        import torch
        ids = np.ascontiguousarray(ids, np.int32)
        offs = np.zeros(ids.shape[0] + 1, np.int64)
        slots = torch.empty(max(int(cap), 1), dtype=torch.int32, device=device)
        lvq_mean_members(self.handle, ids.ctypes.data, ids.shape[0], offs.ctypes.data, _ptr(slots), int(cap),
                         _stream(stream))
        return offs, slots[:int(offs[-1])]

    def read_rows(self, slots, stream=None):
        import torch
        n = slots.shape[0]
        rows = torch.empty((n, self.row_bytes), dtype=torch.uint8, device=slots.device)
        resid = torch.empty((n, self.resid_bytes), dtype=torch.uint8, device=slots.device) if self.bits2 else None
        lvq_read_rows(self.handle, _ptr(slots), n, _ptr(rows), _ptr(resid), _stream(stream))
        return rows, resid

    def stats(self) -> lvq_stats:
        return lvq_get_stats(self.handle)

    def sync(self, stream=None) -> int:
        return lvq_sync(self.handle, _stream(stream))

    def autotune(self, q, offsets, ids, level=LVQ_PRIMARY, k=0, stream=None):
        return lvq_autotune(self.handle, _ptr(q), q.shape[0], _ptr(offsets), _ptr(ids), ids.shape[0], level, k,
                            _stream(stream))

    def set_tile(self, level, topk, shape):
        lvq_set_tile(self.handle, level, int(topk), shape)

    def tile_key(self, level, topk):
        import torch
        arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
        c = self.cfg
        return "%s|d%d|b%dx%d|layout%d|metric%d|align%d|means%s|level%d|topk%d" % (
            arch, c.dim, c.bits1, c.bits2, c.layout, c.metric, c.align,
            "1" if self._means.shape[0] == 1 else "M", level, int(bool(topk)))

    def use_tuned_tile(self, level, k, q=None, offsets=None, ids=None, retune=False, cache=TILE_CACHE):
        """Apply the tile shape recorded for this device and format in the
        tuning cache (a JSON file); when absent (or retune is set) and a
        representative batch is given, run the autotuner and record it.
        Returns the shape, or -1 when neither is available."""
        import json
        key = self.tile_key(level, k)
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table and not retune:
            shape = int(table[key]["shape"])
            self.set_tile(level, k > 0, shape)
            return shape
        if q is None:
            return -1
        shape, ms = self.autotune(q, offsets, ids, level=level, k=k)
        table[key] = {"shape": shape, "ms": round(ms, 4)}
        try:
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        except OSError:
            pass
        return shape

    def set_timing(self, enable=True):
        lvq_set_timing(self.handle, enable)

    def kernel_time(self):
        return lvq_kernel_time(self.handle)


class Server:
    """Request server over an Index (lvq_server_* of lvq.h): batches of host
    float32 queries are admitted by free stream slots and pool memory, run
    concurrently, and answered at their admission epoch."""

    def __init__(self, index: Index, slots=8, max_batch=512, k=10, k_first=64, precision=LVQ_FP32,
                 scan_level=LVQ_PRIMARY, rerank_level=LVQ_FULL, pool_bytes=0):
        self.index = index
        self.k = k
        self.cfg = lvq_server_config(slots, max_batch, k, k_first, precision, scan_level, rerank_level, pool_bytes)
        self.handle = lvq_server_create(index.handle, self.cfg)

    def submit(self, q) -> int:
        """q: host (numpy) nq x dim float32; copied before return."""
        import numpy as np
        q = np.ascontiguousarray(q, np.float32)
        return lvq_server_submit(self.handle, q.ctypes.data, q.shape[0])

    def wait(self, ticket, nq):
        """(ids nq x k int32, dist nq x k float32, record); raises on a failed batch."""
        import numpy as np
        ids = np.empty((nq, self.k), np.int32)
        dist = np.empty((nq, self.k), np.float32)
        info = lvq_server_wait(self.handle, ticket, ids.ctypes.data, dist.ctypes.data)
        if info.status != LVQ_OK:
            raise LVQError(info.status, "lvq_server_wait")
        return ids, dist, info

    def drain(self):
        lvq_server_drain(self.handle)

    def stats(self) -> lvq_server_stats:
        return lvq_server_get_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            lvq_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mean(x, stream=None):
    import torch
    out = torch.empty(x.shape[1], dtype=torch.float32, device=x.device)
    lvq_mean(_ptr(x), x.shape[0], x.shape[1], _ptr(out), _stream(stream))
    return out


def kmeans(x, k, init_idx, iters=25, stream=None):
    import numpy as np
    import torch
    idx = np.ascontiguousarray(init_idx, np.int64)
    out = torch.empty((k, x.shape[1]), dtype=torch.float32, device=x.device)
    lvq_kmeans(_ptr(x), x.shape[0], x.shape[1], k, idx.ctypes.data, iters, _ptr(out), _stream(stream))
    return out
