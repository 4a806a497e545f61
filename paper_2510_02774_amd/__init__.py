"""MI355X (gfx950) GRNND graph construction -- Python binding of libgrnnd.so.

Every function here marshals arguments to the C ABI declared in
``include/grnnd.h`` and calls it; all computation runs in the library's HIP
kernels. PyTorch supplies device memory and the current HIP stream only.
If the library has not been built, importing the binding fails loudly: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

__all__ = [
    "GrnndError", "Params", "lib",
    "grnnd_version", "grnnd_last_error", "grnnd_params_default", "grnnd_workspace_size",
    "grnnd_build", "grnnd_build_ex", "grnnd_build_noalloc", "NOALLOC_SCRATCH_BYTES",
    "grnnd_init_pools", "grnnd_step", "grnnd_finalize",
    "grnnd_tile_probe", "tile_probe",
    "grnnd_search_workspace_size", "grnnd_search", "grnnd_medoid", "medoid", "grnnd_profile_enable", "grnnd_profile_read",
    "METRIC_L2", "METRIC_IP", "ORDER_DISORDERED", "ORDER_ASCENDING", "ORDER_DESCENDING",
    "STEP_UPDATE", "STEP_REVERSE", "NSTATS", "STAT_NAMES",
    "PREC_FP32", "PREC_BF16", "PREC_FP16", "PREC_FP8_E4M3", "REVERSE_HASH", "REVERSE_NEAREST",
    "workspace", "build_graph", "search",
    "Request", "ServerStats", "grnnd_server_create", "grnnd_server_submit", "grnnd_server_poll",
    "grnnd_server_drain", "grnnd_server_stats_read", "grnnd_server_destroy", "Server",
    "grnnd_server_set_batch", "grnnd_batch_workspace_size", "grnnd_build_batch", "BatchItem",
    "build_batch",
    "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgrnnd.so")

METRIC_L2, METRIC_IP = 0, 1
ORDER_DISORDERED, ORDER_ASCENDING, ORDER_DESCENDING = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_FP16, PREC_FP8_E4M3 = 0, 1, 2, 3
REVERSE_HASH, REVERSE_NEAREST = 0, 1
STEP_UPDATE, STEP_REVERSE = 0, 1
NSTATS = 11
STAT_NAMES = ["tile_pairs", "rechecks", "redirects", "survivors", "items", "candidates",
              "init_dists", "final_pairs", "overflow_items", "long_merges", "deferred_keys"]
_CODES = {-1: "EINVAL", -2: "ENOSPACE", -3: "EDEVICE", -4: "EBUDGET", -5: "ENOTSUP"}
REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2


class GrnndError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("S", C.c_int32), ("T1", C.c_int32), ("T2", C.c_int32), ("rho", C.c_float),
                ("order", C.c_int32), ("precision", C.c_int32), ("reverse", C.c_int32),
                ("check", C.c_int32)]

    def __repr__(self):
        return (f"Params(S={self.S}, T1={self.T1}, T2={self.T2}, rho={self.rho:.3f}, "
                f"order={self.order}, precision={self.precision}, reverse={self.reverse}, "
                f"check={self.check})")


class Request(C.Structure):
    _fields_ = [("points", C.c_void_p), ("n", C.c_int64), ("d", C.c_int32),
                ("metric", C.c_int32), ("R", C.c_int32), ("params", C.POINTER(Params)),
                ("seed", C.c_uint64), ("out_adj", C.c_void_p), ("out_keys", C.c_void_p)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("peak_inflight", C.c_int64), ("peak_arena_bytes", C.c_uint64),
                ("batches", C.c_int64), ("batched_requests", C.c_int64)]


class BatchItem(C.Structure):
    _fields_ = [("points", C.c_void_p), ("n", C.c_int64), ("seed", C.c_uint64),
                ("out_adj", C.c_void_p), ("out_keys", C.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2510_02774_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_size_t
    PP = C.POINTER(Params)
    sig = {
        "grnnd_version": (C.c_int, []),
        "grnnd_last_error": (C.c_char_p, []),
        "grnnd_params_default": (C.c_int, [PP, i32, i32]),
        "grnnd_workspace_size": (C.c_int, [i64, i32, i32, PP, C.POINTER(sz)]),
        "grnnd_build": (C.c_int, [P, i64, i32, i32, i32, i32, u64, P, P, sz, P]),
        "grnnd_build_ex": (C.c_int, [P, i64, i32, i32, i32, PP, u64, P, P, P, P, sz, P]),
        "grnnd_build_noalloc": (C.c_int, [P, i64, i32, i32, i32, PP, u64, P, P, P, P]),
        "grnnd_batch_workspace_size": (C.c_int, [C.POINTER(i64), i32, i32, i32, PP,
                                                 C.POINTER(sz)]),
        "grnnd_build_batch": (C.c_int, [C.POINTER(BatchItem), i32, i32, i32, i32, PP, P, P, sz,
                                        P]),
        "grnnd_server_set_batch": (C.c_int, [P, i32, i64]),
        "grnnd_init_pools": (C.c_int, [P, i64, i32, i32, i32, i32, u64, P, P, P, P, sz, P]),
        "grnnd_step": (C.c_int, [P, i64, i32, i32, i32, P, P, P, P, u64, u32, i32, PP, P, P,
                                 sz, P]),
        "grnnd_finalize": (C.c_int, [P, i64, i32, i32, i32, P, P, P, P, P, P, sz, P]),
        "grnnd_tile_probe": (C.c_int, [P, i64, i32, i32, i32, PP, P, i64, P, P, P, P, sz, P]),
        "grnnd_search_workspace_size": (C.c_int, [i64, i32, i64, C.POINTER(sz)]),
        "grnnd_medoid": (C.c_int, [P, i64, i32, P, P, sz, P]),
        "grnnd_search": (C.c_int, [P, i64, i32, i32, P, i32, i64, P, i64, i32, i32, P, P, P,
                                   sz, P]),
        "grnnd_profile_enable": (C.c_int, [C.c_int]),
        "grnnd_server_create": (C.c_int, [P, sz, i32, C.POINTER(C.c_void_p)]),
        "grnnd_server_submit": (C.c_int, [P, C.POINTER(Request), C.POINTER(u64)]),
        "grnnd_server_poll": (C.c_int, [P, u64, C.POINTER(i32), C.POINTER(C.c_double)]),
        "grnnd_server_drain": (C.c_int, [P]),
        "grnnd_server_stats_read": (C.c_int, [P, C.POINTER(ServerStats)]),
        "grnnd_server_destroy": (C.c_int, [P]),
        "grnnd_profile_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


# ---------------------------------------------------------------- marshalling
def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError("tensors passed to libgrnnd must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to libgrnnd must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check(rc: int):
    if rc != 0:
        raise GrnndError(rc, lib().grnnd_last_error().decode())


def _params(p):
    if p is None:
        return None
    return C.byref(p)


# ----------------------------------------------------------- C ABI, same names
def grnnd_version() -> int:
    return int(lib().grnnd_version())


def grnnd_last_error() -> str:
    return lib().grnnd_last_error().decode()


def grnnd_params_default(R: int, iters: int) -> Params:
    p = Params()
    _check(lib().grnnd_params_default(C.byref(p), R, iters))
    return p


def grnnd_workspace_size(n: int, d: int, R: int, params: Params | None = None) -> int:
    b = C.c_size_t(0)
    _check(lib().grnnd_workspace_size(n, d, R, _params(params), C.byref(b)))
    return int(b.value)


def grnnd_build(points, metric, R, iters, seed, out_adj, workspace, stream=None):
    n, d = points.shape
    _check(lib().grnnd_build(_ptr(points), n, d, metric, R, iters, seed, _ptr(out_adj),
                             _ptr(workspace), workspace.numel() * workspace.element_size(),
                             _stream(stream)))


def grnnd_build_ex(points, metric, R, params, seed, out_adj, out_keys, dev_stats, workspace,
                   stream=None):
    n, d = points.shape
    _check(lib().grnnd_build_ex(_ptr(points), n, d, metric, R, _params(params), seed,
                                _ptr(out_adj), _ptr(out_keys), _ptr(dev_stats), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 128 << 20


def grnnd_build_noalloc(points, metric, R, params, seed, out_adj, out_keys, dev_stats,
                        stream=None):
    n, d = points.shape
    _check(lib().grnnd_build_noalloc(_ptr(points), n, d, metric, R, _params(params), seed,
                                     _ptr(out_adj), _ptr(out_keys), _ptr(dev_stats),
                                     _stream(stream)))


def grnnd_batch_workspace_size(ns, d: int, R: int, params: Params | None = None) -> int:
    arr = (C.c_int64 * len(ns))(*[int(x) for x in ns])
    b = C.c_size_t(0)
    _check(lib().grnnd_batch_workspace_size(arr, len(ns), d, R, _params(params), C.byref(b)))
    return int(b.value)


def grnnd_build_batch(items, d, metric, R, params, dev_stats, workspace, stream=None):
    """items: sequence of (points, seed, out_adj, out_keys or None) with device tensors."""
    arr = (BatchItem * len(items))()
    for i, (X, seed, adj, keys) in enumerate(items):
        if X.shape[1] != d:
            raise ValueError("every collection of a batch has the same d")
        arr[i] = BatchItem(points=_ptr(X), n=X.shape[0], seed=seed, out_adj=_ptr(adj),
                           out_keys=_ptr(keys) if keys is not None else None)
    _check(lib().grnnd_build_batch(arr, len(items), d, metric, R, _params(params),
                                   _ptr(dev_stats), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(),
                                   _stream(stream)))


def build_batch(points_list, R: int, params: Params | None = None, seeds=None,
                metric: int = METRIC_L2):
    """One batched build over several collections of the same d; returns
    [(adj, keys)] per collection."""
    d = points_list[0].shape[1]
    if params is None:
        params = grnnd_params_default(R, 4)
    seeds = seeds or [42] * len(points_list)
    dev = points_list[0].device
    ws = workspace(grnnd_batch_workspace_size([X.shape[0] for X in points_list], d, R, params),
                   dev)
    outs = [(torch.empty((X.shape[0], R), dtype=torch.int32, device=dev),
             torch.empty((X.shape[0], R), dtype=torch.float32, device=dev)) for X in points_list]
    grnnd_build_batch([(X, s, a, k) for X, s, (a, k) in zip(points_list, seeds, outs)], d, metric,
                      R, params, None, ws)
    return outs


def grnnd_init_pools(points, metric, R, S, seed, out_ids, out_keys, dev_stats, workspace,
                     stream=None):
    n, d = points.shape
    _check(lib().grnnd_init_pools(_ptr(points), n, d, metric, R, S, seed, _ptr(out_ids),
                                  _ptr(out_keys), _ptr(dev_stats), _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), _stream(stream)))


def grnnd_step(points, metric, R, in_ids, in_keys, out_ids, out_keys, seed, round, kind,
               params, dev_stats, workspace, stream=None):
    n, d = points.shape
    _check(lib().grnnd_step(_ptr(points), n, d, metric, R, _ptr(in_ids), _ptr(in_keys),
                            _ptr(out_ids), _ptr(out_keys), seed, round, kind, _params(params),
                            _ptr(dev_stats), _ptr(workspace),
                            workspace.numel() * workspace.element_size(), _stream(stream)))


def grnnd_finalize(points, metric, R, in_ids, in_keys, out_adj, out_keys, dev_stats,
                   workspace, stream=None):
    n, d = points.shape
    _check(lib().grnnd_finalize(_ptr(points), n, d, metric, R, _ptr(in_ids), _ptr(in_keys),
                                _ptr(out_adj), _ptr(out_keys), _ptr(dev_stats), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream)))


def grnnd_tile_probe(points, metric, R, params, ids, out_tile, out_band, out_canon, workspace,
                     stream=None):
    n, d = points.shape
    nv = ids.shape[0]
    _check(lib().grnnd_tile_probe(_ptr(points), n, d, metric, R, _params(params), _ptr(ids), nv,
                                  _ptr(out_tile), _ptr(out_band), _ptr(out_canon),
                                  _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _stream(stream)))


def tile_probe(points: torch.Tensor, ids: torch.Tensor, params: Params | None = None,
               metric: int = METRIC_L2):
    """Tile distance, recheck band and canonical distance of every ordered
    pair of each candidate set (rows of ids); unwritten entries are NaN."""
    n, d = points.shape
    nv, R = ids.shape
    if params is None:
        params = grnnd_params_default(R, 4)
    ws = workspace(grnnd_workspace_size(n, d, R, params), points.device)
    outs = [torch.full((nv, R, R), float("nan"), dtype=torch.float32, device=points.device)
            for _ in range(3)]
    grnnd_tile_probe(points, metric, R, params, ids, *outs, ws)
    return tuple(outs)


def grnnd_search_workspace_size(n: int, d: int, nq: int) -> int:
    b = C.c_size_t(0)
    _check(lib().grnnd_search_workspace_size(n, d, nq, C.byref(b)))
    return int(b.value)


def grnnd_search(points, metric, adj, entry, queries, k, L, out_ids, out_keys, workspace,
                 stream=None):
    n, d = points.shape
    R = adj.shape[1]
    nq = queries.shape[0]
    ws_ptr = _ptr(workspace) if workspace is not None else None
    ws_b = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().grnnd_search(_ptr(points), n, d, metric, _ptr(adj), R, entry, _ptr(queries), nq,
                              k, L, _ptr(out_ids), _ptr(out_keys), ws_ptr, ws_b,
                              _stream(stream)))


def grnnd_medoid(points, out_entry, workspace, stream=None):
    n, d = points.shape
    _check(lib().grnnd_medoid(_ptr(points), n, d, _ptr(out_entry), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream)))


def medoid(points: torch.Tensor) -> torch.Tensor:
    """Device int64 tensor (1,) holding the approximate medoid's id."""
    n, d = points.shape
    ws = workspace(grnnd_search_workspace_size(n, d, 0), points.device)
    out = torch.empty(1, dtype=torch.int64, device=points.device)
    grnnd_medoid(points, out, ws)
    return out


PROF_NAMES = ["init", "update", "merge", "reverse", "final", "search"]


def grnnd_profile_enable(on: bool) -> None:
    _check(lib().grnnd_profile_enable(1 if on else 0))


def grnnd_profile_read() -> dict:
    """{kernel class: (total ms, launches)} of the launches timed since the
    last read; waits for their events."""
    ms = (C.c_double * len(PROF_NAMES))()
    cnt = (C.c_int64 * len(PROF_NAMES))()
    _check(lib().grnnd_profile_read(ms, cnt))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROF_NAMES)}


# ---------------------------------------------------------- allocation helpers
def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """A device byte buffer usable as a workspace (256-byte aligned by torch)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def build_graph(points: torch.Tensor, R: int, params: Params | None = None, seed: int = 42,
                metric: int = METRIC_L2, stats: bool = False):
    """Allocates outputs and workspace, runs grnnd_build_ex on the current
    stream and returns (adj, keys[, stats])."""
    n, d = points.shape
    if params is None:
        params = grnnd_params_default(R, 4)
    ws = workspace(grnnd_workspace_size(n, d, R, params), points.device)
    adj = torch.empty((n, R), dtype=torch.int32, device=points.device)
    keys = torch.empty((n, R), dtype=torch.float32, device=points.device)
    st = torch.zeros(NSTATS, dtype=torch.int64, device=points.device)
    grnnd_build_ex(points, metric, R, params, seed, adj, keys, st, ws)
    return (adj, keys, st) if stats else (adj, keys)


def search(points: torch.Tensor, adj: torch.Tensor, queries: torch.Tensor, k: int = 10,
           L: int = 64, entry: int = -1, metric: int = METRIC_L2):
    """grnnd_search with fresh outputs; entry -1 starts from the medoid."""
    n, d = points.shape
    nq = queries.shape[0]
    ws = workspace(grnnd_search_workspace_size(n, d, nq), points.device)
    ids = torch.empty((nq, k), dtype=torch.int32, device=points.device)
    keys = torch.empty((nq, k), dtype=torch.float32, device=points.device)
    grnnd_search(points, metric, adj, entry, queries, k, L, ids, keys, ws)
    return ids, keys


# ------------------------------------------------------------- build server
def grnnd_server_create(arena: torch.Tensor, slots: int = 4):
    """Server over a device arena tensor (its bytes are the budget)."""
    h = C.c_void_p()
    _check(lib().grnnd_server_create(_ptr(arena), arena.numel() * arena.element_size(), slots,
                                     C.byref(h)))
    return h


def grnnd_server_submit(server, req: Request) -> int:
    t = C.c_uint64(0)
    _check(lib().grnnd_server_submit(server, C.byref(req), C.byref(t)))
    return int(t.value)


def grnnd_server_poll(server, ticket: int):
    st, lat = C.c_int32(0), C.c_double(0.0)
    _check(lib().grnnd_server_poll(server, ticket, C.byref(st), C.byref(lat)))
    return int(st.value), float(lat.value)


def grnnd_server_set_batch(server, max_requests: int, max_points: int):
    _check(lib().grnnd_server_set_batch(server, max_requests, max_points))


def grnnd_server_drain(server):
    _check(lib().grnnd_server_drain(server))


def grnnd_server_stats_read(server) -> ServerStats:
    out = ServerStats()
    _check(lib().grnnd_server_stats_read(server, C.byref(out)))
    return out


def grnnd_server_destroy(server):
    _check(lib().grnnd_server_destroy(server))


class Server:
    """Owns a device arena and a server; keeps every submitted request's
    tensors alive until the server is closed."""

    def __init__(self, budget_bytes: int, slots: int = 4, device=None):
        self.arena = torch.empty(budget_bytes, dtype=torch.uint8, device=device or "cuda")
        self.h = grnnd_server_create(self.arena, slots)
        self._keep = {}

    def submit(self, points: torch.Tensor, R: int, params: Params | None = None, seed: int = 42,
               metric: int = METRIC_L2, keys: bool = True):
        n, d = points.shape
        adj = torch.empty((n, R), dtype=torch.int32, device=points.device)
        kk = torch.empty((n, R), dtype=torch.float32, device=points.device) if keys else None
        pp = C.pointer(params) if params is not None else None
        req = Request(points=_ptr(points), n=n, d=d, metric=metric, R=R, params=pp, seed=seed,
                      out_adj=_ptr(adj), out_keys=_ptr(kk) if kk is not None else None)
        # the server's streams do not wait for torch's: the points must be
        # complete before the request is queued
        torch.cuda.current_stream(points.device).synchronize()
        t = grnnd_server_submit(self.h, req)
        self._keep[t] = (points, adj, kk, params)
        return t, adj, kk

    def set_batch(self, max_requests: int, max_points: int = 1 << 18):
        grnnd_server_set_batch(self.h, max_requests, max_points)

    def poll(self, ticket: int):
        return grnnd_server_poll(self.h, ticket)

    def drain(self):
        grnnd_server_drain(self.h)

    def stats(self) -> ServerStats:
        return grnnd_server_stats_read(self.h)

    def close(self):
        if self.h is not None:
            grnnd_server_destroy(self.h)
            self.h = None
            self._keep.clear()
            self.arena = None  # the budget's device memory goes back to torch
