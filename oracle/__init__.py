"""Plain CPU oracle for GRNND graph construction (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never does; the two
share no code. See ``grnnd_oracle.c`` for the semantics and the readings of
the paper that it fixes.

Besides the C routines this module holds the numpy helpers that the checks
need: brute-force FP64 k-NN ground truth and recall.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grnnd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# GRNND_ORACLE_SANITIZE=1 builds and loads an AddressSanitizer + UBSan copy
# instead (the Python process then needs the sanitizer runtime preloaded:
# LD_PRELOAD=$(gcc -print-file-name=libasan.so))
_SANITIZE = os.environ.get("GRNND_ORACLE_SANITIZE", "") == "1"
if _SANITIZE:
    _LIB = os.path.join(_HERE, "liboracle_san.so")

L2, IP = 0, 1
DISORDERED, ASCENDING, DESCENDING = 0, 1, 2
REVERSE_HASH, REVERSE_NEAREST = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        san = (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-g",
                "-fno-omit-frame-pointer"] if _SANITIZE else [])
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", *san, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, u32, u64, f32, f64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float, C.c_double
        sig = {
            "orc_set_threads": (None, [C.c_int]),
            "orc_get_threads": (C.c_int, []),
            "orc_mix": (u64, [u64]),
            "orc_hash": (u64, [u64, u64, u64, u64]),
            "orc_dist": (f32, [P, i32, i32, i64, i64]),
            "orc_dist_exact": (f64, [P, i32, i32, i64, i64]),
            "orc_scan_vertex": (i32, [P, i32, i32, i32, P, P, i64, u64, u32, i32, f64,
                                      P, P, P, P, P, P]),
            "orc_merge": (None, [i64, i32, i64, P, P, P, P, P, P, f64, P]),
            "orc_init": (None, [P, i64, i32, i32, i32, i32, u64, P, P, f64, P]),
            "orc_update_round": (None, [P, i64, i32, i32, i32, P, P, u64, u32, i32, P, P,
                                        f64, P, P]),
            "orc_reverse_round": (None, [i64, i32, P, P, u64, u32, f32, i32, P, P]),
            "orc_finalize": (None, [P, i64, i32, i32, i32, P, P, P, P, f64, P, P]),
            "orc_build": (None, [P, i64, i32, i32, i32, i32, i32, i32, f32, i32, i32, u64, P,
                                 P, P]),
            "orc_rnn_descent_seq": (None, [P, i64, i32, i32, i32, i32, i32, i32, u64, P, P]),
            "orc_search": (None, [P, i64, i32, i32, P, i32, i64, P, i64, i32, i32, P, P]),
            "orc_medoid": (i64, [P, i64, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


MAX_R = 256  # the C routines keep one pool row on the stack (ORC_MAXR)


def _check_R(R: int) -> None:
    if not 1 <= int(R) <= MAX_R:
        raise ValueError(f"pool width R={R} outside [1, {MAX_R}]")


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def mix(x: int) -> int:
    return int(lib().orc_mix(x & (2**64 - 1)))


def hash4(seed: int, a: int, b: int, c: int) -> int:
    m = 2**64 - 1
    return int(lib().orc_hash(seed & m, a & m, b & m, c & m))


def dist(X, a: int, b: int, metric: int = L2) -> float:
    X = _f32(X)
    return float(lib().orc_dist(_p(X), X.shape[1], metric, a, b))


def dist_exact(X, a: int, b: int, metric: int = L2) -> float:
    X = _f32(X)
    return float(lib().orc_dist_exact(_p(X), X.shape[1], metric, a, b))


def scan_vertex(X, ids_row, keys_row, v: int, seed: int = 0, round: int = 0,
                order: int = DISORDERED, metric: int = L2, tau: float = 0.0):
    """Items emitted by vertex v's update: list of (dest, cand, key); plus near-tie flag."""
    X = _f32(X)
    ids_row = _i32(ids_row)
    keys_row = _f32(keys_row)
    R = ids_row.shape[0]
    _check_R(R)
    dst = np.empty(R, np.int32); cnd = np.empty(R, np.int32)
    ky = np.empty(R, np.float32); es = np.empty(R, np.float64)
    near = np.zeros(1, np.int32); ncmp = np.zeros(1, np.int64)
    k = lib().orc_scan_vertex(_p(X), X.shape[1], metric, R, _p(ids_row), _p(keys_row), v,
                              seed, round, order, tau, _p(dst), _p(cnd), _p(ky), _p(es),
                              _p(near), _p(ncmp))
    return [(int(dst[i]), int(cnd[i]), float(ky[i])) for i in range(k)], bool(near[0])


def merge(n: int, R: int, dest, cand, key, es=None, tau: float = 0.0):
    dest = _i32(dest); cand = _i32(cand); key = _f32(key)
    es = None if es is None else np.ascontiguousarray(es, dtype=np.float64)
    oi = np.empty((n, R), np.int32); ok = np.empty((n, R), np.float32)
    tag = np.zeros(n, np.uint8)
    lib().orc_merge(n, R, dest.shape[0], _p(dest), _p(cand), _p(key), _p(es), _p(oi),
                    _p(ok), tau, _p(tag))
    return oi, ok, tag.astype(bool)


def init(X, R: int, S: int | None = None, seed: int = 42, metric: int = L2,
         tau: float = 0.0):
    X = _f32(X)
    n, d = X.shape
    S = R if S is None else S
    _check_R(R)
    assert 1 <= S <= R
    oi = np.empty((n, R), np.int32); ok = np.empty((n, R), np.float32)
    tag = np.zeros(n, np.uint8)
    lib().orc_init(_p(X), n, d, metric, R, S, seed, _p(oi), _p(ok), tau, _p(tag))
    return oi, ok, tag.astype(bool)


def update_round(X, ids, keys, seed: int, round: int, order: int = DISORDERED,
                 metric: int = L2, tau: float = 0.0):
    X = _f32(X); ids = _i32(ids); keys = _f32(keys)
    n, d = X.shape
    R = ids.shape[1]
    _check_R(R)
    oi = np.empty((n, R), np.int32); ok = np.empty((n, R), np.float32)
    tag = np.zeros(n, np.uint8); st = np.zeros(8, np.int64)
    lib().orc_update_round(_p(X), n, d, metric, R, _p(ids), _p(keys), seed, round, order,
                           _p(oi), _p(ok), tau, _p(tag), _p(st))
    return oi, ok, tag.astype(bool), st


def reverse_round(ids, keys, seed: int, t1: int, rho: float = 0.6, mode: int = REVERSE_HASH):
    """Reverse-edge sampling (Section 3.6); mode REVERSE_HASH sends v to the
    floor(rho k) hash-first entries of its row, REVERSE_NEAREST to the
    floor(rho k) nearest."""
    ids = _i32(ids); keys = _f32(keys)
    n, R = ids.shape
    _check_R(R)
    oi = np.empty((n, R), np.int32); ok = np.empty((n, R), np.float32)
    lib().orc_reverse_round(n, R, _p(ids), _p(keys), seed, t1, rho, mode, _p(oi), _p(ok))
    return oi, ok


def finalize(X, ids, keys, metric: int = L2, tau: float = 0.0):
    X = _f32(X); ids = _i32(ids); keys = _f32(keys)
    n, d = X.shape
    R = ids.shape[1]
    _check_R(R)
    oa = np.empty((n, R), np.int32); ok = np.empty((n, R), np.float32)
    tag = np.zeros(n, np.uint8); st = np.zeros(8, np.int64)
    lib().orc_finalize(_p(X), n, d, metric, R, _p(ids), _p(keys), _p(oa), _p(ok), tau,
                       _p(tag), _p(st))
    return oa, ok, tag.astype(bool)


def build_graph(X, R: int, T1: int, T2: int = 4, S: int | None = None, rho: float = 0.6,
                order: int = DISORDERED, seed: int = 42, metric: int = L2,
                reverse: int = REVERSE_HASH):
    """Full construction; returns (adj, keys, stats). stats: 0 tile pairs,
    1 comparisons, 2 redirects, 3 survivors, 4 items, 5 near-tie vertices,
    6 initial distances, 7 output-pass pairs."""
    X = _f32(X)
    n, d = X.shape
    S = R if S is None else S
    _check_R(R)
    oa = np.empty((n, R), np.int32); ok = np.empty((n, R), np.float32)
    st = np.zeros(8, np.int64)
    lib().orc_build(_p(X), n, d, metric, R, S, T1, T2, rho, order, reverse, seed, _p(oa),
                    _p(ok), _p(st))
    return oa, ok, st


def rnn_descent_seq(X, R: int, T1: int, T2: int = 4, S: int | None = None, seed: int = 42,
                    metric: int = L2):
    """The sequential in-place RNN-Descent (Alg. 1 with Alg. 2's update) as a
    second reference graph; returns (adj, keys) after the same output pass."""
    X = _f32(X)
    n, d = X.shape
    S = R if S is None else S
    _check_R(R)
    oa = np.empty((n, R), np.int32); ok = np.empty((n, R), np.float32)
    lib().orc_rnn_descent_seq(_p(X), n, d, metric, R, S, T1, T2, seed, _p(oa), _p(ok))
    return oa, ok


def search(X, adj, Q, k: int = 10, L: int = 64, entry: int | None = None,
           metric: int = L2):
    X = _f32(X); Q = _f32(Q); adj = _i32(adj)
    n, d = X.shape
    R = adj.shape[1]
    if entry is None:
        entry = medoid(X)
    nq = Q.shape[0]
    oi = np.empty((nq, k), np.int32); ok = np.empty((nq, k), np.float32)
    lib().orc_search(_p(X), n, d, metric, _p(adj), R, entry, _p(Q), nq, k, L, _p(oi),
                     _p(ok))
    return oi, ok


def medoid(X) -> int:
    X = _f32(X)
    return int(lib().orc_medoid(_p(X), X.shape[0], X.shape[1]))


# ----------------------------------------------------------------- numpy helpers
def _knn_candidates(X64, xn, q, k, metric):
    """Ids of every point whose Gram-form FP64 key is within a rounding
    tolerance of the k-th smallest such key: a superset of the exact k
    nearest and of every point tied with the k-th (the Gram form's error is
    below 1e-12 of the squared norms involved)."""
    if metric == L2:
        qn = (q * q).sum(1)
        dd = qn[:, None] + xn[None, :] - 2.0 * (q @ X64.T)
        tol = 1e-9 * (qn + xn.max() + 1.0)
    else:
        dd = -(q @ X64.T)
        tol = 1e-9 * (np.abs(q).sum(1) * np.abs(X64).max() * X64.shape[1] + 1.0)
    kk = min(k, dd.shape[1]) - 1
    thr = np.partition(dd, kk, axis=1)[:, kk] + tol
    return [np.nonzero(dd[r] <= thr[r])[0] for r in range(q.shape[0])]


def _exact_keys(X64, c, qr, metric):
    return ((X64[c] - qr) ** 2).sum(1) if metric == L2 else -(X64[c] @ qr)


def knn_exact(X, Q, k: int = 10, metric: int = L2, block: int = 256):
    """Brute-force FP64 k-NN of each query: (ids, dists), the first k of all
    points in (exact direct-form FP64 distance, id) order."""
    X64 = np.asarray(X, dtype=np.float64)
    Q64 = np.asarray(Q, dtype=np.float64)
    xn = (X64 * X64).sum(1)
    ids = np.empty((Q64.shape[0], k), np.int64)
    ds = np.empty((Q64.shape[0], k), np.float64)
    for b0 in range(0, Q64.shape[0], block):
        q = Q64[b0:b0 + block]
        for r, c in enumerate(_knn_candidates(X64, xn, q, k, metric)):
            e = _exact_keys(X64, c, q[r], metric)
            o = np.lexsort((c, e))[:k]
            ids[b0 + r] = c[o]
            ds[b0 + r] = e[o]
    return ids, ds


def knn_kth_dist(X, Q, k: int = 10, metric: int = L2, block: int = 256):
    """Exact FP64 distance of the k-th nearest neighbour of every query."""
    X64 = np.asarray(X, dtype=np.float64)
    Q64 = np.asarray(Q, dtype=np.float64)
    xn = (X64 * X64).sum(1)
    out = np.empty(Q64.shape[0], np.float64)
    for b0 in range(0, Q64.shape[0], block):
        q = Q64[b0:b0 + block]
        for r, c in enumerate(_knn_candidates(X64, xn, q, k, metric)):
            out[b0 + r] = np.sort(_exact_keys(X64, c, q[r], metric))[k - 1]
    return out


def recall_at_k(X, Q, found_ids, kth, k: int = 10, metric: int = L2):
    """Tie-aware Recall@k: a returned id counts if its exact FP64 distance is
    <= the exact k-th nearest distance (Section 2.1 defines recall as the
    fraction of true nearest neighbours retrieved; ties are counted as hits)."""
    X64 = np.asarray(X, dtype=np.float64)
    Q64 = np.asarray(Q, dtype=np.float64)
    hits = 0
    for r in range(Q64.shape[0]):
        ids = np.asarray(found_ids[r][:k])
        ids = ids[ids >= 0]
        if ids.size == 0:
            continue
        if metric == L2:
            e = ((X64[ids] - Q64[r]) ** 2).sum(1)
        else:
            e = -(X64[ids] @ Q64[r])
        hits += int((e <= kth[r] * (1 + 1e-12) + 1e-12).sum())
    return hits / (k * Q64.shape[0])


def check_invariants(X, adj, keys=None, metric: int = L2, exact: bool = False,
                     rtol: float = 1e-5):
    """Invariants of an output graph: ids in range, no self loops, no
    duplicates, rows padded at the end, degree >= 1, keys equal to the
    distances, rows sorted by (key, id), and every kept pair meets Eq. 1
    (d(u,w) >= max(key_u, key_w)). With exact=False the key and Eq. 1
    comparisons allow rtol of the distance's natural scale: |key| for L2,
    |x_u| |x_w| for the inner product."""
    X = _f32(X)
    n, R = adj.shape
    L = lib()
    nrm = np.sqrt((X.astype(np.float64) ** 2).sum(1))

    def scale(a, b, val):
        return abs(val) if metric == L2 else nrm[a] * nrm[b]

    for v in range(n):
        row = adj[v]
        valid = row >= 0
        k = int(valid.sum())
        assert k >= 1, f"vertex {v} has no neighbour"
        assert valid[:k].all() and not valid[k:].any(), f"row {v} not -1 padded at the end"
        ids = row[:k]
        assert ((ids >= 0) & (ids < n)).all(), f"row {v} holds ids outside [0, n)"
        assert (ids != v).all(), f"self loop at {v}"
        assert len(set(ids.tolist())) == k, f"duplicate in row {v}"
        dk = np.array([L.orc_dist(_p(X), X.shape[1], metric, v, int(u)) for u in ids],
                      np.float32)
        if keys is not None:
            kk = keys[v, :k]
            if exact:
                assert np.array_equal(kk, dk), f"keys of row {v} differ from distances"
            else:
                for i, u in enumerate(ids):
                    assert abs(kk[i] - dk[i]) <= rtol * scale(v, u, dk[i]), (v, i)
            for i in range(k - 1):
                assert (kk[i], ids[i]) < (kk[i + 1], ids[i + 1]), f"row {v} not sorted"
        else:
            kk = dk
        for i in range(k):
            for j in range(i):
                dij = L.orc_dist(_p(X), X.shape[1], metric, int(ids[i]), int(ids[j]))
                thr = max(kk[i], kk[j])
                if exact:
                    assert dij >= thr, f"row {v}: kept pair ({ids[j]},{ids[i]}) violates Eq. 1"
                else:
                    tol = 4 * rtol * scale(int(ids[i]), int(ids[j]), thr)
                    assert dij >= thr - tol, (v, i, j)
    return True
