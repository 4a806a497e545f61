"""Pins of the oracle's checking helpers: the invariant checker, exact k-NN
ground truth and Recall@k, bounded-list search, the medoid, and near-tie tags.

Every claim the GPU tests make ("invariants exact", "recall within 0.5
points") goes through these helpers, so each is held to something other than
itself: hand-built graphs that break one invariant at a time, brute-force
distances of every point, search results worked out by hand on small graphs,
and ties built on purpose.
"""
import numpy as np
import pytest

import datagen


# ------------------------------------------------------- invariant checker
@pytest.fixture(scope="module")
def good_graph(orc):
    X = datagen.sift_like(400, d=16, k=8, seed=13)
    adj, keys, _ = orc.build_graph(X, R=12, T1=2, T2=2, seed=3)
    assert orc.check_invariants(X, adj, keys, exact=True)
    return X, adj, keys


def _row_with(adj, keys, minlen=2):
    for v in range(adj.shape[0]):
        if (adj[v] >= 0).sum() >= minlen:
            return v
    raise AssertionError("no row long enough")


def _fails(orc, X, adj, keys, **kw):
    with pytest.raises(AssertionError):
        orc.check_invariants(X, adj, keys, **kw)


def test_check_invariants_rejects_self_loop(orc, good_graph):
    X, adj, keys = good_graph
    a, k = adj.copy(), keys.copy()
    v = _row_with(a, k)
    a[v, 0] = v
    k[v, 0] = 0.0
    _fails(orc, X, a, k, exact=True)
    _fails(orc, X, a, None, exact=True)


def test_check_invariants_rejects_duplicate(orc, good_graph):
    X, adj, keys = good_graph
    a, k = adj.copy(), keys.copy()
    v = _row_with(a, k)
    a[v, 1] = a[v, 0]
    k[v, 1] = k[v, 0]
    _fails(orc, X, a, k, exact=True)


def test_check_invariants_rejects_unsorted_row(orc, good_graph):
    X, adj, keys = good_graph
    a, k = adj.copy(), keys.copy()
    v = _row_with(a, k)
    a[v, [0, 1]] = a[v, [1, 0]]
    k[v, [0, 1]] = k[v, [1, 0]]
    _fails(orc, X, a, k, exact=True)


def test_check_invariants_rejects_wrong_key(orc, good_graph):
    X, adj, keys = good_graph
    a, k = adj.copy(), keys.copy()
    v = _row_with(a, k, 1)
    k[v, 0] = np.nextafter(k[v, 0], np.float32(np.inf))
    _fails(orc, X, a, k, exact=True)
    k2 = keys.copy()
    k2[v, 0] = k2[v, 0] * 1.5 + 1.0
    _fails(orc, X, a, k2, exact=False)


def test_check_invariants_rejects_padding_and_range(orc, good_graph):
    X, adj, keys = good_graph
    v = _row_with(adj, keys, 2)
    a, k = adj.copy(), keys.copy()
    a[v, 0] = -1                                  # hole before a valid entry
    _fails(orc, X, a, k, exact=True)
    a, k = adj.copy(), keys.copy()
    a[v, :] = -1                                  # no neighbour at all
    k[v, :] = np.inf
    _fails(orc, X, a, k, exact=True)
    a = adj.copy()
    a[v, 0] = X.shape[0]                          # id outside [0, n)
    _fails(orc, X, a, None, exact=True)


def test_check_invariants_rejects_eq1_violation(orc):
    """A row holding two neighbours u, w with d(u, w) < max(key_u, key_w):
    points on a line, v = 0 at the origin with 1 and 2 on the same side."""
    X = np.array([[0.0], [1.0], [3.0], [-2.0]], np.float32)
    good = np.array([[1, 3], [0, 2], [1, -1], [0, -1]], np.int32)
    keys = np.array([[1, 4], [1, 4], [4, np.inf], [4, np.inf]], np.float32)
    assert orc.check_invariants(X, good, keys, exact=True)
    bad = good.copy()
    bk = keys.copy()
    bad[0] = [1, 2]                               # d(1, 2) = 4 < max(1, 9)
    bk[0] = [1, 9]
    _fails(orc, X, bad, bk, exact=True)
    _fails(orc, X, bad, None, exact=True)
    _fails(orc, X, bad, bk, exact=False)


# --------------------------------------------- ground truth and Recall@k
def _tie_heavy(seed=4, n=300, nq=40, d=3):
    rng = np.random.default_rng(seed)
    X = rng.integers(0, 3, size=(n, d)).astype(np.float32)       # 27 cells, many repeats
    Q = rng.integers(0, 3, size=(nq, d)).astype(np.float32)
    return X, Q


def _brute(X, q, metric):
    X64, q64 = X.astype(np.float64), q.astype(np.float64)
    return ((X64 - q64) ** 2).sum(1) if metric == 0 else -(X64 @ q64)


@pytest.mark.parametrize("metric", [0, 1])
def test_knn_helpers_equal_brute_force_on_ties(orc, metric):
    """knn_exact's ids are the first k of all points sorted by (exact
    distance, id), and knn_kth_dist is the k-th of all exact distances, on
    integer data where most distances are tied."""
    X, Q = _tie_heavy()
    k = 10
    ids, ds = orc.knn_exact(X, Q, k, metric=metric)
    kth = orc.knn_kth_dist(X, Q, k, metric=metric)
    for r in range(Q.shape[0]):
        e = _brute(X, Q[r], metric)
        order = np.lexsort((np.arange(X.shape[0]), e))
        assert ids[r].tolist() == order[:k].tolist()
        assert np.array_equal(ds[r], e[order[:k]])
        assert kth[r] == np.sort(e)[k - 1]


def test_knn_kth_dist_small_sets(orc):
    """Fewer points than k + 8 candidates: still the k-th exact distance."""
    X = np.arange(12, dtype=np.float32)[:, None]
    Q = np.array([[0.2], [11.0]], np.float32)
    kth = orc.knn_kth_dist(X, Q, 10)
    assert kth.tolist() == [(9.0 - np.float64(np.float32(0.2))) ** 2, 81.0]


def test_recall_hand_counted(orc):
    """Tie-aware Recall@k on a line: a returned id counts when its exact
    distance is at most the k-th true distance, padding never counts."""
    X = np.array([[0.0], [1.0], [-1.0], [2.0], [5.0], [-6.0]], np.float32)
    Q = np.array([[0.0], [0.0]], np.float32)
    kth = orc.knn_kth_dist(X, Q, 2)                # distances 0, 1, 1, 4, ...: kth = 1
    assert kth.tolist() == [1.0, 1.0]
    # query 0 returns {0, 2}: both within the tie at distance 1 -> 2 hits;
    # query 1 returns {3, -1}: distance 4 > 1 and padding -> 0 hits
    found = np.array([[0, 2], [3, -1]])
    assert orc.recall_at_k(X, Q, found, kth, k=2) == 2 / 4
    found = np.array([[1, 2], [0, 1]])
    assert orc.recall_at_k(X, Q, found, kth, k=2) == 1.0
    found = np.array([[4, 5], [5, 4]])
    assert orc.recall_at_k(X, Q, found, kth, k=2) == 0.0


# ------------------------------------------------------ bounded-list search
def test_search_bounded_list_by_hand(orc):
    """Best-first search with L smaller than the graph on a graph built to
    trap a short list. Points on a line: A=0 (entry), B=4, C=-3, D=8; edges
    A->{B, C}, B->{A}, C->{D}, D->{C}; query at 8 (keys A 64, B 16, C 121,
    D 0). L = 1 and L = 2 drop C when A is expanded (B is closer, C does not
    fit or is not better), so D is never reached: the answer is B. With
    L = 3, C is kept, expanded after B, and reaches D."""
    X = np.array([[0.0], [4.0], [-3.0], [8.0]], np.float32)
    adj = np.array([[1, 2], [0, -1], [3, -1], [2, -1]], np.int32)
    Q = np.array([[8.0]], np.float32)
    for L, want in ((1, [1]), (2, [1, 0]), (3, [3, 1, 0]), (4, [3, 1, 0, 2])):
        ids, keys = orc.search(X, adj, Q, k=L, L=L, entry=0)
        assert ids[0].tolist() == want, (L, ids)
    ids, keys = orc.search(X, adj, Q, k=3, L=2, entry=0)
    assert ids[0].tolist() == [1, 0, -1] and np.isinf(keys[0, 2])


def test_search_path_graph_short_list(orc):
    """A path graph 0 - 1 - ... - 99 on a line, entry 0, L = 4: the search
    walks the path and stops after the four points nearest to the query."""
    n = 100
    X = np.arange(n, dtype=np.float32)[:, None]
    adj = np.full((n, 2), -1, np.int32)
    for i in range(n):
        nb = [j for j in (i - 1, i + 1) if 0 <= j < n]
        adj[i, :len(nb)] = nb
    Q = np.array([[57.3], [-5.0], [120.0]], np.float32)
    ids, keys = orc.search(X, adj, Q, k=4, L=4, entry=0)
    assert ids[0].tolist() == [57, 58, 56, 59]
    assert ids[1].tolist() == [0, 1, 2, 3]
    assert ids[2].tolist() == [99, 98, 97, 96]
    q = np.float64(np.float32(57.3))
    assert keys[0].tolist() == [np.float32((q - v) ** 2) for v in (57, 58, 56, 59)]


def test_medoid_ties_and_mean(orc):
    """Nearest point to the mean, ties broken by the smaller id."""
    assert orc.medoid(np.array([[-1.0], [1.0]], np.float32)) == 0
    assert orc.medoid(np.array([[1.0], [-1.0]], np.float32)) == 0
    X = np.array([[0, 0], [4, 0], [0, 4], [4, 4], [2, 2], [2.1, 2]], np.float32)
    assert orc.medoid(X) == 4                       # mean (2.01667, 2): 4 is nearer than 5
    X = np.array([[10, 10], [0, 0], [1, 1], [2, 2]], np.float32)
    assert orc.medoid(X) == 3                       # mean (3.25, 3.25)


# --------------------------------------------------------- near-tie tags
def test_near_tie_tag_on_exact_merge_tie(orc):
    """Two items for the same destination with exactly equal keys at the
    capacity cut: (key, id) keeps the smaller id, and the row is tagged as
    rounding-dependent when tau > 0 -- raising the kept one's key by one ulp
    indeed swaps the result. Keys apart by much more than tau times their
    scale are not tagged."""
    dest = [0, 0, 1, 1]
    cand = [5, 3, 2, 4]
    key = np.array([2.0, 2.0, 1.0, 3.0], np.float32)
    es = [2.0, 2.0, 1.0, 3.0]
    oi, ok, tag = orc.merge(6, 1, dest, cand, key, es, tau=1e-6)
    assert oi[0].tolist() == [3] and oi[1].tolist() == [2]
    assert tag[0] and not tag[1] and not tag[2:].any()
    k2 = key.copy()
    k2[1] = np.nextafter(k2[1], np.float32(np.inf))
    oi2, _, _ = orc.merge(6, 1, dest, cand, k2, es, tau=1e-6)
    assert oi2[0].tolist() == [5]
    _, _, tag0 = orc.merge(6, 1, dest, cand, key, es, tau=0.0)
    assert not tag0.any()


def test_near_tie_tag_propagates_from_scan(orc):
    """A near tie inside v's scan tags v and every vertex v could send an
    item to (its pool members); vertices not touched by v stay untagged."""
    # v = 0 at the origin; d(1, 2) = 5 = key_2 exactly (strict test: kept)
    X = np.array([[0, 0], [2, 0], [1, 2], [40, 40], [43, 40], [40, 44]], np.float32)
    R = 2
    ids = np.full((6, R), -1, np.int32)
    ks = np.full((6, R), np.inf, np.float32)
    rows = {0: [1, 2], 3: [4, 5], 4: [3], 5: [3]}
    for v, c in rows.items():
        kk = [orc.dist(X, v, u) for u in c]
        o = sorted(range(len(c)), key=lambda i: (kk[i], c[i]))
        ids[v, :len(c)] = [c[i] for i in o]
        ks[v, :len(c)] = [kk[i] for i in o]
    _, _, tag, st = orc.update_round(X, ids, ks, seed=1, round=0, order=orc.ASCENDING,
                                     tau=1e-6)
    assert tag[0] and tag[1] and tag[2]
    assert not tag[3] and not tag[4] and not tag[5]
    assert st[5] == 1
    _, _, tag0, _ = orc.update_round(X, ids, ks, seed=1, round=0, order=orc.ASCENDING, tau=0.0)
    assert not tag0.any()


def test_oracle_rejects_pool_widths_beyond_its_buffers(orc):
    X = np.zeros((4, 2), np.float32)
    ids = np.full((4, 300), -1, np.int32)
    keys = np.full((4, 300), np.inf, np.float32)
    with pytest.raises(ValueError):
        orc.update_round(X, ids, keys, seed=1, round=0)
    with pytest.raises(ValueError):
        orc.build_graph(X, R=300, T1=1)
    with pytest.raises(ValueError):
        orc.scan_vertex(X, ids[0], keys[0], 0)
