"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's own formulas: each checks a closed
form, a published test vector, a worked example of the paper, a textbook rule
the method reduces to, a brute-force result, or an invariant.
"""
import json
import os
import random

import numpy as np
import pytest

import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = 2**64 - 1
GAMMA = 0x9E3779B97F4A7C15


def _row(orc, X, v, cands, R, metric=0):
    """A canonical pool row for v: candidates sorted by (key, id), padded."""
    keys = [orc.dist(X, v, c, metric) for c in cands]
    order = sorted(range(len(cands)), key=lambda i: (keys[i], cands[i]))
    ids = np.full(R, -1, np.int32)
    ks = np.full(R, np.inf, np.float32)
    for j, i in enumerate(order):
        ids[j] = cands[i]
        ks[j] = keys[i]
    return ids, ks


def _orders(n_seeds=12):
    import oracle
    yield oracle.ASCENDING, 0
    yield oracle.DESCENDING, 0
    for s in range(n_seeds):
        yield oracle.DISORDERED, s


# ----------------------------------------------------------------- hash
def test_splitmix64_published_vectors(orc):
    """mix() is the SplitMix64 output function: its outputs on the generator's
    state sequence reproduce the published test vectors."""
    n = 0
    with open(os.path.join(GOLDEN, "splitmix64_vectors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            seed, idx, out = (int(t) for t in line.split())
            assert orc.mix((seed + idx * GAMMA) & M64) == out
            n += 1
    assert n == 8


def test_hash_chain_definition(orc):
    """h(seed,a,b,c) chains mix with xor (checked on composed published values)."""
    s = 1234567
    # mix(s) is a published value; h(s,0,0,0) must equal mix(mix(mix(mix(s))))
    # built from the published single-step outputs.
    m1 = 6457827717110365317
    assert orc.mix(s) == m1
    assert orc.hash4(s, 0, 0, 0) == orc.mix(orc.mix(orc.mix(m1)))
    assert orc.hash4(s, 1, 2, 3) == orc.mix(orc.mix(orc.mix(m1 ^ 1) ^ 2) ^ 3)
    assert orc.hash4(s, 1, 2, 3) != orc.hash4(s, 1, 2, 4)


# -------------------------------------------------------------- distance
def test_distance_closed_forms(orc):
    X = np.array([[0, 0, 0, 0], [3, 4, 0, 0], [1, 2, 3, 4], [4, 3, 2, 1]], np.float32)
    assert orc.dist(X, 0, 1) == 25.0                       # 3-4-5 triangle
    assert orc.dist(X, 1, 0) == 25.0
    assert orc.dist(X, 2, 3) == 9 + 1 + 1 + 9
    assert orc.dist(X, 2, 3, metric=orc.IP) == -(4 + 6 + 6 + 4)
    d = 128
    Y = np.zeros((2, d), np.float32)
    Y[1] = 255.0
    assert orc.dist(Y, 0, 1) == d * 255.0**2               # exact in FP32 (8.3e6 < 2^24)
    # nine unit differences: exactly 9
    Z = np.zeros((2, 9), np.float32)
    Z[1] = np.float32(1.0)
    assert orc.dist(Z, 0, 1) == np.float32(9.0)


# -------------------------------------------------------------- prune rule
def test_pin_ray_keeps_only_nearest(orc):
    """P1: v at the origin, candidates on one ray. Every pair (a<b) has
    (b-a)^2 < b^2, so Eq. 2 always fires and only the nearest survives, in
    any arrival order; each pruned point goes to a closer candidate."""
    K = 12
    X = np.zeros((K + 1, 2), np.float32)
    X[1:, 0] = np.arange(1, K + 1)
    ids, ks = _row(orc, X, 0, list(range(1, K + 1)), 16)
    for order, seed in _orders():
        items, _ = orc.scan_vertex(X, ids, ks, 0, seed=seed, round=3, order=order)
        assert len(items) == K
        surv = [c for (dst, c, k) in items if dst == 0]
        assert surv == [1]
        for dst, c, k in items:
            if dst != 0:
                assert X[dst, 0] < X[c, 0]
                assert k == (X[c, 0] - X[dst, 0]) ** 2


def test_pin_line_keeps_nearest_each_side(orc):
    """P2: candidates on both sides of v on a line: survivors are the nearest
    on the left and the nearest on the right, for any order."""
    pos = [0, -5, -3, -1, 2, 4, 7, 9]
    X = np.array([[p, 0.0] for p in pos], np.float32)
    ids, ks = _row(orc, X, 0, list(range(1, len(pos))), 8)
    for order, seed in _orders():
        items, _ = orc.scan_vertex(X, ids, ks, 0, seed=seed, order=order)
        surv = sorted(c for (dst, c, k) in items if dst == 0)
        assert surv == [3, 4]


def test_pin_orthogonal_star_prunes_nothing(orc):
    """P3: candidates r_i e_i on distinct axes: d = r_i^2 + r_j^2 > max, so no
    pair meets Eq. 2; the round leaves the pool unchanged."""
    d = 6
    X = np.zeros((d + 1, d), np.float32)
    for i in range(d):
        X[i + 1, i] = i + 1
    R = 8
    ids, ks = _row(orc, X, 0, list(range(1, d + 1)), R)
    for order, seed in _orders():
        items, _ = orc.scan_vertex(X, ids, ks, 0, seed=seed, order=order)
        assert sorted(c for (dst, c, k) in items if dst == 0) == list(range(1, d + 1))
    P1i = np.full((d + 1, R), -1, np.int32)
    P1k = np.full((d + 1, R), np.inf, np.float32)
    P1i[0], P1k[0] = ids, ks
    P2i, P2k, _, _ = orc.update_round(X, P1i, P1k, seed=5, round=0)
    assert np.array_equal(P2i[0], ids) and np.array_equal(P2k[0], ks)
    assert (P2i[1:] == -1).all()


def test_pin_duplicate_points_tie_rule(orc):
    """P4: two identical points (d = 0): the one with the larger (key, id) is
    redirected to the other with key 0, in any order."""
    X = np.array([[0, 0], [1, 0], [1, 0], [0, 3]], np.float32)
    ids, ks = _row(orc, X, 0, [1, 2, 3], 4)
    for order, seed in _orders():
        items, _ = orc.scan_vertex(X, ids, ks, 0, seed=seed, order=order)
        assert sorted(items) == sorted([(0, 1, 1.0), (1, 2, 0.0), (0, 3, 9.0)])


def _textbook_rng_select(X, v):
    """Strict relative-neighbourhood selection (the MRNG / HNSW-heuristic
    rule): scan all other points by ascending (distance, id); keep u iff no
    kept w has d(u, w) < d(v, u)."""
    X64 = X.astype(np.float64)
    d = lambda a, b: np.float32(((X64[a] - X64[b]) ** 2).sum())
    others = sorted((u for u in range(len(X)) if u != v), key=lambda u: (d(v, u), u))
    kept = []
    for u in others:
        if all(d(u, w) >= d(v, u) for w in kept):
            kept.append(u)
    return kept


def test_pin_ascending_mode_is_textbook_rng(orc):
    """P5: with a complete pool and ascending order the survivor set of the
    scan is the strict RNG selection of the point set around v."""
    rng = np.random.default_rng(7)
    for trial in range(25):
        n = int(rng.integers(5, 40))
        X = rng.standard_normal((n, 3)).astype(np.float32)
        v = int(rng.integers(0, n))
        ids, ks = _row(orc, X, v, [u for u in range(n) if u != v], n - 1)
        items, _ = orc.scan_vertex(X, ids, ks, v, order=orc.ASCENDING)
        surv = [c for (dst, c, k) in items if dst == v]
        assert surv == _textbook_rng_select(X, v)


def test_disordered_survivors_pairwise_rng(orc):
    """Whatever the arrival order, the survivors of a scan are pairwise
    RNG-consistent (no kept pair meets Eq. 2), the closest candidate always
    survives, and each candidate yields exactly one item."""
    rng = np.random.default_rng(3)
    for trial in range(30):
        n = 60
        X = rng.standard_normal((n, 5)).astype(np.float32)
        v = int(rng.integers(0, n))
        cands = [int(c) for c in rng.choice([u for u in range(n) if u != v], 24, replace=False)]
        ids, ks = _row(orc, X, v, cands, 32)
        key = {int(i): float(k) for i, k in zip(ids, ks) if i >= 0}
        items, _ = orc.scan_vertex(X, ids, ks, v, seed=trial, round=trial)
        assert sorted(c for _, c, _ in items) == sorted(cands)
        surv = [c for (dst, c, k) in items if dst == v]
        assert int(ids[0]) in surv
        for i, a in enumerate(surv):
            for b in surv[:i]:
                assert orc.dist(X, a, b) >= max(key[a], key[b])
        for dst, c, k in items:
            if dst != v:
                assert k == orc.dist(X, dst, c)
                assert k < max(key[dst], key[c])
                assert (key[dst], dst) < (key[c], c)


def test_pin_paper_examples(orc):
    """P6: the worked examples of Section 2.2 (Figure 1) and Section 3.1."""
    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        ex = json.load(f)
    for name in ("fig1_rng", "vertex1_example"):
        e = ex[name]
        X = np.array(e["points"], np.float32)
        v = e["v"]
        n = len(X)
        ids, ks = _row(orc, X, v, [u for u in range(n) if u != v], 4)
        for order, seed in _orders():
            items, _ = orc.scan_vertex(X, ids, ks, v, seed=seed, order=order)
            assert sorted(c for (dst, c, k) in items if dst == v) == sorted(e["expect_kept"])
            red = sorted([c, dst] for (dst, c, k) in items if dst != v)
            assert red == sorted(e["expect_redirect"])


def test_near_tie_tagging(orc):
    """An exact tie d(u,w) == max(key_u, key_w) is not pruned (strict test) and
    is flagged as a near tie when tau > 0, not when tau == 0."""
    X = np.array([[0, 0], [2, 0], [1, 2]], np.float32)     # d(1,2) = 5 = key_2
    ids, ks = _row(orc, X, 0, [1, 2], 2)
    items, near = orc.scan_vertex(X, ids, ks, 0, order=orc.ASCENDING, tau=1e-6)
    assert sorted(c for (dst, c, k) in items if dst == 0) == [1, 2]
    assert near
    _, near0 = orc.scan_vertex(X, ids, ks, 0, order=orc.ASCENDING, tau=0.0)
    assert not near0


# ------------------------------------------------------------------ merge
def _alg6_literal(seq, R):
    """Sequential insertion into a fixed-capacity pool: skip a duplicate id;
    append while not full; else replace the farthest (by (key, id)) if the
    new item is closer."""
    pool = []
    for c, k in seq:
        if any(p[0] == c for p in pool):
            continue
        if len(pool) < R:
            pool.append((c, k))
            continue
        far = max(range(len(pool)), key=lambda i: (pool[i][1], pool[i][0]))
        if (k, c) < (pool[far][1], pool[far][0]):
            pool[far] = (c, k)
    return sorted(pool, key=lambda p: (p[1], p[0]))


def test_pin_merge_equals_sequential_insertion(orc):
    """P7: the merge equals Alg. 6 applied sequentially, for any insertion order
    (keys are a function of the (dest, cand) pair, as distances are)."""
    rng = np.random.default_rng(11)
    n, R = 40, 6
    tab = rng.integers(0, 50, size=(n, n)).astype(np.float32)  # many equal keys
    tab = np.minimum(tab, tab.T)
    items = []
    for _ in range(900):
        a, b = (int(t) for t in rng.integers(0, n, 2))
        if a != b:
            items.append((a, b, float(tab[a, b])))
    dest = np.array([i[0] for i in items]); cand = np.array([i[1] for i in items])
    key = np.array([i[2] for i in items])
    oi, ok, _ = orc.merge(n, R, dest, cand, key)
    for trial in range(5):
        perm = list(range(len(items)))
        random.Random(trial).shuffle(perm)
        for x in range(n):
            seq = [(items[p][1], items[p][2]) for p in perm if items[p][0] == x]
            exp = _alg6_literal(seq, R)
            got = [(int(c), float(k)) for c, k in zip(oi[x], ok[x]) if c >= 0]
            assert got == exp
            assert (oi[x, len(exp):] == -1).all()


def test_merge_drops_self_and_keeps_min_key(orc):
    oi, ok, _ = orc.merge(3, 4, [0, 0, 0, 0, 1], [0, 2, 2, 1, 1], [0.5, 3.0, 2.0, 7.0, 1.0])
    assert oi[0].tolist() == [2, 1, -1, -1] and ok[0, :2].tolist() == [2.0, 7.0]
    assert (oi[1] == -1).all() and (oi[2] == -1).all()


# ----------------------------------------------------------------- reverse
def _canonical_pools(orc, X, R, K, seed):
    n = X.shape[0]
    raw = datagen.random_pool(n, R, K, seed)
    ids = np.full((n, R), -1, np.int32)
    ks = np.full((n, R), np.inf, np.float32)
    for v in range(n):
        ids[v], ks[v] = _row(orc, X, v, raw[v, :K].tolist(), R)
    return ids, ks


@pytest.mark.parametrize("mode", [0, 1])
def test_pin_reverse_sampling_by_sets(orc, mode):
    """P8: after reverse sampling, pool[x] = first R by (key, id) of
    pool[x] + {v : x among the floor(rho*k_v) sampled entries of pool[v]};
    sampled = hash-first (mode 0) or nearest by (key, id) (mode 1)."""
    rng = np.random.default_rng(5)
    n, R = 80, 8
    X = rng.standard_normal((n, 4)).astype(np.float32)
    ids, ks = _canonical_pools(orc, X, R, 5, seed=9)
    ids[3, 2:] = -1; ks[3, 2:] = np.inf                     # a short row
    seed, t1, rho = 77, 2, 0.6
    got_i, got_k = orc.reverse_round(ids, ks, seed, t1, rho, mode=mode)
    inc = {x: {} for x in range(n)}
    for v in range(n):
        ent = [(int(i), float(k)) for i, k in zip(ids[v], ks[v]) if i >= 0]
        for i, k in ent:
            inc[v][i] = min(k, inc[v].get(i, np.inf))
        m = int(np.floor(np.float64(np.float32(rho)) * len(ent)))
        if mode == 0:
            order = sorted(ent, key=lambda e: ((orc.hash4(seed, 0x2000 + t1, v, e[0]) >> 32), e[0]))
        else:
            order = sorted(ent, key=lambda e: (e[1], e[0]))
        for i, k in order[:m]:
            inc[i][v] = min(k, inc[i].get(v, np.inf))
    for x in range(n):
        exp = sorted(((k, c) for c, k in inc[x].items() if c != x))[:R]
        got = [(float(k), int(c)) for c, k in zip(got_i[x], got_k[x]) if c >= 0]
        assert got == exp


def test_pin_reverse_nearest_worked_example(orc):
    """The nearest-m reading on a line with doubling gaps (0, 1, 3, 7, 15),
    each pool holding its two nearest points and m = floor(0.5 * 2) = 1: every
    point sends itself to its single nearest neighbour (0->1, 1->0, 3->1,
    7->3, 15->7), so 3 gains 7 and 7 gains 15, worked out by hand."""
    pos = [0.0, 1.0, 3.0, 7.0, 15.0]
    X = np.array(pos, np.float32)[:, None]
    R = 3
    two = {0: [1, 2], 1: [0, 2], 2: [1, 0], 3: [2, 1], 4: [3, 2]}
    ids = np.full((5, R), -1, np.int32)
    ks = np.full((5, R), np.inf, np.float32)
    for v, c in two.items():
        ids[v, :2] = c
        ks[v, :2] = [(pos[v] - pos[u]) ** 2 for u in c]
    got_i, got_k = orc.reverse_round(ids, ks, seed=3, t1=1, rho=0.5, mode=orc.REVERSE_NEAREST)
    want = {0: [1, 2, -1], 1: [0, 2, -1], 2: [1, 0, 3], 3: [2, 1, 4], 4: [3, 2, -1]}
    for v, w in want.items():
        assert got_i[v].tolist() == w
        assert got_k[v, :sum(u >= 0 for u in w)].tolist() == \
            [(pos[v] - pos[u]) ** 2 for u in w if u >= 0]


# -------------------------------------------------------------------- init
def test_init_draw_rule(orc):
    """Initial pools: the first min(S, n-1) distinct non-self ids of the hash
    stream h(seed, 0x3000, v, j) mod n, sorted by (key, id)."""
    rng = np.random.default_rng(1)
    n, R, S = 50, 12, 10
    X = rng.standard_normal((n, 3)).astype(np.float32)
    oi, ok, _ = orc.init(X, R, S, seed=123)
    for v in range(n):
        want, j = [], 0
        while len(want) < S:
            c = orc.hash4(123, 0x3000, v, j) % n
            j += 1
            if c != v and c not in want:
                want.append(c)
        row = [int(c) for c in oi[v] if c >= 0]
        assert sorted(row) == sorted(want)
        ks = [orc.dist(X, v, c) for c in row]
        assert ok[v, :S].tolist() == ks
        assert [(k, c) for k, c in zip(ks, row)] == sorted(zip(ks, row))
    oi2, _, _ = orc.init(X[:4], R=8, S=8, seed=1)                 # S > n-1
    assert ((oi2 >= 0).sum(1) == 3).all()


# ------------------------------------------------------------------ builds
def test_pin_build_invariants_integer_exact(orc):
    """P9 (exact form): integer-valued data, every key is an exact distance."""
    X = datagen.sift_like(3000, d=32, k=30, seed=3)
    adj, keys, st = orc.build_graph(X, R=16, T1=3, T2=3, seed=9)
    orc.check_invariants(X, adj, keys, exact=True)
    adj, keys, st = orc.build_graph(X, R=16, T1=3, T2=3, seed=9, reverse=orc.REVERSE_NEAREST)
    orc.check_invariants(X, adj, keys, exact=True)


def test_pin_build_invariants_float(orc):
    X = datagen.mixture(2000, d=16, k=20, sigma=0.2, seed=4)
    adj, keys, st = orc.build_graph(X, R=24, T1=2, T2=3, seed=5)
    orc.check_invariants(X, adj, keys, exact=True)       # same FP32 keys on both sides
    adj2, keys2, _ = orc.build_graph(X, R=24, T1=2, T2=3, seed=5, order=orc.ASCENDING)
    orc.check_invariants(X, adj2, keys2, exact=True)


def test_pin_line_build_is_path_like(orc):
    """P2 (build form): on distinct points of a line the output has at most one
    neighbour per side, and nearly all path edges are found."""
    rng = np.random.default_rng(2)
    n = 600
    pos = rng.permutation(n).astype(np.float32) * 1.0
    X = pos[:, None].copy()
    adj, keys, _ = orc.build_graph(X, R=16, T1=4, T2=4, seed=1)
    found = 0
    for v in range(n):
        nb = [int(u) for u in adj[v] if u >= 0]
        left = [u for u in nb if pos[u] < pos[v]]
        right = [u for u in nb if pos[u] > pos[v]]
        assert len(left) <= 1 and len(right) <= 1
        found += sum(1 for u in nb if abs(pos[u] - pos[v]) == 1)
    assert found / (2 * (n - 1)) >= 0.95


def test_pin_build_quality_mixture(orc):
    """P11: on the 10k x 128 mixture the oracle graph reaches Recall@10 >= 0.95
    with list size 64 (brute-force FP64 ground truth)."""
    X, Q, metric, R = datagen.workload("mixture10k_d128", nq=300)
    adj, keys, st = orc.build_graph(X, R=R, T1=4, T2=4, seed=42)
    kth = orc.knn_kth_dist(X, Q, 10)
    ids, _ = orc.search(X, adj, Q, k=10, L=64)
    assert orc.recall_at_k(X, Q, ids, kth) >= 0.95


def test_pin_determinism_threads(orc):
    """P12: the round is order-independent: 1 thread and many give the same bits."""
    X = datagen.mixture(1500, d=24, k=10, seed=8)
    t0 = orc.get_threads()
    try:
        orc.set_threads(1)
        a1, k1, s1 = orc.build_graph(X, R=16, T1=2, T2=2, seed=3)
        orc.set_threads(max(2, os.cpu_count() or 2))
        a2, k2, s2 = orc.build_graph(X, R=16, T1=2, T2=2, seed=3)
    finally:
        orc.set_threads(t0)
    assert np.array_equal(a1, a2) and np.array_equal(k1, k2) and np.array_equal(s1, s2)


def test_pin_resume_equals_build(orc):
    """P13: a build equals init, rounds and reverse passes chained by hand."""
    X = datagen.mixture(800, d=8, k=6, seed=2)
    R, T1, T2, seed, rho = 12, 3, 2, 17, 0.6
    adj, keys, _ = orc.build_graph(X, R=R, T1=T1, T2=T2, seed=seed, rho=rho)
    ids, ks, _ = orc.init(X, R, R, seed)
    for t1 in range(1, T1 + 1):
        for t2 in range(1, T2 + 1):
            ids, ks, _, _ = orc.update_round(X, ids, ks, seed, (t1 - 1) * T2 + (t2 - 1))
        if t1 != T1:
            ids, ks = orc.reverse_round(ids, ks, seed, t1, rho)
    a2, k2, _ = orc.finalize(X, ids, ks)
    assert np.array_equal(adj, a2) and np.array_equal(keys, k2)


# ------------------------------------------------------------------ search
def test_pin_search_on_complete_graph_is_exact(orc):
    """On the complete graph with a list as large as the data set, best-first
    search visits every point and returns the exact k nearest."""
    rng = np.random.default_rng(12)
    n, d = 120, 6
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((20, d)).astype(np.float32)
    adj = np.array([[u for u in range(n) if u != v] for v in range(n)], np.int32)
    ids, keys = orc.search(X, adj, Q, k=10, L=n, entry=0)
    gt, gd = orc.knn_exact(X, Q, 10)
    assert np.array_equal(ids, gt)
    ids_ip, _ = orc.search(X, adj, Q, k=10, L=n, entry=5, metric=orc.IP)
    gt_ip, _ = orc.knn_exact(X, Q, 10, metric=orc.IP)
    assert np.array_equal(ids_ip, gt_ip)


def test_pin_medoid_symmetric(orc):
    pos = np.array([3, -2, 0, 2, -3, 1, -1], np.float32)
    assert orc.medoid(pos[:, None]) == 2


# ------------------------------------------- sequential RNN-Descent reference
def test_rnn_descent_seq_line_is_path_like(orc):
    """The sequential RNN-Descent (Alg. 1 with Alg. 2) on distinct points of a
    line: at most one neighbour per side (the RNG of a line is its path), and
    nearly all path edges are found."""
    rng = np.random.default_rng(2)
    n = 600
    pos = rng.permutation(n).astype(np.float32)
    X = pos[:, None].copy()
    adj, _ = orc.rnn_descent_seq(X, R=16, T1=4, T2=4, seed=1)
    found = 0
    for v in range(n):
        nb = [int(u) for u in adj[v] if u >= 0]
        assert len([u for u in nb if pos[u] < pos[v]]) <= 1
        assert len([u for u in nb if pos[u] > pos[v]]) <= 1
        found += sum(1 for u in nb if abs(pos[u] - pos[v]) == 1)
    assert found / (2 * (n - 1)) >= 0.95


def test_rnn_descent_seq_rows_are_rng_rows(orc):
    """On integer data (exact distances) every output row of the sequential
    method is sorted by (key, id), holds no self id and no repeat, keys are
    the exact distances, and no two kept neighbours violate the strict RNG
    test of Eq. 1 against each other."""
    X = datagen.sift_like(2000, d=32, k=20, seed=7)
    adj, keys = orc.rnn_descent_seq(X, R=24, T1=3, T2=3, seed=5)
    assert orc.check_invariants(X, adj, keys, exact=True)
    assert (adj >= 0).sum(1).min() >= 1


def test_grnnd_quality_matches_rnn_descent(orc):
    """The paper's claim that the parallel method keeps the sequential
    method's graph quality, on the 5k x 64 mixture: Recall@10 of both graphs
    with the same search routine agrees within 2 points at L = 16, 32, 64."""
    X = datagen.mixture(5000, d=64, k=40, sigma=0.15, seed=1)
    Q = datagen.mixture(400, d=64, k=40, sigma=0.15, seed=1, stream=1)
    seq, seqk = orc.rnn_descent_seq(X, R=32, T1=4, T2=4, seed=42)
    par, park, _ = orc.build_graph(X, R=32, T1=4, T2=4, seed=42)
    assert orc.check_invariants(X, seq, seqk)
    kth = orc.knn_kth_dist(X, Q, 10)
    e = orc.medoid(X)
    for L in (16, 32, 64):
        rs = orc.recall_at_k(X, Q, orc.search(X, seq, Q, 10, L, e)[0], kth)
        rp = orc.recall_at_k(X, Q, orc.search(X, par, Q, 10, L, e)[0], kth)
        assert abs(rs - rp) <= 0.02, (L, rs, rp)
    assert rs >= 0.99
