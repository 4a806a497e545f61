"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (stated per test):
  * integer-valued data: every FP32 distance is exact in any summation
    order, so ids AND keys must match bit for bit;
  * float data: rows the oracle does not tag as near ties (tau = 2e-6 of a
    distance's natural scale, above the canonical FP32 distance's error
    bound for d <= 1024) must match bit for bit in ids, keys within 1e-5
    relative; the tagged fraction is bounded;
  * full builds on float data: Recall@10 within 0.5 points of the oracle
    graph's, with the same search routine and list size.
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

TAU = 2e-6


@pytest.fixture(scope="module")
def g():
    import paper_2510_02774_amd as g
    g.lib()
    assert torch.cuda.is_available()
    return g


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def params(g, R, T1=1, T2=4, S=None, order=0, rho=0.6):
    p = g.grnnd_params_default(R, T1)
    p.T2 = T2
    p.S = R if S is None else S
    p.order = order
    p.rho = rho
    return p


def gpu_init(g, X, R, S, seed, metric=0):
    n, d = X.shape
    p = params(g, R, S=S)
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, p))
    ids = torch.empty((n, R), dtype=torch.int32, device="cuda")
    keys = torch.empty((n, R), dtype=torch.float32, device="cuda")
    g.grnnd_init_pools(dev(X), metric, R, S, seed, ids, keys, None, ws)
    return host(ids), host(keys)


def gpu_step(g, X, ids, keys, seed, rnd, kind, p, metric=0):
    n, d = X.shape
    R = ids.shape[1]
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, p))
    oi = torch.empty((n, R), dtype=torch.int32, device="cuda")
    ok = torch.empty((n, R), dtype=torch.float32, device="cuda")
    st = torch.zeros(g.NSTATS, dtype=torch.int64, device="cuda")
    g.grnnd_step(dev(X), metric, R, dev(ids), dev(keys), oi, ok, seed, rnd, kind, p, st, ws)
    return host(oi), host(ok), host(st)


def gpu_final(g, X, ids, keys, metric=0):
    n, d = X.shape
    R = ids.shape[1]
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, None))
    oa = torch.empty((n, R), dtype=torch.int32, device="cuda")
    ok = torch.empty((n, R), dtype=torch.float32, device="cuda")
    g.grnnd_finalize(dev(X), metric, R, dev(ids), dev(keys), oa, ok, None, ws)
    return host(oa), host(ok)


def gpu_build(g, X, R, p, seed, metric=0):
    adj, keys, st = g.build_graph(dev(X), R, p, seed=seed, metric=metric, stats=True)
    return host(adj), host(keys), host(st)


def int_data(n, d, seed=5, k=40):
    return datagen.sift_like(n, d=d, k=k, seed=seed)


def state(orc, X, R, seed=3, rounds=1, metric=0):
    """A realistic frozen pool state produced by the oracle alone."""
    ids, keys, _ = orc.init(X, R, R, seed=seed, metric=metric)
    for r in range(rounds):
        ids, keys, _, _ = orc.update_round(X, ids, keys, seed=seed, round=r, metric=metric)
    return ids, keys


def assert_rows_equal(gi, gk, oi, ok, mask=None, rtol=0.0, atol=0.0):
    """Ids equal on the compared rows; keys equal (rtol == 0) or within
    rtol * |key| + atol. For the inner-product metric the FP32 error bound is
    relative to sum |a_k b_k| (<= 1 for unit vectors), not to |key|, so such
    tests pass an absolute term."""
    rows = np.arange(gi.shape[0]) if mask is None else np.nonzero(~mask)[0]
    bad = [int(r) for r in rows if not np.array_equal(gi[r], oi[r])]
    assert not bad, (f"{len(bad)} of {len(rows)} rows differ in ids, e.g. row {bad[0]}: "
                     f"{gi[bad[0]].tolist()} vs {oi[bad[0]].tolist()}")
    if rtol == 0.0 and atol == 0.0:
        badk = [int(r) for r in rows if not np.array_equal(gk[r], ok[r])]
        assert not badk, f"{len(badk)} rows differ in keys, e.g. row {badk[0]}"
    else:
        a, b = gk[rows], ok[rows]
        fin = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), fin), "padding differs"
        err = np.abs(a[fin] - b[fin])
        lim = rtol * np.abs(b[fin]) + atol
        assert (err <= lim).all(), f"max key error {err.max():.3g} (limit there {lim[err.argmax()]:.3g})"


# ----------------------------------------------------------------- init
@pytest.mark.parametrize("n,d,R", [(3000, 128, 32), (1500, 36, 20), (2000, 64, 48),
                                   (1200, 16, 64), (700, 5, 16), (40, 8, 48)])
def test_init_bit_exact_integer(g, orc, n, d, R):
    X = int_data(n, d)
    S = min(R, 32)
    gi, gk = gpu_init(g, X, R, S, seed=7)
    oi, ok, _ = orc.init(X, R, S, seed=7)
    assert_rows_equal(gi, gk, oi, ok)


# ---------------------------------------------------------- update step
@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("n,d,R", [(3000, 128, 32), (2000, 64, 48), (1500, 40, 20),
                                   (1000, 16, 64)])
def test_update_step_bit_exact_integer(g, orc, order, n, d, R):
    X = int_data(n, d)
    ids, keys = state(orc, X, R)
    p = params(g, R, order=order)
    gi, gk, st = gpu_step(g, X, ids, keys, 11, 5, g.STEP_UPDATE, p)
    oi, ok, _, ost = orc.update_round(X, ids, keys, seed=11, round=5, order=order)
    assert_rows_equal(gi, gk, oi, ok)
    # counters agree with the oracle's (pairs, redirects, survivors, items)
    assert st[0] == ost[0] and st[2] == ost[2] and st[3] == ost[3] and st[4] == ost[4]


def test_update_step_float_tagged(g, orc):
    X = datagen.mixture(6000, d=128, k=50, sigma=0.15, seed=1)
    R = 32
    ids, keys = state(orc, X, R, rounds=2)
    p = params(g, R)
    gi, gk, _ = gpu_step(g, X, ids, keys, 42, 3, g.STEP_UPDATE, p)
    oi, ok, tag, _ = orc.update_round(X, ids, keys, seed=42, round=3, tau=TAU)
    assert tag.mean() < 0.05, tag.mean()
    assert_rows_equal(gi, gk, oi, ok, mask=tag, rtol=1e-5)


def test_update_step_ip_tagged(g, orc):
    X = datagen.angular(5000, d=100, k=200, seed=31)
    R = 32
    ids, keys = state(orc, X, R, rounds=1, metric=1)
    p = params(g, R)
    gi, gk, _ = gpu_step(g, X, ids, keys, 9, 2, g.STEP_UPDATE, p, metric=1)
    oi, ok, tag, _ = orc.update_round(X, ids, keys, seed=9, round=2, tau=TAU, metric=1)
    assert tag.mean() < 0.05, tag.mean()
    assert_rows_equal(gi, gk, oi, ok, mask=tag, rtol=1e-5, atol=1e-6)


def test_update_step_ragged_pools(g, orc):
    """Rows with every fill level 0..R, including empty and single-entry rows."""
    X = int_data(900, 24)
    R = 24
    ids, keys = state(orc, X, R)
    for v in range(X.shape[0]):
        k = v % (R + 1)
        ids[v, k:] = -1
        keys[v, k:] = np.inf
    p = params(g, R)
    gi, gk, _ = gpu_step(g, X, ids, keys, 5, 1, g.STEP_UPDATE, p)
    oi, ok, _, _ = orc.update_round(X, ids, keys, seed=5, round=1)
    assert_rows_equal(gi, gk, oi, ok)


def hub_state(orc, n=3000, d=64, R=32, seed=3):
    """Integer points h + s_i, s_i in {-3..3}^d, around one hub h (id 0):
    every point is about twice as far from the others as from h. Each pool of
    an oracle-made state gets h in place of its farthest entry, so in a round
    almost every other candidate u of a pool meets h with d(u, h) < key_u and
    is redirected to h: h receives far more items than its R-slot bucket
    holds and its merge takes the chunked path for inputs above 64 items."""
    rng = np.random.default_rng(seed)
    X = (100 + rng.integers(-3, 4, size=(n, d))).astype(np.float32)
    X[0] = 100.0
    ids, keys = state(orc, X, R, seed=seed)
    for v in range(1, n):
        row = [(float(k), int(i)) for i, k in zip(ids[v], keys[v]) if i >= 0 and i != 0]
        row = sorted(row)[:R - 1] + [(orc.dist(X, v, 0), 0)]
        row.sort()
        ids[v] = [i for _, i in row] + [-1] * (R - len(row))
        keys[v] = [k for k, _ in row] + [np.inf] * (R - len(row))
    return X, ids, keys


@pytest.mark.parametrize("kind", ["update", "reverse"])
def test_step_hub_overflow_and_long_merge(g, orc, kind):
    """A hub receiving thousands of items in one step: bucket overflow and the
    chunked merge (both seen in the device counters) stay bit-exact."""
    X, ids, keys = hub_state(orc)
    R = ids.shape[1]
    p = params(g, R, rho=0.6)
    if kind == "update":
        gi, gk, st = gpu_step(g, X, ids, keys, 7, 3, g.STEP_UPDATE, p)
        oi, ok, _, ost = orc.update_round(X, ids, keys, seed=7, round=3)
        assert st[4] == ost[4]
    else:
        gi, gk, st = gpu_step(g, X, ids, keys, 7, 1, g.STEP_REVERSE, p)
        oi, ok = orc.reverse_round(ids, keys, seed=7, t1=1, rho=0.6)
    assert_rows_equal(gi, gk, oi, ok)
    print(f"{kind}: overflow items {st[8]}, long merges {st[9]}, items {st[4]}")
    assert st[8] > 1000, st[8]       # items beyond the hub's bucket
    assert st[9] >= 1, st[9]         # the hub's merge ran in chunks


# --------------------------------------------------------- reverse step
@pytest.mark.parametrize("n,R,rho", [(2500, 32, 0.6), (2500, 32, 0.25), (2500, 32, 0.95),
                                     (2501, 16, 0.6), (2502, 24, 0.5), (2503, 48, 0.6),
                                     (2500, 32, 0.05), (2501, 16, 0.999)])
def test_reverse_step_bit_exact(g, orc, n, R, rho):
    """Pool widths of every vertex grouping (4, 2 and 1 pools per wave), with
    vertex counts that leave the last wave's groups partly empty, and sampling
    ratios at which most vertices send nothing or all but one entry."""
    X = int_data(n, 32)
    ids, keys = state(orc, X, R, rounds=2)
    p = params(g, R, rho=rho)
    gi, gk, _ = gpu_step(g, X, ids, keys, 17, 2, g.STEP_REVERSE, p)
    oi, ok = orc.reverse_round(ids, keys, seed=17, t1=2, rho=rho)
    assert_rows_equal(gi, gk, oi, ok)


@pytest.mark.parametrize("n,R,rho", [(2500, 32, 0.6), (2501, 16, 0.3), (2503, 48, 0.95)])
def test_reverse_step_nearest_bit_exact(g, orc, n, R, rho):
    """The second reading of Section 3.6's "top rho k" neighbours: v sends
    itself to the floor(rho k) nearest entries of its row."""
    X = int_data(n, 32)
    ids, keys = state(orc, X, R, rounds=2)
    p = params(g, R, rho=rho)
    p.reverse = g.REVERSE_NEAREST
    gi, gk, _ = gpu_step(g, X, ids, keys, 17, 2, g.STEP_REVERSE, p)
    oi, ok = orc.reverse_round(ids, keys, seed=17, t1=2, rho=rho, mode=orc.REVERSE_NEAREST)
    assert_rows_equal(gi, gk, oi, ok)
    hi, hk = orc.reverse_round(ids, keys, seed=17, t1=2, rho=rho)
    assert not np.array_equal(oi, hi)  # the two readings differ on this state


def test_build_nearest_reverse_bit_exact(g, orc):
    X = int_data(3000, 48)
    R = 32
    p = params(g, R, T1=3, T2=2)
    p.reverse = g.REVERSE_NEAREST
    ga, gk, _ = gpu_build(g, X, R, p, seed=23)
    oa, ok, _ = orc.build_graph(X, R=R, T1=3, T2=2, seed=23, reverse=orc.REVERSE_NEAREST)
    assert_rows_equal(ga, gk, oa, ok)


# ----------------------------------------------------------- output pass
@pytest.mark.parametrize("n,d,R", [(3000, 128, 32), (1500, 20, 48)])
def test_finalize_bit_exact_integer(g, orc, n, d, R):
    X = int_data(n, d)
    ids, keys = state(orc, X, R, rounds=3)
    ga, gk = gpu_final(g, X, ids, keys)
    oa, ok, _ = orc.finalize(X, ids, keys)
    assert_rows_equal(ga, gk, oa, ok)


# ---------------------------------------------------------- full builds
@pytest.mark.parametrize("n,d,R,T1,T2", [(4000, 32, 16, 3, 3), (3000, 128, 32, 2, 4)])
def test_build_bit_exact_integer(g, orc, n, d, R, T1, T2):
    X = int_data(n, d)
    p = params(g, R, T1=T1, T2=T2)
    ga, gk, st = gpu_build(g, X, R, p, seed=21)
    oa, ok, ost = orc.build_graph(X, R=R, T1=T1, T2=T2, seed=21)
    assert_rows_equal(ga, gk, oa, ok)
    assert st[0] == ost[0] and st[7] == ost[7] and st[6] == ost[6]
    orc.check_invariants(X, ga, gk, exact=True)


@pytest.mark.parametrize("n,d,R", [(3000, 16, 32), (2000, 12, 16), (2500, 24, 48)])
def test_build_bit_exact_binary_ties(g, orc, n, d, R):
    """0/1 rows: every distance is a small integer, so nearly all keys tie and
    the (key, id) order alone decides every pool, merge and reverse sample;
    repeated rows put distance 0 between distinct ids. Pool widths 16, 32
    and 48 take the merge's 16-, 32- and 64-lane sorting segments."""
    X = datagen.binary(n, d=d, seed=40 + d)
    assert len(np.unique(X, axis=0)) < n  # some rows repeat
    p = params(g, R, T1=2, T2=3)
    ga, gk, st = gpu_build(g, X, R, p, seed=29)
    oa, ok, ost = orc.build_graph(X, R=R, T1=2, T2=3, seed=29)
    assert_rows_equal(ga, gk, oa, ok)
    assert st[0] == ost[0] and st[7] == ost[7] and st[6] == ost[6]
    orc.check_invariants(X, ga, gk, exact=True)


def test_build_mixture10k_recall_parity(g, orc):
    """10k x 128 Gaussian mixture, L2, R=32, 32 random initial neighbours,
    T1=4 (T2=4): GPU graph invariants hold and its Recall@10 is within 0.5
    points of the oracle graph's (same search routine, L=64)."""
    X, Q, metric, R = datagen.workload("mixture10k_d128")
    p = params(g, R, T1=4, T2=4)
    ga, gk, st = gpu_build(g, X, R, p, seed=42)
    oa, ok, _ = orc.build_graph(X, R=R, T1=4, T2=4, seed=42)
    orc.check_invariants(X, ga, gk, exact=False, rtol=1e-5)
    kth = orc.knn_kth_dist(X, Q, 10)
    ent = orc.medoid(X)
    rg = orc.recall_at_k(X, Q, orc.search(X, ga, Q, k=10, L=64, entry=ent)[0], kth)
    ro = orc.recall_at_k(X, Q, orc.search(X, oa, Q, k=10, L=64, entry=ent)[0], kth)
    assert rg >= 0.95
    assert abs(rg - ro) <= 0.005, (rg, ro)


def test_build_quality_matches_sequential_rnn_descent(g, orc):
    """The GPU graph against the sequential in-place RNN-Descent reference
    (Alg. 1 with Alg. 2, in the oracle) on the 10k x 128 mixture: Recall@10
    of both graphs, searched on the device with the same routine and entry,
    agrees within 2 points at L = 16, 32 and 64."""
    X, Q, metric, R = datagen.workload("mixture10k_d128", nq=500)
    ga, gk, _ = gpu_build(g, X, R, params(g, R, T1=4, T2=4), seed=42)
    sa, sk = orc.rnn_descent_seq(X, R=R, T1=4, T2=4, seed=42)
    kth = orc.knn_kth_dist(X, Q, 10)
    ent = orc.medoid(X)
    for L in (16, 32, 64):
        gi, _ = g.search(dev(X), dev(ga), dev(Q), k=10, L=L, entry=ent)
        si, _ = g.search(dev(X), dev(sa), dev(Q), k=10, L=L, entry=ent)
        rg = orc.recall_at_k(X, Q, host(gi), kth)
        rs = orc.recall_at_k(X, Q, host(si), kth)
        assert abs(rg - rs) <= 0.02, (L, rg, rs)


def test_build_angular_ip_recall_parity(g, orc):
    X = datagen.angular(6000, d=100, k=100, seed=31)
    Q = datagen.angular(300, d=100, k=100, seed=31, stream=1)
    R = 32
    p = params(g, R, T1=3, T2=4)
    ga, gk, _ = gpu_build(g, X, R, p, seed=4, metric=1)
    oa, ok, _ = orc.build_graph(X, R=R, T1=3, T2=4, seed=4, metric=1)
    orc.check_invariants(X, ga, gk, metric=1, exact=False, rtol=1e-5)
    kth = orc.knn_kth_dist(X, Q, 10, metric=1)
    rg = orc.recall_at_k(X, Q, orc.search(X, ga, Q, 10, 64, 0, metric=1)[0], kth, metric=1)
    ro = orc.recall_at_k(X, Q, orc.search(X, oa, Q, 10, 64, 0, metric=1)[0], kth, metric=1)
    assert abs(rg - ro) <= 0.005 + 1e-9, (rg, ro)


@pytest.mark.parametrize("R,d,metric", [(24, 48, 0), (16, 40, 1), (48, 20, 0)])
def test_build_deterministic_and_resumable(g, orc, R, d, metric):
    """Same seed twice gives the same bits; the build equals init, steps and
    the output pass chained through the C ABI. The build's merges take the
    single-sort path for canonical keys, the steps' merges (pools handed in
    by the caller) the general one, so this also holds the two merge paths
    to the same bits on non-integer data."""
    X = datagen.mixture(3000, d=d, k=20, seed=6)
    if metric == 1:
        X = (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)
    T1, T2, seed = 3, 2, 99
    p = params(g, R, T1=T1, T2=T2)
    a1, k1, _ = gpu_build(g, X, R, p, seed, metric=metric)
    a2, k2, _ = gpu_build(g, X, R, p, seed, metric=metric)
    assert np.array_equal(a1, a2) and np.array_equal(k1, k2)
    ids, keys = gpu_init(g, X, R, R, seed, metric=metric)
    for t1 in range(1, T1 + 1):
        for t2 in range(1, T2 + 1):
            ids, keys, _ = gpu_step(g, X, ids, keys, seed, (t1 - 1) * T2 + (t2 - 1),
                                    g.STEP_UPDATE, p, metric=metric)
        if t1 != T1:
            ids, keys, _ = gpu_step(g, X, ids, keys, seed, t1, g.STEP_REVERSE, p, metric=metric)
    a3, k3 = gpu_final(g, X, ids, keys, metric=metric)
    assert np.array_equal(a1, a3) and np.array_equal(k1, k3)


@pytest.mark.parametrize("n,R", [(2, 4), (3, 16), (17, 32), (65, 64)])
def test_build_tiny_sets(g, orc, n, R):
    X = int_data(n, 12, k=3)
    p = params(g, R, T1=2, T2=2)
    ga, gk, _ = gpu_build(g, X, R, p, seed=1)
    oa, ok, _ = orc.build_graph(X, R=R, T1=2, T2=2, seed=1)
    assert_rows_equal(ga, gk, oa, ok)


# ---------------------------------------------------------------- search
def test_search_bit_exact_integer(g, orc):
    X = int_data(5000, 64)
    Q = datagen.sift_like(400, d=64, k=40, seed=5, stream=1)
    R = 24
    adj, keys, _ = orc.build_graph(X, R=R, T1=2, T2=3, seed=2)
    ent = orc.medoid(X)
    for L in (10, 32, 64, 100, 256):
        oi, ok = orc.search(X, adj, Q, k=10, L=L, entry=ent)
        gi, gk = g.search(dev(X), dev(adj), dev(Q), k=10, L=L, entry=ent)
        assert np.array_equal(host(gi), oi)
        assert np.array_equal(host(gk), ok)


def test_search_float_recall_matches(g, orc):
    X, Q, metric, R = datagen.workload("mixture10k_d128", nq=500)
    adj, keys, _ = orc.build_graph(X, R=R, T1=2, T2=2, seed=3)
    ent = orc.medoid(X)
    kth = orc.knn_kth_dist(X, Q, 10)
    oi, _ = orc.search(X, adj, Q, k=10, L=32, entry=ent)
    gi, _ = g.search(dev(X), dev(adj), dev(Q), k=10, L=32, entry=ent)
    r_o = orc.recall_at_k(X, Q, oi, kth)
    r_g = orc.recall_at_k(X, Q, host(gi), kth)
    assert abs(r_o - r_g) <= 0.002
    assert (host(gi) == oi).all(axis=1).mean() > 0.98


# ------------------------------------------------------- high dimension
def small_int_data(n, d, hi=60, seed=9):
    """Integer-valued rows in [0, hi]: with d * hi^2 * 2 < 2^24 every FP32
    distance and Gram entry is exact, so the bit-exact bar applies at d = 960."""
    rng = np.random.default_rng(seed)
    c = rng.integers(0, hi + 1, size=(40, d))
    lab = rng.integers(0, 40, size=n)
    X = np.clip(c[lab] + rng.integers(-8, 9, size=(n, d)), 0, hi)
    return X.astype(np.float32)


@pytest.mark.parametrize("order", [0, 1])
def test_update_step_bit_exact_integer_d960(g, orc, order):
    X = small_int_data(1200, 960)
    R = 48
    ids, keys = state(orc, X, R)
    p = params(g, R, order=order)
    gi, gk, st = gpu_step(g, X, ids, keys, 13, 2, g.STEP_UPDATE, p)
    oi, ok, _, ost = orc.update_round(X, ids, keys, seed=13, round=2, order=order)
    assert_rows_equal(gi, gk, oi, ok)
    assert st[0] == ost[0] and st[2] == ost[2] and st[3] == ost[3] and st[4] == ost[4]


def test_build_bit_exact_integer_d960(g, orc):
    X = small_int_data(1500, 960, seed=10)
    R = 48
    p = params(g, R, T1=2, T2=2)
    gi, gk, st = gpu_build(g, X, R, p, seed=5)
    oi, ok, ost = orc.build_graph(X, R, S=R, T1=2, T2=2, seed=5)
    assert_rows_equal(gi, gk, oi, ok)
    # tile pairs, redirects, survivors, initial and output-pass pairs (the
    # library's item count also covers the reverse-sampling merges)
    for i in (0, 2, 3, 6, 7):
        assert st[i] == ost[i], (i, st[i], ost[i])
    assert st[10] == 0  # every redirect key came exactly from the tile
    orc.check_invariants(X, gi, gk, exact=True)


def test_build_bit_exact_mixed_row_flags(g, orc):
    """Rows of two kinds, integers and half-integers (all BF16 values): the
    build-wide summary of the row flags differs between its AND and OR, so
    the round kernels read each candidate's own flags. Every distance is a
    multiple of 1/4 far below 2^22, hence exact in FP32: the graph must equal
    the oracle's bit for bit."""
    X = small_int_data(2000, 64, hi=60, seed=12)
    X[1::2] += 0.5
    R = 32
    p = params(g, R, T1=2, T2=2)
    gi, gk, st = gpu_build(g, X, R, p, seed=9)
    oi, ok, ost = orc.build_graph(X, R, S=R, T1=2, T2=2, seed=9)
    assert_rows_equal(gi, gk, oi, ok)
    for i in (0, 2, 3, 6, 7):
        assert st[i] == ost[i], (i, st[i], ost[i])


@pytest.mark.parametrize("d,hi", [(960, 115), (600, 150)])
def test_build_bit_exact_integer_deferred_keys(g, orc, d, hi):
    """Rows of at least 512 elements leave the redirect keys that the tile
    does not give exactly to the destination's merge. Here most of the rows
    have squared norms of 2^22 or more, so most redirects are such
    deferred keys (at d = 960 a quarter of the rows stay below, so pools mix
    exact and deferred keys), while every canonical distance (below
    d hi^2 < 2^24) is still exact: the graph must equal the oracle's bit for
    bit."""
    print(f"case: integer d={d} hi={hi}", flush=True)
    X = small_int_data(1500, d, hi=hi, seed=11)
    big = ((X.astype(np.float64) ** 2).sum(1) >= 2.0 ** 22).mean()
    assert big > 0.5, big
    R = 48
    p = params(g, R, T1=2, T2=2)
    gi, gk, st = gpu_build(g, X, R, p, seed=5)
    oi, ok, ost = orc.build_graph(X, R, S=R, T1=2, T2=2, seed=5)
    assert_rows_equal(gi, gk, oi, ok)
    for i in (0, 2, 3, 6, 7):
        assert st[i] == ost[i], (i, st[i], ost[i])
    # the merge computed deferred keys, at most one per redirect
    assert 0 < st[10] <= st[2], (st[10], st[2])


def test_update_step_gistlike_float_tagged(g, orc):
    """At d = 960 the canonical FP32 distance (d / 16 chained FMAs per lane,
    then four additions, each term's difference rounded once) is within about
    (d / 16 + 6) u = 3.9e-6 of the exact value relative to it, so the near-tie
    band is widened to 5e-6; with R = 48 (1128 pairs per pool) about 11% of the
    rows are then tagged on this data, and every other row must match."""
    X = datagen.gist_like(2500, d=960, k=40, seed=21)
    R = 48
    ids, keys = state(orc, X, R)
    p = params(g, R)
    gi, gk, _ = gpu_step(g, X, ids, keys, 17, 1, g.STEP_UPDATE, p)
    oi, ok, tag, _ = orc.update_round(X, ids, keys, seed=17, round=1, tau=5e-6)
    assert tag.mean() < 0.15, tag.mean()
    assert_rows_equal(gi, gk, oi, ok, mask=tag, rtol=1e-5)


def test_search_bit_exact_integer_d960(g, orc):
    X = small_int_data(2000, 960, seed=12)
    Q = small_int_data(200, 960, seed=13)
    R = 48
    adj, _, _ = orc.build_graph(X, R, S=R, T1=2, T2=2, seed=3)
    entry = orc.medoid(X)
    oi, ok = orc.search(X, adj, Q, k=10, L=64, entry=entry)
    import paper_2510_02774_amd as gg
    gi, gk = gg.search(dev(X), dev(adj), dev(Q), k=10, L=64, entry=entry)
    assert np.array_equal(host(gi), oi)
    assert np.array_equal(host(gk), ok)


# ------------------------------------------- full size, sampled parity
def test_full_size_step_sampled_parity_siftlike1m(g, orc):
    """One update round at the benchmark's full size (1,000,000 x 128
    integer-valued, R = 32, the launch configuration the benchmark times),
    after GPU initial pools and one GPU round. For 256 sampled destinations x,
    the oracle recomputes every item sent to x -- x's own scan and the scan of
    every vertex whose pool holds x (only those can redirect to x) -- merges
    them, and the GPU's new pool of x must equal it bit for bit."""
    X, _, metric, R = datagen.workload("siftlike1m_d128", nq=1)
    n, d = X.shape
    p = params(g, R)
    Xd = dev(X)
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, p))
    i0 = torch.empty((n, R), dtype=torch.int32, device="cuda")
    k0 = torch.empty((n, R), dtype=torch.float32, device="cuda")
    i1, k1 = torch.empty_like(i0), torch.empty_like(k0)
    i2, k2 = torch.empty_like(i0), torch.empty_like(k0)
    g.grnnd_init_pools(Xd, metric, R, R, 42, i0, k0, None, ws)
    g.grnnd_step(Xd, metric, R, i0, k0, i1, k1, 42, 0, g.STEP_UPDATE, p, None, ws)
    g.grnnd_step(Xd, metric, R, i1, k1, i2, k2, 42, 1, g.STEP_UPDATE, p, None, ws)
    P1, K1 = host(i1), host(k1)
    P2, K2 = host(i2), host(k2)
    flat = P1.ravel()
    srt = np.argsort(flat, kind="stable")
    fs = flat[srt]
    rng = np.random.default_rng(7)
    xs = rng.choice(n, 256, replace=False)
    for x in xs:
        lo, hi = np.searchsorted(fs, x), np.searchsorted(fs, x, side="right")
        srcs = sorted(set((srt[lo:hi] // R).tolist()) | {int(x)})
        dst, cnd, key = [], [], []
        for u in srcs:
            items, _ = orc.scan_vertex(X, P1[u], K1[u], u, seed=42, round=1)
            for dd, cc, kk in items:
                if dd == x:
                    dst.append(dd)
                    cnd.append(cc)
                    key.append(kk)
        # merge as destination z, a small id no item names (x never appears
        # as a candidate of its own items, so only the self-drop differs)
        z = min(set(range(len(cnd) + 2)) - set(cnd))
        mi, mk, _ = orc.merge(z + 1, R, np.full(len(dst), z, np.int32), np.array(cnd, np.int32),
                              np.array(key, np.float32))
        assert np.array_equal(P2[x], mi[z]), (int(x), P2[x], mi[z])
        assert np.array_equal(K2[x], mk[z]), int(x)


# --------------------------------------------------- narrow distance tiles
NARROW = ("bf16", "fp16", "fp8")


def prec_code(g, name):
    return {"fp32": g.PREC_FP32, "bf16": g.PREC_BF16, "fp16": g.PREC_FP16,
            "fp8": g.PREC_FP8_E4M3}[name]


@pytest.mark.parametrize("case", ["siftlike", "mixture", "angular_ip", "gistlike_d960"])
def test_narrow_build_equals_fp32_build(g, case):
    """A build with BF16, FP16 or FP8 tiles decides every comparison exactly as
    the FP32 tile does (comparisons inside the narrow tile's per-pair error
    bound are re-decided with the canonical FP32 distance), so its graph and
    keys equal the FP32 build's bit for bit; only the recheck count differs."""
    if case == "siftlike":
        X, metric, R = int_data(3000, 128), 0, 32
    elif case == "mixture":
        X, metric, R = datagen.mixture(4000, d=128, k=50, sigma=0.15, seed=1), 0, 32
    elif case == "angular_ip":
        X, metric, R = datagen.angular(4000, d=100, k=200, seed=31), 1, 32
    else:
        X, metric, R = datagen.gist_like(1500, d=960, k=40, seed=21), 0, 48
    ref = gpu_build(g, X, R, params(g, R, T1=2, T2=3), seed=19, metric=metric)
    for name in NARROW:
        p = params(g, R, T1=2, T2=3)
        p.precision = prec_code(g, name)
        ga, gk, st = gpu_build(g, X, R, p, seed=19, metric=metric)
        assert np.array_equal(ga, ref[0]), name
        assert np.array_equal(gk, ref[1]), name
        for i in (0, 2, 3, 6, 7):
            assert st[i] == ref[2][i], (name, i)


def test_build_gistlike_d960_recall_parity_all_precisions(g, orc):
    """Float gist-like data at d = 960, R = 48, 8,000 points: the GPU graph of
    every tile precision (FP32, BF16, FP16, FP8-e4m3) against the oracle's
    graph, both searched by the oracle's routine from the medoid (L = 64):
    Recall@10 within 0.5 points, and the narrow graphs equal the FP32 one."""
    X = datagen.gist_like(8000, d=960, k=80, seed=21)
    Q = datagen.gist_like(400, d=960, k=80, seed=21, stream=1)
    R, T1, T2 = 48, 3, 3
    oa, ok, _ = orc.build_graph(X, R=R, T1=T1, T2=T2, seed=8)
    kth = orc.knn_kth_dist(X, Q, 10)
    ent = orc.medoid(X)
    ro = orc.recall_at_k(X, Q, orc.search(X, oa, Q, k=10, L=64, entry=ent)[0], kth)
    ref = None
    for name in ("fp32",) + NARROW:
        print(f"case: gistlike d960 {name}", flush=True)
        p = params(g, R, T1=T1, T2=T2)
        p.precision = prec_code(g, name)
        ga, gk, _ = gpu_build(g, X, R, p, seed=8)
        if ref is None:
            ref = (ga, gk)
            orc.check_invariants(X, ga, gk, exact=False, rtol=1e-5)
            rg = orc.recall_at_k(X, Q, orc.search(X, ga, Q, k=10, L=64, entry=ent)[0], kth)
            assert abs(rg - ro) <= 0.005, (name, rg, ro)
        else:
            assert np.array_equal(ga, ref[0]) and np.array_equal(gk, ref[1]), name


def test_narrow_step_equals_fp32_step_integer(g, orc):
    """One update step with narrow tiles on integer data equals the oracle bit
    for bit (BF16 and FP16 hold these values exactly; FP8 does not, and its
    comparisons near a threshold are re-decided)."""
    X = int_data(3000, 128)
    R = 32
    ids, keys = state(orc, X, R)
    oi, ok, _, _ = orc.update_round(X, ids, keys, seed=11, round=5)
    for name in NARROW:
        p = params(g, R)
        p.precision = prec_code(g, name)
        gi, gk, _ = gpu_step(g, X, ids, keys, 11, 5, g.STEP_UPDATE, p)
        assert_rows_equal(gi, gk, oi, ok)
