"""GPU tests of the build server (continuous batching of many builds).

The bar: every build's result, run in the mix with others (overlapping on
the device, admitted as slots and arena room free up), equals the same build
run alone with grnnd_build_ex, bit for bit; the arena never exceeds its
budget; a request that can never fit is refused with EBUDGET.
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2510_02774_amd as g
    g.lib()
    assert torch.cuda.is_available()
    return g


def _requests():
    """A ragged mix: sizes, dimensions, metrics, pool widths and tile
    precisions all vary (inner-product rows are unit-normalised)."""
    rng = np.random.default_rng(5)
    out = []
    for i in range(14):
        n = int(np.exp(rng.uniform(np.log(2000), np.log(20000))))
        d = int(rng.choice([96, 128, 384, 768]))
        metric = int(i % 2)
        R = int(rng.choice([16, 32]))
        X = datagen.mixture(n, d=d, k=int(rng.integers(20, 200)), sigma=0.15, seed=1000 + i)
        if metric == 1:
            X = (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)
        prec = [0, 0, 1, 2][i % 4]
        out.append((X, metric, R, prec, 1000 + i))
    return out


def _params(g, R, prec):
    p = g.grnnd_params_default(R, 2)
    p.T2 = 2
    p.precision = prec
    return p


def _alone(g, X, metric, R, prec, seed):
    adj, keys = g.build_graph(torch.from_numpy(X).cuda(), R, _params(g, R, prec), seed=seed,
                              metric=metric)
    torch.cuda.synchronize()
    return adj.cpu().numpy(), keys.cpu().numpy()


def _serve(g, reqs, budget, slots):
    srv = g.Server(budget, slots=slots)
    try:
        subs = []
        for X, metric, R, prec, seed in reqs:
            t, adj, keys = srv.submit(torch.from_numpy(X).cuda(), R, _params(g, R, prec),
                                      seed=seed, metric=metric)
            subs.append((t, adj, keys))
        srv.drain()
        st = srv.stats()
        res = []
        for t, adj, keys in subs:
            state, lat = srv.poll(t)
            assert state == g.REQ_DONE, state
            assert lat > 0.0
            res.append((adj.cpu().numpy(), keys.cpu().numpy()))
        return res, st
    finally:
        srv.close()


def test_server_mix_equals_alone(g):
    reqs = _requests()
    res, st = _serve(g, reqs, budget=6 << 30, slots=4)
    assert st.submitted == len(reqs) and st.completed == len(reqs) and st.failed == 0
    assert st.peak_inflight >= 2, st.peak_inflight  # builds overlapped on the device
    for (X, metric, R, prec, seed), (adj, keys) in zip(reqs, res):
        a0, k0 = _alone(g, X, metric, R, prec, seed)
        assert np.array_equal(adj, a0), (X.shape, metric, R, prec)
        assert np.array_equal(keys, k0), (X.shape, metric, R, prec)


def test_server_budget_admission(g):
    """A budget that holds only about two of the largest workspaces: requests
    wait for arena room, peak use stays within the budget, results unchanged."""
    reqs = _requests()[:8]
    sizes = [g.grnnd_workspace_size(X.shape[0], X.shape[1], R, _params(g, R, prec))
             for X, metric, R, prec, _ in reqs]
    budget = int(2.2 * max(sizes)) // 256 * 256
    res, st = _serve(g, reqs, budget=budget, slots=8)
    assert st.completed == len(reqs)
    assert st.peak_arena_bytes <= budget
    for (X, metric, R, prec, seed), (adj, keys) in zip(reqs, res):
        a0, k0 = _alone(g, X, metric, R, prec, seed)
        assert np.array_equal(adj, a0) and np.array_equal(keys, k0)


def test_server_refuses_what_never_fits(g):
    srv = g.Server(1 << 20, slots=1)
    try:
        X = torch.from_numpy(datagen.mixture(5000, d=128, k=20, seed=3)).cuda()
        with pytest.raises(g.GrnndError) as e:
            srv.submit(X, 32, _params(g, 32, 0))
        assert e.value.code == -4
    finally:
        srv.close()


def test_served_requests_match_the_oracle(g, orc):
    """Serving-shaped requests against the oracle's graph. Integer-valued rows
    make every FP32 distance exact (d * max|a_k b_k| or d * max|a_k - b_k|^2
    well below 2^24), so a served L2 request at d = 384 and a served IP request
    at d = 768 equal the oracle's build bit for bit; a float L2 request at
    d = 384 (unit-free mixture) is held to Recall@10 within 0.5 points of the
    oracle graph's. They run in the server mixed with float requests."""
    rng = np.random.default_rng(77)
    n1, n2, n3 = 3000, 2500, 3000
    c1 = rng.integers(0, 61, size=(30, 384))
    X1 = np.clip(c1[rng.integers(0, 30, n1)] + rng.integers(-6, 7, size=(n1, 384)), 0, 60)
    c2 = rng.integers(-8, 9, size=(25, 768))
    X2 = np.clip(c2[rng.integers(0, 25, n2)] + rng.integers(-2, 3, size=(n2, 768)), -8, 8)
    X1, X2 = X1.astype(np.float32), X2.astype(np.float32)
    X3 = datagen.mixture(n3, d=384, k=40, sigma=0.15, seed=4242)
    reqs = [(X1, 0, 32, 0, 501), (X2, 1, 16, 0, 502), (X3, 0, 32, 0, 503)]
    reqs += _requests()[:4]
    res, st = _serve(g, reqs, budget=4 << 30, slots=4)
    assert st.completed == len(reqs) and st.failed == 0
    for k in range(2):
        X, metric, R, _, seed = reqs[k]
        oa, ok, _ = orc.build_graph(X, R=R, T1=2, T2=2, seed=seed, metric=metric)
        assert np.array_equal(res[k][0], oa), (k, metric)
        assert np.array_equal(res[k][1], ok), (k, metric)
    X, metric, R, _, seed = reqs[2]
    Q = datagen.mixture(300, d=384, k=40, sigma=0.15, seed=4242, stream=1)
    oa, _, _ = orc.build_graph(X, R=R, T1=2, T2=2, seed=seed)
    kth = orc.knn_kth_dist(X, Q, 10)
    ent = orc.medoid(X)
    rg = orc.recall_at_k(X, Q, orc.search(X, res[2][0], Q, k=10, L=64, entry=ent)[0], kth)
    ro = orc.recall_at_k(X, Q, orc.search(X, oa, Q, k=10, L=64, entry=ent)[0], kth)
    assert abs(rg - ro) <= 0.005, (rg, ro)
