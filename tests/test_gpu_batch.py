"""Batched builds (shared launches over several collections, the serving
form) through the C ABI.

Bar: every collection of a batch equals grnnd_build_ex on it alone with its
seed, bit for bit (ids, keys); on integer-valued data also the oracle's
build. The server, given many queued requests of one class, batches them
(its counters show it) and every result still equals the build alone."""
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


def _params(g, R, T1=2, T2=2, prec=0):
    p = g.grnnd_params_default(R, T1)
    p.T2 = T2
    p.precision = prec
    return p


def _alone(g, X, R, p, seed, metric):
    a, k = g.build_graph(torch.from_numpy(X).cuda(), R, p, seed=seed, metric=metric)
    torch.cuda.synchronize()
    return a.cpu().numpy(), k.cpu().numpy()


@pytest.mark.parametrize("case", ["mixture_l2_d128", "angular_ip_d100", "integer_d130",
                                  "bf16_l2_d96", "tiny_and_large_r48", "gist_l2_d640",
                                  "angular_ip_d768"])
def test_batch_equals_alone(g, case):
    rng = np.random.default_rng(3)
    if case == "mixture_l2_d128":
        d, R, metric, prec = 128, 32, 0, 0
        Xs = [datagen.mixture(int(n), d=d, k=20, seed=100 + i)
              for i, n in enumerate([3000, 517, 12000, 2, 4099])]
    elif case == "angular_ip_d100":
        d, R, metric, prec = 100, 16, 1, 0
        Xs = [datagen.angular(int(n), d=d, k=30, seed=200 + i)
              for i, n in enumerate([2500, 7001, 64])]
    elif case == "integer_d130":
        d, R, metric, prec = 130, 24, 0, 0
        Xs = [datagen.sift_like(int(n), d=d, k=25, seed=300 + i)
              for i, n in enumerate([1800, 2600, 999])]
    elif case == "bf16_l2_d96":
        d, R, metric, prec = 96, 32, 0, 1
        Xs = [datagen.mixture(int(n), d=d, k=15, seed=400 + i) for i, n in enumerate([3500, 2100])]
    elif case == "gist_l2_d640":  # rows of 512 or more: redirect keys computed in the merge
        d, R, metric, prec = 640, 48, 0, 0
        Xs = [datagen.gist_like(int(n), d=d, k=30, seed=700 + i)
              for i, n in enumerate([2500, 900, 4000])]
    elif case == "angular_ip_d768":
        d, R, metric, prec = 768, 32, 1, 0
        Xs = [datagen.angular(int(n), d=d, k=30, seed=800 + i) for i, n in enumerate([1500, 3000])]
    else:
        d, R, metric, prec = 64, 48, 0, 0
        Xs = [datagen.mixture(int(n), d=d, k=40, seed=500 + i)
              for i, n in enumerate([3, 20000, 49, 6000])]
    print(f"case: {case}", flush=True)
    p = _params(g, R, prec=prec)
    seeds = [int(s) for s in rng.integers(1, 1 << 40, size=len(Xs))]
    outs = g.build_batch([torch.from_numpy(X).cuda() for X in Xs], R, p, seeds=seeds, metric=metric)
    torch.cuda.synchronize()
    for X, s, (a, k) in zip(Xs, seeds, outs):
        a0, k0 = _alone(g, X, R, p, s, metric)
        assert np.array_equal(a.cpu().numpy(), a0), (case, X.shape)
        assert np.array_equal(k.cpu().numpy(), k0), (case, X.shape)


def test_batch_integer_equals_oracle(g, orc):
    Xs = [datagen.sift_like(n, d=48, k=20, seed=600 + i) for i, n in enumerate([2000, 3100, 700])]
    R, seeds = 16, [5, 6, 7]
    p = _params(g, R, T1=3, T2=2)
    outs = g.build_batch([torch.from_numpy(X).cuda() for X in Xs], R, p, seeds=seeds)
    torch.cuda.synchronize()
    for X, s, (a, k) in zip(Xs, seeds, outs):
        oa, ok, _ = orc.build_graph(X, R=R, T1=3, T2=2, seed=s)
        assert np.array_equal(a.cpu().numpy(), oa)
        assert np.array_equal(k.cpu().numpy(), ok)


def test_server_batches_queued_requests(g):
    """Twenty requests of two classes queued on a one-slot server: the
    server runs them as batched builds, and each result equals its build
    alone."""
    reqs = []
    for i in range(20):
        d, metric = (128, 0) if i % 2 == 0 else (96, 1)
        n = [2000, 3500, 800, 6000][i % 4]
        X = datagen.mixture(n, d=d, k=20, seed=700 + i)
        if metric == 1:
            X = (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)
        reqs.append((X, metric, 16 if metric else 32, 900 + i))
    srv = g.Server(4 << 30, slots=1)
    try:
        srv.set_batch(8, 1 << 16)
        subs = [srv.submit(torch.from_numpy(X).cuda(), R, _params(g, R), seed=s, metric=m)
                for X, m, R, s in reqs]
        srv.drain()
        st = srv.stats()
        assert st.completed == len(reqs) and st.failed == 0
        assert st.batches >= 2 and st.batched_requests >= 8, (st.batches, st.batched_requests)
        for (X, m, R, s), (t, adj, keys) in zip(reqs, subs):
            a0, k0 = _alone(g, X, R, _params(g, R), s, m)
            assert np.array_equal(adj.cpu().numpy(), a0)
            assert np.array_equal(keys.cpu().numpy(), k0)
    finally:
        srv.close()
