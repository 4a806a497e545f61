"""The library's approximate medoid (the default entry point of the search,
Section 4.1) against the oracle's, through the C ABI.

Bars: on integer-valued data every FP64 column sum is exact in any order, so
the mean, every distance to it and the chosen id must equal the oracle's
exactly (including the smaller-id rule on exact ties); on float data the
column sums may round differently, so the chosen id must be the oracle's or
a point whose exact distance to the exact mean is within 1e-12 relative of
the smallest one."""
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


def _gpu_medoid(g, X):
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    out = g.medoid(Xd)
    torch.cuda.synchronize()
    return int(out.item())


def _near_min(X, e):
    X64 = X.astype(np.float64)
    m = X64.mean(0)
    dd = ((X64 - m) ** 2).sum(1)
    return dd[e] <= dd.min() * (1.0 + 1e-12) + 1e-300


@pytest.mark.parametrize("n,d", [(2, 1), (37, 3), (20000, 128), (6001, 130), (3000, 960)])
def test_medoid_integer_exact(g, orc, n, d):
    print(f"case: integer n={n} d={d}", flush=True)
    X = datagen.sift_like(n, d=d, k=max(2, n // 50), seed=13)
    if d == 960:
        X = np.minimum(X, 60.0).astype(np.float32)
    assert _gpu_medoid(g, X) == orc.medoid(X)


def test_medoid_ties_take_the_smaller_id(g, orc):
    # symmetric around the mean: rows 2 and 3 are equally near; 2 wins
    X = np.array([[-3.0], [3.0], [0.5], [-0.5]], np.float32)
    assert orc.medoid(X) == 2 and _gpu_medoid(g, X) == 2
    # duplicate rows nearest the mean: the first copy wins
    X = np.array([[0, 0], [4, 4], [2, 2], [2, 2], [1, 3]], np.float32)
    assert orc.medoid(X) == 2 and _gpu_medoid(g, X) == 2
    X = np.array([[4, 4], [2, 2], [0, 0], [2, 2]], np.float32)
    assert orc.medoid(X) == 1 and _gpu_medoid(g, X) == 1


@pytest.mark.parametrize("name,n,d", [("mixture", 30000, 128), ("gist", 5000, 960),
                                      ("angular", 20000, 100)])
def test_medoid_float_valid(g, orc, name, n, d):
    print(f"case: float {name} n={n} d={d}", flush=True)
    X = {"mixture": lambda: datagen.mixture(n, d=d, k=50, seed=3),
         "gist": lambda: datagen.gist_like(n, d=d, k=100, seed=4),
         "angular": lambda: datagen.angular(n, d=d, k=200, seed=5)}[name]()
    e = _gpu_medoid(g, X)
    o = orc.medoid(X)
    assert e == o or _near_min(X, e), (e, o)


def test_search_default_entry_is_the_medoid(g, orc):
    """grnnd_search with entry < 0 starts from the medoid: on integer data its
    results equal the oracle's search from the oracle's medoid, bit for bit."""
    X = datagen.sift_like(8000, d=64, k=40, seed=21)
    Q = datagen.sift_like(300, d=64, k=40, seed=21, stream=1)
    adj, _, _ = orc.build_graph(X, R=16, T1=2, T2=2, seed=3)
    oi, ok = orc.search(X, adj, Q, k=10, L=32, entry=orc.medoid(X))
    gi, gk = g.search(torch.from_numpy(X).cuda(), torch.from_numpy(adj).cuda(),
                      torch.from_numpy(Q).cuda(), k=10, L=32, entry=-1)
    torch.cuda.synchronize()
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gk.cpu().numpy(), ok)
