"""The allocation-free construction (grnnd_build_noalloc, scratch in a static
device array) against grnnd_build_ex with a caller workspace, through the C
ABI: two calls in a row on one GPU, the second smaller than the first, must
each equal the workspace build bit for bit (ids, keys and counters); the
scratch array keeps the first call's contents, so the second call also shows
that everything that must start at zero is cleared."""
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


def _pair(g, X, R, metric, T1, T2, precision, seed):
    n, d = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    p = g.grnnd_params_default(R, T1)
    p.T2 = T2
    p.precision = precision
    assert g.grnnd_workspace_size(n, d, R, p) <= g.NOALLOC_SCRATCH_BYTES
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, p))
    out = []
    for noalloc in (False, True):
        adj = torch.full((n, R), -7, dtype=torch.int32, device="cuda")
        keys = torch.full((n, R), -7.0, dtype=torch.float32, device="cuda")
        st = torch.zeros(g.NSTATS, dtype=torch.int64, device="cuda")
        if noalloc:
            g.grnnd_build_noalloc(Xd, metric, R, p, seed, adj, keys, st)
        else:
            g.grnnd_build_ex(Xd, metric, R, p, seed, adj, keys, st, ws)
        torch.cuda.synchronize()
        out.append((adj.cpu().numpy(), keys.cpu().numpy(), st.cpu().numpy()))
    return out


CASES = [
    # (name, n, d, R, metric, T1, T2, precision)
    ("float mixture 40000 x 128 L2 R32", 40000, 128, 32, 0, 3, 3, 0),
    ("float angular 9000 x 100 IP R16", 9000, 100, 16, 1, 2, 3, 0),
    ("integer 6000 x 96 L2 R32 BF16 tiles", 6000, 96, 32, 0, 2, 2, 1),
]


def _data(name, n, d):
    if name.startswith("integer"):
        return datagen.sift_like(n, d=d, k=20, seed=3)
    if "angular" in name:
        return datagen.angular(n, d=d, k=40, seed=4)
    return datagen.mixture(n, d=d, k=30, seed=5)


def test_noalloc_equals_workspace_build_two_calls_shrinking():
    import paper_2510_02774_amd as g
    for name, n, d, R, metric, T1, T2, prec in CASES:
        print(f"case: {name}", flush=True)
        X = _data(name, n, d)
        (a0, k0, s0), (a1, k1, s1) = _pair(g, X, R, metric, T1, T2, prec, seed=11)
        assert np.array_equal(a0, a1), name
        assert np.array_equal(k0.view(np.uint32), k1.view(np.uint32)), name
        assert np.array_equal(s0, s1), name
        assert (a1[:, 0] >= 0).all(), name


def test_noalloc_refuses_too_large_and_keeps_working():
    import paper_2510_02774_amd as g
    X = torch.zeros((1, 4), dtype=torch.float32, device="cuda")
    adj = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    L = g.lib()
    import ctypes as C
    rc = L.grnnd_build_noalloc(C.c_void_p(X.data_ptr()), 1_000_000, 128, 0, 32, None, 1,
                               C.c_void_p(adj.data_ptr()), None, None, None)
    assert rc == -2 and "scratch" in g.grnnd_last_error()
    Xs = datagen.sift_like(3000, d=64, k=10, seed=9)
    (a0, k0, _), (a1, k1, _) = _pair(g, Xs, 16, 0, 2, 2, 0, seed=5)
    assert np.array_equal(a0, a1) and np.array_equal(k0, k1)
