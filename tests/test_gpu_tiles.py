"""GPU tests of the distance tiles the update rounds decide Eq. 2 from, read
back through grnnd_tile_probe on candidate sets taken from real pools (the
pools after the initial draw and one update round).

Bars:
  * integer-valued data: the FP32 tile, and the BF16 / FP16 tiles of
    integers they hold exactly, equal the canonical distance, which equals
    the exact distance, bit for bit;
  * every precision, float data: for every pair the tile's distance lies
    within the recheck band of the canonical distance, which is what makes a
    decision taken outside the band equal the canonical one;
  * the canonical distance is within its error bound of the exact FP64
    distance ((d/16 + 6) u relative for L2, u = 2^-24; for the inner product
    relative to sum |a_k b_k|).
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16", "fp16", "fp8"]


@pytest.fixture(scope="module")
def g():
    import paper_2510_02774_amd as g
    g.lib()
    assert torch.cuda.is_available()
    return g


def prec_code(g, name):
    return {"fp32": g.PREC_FP32, "bf16": g.PREC_BF16, "fp16": g.PREC_FP16,
            "fp8": g.PREC_FP8_E4M3}[name]


def real_sets(g, X, R, metric, nsample, seed=3):
    """Candidate sets of nsample vertices after init and one update round."""
    n, d = X.shape
    p = g.grnnd_params_default(R, 1)
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, p))
    Xd = torch.from_numpy(X).cuda()
    ids = torch.empty((n, R), dtype=torch.int32, device="cuda")
    keys = torch.empty((n, R), dtype=torch.float32, device="cuda")
    g.grnnd_init_pools(Xd, metric, R, R, seed, ids, keys, None, ws)
    oi, ok = torch.empty_like(ids), torch.empty_like(keys)
    g.grnnd_step(Xd, metric, R, ids, keys, oi, ok, seed, 0, g.STEP_UPDATE, p, None, ws)
    torch.cuda.synchronize()
    rows = np.random.default_rng(seed).choice(n, size=nsample, replace=False)
    return Xd, oi[torch.from_numpy(rows).cuda()].contiguous()


def probe(g, Xd, sets, metric, prec):
    R = sets.shape[1]
    p = g.grnnd_params_default(R, 1)
    p.precision = prec_code(g, prec)
    t, b, c = g.tile_probe(Xd, sets, p, metric)
    torch.cuda.synchronize()
    return t.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()


def exact(X, sets, metric):
    """FP64 distance of every ordered pair of each set (NaN where absent)."""
    nv, R = sets.shape
    out = np.full((nv, R, R), np.nan)
    X64 = X.astype(np.float64)
    for q in range(nv):
        ids = sets[q][sets[q] >= 0]
        Y = X64[ids]
        if metric == 0:
            D = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
        else:
            D = -(Y @ Y.T)
        k = len(ids)
        out[q, :k, :k] = D
        np.fill_diagonal(out[q], np.nan)
    return out


def scale(X, sets, metric):
    """Natural scale of each pair's canonical error bound."""
    nv, R = sets.shape
    out = np.full((nv, R, R), np.nan)
    A = np.abs(X.astype(np.float64))
    for q in range(nv):
        ids = sets[q][sets[q] >= 0]
        k = len(ids)
        if metric == 0:
            Y = X[ids].astype(np.float64)
            out[q, :k, :k] = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
        else:
            out[q, :k, :k] = A[ids] @ A[ids].T
    return out


def test_probe_integer_tiles_exact(g):
    X = datagen.sift_like(3000, d=128, k=40, seed=5)
    Xd, sets = real_sets(g, X, 32, 0, 200)
    s = sets.cpu().numpy()
    ex = exact(X, s, 0)
    m = ~np.isnan(ex)
    assert m.sum() > 100_000
    for prec in ["fp32", "bf16", "fp16"]:
        t, b, c = probe(g, Xd, sets, 0, prec)
        assert np.array_equal(c[m], ex[m].astype(np.float32)), prec
        assert np.array_equal(t[m], c[m]), prec
        assert (b[m] >= 0).all(), prec
        assert np.isnan(t[~m]).all() and np.isnan(c[~m]).all(), prec


CASES = {
    "mixture_d128": (lambda: datagen.mixture(4000, d=128, k=50, sigma=0.15, seed=1), 0, 32),
    "siftlike_d128": (lambda: datagen.sift_like(4000, d=128, k=40, seed=5), 0, 32),
    "gistlike_d960": (lambda: datagen.gist_like(1500, d=960, k=40, seed=21), 0, 48),
    "angular_ip_d100": (lambda: datagen.angular(4000, d=100, k=200, seed=31), 1, 32),
}


@pytest.mark.parametrize("case", list(CASES))
def test_probe_band_covers_tile_error(g, case):
    make, metric, R = CASES[case]
    X = make()
    Xd, sets = real_sets(g, X, R, metric, 150)
    s = sets.cpu().numpy()
    ex = exact(X, s, metric)
    sc = scale(X, s, metric)
    m = ~np.isnan(ex)
    d16 = -(-X.shape[1] // 16) * 16
    u = 2.0 ** -24
    first = None
    for prec in PRECS:
        t, b, c = probe(g, Xd, sets, metric, prec)
        assert not np.isnan(t[m]).any() and not np.isnan(c[m]).any(), prec
        err = np.abs(t[m].astype(np.float64) - c[m].astype(np.float64))
        assert (err <= b[m]).all(), (prec, float((err - b[m]).max()))
        # the canonical distance is the same whatever the tile precision
        if first is None:
            first = c
        assert np.array_equal(c[m], first[m]), prec
    bound = 1.01 * (d16 / 16 + 6) * u * sc[m]  # first-order bound, 1% for higher terms
    assert (np.abs(first[m].astype(np.float64) - ex[m]) <= bound).all()
