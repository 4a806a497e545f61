"""The pool check of grnnd_step (params.check = 1), through the C ABI.

A step's read pool must be canonical: per row, valid entries first with ids
in [0, n), none the row's own id and none twice, strictly ascending by
(key, id), each key the canonical distance; padding is id -1 with key +inf.
With the check on, a canonical pool steps exactly as without it, and each
kind of damage is refused with GRNND_EINVAL naming the first damaged row.
Pools written by the library (initial draw, update and reverse steps) pass;
so do the oracle's initial pools on integer-valued rows, whose keys are
exact and therefore equal to the canonical FP32 distance."""
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


def _setup(g, n, d, R, S, metric, seed=3):
    if metric == 0:
        X = datagen.sift_like(n, d=d, k=20, seed=seed)
    else:
        X = datagen.angular(n, d=d, k=20, seed=seed)
    Xd = torch.from_numpy(X).cuda()
    p = g.grnnd_params_default(R, 2)
    p.S = S
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, p))
    ids = torch.empty((n, R), dtype=torch.int32, device="cuda")
    keys = torch.empty((n, R), dtype=torch.float32, device="cuda")
    st = torch.zeros(g.NSTATS, dtype=torch.int64, device="cuda")
    g.grnnd_init_pools(Xd, metric, R, S, 7, ids, keys, st, ws)
    torch.cuda.synchronize()
    return X, Xd, p, ws, ids, keys, st


def _step(g, Xd, metric, R, ids, keys, p, ws, st, kind=0, rnd=0):
    oi = torch.empty_like(ids)
    ok = torch.empty_like(keys)
    g.grnnd_step(Xd, metric, R, ids, keys, oi, ok, 7, rnd, kind, p, st, ws)
    torch.cuda.synchronize()
    return oi, ok


@pytest.mark.parametrize("metric,d", [(0, 40), (0, 37), (1, 100)])
def test_check_passes_library_pools_and_changes_nothing(g, metric, d):
    print(f"case: metric={metric} d={d}", flush=True)
    n, R = 3000, 16
    X, Xd, p, ws, ids, keys, st = _setup(g, n, d, R, 12, metric)
    a = _step(g, Xd, metric, R, ids, keys, p, ws, st)
    p.check = 1
    b = _step(g, Xd, metric, R, ids, keys, p, ws, st)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # the update step's and the reverse step's write pools are canonical too
    c = _step(g, Xd, metric, R, b[0], b[1], p, ws, st, kind=1, rnd=0)
    _step(g, Xd, metric, R, c[0], c[1], p, ws, st, kind=0, rnd=1)


def test_check_passes_oracle_pools_on_integer_rows(g, orc):
    n, d, R, S = 2000, 24, 16, 16
    X = datagen.sift_like(n, d=d, k=20, seed=5)
    oi, okk, _ = orc.init(X, R, S=S, seed=11, metric=0)
    Xd = torch.from_numpy(X).cuda()
    p = g.grnnd_params_default(R, 2)
    p.check = 1
    ws = g.workspace(g.grnnd_workspace_size(n, d, R, p))
    st = torch.zeros(g.NSTATS, dtype=torch.int64, device="cuda")
    _step(g, Xd, 0, R, torch.from_numpy(oi).cuda(), torch.from_numpy(okk).cuda(), p, ws, st)


def _damaged(g, Xd, metric, R, ids, keys, p, ws, st, fn):
    i = ids.cpu().numpy().copy()
    k = keys.cpu().numpy().copy()
    fn(i, k)
    p.check = 1
    with pytest.raises(g.GrnndError) as e:
        _step(g, Xd, metric, R, torch.from_numpy(i).cuda(), torch.from_numpy(k).cuda(), p, ws,
              st)
    return str(e.value)


def test_check_names_each_kind_of_damage(g):
    n, d, R, S, metric = 3000, 40, 16, 12, 0
    X, Xd, p, ws, ids, keys, st = _setup(g, n, d, R, S, metric)
    r = 1234

    def out_of_range(i, k):
        i[r, 0] = n
    assert f"row {r} " in (m := _damaged(g, Xd, metric, R, ids, keys, p, ws, st, out_of_range)) \
        and "outside" in m

    def negative(i, k):
        i[r, 3] = -7
    assert "outside" in _damaged(g, Xd, metric, R, ids, keys, p, ws, st, negative)

    def self_id(i, k):
        i[r, 0] = r
    assert "own id" in _damaged(g, Xd, metric, R, ids, keys, p, ws, st, self_id)

    def hole(i, k):
        i[r, 0] = -1
        k[r, 0] = np.inf
    assert "after padding" in _damaged(g, Xd, metric, R, ids, keys, p, ws, st, hole)

    def pad_key(i, k):
        k[r, S] = 1.0
    assert "padding" in _damaged(g, Xd, metric, R, ids, keys, p, ws, st, pad_key)

    def duplicate(i, k):
        i[r, 1] = i[r, 0]
    assert "twice" in _damaged(g, Xd, metric, R, ids, keys, p, ws, st, duplicate)

    def swapped(i, k):
        i[r, [0, 1]] = i[r, [1, 0]]
        k[r, [0, 1]] = k[r, [1, 0]]
    assert "ascending" in _damaged(g, Xd, metric, R, ids, keys, p, ws, st, swapped)

    def wrong_key(i, k):
        k[r, S - 1] = np.nextafter(k[r, S - 1], np.float32(np.inf))
    assert "canonical distance" in _damaged(g, Xd, metric, R, ids, keys, p, ws, st, wrong_key)

    def two_rows(i, k):
        i[2900, 0] = 2900
        k[17, 2] = np.float32(k[17, 2] * 0.5)
    m = _damaged(g, Xd, metric, R, ids, keys, p, ws, st, two_rows)
    assert "row 17 " in m
