"""Host logic of the benchmark's recall measurement, on the CPU: the exact
ground truth (FP32 pre-filter per chunk of points, FP64 re-rank) against
brute force, the tie-aware Recall@k and the plain id-overlap form (the
paper's Recall@k definition, Section 2.1)."""
import numpy as np
import pytest
import torch

import bench


def _brute(X, Q, metric):
    X64, Q64 = X.astype(np.float64), Q.astype(np.float64)
    if metric == 0:
        return ((X64[None, :, :] - Q64[:, None, :]) ** 2).sum(-1)
    return -(Q64 @ X64.T)


@pytest.mark.parametrize("metric", [0, 1])
def test_ground_truth_equals_brute_force(metric):
    rng = np.random.default_rng(4)
    X = rng.integers(0, 40, size=(3000, 16)).astype(np.float32)
    Q = rng.integers(0, 40, size=(40, 16)).astype(np.float32)
    kth, top = bench._ground_truth(torch.from_numpy(X), torch.from_numpy(Q), metric, 10,
                                   chunk=700)
    E = _brute(X, Q, metric)
    for qi in range(Q.shape[0]):
        order = np.lexsort((np.arange(X.shape[0]), E[qi]))  # by (key, id)
        assert kth[qi].item() == E[qi, order[9]]
        assert np.array_equal(top[qi].numpy(), order[:10])


def test_ground_truth_keeps_the_kth_key_under_heavy_ties():
    # four values per coordinate: thousands of exact ties at every distance;
    # the k-th key is still exact and the returned ids carry the k smallest keys
    rng = np.random.default_rng(3)
    X = rng.integers(0, 4, size=(3000, 8)).astype(np.float32)
    Q = rng.integers(0, 4, size=(30, 8)).astype(np.float32)
    kth, top = bench._ground_truth(torch.from_numpy(X), torch.from_numpy(Q), 0, 10, chunk=700)
    E = _brute(X, Q, 0)
    for qi in range(Q.shape[0]):
        srt = np.sort(E[qi])
        assert kth[qi].item() == srt[9]
        assert np.array_equal(np.sort(E[qi, top[qi].numpy()]), srt[:10])


def test_recall_forms_by_hand():
    X = np.array([[0.0], [1.0], [2.0], [2.0], [5.0]], np.float32)
    Q = np.array([[0.0]], np.float32)
    Xd, Qd = torch.from_numpy(X), torch.from_numpy(Q)
    kth, top = bench._ground_truth(Xd, Qd, 0, 3)
    assert kth[0].item() == 4.0 and top[0].tolist() == [0, 1, 2]
    # ids 0, 1, 3: tie-aware counts all three (d(3) = 4 <= 4), id overlap two
    ids = torch.tensor([[0, 1, 3]], dtype=torch.int32)
    assert bench._recall(Xd, Qd, ids, kth, 0, k=3) == 1.0
    assert abs(bench._id_overlap(ids, top, k=3) - 2.0 / 3.0) < 1e-12
    # a missing result (-1) counts for neither
    ids = torch.tensor([[0, -1, 4]], dtype=torch.int32)
    assert abs(bench._recall(Xd, Qd, ids, kth, 0, k=3) - 1.0 / 3.0) < 1e-12
    assert abs(bench._id_overlap(ids, top, k=3) - 1.0 / 3.0) < 1e-12
