"""Training targets of the placement network (host logic, no GPU): the
label standardised within its scene, the scene's highest labels always
sampled, the rest drawn uniformly and reproducibly."""
import numpy as np
import torch

from paper_2305_08343_amd import placement


def _labels(S, seed=1):
    rng = np.random.default_rng(seed)
    y = np.where(rng.random(S) < 0.7, 0.0, rng.exponential(3.0, S))
    return torch.from_numpy(y.astype(np.float32))


def test_small_scene_keeps_every_slot_and_standardises():
    y = _labels(1000)
    idx, t = placement.scene_targets(y, 4096, seed=3)
    assert np.array_equal(idx, np.arange(1000))
    yy = y.numpy().astype(np.float64)
    assert np.allclose(t, (yy - yy.mean()) / yy.std(), atol=1e-6)
    assert abs(float(np.mean(t))) < 1e-5 and abs(float(np.std(t)) - 1.0) < 1e-5


def test_large_scene_samples_top_quarter_plus_uniform_rest():
    S, M = 50_000, 4096
    y = _labels(S)
    idx, t = placement.scene_targets(y, M, seed=7)
    assert idx.size == M and np.all(np.diff(idx) > 0)
    yy = y.numpy().astype(np.float64)
    top = np.argsort(-yy, kind="stable")[:M // 4]
    assert np.isin(top, idx).all()
    # targets are standardised over all S slots, not over the sample
    assert np.allclose(t, ((yy - yy.mean()) / yy.std())[idx], atol=1e-6)
    # the rest is a uniform draw: its mean label is close to the mean outside the top
    rest = np.setdiff1d(idx, top)
    outside = np.setdiff1d(np.arange(S), top)
    assert abs(yy[rest].mean() - yy[outside].mean()) < 0.15
    idx2, t2 = placement.scene_targets(y, M, seed=7)
    assert np.array_equal(idx, idx2) and np.array_equal(t, t2)


def test_constant_labels_give_zero_targets():
    idx, t = placement.scene_targets(torch.zeros(10_000), 512, seed=0)
    assert idx.size == 512 and np.all(t == 0.0)
