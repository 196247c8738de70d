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


def test_residual_targets_fit_the_heuristic_slope():
    rng = np.random.default_rng(5)
    hs = [placement.standardise(rng.normal(size=n)) for n in (100, 300)]
    noise = [rng.normal(scale=0.1, size=h.size) for h in hs]
    ts = [0.8 * h + e for h, e in zip(hs, noise)]
    a, r = placement.residual_targets(ts, hs)
    h, t = np.concatenate(hs), np.concatenate(ts)
    # the least-squares slope through the origin, and residuals orthogonal to h
    assert abs(a - float((t * h).sum() / (h * h).sum())) < 1e-12
    assert abs(a - 0.8) < 0.05
    assert np.allclose(r, t - a * h, atol=1e-6)
    assert abs(float((r.astype(np.float64) * h).sum())) < 1e-3
    # labels that are exactly a multiple of h leave nothing to learn
    a2, r2 = placement.residual_targets([2.0 * hs[0]], [hs[0]])
    assert abs(a2 - 2.0) < 1e-12 and np.abs(r2).max() < 1e-6


def test_heuristic_log_orders_slots_as_area_times_emptiness():
    rng = np.random.default_rng(2)
    X = torch.zeros((500, 12), dtype=torch.float32)
    X[:, 3] = torch.from_numpy(rng.uniform(-0.6, 0.0, 500).astype(np.float32))   # log2(area) / 32
    X[:, 6] = torch.from_numpy(rng.choice(np.arange(0, 216) / 216.0, 500).astype(np.float32))
    h = placement.heuristic_log(X).numpy()
    s = placement.heuristic_scores(X)
    keep = s > 0
    assert (np.argsort(-h[keep], kind="stable") == np.argsort(-s[keep], kind="stable")).mean() > 0.99
    # a full mask gets the floor, below every non-full slot of the same area
    X2 = X.clone()
    X2[:, 6] = 1.0
    assert (placement.heuristic_log(X2).numpy() < h - 1e-6).all()
    sd = placement.standardise(h)
    assert abs(sd.mean()) < 1e-9 and abs(sd.std() - 1.0) < 1e-9
    assert (placement.standardise(np.ones(7)) == 0).all()
