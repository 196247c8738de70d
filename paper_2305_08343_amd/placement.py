"""Learned mask placement (growth direction of the culling method).

Masks cost memory (27 bytes per slot at R = 6) and a test per slab hit; most
of the false-positive removal comes from few slots. A small MLP predicts,
from 12 geometric features of a child slot (its box relative to its parent
and to the root, depth, triangle count and thinness, mask occupancy, and where
its box sits in the scene), how many false-positive slab hits the slot's mask
removes; masks are then placed on the highest-scoring slots
until a budget of `beta` bytes per inner node is spent (SC_MASK_SPARSE). A
slot without a mask is traversed exactly as in plain BVH traversal, so every
placement returns the same hits as all masks and as no masks.

Training data: for each training scene, the shadow trace (culling off,
masks evaluated) counts per slot the slab hits whose mask test fails; the
label is log2(1 + 1e6 * count / rays). Placement only ranks the slots of one
scene against each other, so labels are standardised within their scene
(minus the scene's mean, over its standard deviation): the scene-wide level
of false positives, which the geometric features cannot see, no longer has
to be fitted. The network learns a correction to the importance the paper
gives a mask (surface area, here times emptiness, Sect. 3.2.2): with h the
log2 of area x emptiness standardised within its scene, and a the
least-squares slope of the standardised label on h over all training
samples, the regression target is label - a * h, and a slot's placement score
is a * h + the network's output. A network that outputs zero ranks exactly as
the heuristic; training moves the ranking where the features say the
heuristic is wrong. Each scene contributes its highest-label slots (a quarter
of its sample) plus a uniform draw of the rest, since the budget places masks
on the top few percent only. Training runs on the GPU through the library's
MLP kernels (forward, backward, Adam). This module only orchestrates:
sampling of batches, the label and heuristic transforms and bookkeeping use
torch tensors as plumbing.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import binding

MASK_BYTES_R6 = 27  # 216 bits


def he_init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the library's parameter layout."""
    rng = np.random.default_rng(seed)
    p = np.zeros(5057, np.float32)
    p[0:768] = rng.normal(0.0, math.sqrt(2.0 / 12), 768)              # W1 [64][12]
    p[832:4928] = rng.normal(0.0, math.sqrt(2.0 / 64), 4096)          # W2 [64][64]
    p[4992:5056] = rng.normal(0.0, math.sqrt(2.0 / 64), 64)           # W3 [64]
    return p


def slot_dataset(ctx, tris, rays, R: int = 6):
    """Features [S, 12] and labels [S] (device tensors) of one scene's slots."""
    import torch
    scene = binding.Scene(ctx, tris, R=R, mode="raw")
    S = 2 * scene.info["n_inner"]
    fp = torch.zeros(max(S, 1), dtype=torch.int32, device=f"cuda:{ctx.device}")
    rays_dev = torch.from_numpy(np.ascontiguousarray(rays, np.float32)).cuda(ctx.device)
    scene.trace(rays_dev, cull=False, shadow=True, slot_fp=fp, extra=False)
    X = scene.features()
    y = torch.log2(1.0 + 1e6 * fp[:S].double() / rays.shape[0]).float()
    info = dict(scene.info)
    scene.close()
    return X.contiguous(), y.contiguous(), info


def save_checkpoint(path: str, params, m, v, step: int, epoch: int, rng, hist) -> None:
    """Training state after `epoch` epochs: parameters, Adam moments and step, the batch-order
    generator's state and the loss history (an .npz written atomically)."""
    import json
    import os
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
             step=np.int64(step), epoch=np.int64(epoch), hist=np.asarray(hist, np.float64),
             rng=np.frombuffer(json.dumps(rng.bit_generator.state).encode(), np.uint8))
    os.replace(tmp, path)


def load_checkpoint(path: str, device):
    """(params, m, v, step, epoch, rng, hist) as written by save_checkpoint."""
    import json

    import torch
    with np.load(path, allow_pickle=False) as z:
        rng = np.random.default_rng()
        rng.bit_generator.state = json.loads(bytes(z["rng"]).decode())
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return (t(z["params"]), t(z["m"]), t(z["v"]), int(z["step"]), int(z["epoch"]), rng,
                [float(x) for x in z["hist"]])


def train(ctx, X, y, *, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 0, log=None,
          checkpoint: str | None = None, resume: bool = False):
    """Adam on the mean squared error; returns (params device tensor, loss history). With
    `checkpoint`, the training state is written there after every epoch; with `resume` as well,
    training continues from the state stored there (the same result as an uninterrupted run: the
    kernels are deterministic and the batch order's generator is restored)."""
    import os

    import torch
    dev = X.device
    N = X.shape[0]
    params = torch.from_numpy(he_init(seed)).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    act = torch.empty((batch, 128), dtype=torch.float32, device=dev)
    grad = torch.empty_like(params)
    work = torch.empty(binding.mlp_work_floats(batch), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    step, hist, start = 0, [], 0
    if checkpoint and resume and os.path.exists(checkpoint):
        params, m, v, step, start, rng, hist = load_checkpoint(checkpoint, dev)
        if log:
            log(f"resumed from {checkpoint} after epoch {start} (step {step})")
    for ep in range(start, epochs):
        perm = torch.from_numpy(rng.permutation(N)).to(dev)
        acc, nb = 0.0, 0
        for b0 in range(0, N - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb, yb = X[idx].contiguous(), y[idx].contiguous()
            pred = ctx.mlp_forward(params, xb, act)
            ctx.mlp_backward(params, xb, act, pred, yb, grad, work, loss)
            step += 1
            ctx.mlp_adam(params, grad, m, v, step, lr=lr)
            if nb % 64 == 0:
                acc += loss.item()
            nb += 1
        hist.append(acc / max(1, (nb + 63) // 64))
        if log:
            log(f"epoch {ep + 1}/{epochs}: {nb} steps, sampled mse {hist[-1]:.4f}")
        if checkpoint:
            save_checkpoint(checkpoint, params, m, v, step, ep + 1, rng, hist)
    return params, hist


def predict(ctx, params, X, chunk: int = 1 << 20):
    import torch
    out = []
    for i in range(0, X.shape[0], chunk):
        out.append(ctx.mlp_forward(params, X[i:i + chunk].contiguous()))
    return torch.cat(out) if out else torch.empty(0, device=X.device)


def budget_masks(beta: float, n_inner: int, mask_bytes: int = MASK_BYTES_R6) -> int:
    """Masks affordable with beta bytes per inner node."""
    return int(math.floor(beta * n_inner / mask_bytes))


def heuristic_log(X):
    """log2 of surface area (relative to the root) times emptiness, from the slot features
    (feature 3 = log2(area / root area) / 32, feature 6 = occupied fraction); emptiness is
    floored at 2^-9 (a mask that is not full at R = 6 has at least 1/216 empty)."""
    import torch
    return X[:, 3] * 32.0 + torch.log2(torch.clamp(1.0 - X[:, 6], min=2.0 ** -9))


def standardise(v):
    """(v - mean) / std over all entries (zeros where the std is 0), float64 numpy."""
    vv = np.asarray(v, np.float64)
    sd = float(vv.std()) if vv.size else 0.0
    return (vv - vv.mean()) / sd if sd > 0.0 else np.zeros_like(vv)


def heuristic_scores(X) -> np.ndarray:
    """Surface area times emptiness: SA(N) (1 - O_m(N)/R^3), the paper's
    mask importance (Sect. 3.2.2) turned towards masks that can cull."""
    f = X.cpu().numpy().astype(np.float64)
    return (np.exp2(f[:, 3] * 32.0) * (1.0 - f[:, 6])).astype(np.float32)


@dataclass
class Evaluation:
    name: str
    beta: float | None
    n_masks: int
    tests_per_ray: float
    box_per_ray: float
    tri_per_ray: float
    ms: float
    rays_per_s: float
    hits_equal: bool
    mask_per_ray: float = 0.0


def evaluate(ctx, tris, rays_dev, placement, ref_hits, *, R: int = 6, name: str = "", beta=None,
             reps: int = 5, mode: str = "sparse") -> Evaluation:
    """Trace with a placement (or mode "raw"/"none") and report counts and speed."""
    import torch
    if mode == "sparse":
        scene = binding.Scene(ctx, tris, R=R, mode="sparse", placement=placement)
    else:
        scene = binding.Scene(ctx, tris, R=R, mode=mode)
    n = rays_dev.shape[0]
    hits = torch.empty((n, 4), dtype=torch.int32, device=rays_dev.device)
    extra = scene.trace(rays_dev, hits=hits, extra=True).extra
    h = hits.cpu().numpy()
    mask_tests = float(extra[:, 0].double().sum().item()) if n else 0.0
    same = bool(ref_hits is None or ((h[:, 0] == ref_hits[:, 0]).all() and (h[:, 1] == ref_hits[:, 1]).all()))
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        scene.trace(rays_dev, hits=hits, extra=False)
        b.record()
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
    n_masks = scene.info["n_masked"] if mode == "sparse" else (2 * scene.info["n_inner"] if mode == "raw" else 0)
    scene.close()
    box = h[:, 2].astype(np.float64).sum() / n
    tri = h[:, 3].astype(np.float64).sum() / n
    return Evaluation(name, beta, int(n_masks), box + tri, box, tri, ms, n / (ms * 1e-3), same,
                      mask_tests / max(n, 1))


def placeable(scores, X) -> np.ndarray:
    """Scores with every slot whose exact mask is full (occupied fraction 1)
    moved last: a full mask always overlaps the ray mask, is never tested and
    would only use up the budget."""
    s = np.asarray(scores, np.float32).copy()
    s[X[:, 6].detach().cpu().numpy() >= 1.0] = -np.inf
    return s


def placements(scores_by_name: dict, n_place: int, X=None) -> dict:
    """uint8 placements of the n_place highest scores for each named scoring
    (full-mask slots last when the features X are given)."""
    return {k: binding.place_top(placeable(v, X) if X is not None else v, n_place)
            for k, v in scores_by_name.items()}


def scene_targets(y, max_slots: int, seed: int, top_share: float = 0.25):
    """Sample of one scene's slots and their standardised targets: the
    top_share * max_slots highest labels (ties: lower slot) plus a uniform
    draw from the other slots, (label - mean) / std over all of the scene's
    slots (0 where the std is 0). Returns (slot indices ascending, targets)."""
    yy = y.detach().cpu().numpy().astype(np.float64)
    S = yy.size
    mu, sd = float(yy.mean()) if S else 0.0, float(yy.std()) if S else 0.0
    t = (yy - mu) / sd if sd > 0.0 else np.zeros_like(yy)
    if S <= max_slots:
        idx = np.arange(S)
    else:
        n_top = int(max_slots * top_share)
        order = np.argsort(-yy, kind="stable")
        rest = np.random.default_rng(seed).choice(order[n_top:], max_slots - n_top, replace=False)
        idx = np.sort(np.concatenate([order[:n_top], rest]))
    return idx, t[idx].astype(np.float32)


def residual_targets(ts, hs):
    """Least-squares slope a of the standardised labels on the standardised log heuristic over
    all training samples, and the targets label - a * h. ts, hs: per-scene float arrays."""
    t = np.concatenate(ts).astype(np.float64) if ts else np.zeros(0)
    h = np.concatenate(hs).astype(np.float64) if hs else np.zeros(0)
    hh = float((h * h).sum())
    a = float((t * h).sum()) / hh if hh > 0.0 else 0.0
    return a, (t - a * h).astype(np.float32)


def build_training_set(ctx, specs, *, max_slots: int = 65536, log=None):
    """Concatenated features (device tensor), residual targets (device tensor) and the slope a
    over the training scenes."""
    import torch
    from . import scenes
    Xs, ts, hs = [], [], []
    for i, sp in enumerate(specs):
        tris, rays = scenes.placement_scene(sp)
        X, y, info = slot_dataset(ctx, tris, rays)
        idx, t = scene_targets(y, max_slots, sp.seed)
        h = standardise(heuristic_log(X).cpu().numpy())
        sel = torch.from_numpy(idx).to(X.device)
        Xs.append(X[sel])
        ts.append(t)
        hs.append(h[idx])
        if log and (i % 10 == 0 or i == len(specs) - 1):
            log(f"train scene {i + 1}/{len(specs)}: {sp.kind} {tris.shape[0]} tris, "
                f"{info['n_inner']} inner nodes, mean label {y.mean().item():.3f}")
    a, r = residual_targets(ts, hs)
    X = torch.cat(Xs).contiguous()
    return X, torch.from_numpy(r).to(X.device).contiguous(), a


def learned_scores(ctx, params, a: float, X) -> np.ndarray:
    """Placement scores of one scene's slots: a * h + the network's correction."""
    h = standardise(heuristic_log(X).cpu().numpy())
    return (a * h + predict(ctx, params, X).cpu().numpy().astype(np.float64)).astype(np.float32)


def evaluate_scene(ctx, params, a, tris, rays, *, betas=(0.5, 1.0, 2.0), seed: int = 0, reps: int = 5,
                   log=None, placements_out=None) -> list:
    """All placements of one held-out scene: learned, heuristic, random and
    true-label at each budget, plus all masks (raw) and no masks. With a dict
    `placements_out`, the uint8 placement of each (name, beta) is stored there."""
    import torch
    X, y, info = slot_dataset(ctx, tris, rays)
    S = X.shape[0]
    pred = learned_scores(ctx, params, a, X)
    rng = np.random.default_rng(seed)
    scores = {"learned": pred, "heuristic": heuristic_scores(X),
              "random": rng.random(S).astype(np.float32), "true_label": y.cpu().numpy()}
    rays_dev = torch.from_numpy(np.ascontiguousarray(rays, np.float32)).cuda(ctx.device)
    sc = binding.Scene(ctx, tris, R=6, mode="none")
    ref = sc.trace(rays_dev, extra=False).hits.cpu().numpy()
    sc.close()
    out = [evaluate(ctx, tris, rays_dev, None, ref, mode="none", name="no_masks", reps=reps),
           evaluate(ctx, tris, rays_dev, None, ref, mode="raw", name="all_masks", reps=reps)]
    for beta in betas:
        M = budget_masks(beta, info["n_inner"])
        for name, pl in placements(scores, M, X).items():
            out.append(evaluate(ctx, tris, rays_dev, pl, ref, name=name, beta=beta, reps=reps))
            if placements_out is not None:
                placements_out[(name, beta)] = pl
    if log:
        for e in out:
            log(f"  {e.name:>10} beta={e.beta}: masks {e.n_masks}, tests/ray {e.tests_per_ray:.2f}, "
                f"{e.rays_per_s / 1e6:.1f} Mrays/s, hits equal {e.hits_equal}")
    return out


def run_experiment(ctx, train_specs, heldout, *, betas=(0.5, 1.0, 2.0), epochs: int = 30,
                   batch: int = 4096, lr: float = 1e-3, max_slots: int = 65536, seed: int = 0, log=None,
                   placements_out=None):
    """Train on the training scenes, evaluate every placement on each held-out
    (tris, rays) pair. Returns (params, loss history, [[Evaluation]]); with a list
    `placements_out`, each held-out scene appends its {(name, beta): placement}."""
    t0 = time.time()
    X, y, a = build_training_set(ctx, train_specs, max_slots=max_slots, log=log)
    if log:
        log(f"training set: {X.shape[0]} slots from {len(train_specs)} scenes ({time.time() - t0:.1f} s), "
            f"heuristic slope a = {a:.4f}")
    t1 = time.time()
    params, hist = train(ctx, X, y, epochs=epochs, batch=min(batch, X.shape[0]), lr=lr, seed=seed, log=log)
    if log:
        log(f"training: {epochs} epochs in {time.time() - t1:.1f} s")
    results = []
    for k, (tris, rays) in enumerate(heldout):
        if log:
            log(f"held-out scene {k}: {tris.shape[0]} tris, {rays.shape[0]} rays")
        kept = {} if placements_out is not None else None
        results.append(evaluate_scene(ctx, params, a, tris, rays, betas=betas, seed=seed + k, log=log,
                                      placements_out=kept))
        if placements_out is not None:
            placements_out.append(kept)
    return params, hist, results
