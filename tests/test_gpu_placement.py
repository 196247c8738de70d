"""GPU kernels of the learned placement against the float64 oracle:
per-slot features, MLP forward, gradients (rtol 1e-4, atol 1e-6), Adam,
determinism of the fixed-order reductions, and that training lowers the loss."""
import numpy as np
import pytest

import oracle
from oracle import features as ofeat
from paper_2305_08343_amd import binding
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("R", [4, 6])
def test_slot_features_match_oracle(ctx, small_scene, small_oracle, R):
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    print(f"[gpu] features R={R}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode="raw")
    f = s.features().cpu().numpy()
    s.close()
    ref = ofeat.slot_features(tris, small_oracle["bvh"], small_oracle[f"masks{R}"], R)
    assert f.shape == ref.shape
    assert np.allclose(f, ref, rtol=1e-4, atol=2e-5), np.abs(f - ref).max(0)


@pytest.mark.parametrize("name", ["segments", "flat"])
def test_slot_features_of_degenerate_boxes_match_oracle(ctx, name):
    """Zero-area triangles along x (leaf boxes are segments: extent ratios 0 on y and z, areas
    clamped at 2^-40 of the root's) and a scene flat in z (position 0 on the flat axis)."""
    from paper_2305_08343_amd import scenes
    tris = scenes.segment_rows(0)
    if name == "flat":
        tris = scenes.lattice_copies(5)
        tris[..., 2] = np.float32(0.5)
    print(f"[gpu] features of {name}", flush=True)
    bvh = oracle.bvh_build(tris)
    _, delta = oracle.default_bounds(tris)
    m = oracle.object_masks(tris, bvh, 6, delta)
    s = binding.Scene(ctx, tris, R=6, mode="raw")
    f = s.features().cpu().numpy()
    s.close()
    ref = ofeat.slot_features(tris, bvh, m, 6)
    assert f.shape == ref.shape
    assert np.allclose(f, ref, rtol=1e-4, atol=2e-5), np.abs(f - ref).max(0)
    if name == "flat":
        assert (f[:, 10] == 0.0).all()


def test_mlp_forward_and_gradients_match_oracle(ctx):
    import torch
    rng = np.random.default_rng(0)
    p = omlp.init_params(3) + rng.normal(0, 0.02, omlp.N_PARAMS)
    n = 1000
    x = rng.normal(size=(n, 12))
    t = rng.normal(size=n)
    p32, x32, t32 = p.astype(np.float32), x.astype(np.float32), t.astype(np.float32)
    dp, dx, dt = _dev(p32), _dev(x32), _dev(t32)
    act = torch.empty((n, 128), dtype=torch.float32, device="cuda")
    y = ctx.mlp_forward(dp, dx, act)
    y_ref, _ = omlp.forward(p32.astype(np.float64), x32.astype(np.float64))
    assert np.allclose(y.cpu().numpy(), y_ref, rtol=1e-4, atol=1e-5)
    grad = torch.empty(omlp.N_PARAMS, dtype=torch.float32, device="cuda")
    work = torch.empty(binding.mlp_work_floats(n), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ctx.mlp_backward(dp, dx, act, y, dt, grad, work, loss)
    g_ref = omlp.grad(p32.astype(np.float64), x32.astype(np.float64), t32.astype(np.float64))
    g = grad.cpu().numpy()
    assert np.allclose(g, g_ref, rtol=1e-4, atol=1e-6), np.abs(g - g_ref).max()
    assert np.isclose(loss.item(), omlp.loss(p32.astype(np.float64), x32.astype(np.float64),
                                             t32.astype(np.float64)), rtol=1e-5)
    # fixed-order reductions: a second run gives the same bits
    grad2 = torch.empty_like(grad)
    ctx.mlp_backward(dp, dx, act, y, dt, grad2, work)
    assert (grad.cpu().numpy().view(np.uint32) == grad2.cpu().numpy().view(np.uint32)).all()


def test_zero_weights_give_output_bias(ctx):
    import torch
    p = np.zeros(omlp.N_PARAMS, np.float32)
    p[-1] = 0.25
    y = ctx.mlp_forward(_dev(p), _dev(np.random.default_rng(1).normal(size=(77, 12))))
    assert (y.cpu().numpy() == np.float32(0.25)).all()


def test_adam_matches_oracle(ctx):
    import torch
    rng = np.random.default_rng(2)
    p = rng.normal(size=omlp.N_PARAMS)
    m = rng.normal(size=omlp.N_PARAMS) * 0.01
    v = np.abs(rng.normal(size=omlp.N_PARAMS)) * 0.001
    g = rng.normal(size=omlp.N_PARAMS) * 0.1
    dp, dm, dv, dg = _dev(p), _dev(m), _dev(v), _dev(g)
    ctx.mlp_adam(dp, dg, dm, dv, 7, lr=1e-3)
    p2, m2, v2 = omlp.adam_step(p.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64),
                                m.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64), 7)
    # float32 has a spacing of ~1.2e-7 relative: a few roundings per update
    assert np.allclose(dp.cpu().numpy(), p2, rtol=1e-5, atol=1e-7)
    assert np.allclose(dm.cpu().numpy(), m2, rtol=1e-5, atol=4 * np.spacing(np.float32(np.abs(m2).max())))
    assert np.allclose(dv.cpu().numpy(), v2, rtol=1e-5, atol=4 * np.spacing(np.float32(np.abs(v2).max())))


def test_training_steps_track_the_oracle(ctx):
    """Ten Adam steps on a fixed batch: GPU float32 and oracle float64 agree."""
    import torch
    rng = np.random.default_rng(4)
    n = 512
    x = rng.normal(size=(n, 12)).astype(np.float32)
    t = (x[:, 0] * 0.5 - x[:, 3] ** 2 * 0.2).astype(np.float32)
    p = omlp.init_params(5).astype(np.float32)
    dp, dx, dt = _dev(p), _dev(x), _dev(t)
    dm = torch.zeros(omlp.N_PARAMS, device="cuda")
    dv = torch.zeros(omlp.N_PARAMS, device="cuda")
    act = torch.empty((n, 128), device="cuda")
    grad = torch.empty(omlp.N_PARAMS, device="cuda")
    work = torch.empty(binding.mlp_work_floats(n), device="cuda")
    loss = torch.empty(1, device="cuda")
    P, M, V = p.astype(np.float64), np.zeros(omlp.N_PARAMS), np.zeros(omlp.N_PARAMS)
    losses = []
    for step in range(1, 11):
        y = ctx.mlp_forward(dp, dx, act)
        ctx.mlp_backward(dp, dx, act, y, dt, grad, work, loss)
        ctx.mlp_adam(dp, grad, dm, dv, step, lr=1e-2)
        losses.append(loss.item())
        P, M, V = omlp.adam_step(P, omlp.grad(P, x.astype(np.float64), t.astype(np.float64)), M, V, step, lr=1e-2)
    assert losses[-1] < losses[0]
    assert np.allclose(dp.cpu().numpy(), P, rtol=1e-3, atol=1e-4)


def test_training_checkpoint_resume_equals_uninterrupted(ctx, tmp_path):
    """Six epochs in one run, and two runs of three epochs with the state written to a checkpoint
    and read back in between: parameters, Adam state and loss history are bit-identical."""
    import torch
    from paper_2305_08343_amd import placement
    rng = np.random.default_rng(11)
    X = _dev(rng.normal(size=(8192 + 37, 12)))
    y = _dev(rng.normal(size=8192 + 37))
    print("[gpu] checkpoint / resume", flush=True)
    p_all, h_all = placement.train(ctx, X, y, epochs=6, batch=1024, seed=3)
    ck = str(tmp_path / "mlp.npz")
    p_half, h_half = placement.train(ctx, X, y, epochs=3, batch=1024, seed=3, checkpoint=ck)
    assert len(h_half) == 3
    p_res, h_res = placement.train(ctx, X, y, epochs=6, batch=1024, seed=3, checkpoint=ck, resume=True)
    torch.cuda.synchronize()
    assert torch.equal(p_all, p_res)
    assert h_all == h_res
    params, m, v, step, epoch, _, hist = placement.load_checkpoint(ck, X.device)
    assert epoch == 6 and step == 6 * 8 and torch.equal(params, p_res) and hist == h_res
    assert not torch.equal(p_half, p_res)
