"""GPU parity of the 2-D bit table (Sect. 3.2.2): the device table equals the
oracle's bit for bit, and traces that test compressed masks through it give
exactly the oracle's compressed-mask results (same predicate), culled and in
shadow mode, on both BVH widths."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _compare(dev, ora):
    for k, o in (("prim", ora.prim), ("box_tests", ora.box_tests), ("tri_tests", ora.tri_tests),
                 ("mask_tests", ora.mask_tests), ("mask_culls", ora.mask_culls)):
        bad = np.flatnonzero(dev[k] != o)
        assert bad.size == 0, f"{k}: {bad.size} rays differ, first {bad[:5]}"
    assert (dev["t"].view(np.uint32) == ora.t.view(np.uint32)).all()


@pytest.mark.parametrize("R,K,width", [(4, 256, 2), (4, 256, 4), (6, 256, 2), (6, 256, 4), (6, 4096, 4),
                                       (4, 4096, 2)])
def test_bit_table_and_traces(ctx, small_scene, small_oracle, R, K, width):
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    bvh = small_oracle["bvh"]
    print(f"[gpu-bits] R={R} K={K} width={width}", flush=True)
    cb, idx = oracle.compress(small_oracle[f"masks{R}"], bvh.slot_boxes(), R, K)
    s = binding.Scene(ctx, tris, R=R, mode="lut", K=K, width=width, bit_table=True)
    assert s.info["bit_table"] == 1
    assert (s.export_bit_table() == oracle.bit_table(R, cb)).all()
    kw = dict(mode="lut", R=R, codebook=cb, cidx=idx, origin_bound=small_oracle["origin_bound"])
    ora_trace = (lambda **k: oracle.trace4(tris, bvh, oracle.bvh4_collapse(bvh), rays, **k)) if width == 4 else \
        (lambda **k: oracle.trace(tris, bvh, rays, **k))
    _compare(s.trace(rays).numpy(), ora_trace(**kw))
    fp = torch.zeros(2 * bvh.n_inner, dtype=torch.int32, device="cuda:0")
    dev = s.trace(rays, cull=False, shadow=True, slot_fp=fp).numpy()
    ora = ora_trace(cull=False, shadow=True, **kw)
    _compare(dev, ora)
    assert (fp.cpu().numpy().view(np.uint32) == ora.slot_fp).all()
    s.close()
