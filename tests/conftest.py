import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: large inputs")


def pytest_sessionfinish(session, exitstatus):
    # with SUBCULL_DEBUG=1 every context runs the checked traversal kernels: a check that failed in
    # a context the tests did not reset fails the session
    if os.environ.get("SUBCULL_DEBUG") != "1" or "paper_2305_08343_amd.binding" not in sys.modules:
        return
    failures = sys.modules["paper_2305_08343_amd.binding"].CHECK_FAILURES
    if failures:
        print(f"\n[device checks] failed checks in {len(failures)} context(s): {failures}", flush=True)
        session.exitstatus = 1
    else:
        print("\n[device checks] no check failed", flush=True)


@pytest.fixture(scope="session")
def small_scene():
    from paper_2305_08343_amd import scenes
    return scenes.scene_small(0), scenes.rays_small(256)


@pytest.fixture(scope="session")
def small_oracle(small_scene):
    """Oracle BVH, bounds, masks (R=4, R=6) for the 4,096-triangle strand scene."""
    import oracle
    tris, _ = small_scene
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    return {
        "bvh": bvh, "origin_bound": ob, "delta": delta,
        "masks4": oracle.object_masks(tris, bvh, 4, delta),
        "masks6": oracle.object_masks(tris, bvh, 6, delta),
        "lut4": oracle.raymask_lut(4), "lut6": oracle.raymask_lut(6),
    }


def popcount64(a):
    a = np.asarray(a, np.uint64)
    return np.unpackbits(a.view(np.uint8), axis=-1).reshape(*a.shape[:-1], -1).sum(-1)
