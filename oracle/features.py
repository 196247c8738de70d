"""Float64 reference of the per-slot placement features -- TEST INFRASTRUCTURE ONLY.

For child slot s = 2*node + c of an oracle BVH (see sc_slot_features in the
library header for the same list):
  0-2  child box extent / parent box extent per axis (0 if the parent is flat)
  3    log2(max(SA(child) / SA(root box), 2^-40)) / 32
  4    depth of the parent node (root 1) / tree depth
  5    log2(1 + triangles under the child) / 24
  6    set bits of the child's exact mask / R^3
  7    mean thinness 1 - 4 sqrt(3) area / (sum of squared edges), clipped to [0, 1]
  8-10 centre of the child box relative to the root box per axis: (mid - root lo) / root
       extent, 0 where the root box is flat on that axis
  11   1 if the child is a leaf
"""
from __future__ import annotations

import numpy as np


def tri_thinness(tris):
    """[n]: 1 - 4 sqrt(3) area / (sum of squared edge lengths), clipped to [0, 1]; 1 when the
    edges have zero length (float64)."""
    v = np.asarray(tris, np.float64)
    e = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 1], v[:, 0] - v[:, 2]], 1)  # [n, 3 edges, 3]
    l2 = (e * e).sum(-1)
    area = 0.5 * np.linalg.norm(np.cross(e[:, 0], e[:, 1]), axis=-1)
    s = l2.sum(-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        thin = np.where(s > 0, 1.0 - 4.0 * np.sqrt(3.0) * area / s, 1.0)
    return np.clip(thin, 0.0, 1.0)


def slot_features(tris, bvh, masks, R):
    n_inner = bvh.n_inner
    S = 2 * n_inner
    out = np.zeros((S, 12))
    if n_inner == 0:
        return out
    depth = np.zeros(n_inner, np.int64)
    depth[0] = 1
    for i in range(n_inner):
        for c in range(2):
            r = int(bvh.cref[i, c])
            if not r & 0x80000000:
                depth[r] = depth[i] + 1
    box = bvh.cbox.astype(np.float64).reshape(n_inner, 2, 6)
    plo = np.minimum(box[:, 0, :3], box[:, 1, :3])
    phi = np.maximum(box[:, 0, 3:], box[:, 1, 3:])

    def area(lo, hi):
        d = hi - lo
        return 2.0 * ((d[..., 0] * d[..., 1] + d[..., 1] * d[..., 2]) + d[..., 2] * d[..., 0])

    root_lo, root_hi = plo[0], phi[0]
    root_area = area(root_lo, root_hi)
    root_ext = root_hi - root_lo
    thin = tri_thinness(np.asarray(tris)[bvh.perm])  # leaf order
    pre = np.concatenate([[0.0], np.cumsum(thin)])
    m = np.ascontiguousarray(masks, np.uint64)
    pc = np.unpackbits(m.view(np.uint8), axis=-1).reshape(m.shape[0], -1).sum(-1)
    for s in range(S):
        i, c = s >> 1, s & 1
        lo, hi = box[i, c, :3], box[i, c, 3:]
        pe = phi[i] - plo[i]
        out[s, 0:3] = np.where(pe > 0, (hi - lo) / np.where(pe > 0, pe, 1.0), 0.0)
        out[s, 3] = np.log2(max(area(lo, hi) / root_area, 2.0 ** -40)) / 32.0
        out[s, 4] = depth[i] / bvh.depth
        ref = int(bvh.cref[i, c])
        if ref & 0x80000000:
            first, count = ref & 0x1FFFFFFF, ((ref >> 29) & 3) + 1
        else:
            first, count = (int(x) for x in bvh.range[ref])
        out[s, 5] = np.log2(1.0 + count) / 24.0
        out[s, 6] = pc[s] / R ** 3
        out[s, 7] = (pre[first + count] - pre[first]) / count
        mid = (lo + hi) * 0.5
        out[s, 8:11] = np.where(root_ext > 0, (mid - root_lo) / np.where(root_ext > 0, root_ext, 1.0), 0.0)
        out[s, 11] = 1.0 if ref & 0x80000000 else 0.0
    return out
