"""Structural check of the BVH the library builds (host build, no GPU):
every triangle is referenced by exactly one leaf and carries its own
vertices, every node is reached exactly once from the root, every child box
contains everything below it, empty slots have empty boxes, leaves hold at
most 8 triangles, and the reported depth is the tree's."""
import numpy as np
import pytest

import workloads as w

EMPTY = 0xFFFFFFFF
LEAF = 0x80000000


def _check(V, F):
    import paper_2607_23122_amd as ocr
    nodes, tris, depth = ocr.build_bvh_host(V, F)
    nt = F.shape[0]
    nn = nodes.size
    assert nn >= 1
    ids = tris[:, 0, 3].view(np.uint32)
    # the triangles, in leaf order, are the scene's: a permutation of the rows
    assert np.array_equal(np.sort(ids), np.arange(nt, dtype=np.uint32))
    assert np.array_equal(tris[:, :, :3], V[F[ids]])
    lo = np.stack([nodes["lo_x"], nodes["lo_y"], nodes["lo_z"]], -1)  # [nn, 4, 3]
    hi = np.stack([nodes["hi_x"], nodes["hi_y"], nodes["hi_z"]], -1)
    ch = nodes["child"]
    empty = ch == EMPTY
    leaf = ~empty & ((ch & LEAF) != 0)
    inner = ~empty & ~leaf
    # empty slots have empty boxes, and are never entered
    assert (lo[empty] == np.inf).all() and (hi[empty] == -np.inf).all()
    assert (~empty).any(axis=1).all()
    # each node is the child of exactly one slot (the root of none)
    kids = ch[inner]
    assert (kids < nn).all()
    seen = np.bincount(kids, minlength=nn)
    assert seen[0] == 0 and (seen[1:] == 1).all()
    # leaves partition the leaf-ordered triangles
    first = (ch[leaf] & 0x07FFFFFF).astype(np.int64)
    count = (((ch[leaf] >> 27) & 0xF) + 1).astype(np.int64)
    assert count.max() <= 8
    cover = np.zeros(nt, np.int64)
    for f, c in zip(first, count):
        cover[f:f + c] += 1
    assert (cover == 1).all()
    # an interior child's box holds its node's non-empty child boxes
    pn, ps = np.nonzero(inner)
    c = ch[pn, ps]
    cl = np.where(empty[c][..., None], np.inf, lo[c]).min(axis=1)
    chh = np.where(empty[c][..., None], -np.inf, hi[c]).max(axis=1)
    assert (lo[pn, ps] <= cl).all() and (hi[pn, ps] >= chh).all()
    # a leaf child's box holds its triangles' vertices
    ln, ls = np.nonzero(leaf)
    for n_, s_, f, k in zip(ln, ls, first, count):
        v = tris[f:f + k, :, :3].reshape(-1, 3)
        assert (lo[n_, s_] <= v.min(axis=0)).all() and (hi[n_, s_] >= v.max(axis=0)).all()
    # depth: levels of nodes from the root
    level = np.zeros(nn, np.int64)
    level[0] = 1
    order = [0]
    for n_ in order:
        for k in ch[n_][inner[n_]]:
            level[k] = level[n_] + 1
            order.append(int(k))
    assert len(order) == nn
    assert level.max() == depth
    return nodes, depth


def test_boxes_scene():
    s = w.boxes_scene(1)
    _check(s.V, s.F)


@pytest.mark.parametrize("n", [1, 2, 9, 1000])
def test_random_soups(n):
    rng = np.random.default_rng(n)
    V = (rng.uniform(-5, 5, (n, 1, 3)) + rng.normal(0, 0.5, (n, 3, 3))).reshape(-1, 3).astype(np.float32)
    F = np.arange(3 * n, dtype=np.uint32).reshape(-1, 3)
    _check(V, F)


def test_coincident_triangles():
    # identical triangles cannot be split by centroid: leaves of at most 8
    # still, with a tree above them
    V = np.tile(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), (40, 1))
    F = np.arange(120, dtype=np.uint32).reshape(-1, 3)
    nodes, depth = _check(V, F)
    assert depth >= 2


def test_terrain_scene():
    s = w.terrain_scene(seed=10, cells=128, nspheres=54)
    nodes, depth = _check(s.V, s.F)
    assert nodes.size > 1000
