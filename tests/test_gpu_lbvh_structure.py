"""Structure of the device-built LBVH, checked on the host (rt_scene_export).

The builder (Morton codes, LSD radix sort, Karras hierarchy, level-ordered
refit, 4-wide collapse) is this library's own acceleration structure; the
paper delegates intersection to its renderer.  These checks are independent
of traversal and of the oracle:
* Morton codes equal a NumPy evaluation of the same quantisation of the
  triangle AABB centres (63 bits, 21 per axis, x in the highest bit);
* the slot order equals np.argsort(codes, kind="stable") (the LSD sort is
  stable, so equal codes keep input order);
* the binary tree has n - 1 internal nodes; walking it from the root reaches
  every internal node and every leaf exactly once; every child reference is
  in range; every child box stored in a node is exactly the union of the
  boxes below it, and a leaf's box is its triangle's AABB;
* the 4-wide tree: every child reference is in range or the empty marker,
  every wide node and every leaf is reached exactly once, every child box
  contains everything below it, empty slots hold inverted boxes;
* the reported depth is the deepest leaf's depth.
Scenes: a single triangle, two triangles, identical triangles (all Morton
codes equal), a flat scene (zero extent in z), random soups of ragged sizes,
the tiny and Manhattan scenes and the 1.02 M-triangle scene.
"""
import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu

EMPTY = 0x7FFFFFFF


def _spread21(v):
    x = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    for shift, mask in ((32, 0x001F00000000FFFF), (16, 0x001F0000FF0000FF), (8, 0x100F00F00F00F00F),
                        (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        x = (x | (x << np.uint64(shift))) & np.uint64(mask)
    return x


def reference_morton(V, F):
    """Morton codes of the AABB centres, in FP32 as the builder defines them:
    centre = 0.5 (lo + hi) per axis, quantised to 21 bits from the lower
    corner of the centres' bounding box with one scale for all axes,
    (2^21 - 1) / (largest extent) (0 if every centre coincides)."""
    P = V[F].astype(np.float32)                      # [n, 3 vertices, 3 axes]
    lo = P.min(axis=1)
    hi = P.max(axis=1)
    c = np.float32(0.5) * (lo + hi)
    cl = c.min(axis=0)
    ext = np.float32((c.max(axis=0) - cl).max())
    qmax = np.float32(2097151.0)
    sc = np.float32(qmax / ext) if ext > 0 else np.float32(0)
    q = np.minimum(np.maximum((c - cl) * sc, np.float32(0)), qmax).astype(np.uint32)
    return (_spread21(q[:, 0]) << np.uint64(2)) | (_spread21(q[:, 1]) << np.uint64(1)) | _spread21(q[:, 2])


def tri_boxes(dump):
    T = dump["tris"].reshape(-1, 3, 4)[:, :, :3]
    return T.min(axis=1), T.max(axis=1)


def check_binary(dump, n):
    """Reachability, reference ranges and exact boxes of the binary tree.
    Returns the deepest leaf depth."""
    nodes = dump["nodes"]
    assert nodes.shape == (n - 1, 16)
    refs = nodes[:, 12:14].copy().view(np.int32)
    ok_int = (refs >= 0) & (refs < n - 1)
    ok_leaf = (refs < 0) & (~refs < n)
    assert np.all(ok_int | ok_leaf), "child reference out of range"
    # every node except the root is some node's child, exactly once
    int_refs = refs[refs >= 0]
    assert np.array_equal(np.sort(int_refs), np.arange(1, n - 1)), "internal nodes not reached exactly once"
    leaf_refs = ~refs[refs < 0]
    assert np.array_equal(np.sort(leaf_refs), np.arange(n)), "leaves not reached exactly once"
    # breadth-first walk from the root: depth of every node and leaf
    depth = np.full(n - 1, -1, np.int64)
    depth[0] = 0
    level = np.array([0])
    leaf_depth = np.full(n, -1, np.int64)
    d = 0
    while level.size:
        r = refs[level].ravel()
        leaf_depth[~r[r < 0]] = d + 1
        level = r[r >= 0]
        assert np.all(depth[level] == -1), "a node is reached twice"
        d += 1
        depth[level] = d
    assert np.all(depth >= 0) and np.all(leaf_depth >= 0), "unreachable node or leaf"
    # boxes: node i stores (lo, hi) of both children; a child's box is the
    # union of its own two children, a leaf's box its triangle's AABB
    Llo = np.stack([nodes[:, 0], nodes[:, 2], nodes[:, 8]], 1)
    Lhi = np.stack([nodes[:, 1], nodes[:, 3], nodes[:, 9]], 1)
    Rlo = np.stack([nodes[:, 4], nodes[:, 6], nodes[:, 10]], 1)
    Rhi = np.stack([nodes[:, 5], nodes[:, 7], nodes[:, 11]], 1)
    own_lo = np.minimum(Llo, Rlo)
    own_hi = np.maximum(Lhi, Rhi)
    tlo, thi = tri_boxes(dump)
    for side, (blo, bhi) in enumerate(((Llo, Lhi), (Rlo, Rhi))):
        r = refs[:, side]
        i = r >= 0
        assert np.array_equal(blo[i], own_lo[r[i]]) and np.array_equal(bhi[i], own_hi[r[i]]), "box != union"
        j = ~i
        assert np.array_equal(blo[j], tlo[~r[j]]) and np.array_equal(bhi[j], thi[~r[j]]), "leaf box != AABB"
    return int(leaf_depth.max())


def check_wide(dump, n):
    W = dump["wide"]
    if n < 2:
        assert W.shape[0] == 0
        return
    assert W.shape[0] >= 1
    n4 = W.shape[0]
    lo = np.stack([W[:, 0:4], W[:, 8:12], W[:, 16:20]], 2)     # [n4, 4 children, 3]
    hi = np.stack([W[:, 4:8], W[:, 12:16], W[:, 20:24]], 2)
    refs = W[:, 24:28].copy().view(np.int32)
    empty = refs == EMPTY
    internal = (refs >= 0) & ~empty
    leaf = refs < 0
    assert np.all(refs[internal] < n4), "wide child reference out of range"
    assert np.all(~refs[leaf] < n), "wide leaf slot out of range"
    assert np.all(lo[empty] > hi[empty]), "empty slot without an inverted box"
    assert np.all(internal.sum(1) + leaf.sum(1) >= 2), "wide node with fewer than two children"
    assert np.array_equal(np.sort(refs[internal]), np.arange(1, n4)), "wide nodes not reached exactly once"
    assert np.array_equal(np.sort(~refs[leaf]), np.arange(n)), "leaves not reached exactly once in the wide tree"
    # a child box contains its node's children (union of the child's slots)
    full_lo = np.where(empty[..., None], np.inf, lo).min(1)
    full_hi = np.where(empty[..., None], -np.inf, hi).max(1)
    r = refs[internal]
    assert np.all(lo[internal] <= full_lo[r]) and np.all(hi[internal] >= full_hi[r]), "wide box too small"
    tlo, thi = tri_boxes(dump)
    s = ~refs[leaf]
    assert np.all(lo[leaf] <= tlo[s]) and np.all(hi[leaf] >= thi[s]), "wide leaf box too small"


def check_scene(mesh):
    import paper_2504_21719_amd as rt
    s = rt.scene_from_mesh(mesh)
    info = s.info()
    dump = s.export()
    n = mesh.n_triangles
    V, F = np.asarray(mesh.vertices, np.float32), np.asarray(mesh.triangles, np.int64)
    ref = reference_morton(V, F)
    order = dump["tris"][:, 3].copy().view(np.int32).astype(np.int64)   # original id of every slot
    assert np.array_equal(np.sort(order), np.arange(n)), "slot order is not a permutation"
    assert np.array_equal(dump["morton"], ref[order]), "Morton codes differ from the reference"
    assert np.array_equal(order, np.argsort(ref, kind="stable")), "sort differs from a stable argsort"
    # materials travel with their triangles
    mats = dump["tris"][:, 7].copy().view(np.int32)
    assert np.array_equal(mats, np.asarray(mesh.tri_material)[order])
    if n >= 2:
        assert info.n_nodes == n - 1
        assert check_binary(dump, n) == info.bvh_depth
    else:
        assert dump["nodes"].shape[0] == 0 and info.bvh_depth == 0
    check_wide(dump, n)
    return info


def _mesh(V, F, n_mat=1):
    V = np.asarray(V, np.float32)
    F = np.asarray(F, np.int32)
    M = (np.arange(F.shape[0]) % n_mat).astype(np.int32)
    return sg.Scene(V, F, M, np.array([5.24] * n_mat), np.array([0.12] * n_mat), "t")


def test_single_and_two_triangles():
    check_scene(_mesh([[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 1, 2]]))
    check_scene(_mesh([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 1]], [[0, 1, 2], [1, 3, 2]]))


def test_identical_triangles_share_one_code():
    n = 37
    V = np.tile(np.array([[0, 0, 0], [2, 0, 1], [0, 3, 0]], np.float32), (n, 1))
    F = np.arange(3 * n).reshape(n, 3)
    info = check_scene(_mesh(V, F, 2))
    assert info.bvh_depth >= 6   # equal keys are split by index: a balanced tree over 37 leaves


def test_flat_scene():
    rng = np.random.default_rng(4)
    n = 300
    c = rng.uniform(-100, 100, (n, 1, 3))
    c[..., 2] = 0.0
    d = rng.uniform(-2, 2, (n, 3, 3))
    d[..., 2] = 0.0
    check_scene(_mesh((c + d).reshape(-1, 3), np.arange(3 * n).reshape(n, 3), 3))


@pytest.mark.parametrize("n", [3, 64, 65, 1000, 4097, 50_001])
def test_random_soups(n):
    check_scene(sg.random_soup(n, seed=n))


def test_tiny_and_manhattan():
    check_scene(sg.tiny_scene())
    check_scene(sg.manhattan_scene())


def test_large_scene():
    info = check_scene(sg.large_config().scene)
    assert info.n_triangles == 1_021_074
