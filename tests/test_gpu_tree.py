"""The N-BVH nbvh_build writes (Sec. 5: a shallow BVH whose leaves are the
neural nodes), read back through the documented node layout: every leaf
appears once with its own box, every inner box is the exact min/max union of
its children's boxes (what makes the walk visit exactly the leaves an
every-leaf slab test reports), each inner node splits its leaves in halves at
the median centroid along the widest centroid extent, and the depth is that of
a balanced binary tree."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nbvh_synth import configs

pytestmark = pytest.mark.gpu

EMPTY = 0x7FFFFFFF


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16237_amd as P
    P.load()
    return P


def _check_tree(lib, boxes):
    n = boxes.shape[0]
    sc_lo = boxes[:, :3].min(0)
    side = np.float32((boxes[:, 3:].max(0) - sc_lo).max() * 1.01 + 1e-3)
    m = lib.NBVH(configs.C1_NET, boxes, sc_lo, side, precision="fp32")
    torch.cuda.synchronize()
    cb, ch = m.tree()
    assert cb.shape[0] == max(1, n - 1)
    seen = np.zeros(n, np.int64)
    leaves = {}

    def visit(node):
        """(leaf ids under node, its box, its height)"""
        ids, box, height, parts = [], None, 0, []
        for k in range(2):
            c = int(ch[node, k])
            if c == EMPTY:
                assert n == 1 and k == 1
                continue
            if c < 0:
                leaf = ~c
                seen[leaf] += 1
                assert np.array_equal(cb[node, k], boxes[leaf]), "leaf box differs from the input"
                sub, sb, h = [leaf], boxes[leaf], 0
            else:
                assert c > node, "children come after their parent"
                sub, sb, h = visit(c)
                assert np.array_equal(cb[node, k], sb), "child box is not the union of its children's"
            parts.append(sub)
            ids += sub
            box = sb.copy() if box is None else np.concatenate([np.minimum(box[:3], sb[:3]),
                                                                np.maximum(box[3:], sb[3:])])
            height = max(height, h + 1)
        if len(parts) == 2:
            a, b = parts
            assert len(b) - len(a) in (0, 1), "halves of a median split"
            cen = (np.float32(0.5) * (boxes[ids, :3] + boxes[ids, 3:])).astype(np.float32)
            axis = int(np.argmax(cen.max(0) - cen.min(0)))
            ca = np.float32(0.5) * (boxes[a, axis] + boxes[a, 3 + axis])
            cbb = np.float32(0.5) * (boxes[b, axis] + boxes[b, 3 + axis])
            assert ca.max() <= cbb.min(), "not split along the widest centroid axis"
        leaves[node] = ids
        return ids, box, height

    _, _, height = visit(0)
    assert np.array_equal(seen, np.ones(n, np.int64)), "every leaf appears exactly once"
    assert height == max(1, math.ceil(math.log2(n))), (height, n)
    return height


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 1000])
def test_tree_random_boxes(lib, n):
    rng = np.random.default_rng(100 + n)
    c = rng.uniform(-1, 1, (n, 3))
    h = rng.uniform(0.01, 0.3, (n, 3))
    boxes = np.concatenate([c - h, c + h], 1).astype(np.float32)
    _say("tree over", n, "random boxes")
    _check_tree(lib, boxes)


@pytest.mark.parametrize("n_tris,n_leaves", [(1_003_520, 1024), (3_996_180, 16384)])
def test_tree_workload_scenes(lib, n_tris, n_leaves):
    sc = configs.make_scene(n_tris, n_leaves, with_mesh=False)
    _say("tree over the", n_leaves, "leaves of the", n_tris, "triangle scene")
    assert _check_tree(lib, sc.boxes) == int(math.log2(n_leaves))
