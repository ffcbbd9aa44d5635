"""Host logic of the error-driven construction (Sec. 5.1) and the base BVH
it cuts: split choice and cut expansion on hand cases. CPU only. (Ranks and
acceptance probabilities are library calls, checked against the oracle on the
GPU; the oracle's are pinned in test_oracle_pins.py.)"""
import math

import numpy as np
import pytest

pytest.importorskip("torch")

from nbvh_synth import configs, scene
from paper_2405_16237_amd import construct as C


def _toy_base():
    # root 0 -> (1, 2); 1 -> (3, 4); 2, 3, 4 leaves
    left = np.array([1, 3, -1, -1, -1], dtype=np.int32)
    right = np.array([2, 4, -1, -1, -1], dtype=np.int32)
    lo = np.zeros((5, 3), dtype=np.float32)
    hi = np.ones((5, 3), dtype=np.float32) * np.arange(5, 0, -1, dtype=np.float32)[:, None]
    return dict(lo=lo, hi=hi, left=left, right=right)


def test_choose_splits_and_expand():
    base = _toy_base()
    cut = C.Cut([0])
    assert C.choose_splits(cut, base, np.array([0.0]), 1) == [0]
    cut = C.expand(cut, base, [0])
    assert cut.nodes == [1, 2]
    # node 2 is a leaf of the base BVH: only node 1 can split, whatever the ranks
    assert C.choose_splits(cut, base, np.array([-5.0, 0.0]), 2) == [0]
    cut = C.expand(cut, base, [0])
    assert cut.nodes == [3, 2, 4]
    assert np.array_equal(cut.boxes(base)[:, 3], base["hi"][[3, 2, 4], 0])
    # ties go to the lower position, -inf ranks last
    base2 = dict(base, left=np.array([1, 3, 5, -1, -1], np.int32), right=np.array([2, 4, 6, -1, -1], np.int32))
    assert C.choose_splits(C.Cut([1, 2]), base2, np.array([-1.0, -1.0]), 1) == [0]
    assert C.choose_splits(C.Cut([1, 2]), base2, np.array([-math.inf, -7.0]), 1) == [1]


def test_base_bvh_nests_and_partitions():
    sc = configs.make_scene(20480, 64, with_mesh=False)
    b = scene.base_bvh(sc.verts, sc.tris, leaf_tris=16)
    m = b["lo"].shape[0]
    inner = np.nonzero(b["left"] >= 0)[0]
    assert np.all((b["left"] >= 0) == (b["right"] >= 0))
    for k in (b["left"][inner], b["right"][inner]):
        assert np.all(b["lo"][k] >= b["lo"][inner]) and np.all(b["hi"][k] <= b["hi"][inner])
        assert np.all(k > inner)
    assert np.all(b["n_tris"][inner] == b["n_tris"][b["left"][inner]] + b["n_tris"][b["right"][inner]])
    leaves = b["left"] < 0
    assert b["n_tris"][0] == sc.tris.shape[0] and b["n_tris"][leaves].sum() == sc.tris.shape[0]
    assert b["n_tris"][leaves].max() <= 16 and m == 2 * leaves.sum() - 1
    # the root box holds every vertex
    assert np.all(sc.verts >= b["lo"][0]) and np.all(sc.verts <= b["hi"][0])
