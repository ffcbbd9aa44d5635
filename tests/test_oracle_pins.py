"""Pins of the FP64 oracle against facts fixed outside it: hand-derived
closed forms, invariants of trilinear interpolation, library routines, brute
force, finite differences. CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from nbvh_synth import configs, scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class Net:
    def __init__(self, n_levels, n_features, log2_T, n_samples, level_res, mlp_width=16, mlp_hidden=2, n_out=5):
        self.n_levels, self.n_features, self.log2_T, self.n_samples = n_levels, n_features, log2_T, n_samples
        self.level_res = list(level_res)
        self.mlp_width, self.mlp_hidden, self.n_out = mlp_width, mlp_hidden, n_out


# ---------------------------------------------------------------- traversal
def test_slab_golden_cases():
    with open(os.path.join(GOLDEN, "slab_cases.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        ray = np.array(c["ray"], dtype=np.float32)
        if ray[7] >= 1e30:
            ray[7] = np.inf
        hit, t0, t1 = oracle.slab(ray, np.array(c["box"], dtype=np.float32))
        assert hit == c["hit"], c["name"]
        if hit:
            assert t0 == np.float32(c["t0"]) and t1 == np.float32(c["t1"]), (c["name"], t0, t1)


def _random_rays_boxes(rng, n_rays, n_boxes):
    rays = np.zeros((n_rays, 8), dtype=np.float32)
    rays[:, 0:3] = rng.uniform(-2, 2, size=(n_rays, 3))
    d = rng.normal(size=(n_rays, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # some axis-aligned directions with exact zeros
    ax = rng.integers(0, 4, size=n_rays)
    for a in range(3):
        m = ax == a
        d[m] = 0.0
        d[m, a] = rng.choice([-1.0, 1.0], size=m.sum())
    rays[:, 4:7] = d
    rays[:, 3] = 0.0
    rays[:, 7] = rng.choice([np.inf, 2.5], size=n_rays)
    c = rng.uniform(-1, 1, size=(n_boxes, 3))
    h = rng.uniform(0.05, 0.6, size=(n_boxes, 3))
    boxes = np.concatenate([c - h, c + h], axis=1).astype(np.float32)
    return rays, boxes


def test_slab_against_point_sampling():
    """Brute force: march each ray in fine steps in float64; a sample point
    safely inside a box must lie inside the reported interval, and a reported
    interval longer than the step must have its midpoint inside the box."""
    rng = np.random.default_rng(11)
    rays, boxes = _random_rays_boxes(rng, 300, 40)
    ts = np.linspace(0.0, 6.0, 6001)
    margin = 1e-3
    for r in rays:
        o = r[0:3].astype(np.float64)
        d = r[4:7].astype(np.float64)
        tmax = float(r[7])
        pts = o[None, :] + ts[:, None] * d[None, :]
        for b in boxes:
            lo, hi = b[:3].astype(np.float64), b[3:].astype(np.float64)
            inside = np.all((pts > lo + margin) & (pts < hi - margin), axis=1) & (ts <= tmax - margin)
            hit, t0, t1 = oracle.slab(r, b)
            if inside.any():
                assert hit
                tin = ts[inside]
                assert t0 <= tin.min() + 1e-5 and t1 >= tin.max() - 1e-5
            if hit and t1 - t0 > 2e-3 and np.isfinite(t1):
                mid = o + 0.5 * (t0 + t1) * d
                assert np.all(mid >= lo - 1e-5) and np.all(mid <= hi + 1e-5)
                assert t0 >= 0.0 and t1 <= tmax


def test_traverse_counts_and_order():
    rng = np.random.default_rng(12)
    rays, boxes = _random_rays_boxes(rng, 500, 30)
    off, sr, sl, t0, t1 = oracle.traverse(rays, boxes)
    for i, r in enumerate(rays):
        expect = [(oracle.slab(r, b)[1], j) for j, b in enumerate(boxes) if oracle.slab(r, b)[0]]
        expect.sort()
        got = list(zip(t0[off[i]:off[i + 1]].tolist(), sl[off[i]:off[i + 1]].tolist()))
        assert [(float(a), b) for a, b in expect] == [(float(a), b) for a, b in got]
        assert np.all(sr[off[i]:off[i + 1]] == i)
    assert np.all(t0 <= t1)


def test_nested_boxes_nest_intervals():
    """A box containing another gets an interval containing the inner one
    (what lets a tree of unions reproduce the every-leaf answer)."""
    rng = np.random.default_rng(13)
    rays, boxes = _random_rays_boxes(rng, 400, 20)
    outer = boxes.copy()
    outer[:, :3] -= rng.uniform(0, 0.3, size=(20, 3)).astype(np.float32)
    outer[:, 3:] += rng.uniform(0, 0.3, size=(20, 3)).astype(np.float32)
    for r in rays:
        for b, B in zip(boxes, outer):
            h, a0, a1 = oracle.slab(r, b)
            if h:
                H, A0, A1 = oracle.slab(r, B)
                assert H and A0 <= a0 and A1 >= a1


# ---------------------------------------------------------------- sampling + encoding
def _dense_net():
    # every level dense: (N+1)^3 <= 4096
    return Net(3, 2, 12, 4, [4, 7, 11])


def _cfg(net, lo=(0.0, 0.0, 0.0), side=1.0):
    return oracle.make_cfg(net, np.array(lo, dtype=np.float32), np.float32(side))


def _random_segments(rng, n, lo=-1.0, hi=1.0):
    segs = np.zeros((n, 8), dtype=np.float32)
    segs[:, 0:3] = rng.uniform(lo, hi, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    segs[:, 4:7] = d
    segs[:, 3] = rng.uniform(0.0, 0.3, size=n)
    segs[:, 7] = segs[:, 3] + rng.uniform(0.0, 0.8, size=n)
    return segs


def test_sample_positions_closed_form():
    net = _dense_net()
    lo = np.array([-1.25, -1.0, -1.5], dtype=np.float32)
    cfg = _cfg(net, lo, 3.0)
    rng = np.random.default_rng(21)
    segs = _random_segments(rng, 200)
    x = oracle.sample_positions(cfg, segs).astype(np.float64)
    S = net.n_samples
    for s in range(S):
        ts = segs[:, 3].astype(np.float64) + (s + 0.5) / S * (segs[:, 7] - segs[:, 3]).astype(np.float64)
        p = segs[:, 0:3].astype(np.float64) + ts[:, None] * segs[:, 4:7].astype(np.float64)
        ref = np.clip((p - lo.astype(np.float64)) / 3.0, 0.0, 1.0)
        assert np.abs(x[:, s] - ref).max() < 4e-7


def _dense_vertex_coords(net, l):
    r1 = net.level_res[l] + 1
    e = np.arange(r1 ** 3)
    return np.stack([e % r1, (e // r1) % r1, e // (r1 * r1)], axis=1)


def test_linear_reproduction_dense_levels():
    """Trilinear interpolation reproduces affine functions exactly: with
    theta_l[v][f] = a_f * v_axis(f) / N_l + b_f on collision-free dense levels,
    the feature equals a_f * x_axis(f) + b_f at the sample point."""
    net = _dense_net()
    lo = np.array([-1.0, -1.0, -1.0], dtype=np.float32)
    cfg = _cfg(net, lo, 2.0)
    a = [0.7, -1.3]
    b = [0.1, 0.25]
    axis_of_f = [0, 2]
    table = []
    for l in range(net.n_levels):
        v = _dense_vertex_coords(net, l)
        t = np.zeros((v.shape[0], 2))
        for f in range(2):
            t[:, f] = a[f] * v[:, axis_of_f[f]] / net.level_res[l] + b[f]
        table.append(t.reshape(-1))
    table = np.concatenate(table)
    assert table.size == oracle.n_table_params(cfg)
    rng = np.random.default_rng(22)
    segs = _random_segments(rng, 300, -0.9, 0.9)
    u = oracle.encode(cfg, table, segs).reshape(300, net.n_samples, net.n_levels, 2)
    x = oracle.sample_positions(cfg, segs).astype(np.float64)
    for f in range(2):
        ref = a[f] * x[:, :, axis_of_f[f]] + b[f]
        for l in range(net.n_levels):
            assert np.abs(u[:, :, l, f] - ref).max() < 1e-12


def test_partition_of_unity_all_levels():
    """Constant tables give constant features on dense and hashed levels."""
    net = Net(4, 2, 10, 3, [3, 9, 17, 40])  # levels 0,1 dense; 2,3 hashed
    cfg = _cfg(net, (-1, -1, -1), 2.0)
    dense = [(r + 1) ** 3 <= 1024 for r in net.level_res]
    assert dense == [True, True, False, False]
    table = np.full(oracle.n_table_params(cfg), 0.375)
    rng = np.random.default_rng(23)
    segs = _random_segments(rng, 200)
    u = oracle.encode(cfg, table, segs)
    assert np.abs(u - 0.375).max() < 1e-14


def test_grid_vertices_pick_single_entry():
    """A point exactly on a grid vertex takes that vertex's entry alone.
    Entries hold their own position so the addressed slot is visible; the
    slot is compared with an independent recomputation of the dense index
    (x fastest) and of the spatial hash (primes 1, 2654435761, 805459861;
    Mueller et al. 2022). Hash values themselves are a definition: beyond
    this recomputation and the invariants, their parity is unpinned."""
    res = [8, 16, 32, 64]
    net = Net(4, 2, 10, 1, res)  # 9^3 = 729 <= 1024 dense; the others hashed
    cfg = _cfg(net, (0, 0, 0), 1.0)
    sizes = [(r + 1) ** 3 if (r + 1) ** 3 <= 1024 else 1024 for r in res]
    table = np.concatenate([np.stack([np.arange(s) + 0.0, np.arange(s) + 0.5], axis=1).reshape(-1) for s in sizes])
    rng = np.random.default_rng(24)
    for _ in range(100):
        l = int(rng.integers(0, 4))
        N = res[l]
        k = rng.integers(0, N + 1, size=3)
        # S = 1 sample at t0 + (t1 - t0)/2 along +x from (0, ky/N, kz/N): exact in binary32
        seg = np.array([0.0, k[1] / N, k[2] / N, 0.0, 1.0, 0.0, 0.0, 2.0 * k[0] / N], dtype=np.float32)
        u = oracle.encode(cfg, table, seg[None, :]).reshape(4, 2)
        cell = np.minimum(k, N - 1)
        if (N + 1) ** 3 <= 1024:
            slot = int(k[0] + (N + 1) * (k[1] + (N + 1) * k[2]))
        else:
            h = (int(k[0]) * 1) ^ ((int(k[1]) * 2654435761) & 0xFFFFFFFF) ^ ((int(k[2]) * 805459861) & 0xFFFFFFFF)
            slot = h & 1023
        assert (cell <= N - 1).all()
        assert u[l, 0] == slot and u[l, 1] == slot + 0.5, (l, k, u[l], slot)


def test_encode_feature_order():
    """Concatenation order s*L*F + l*F + f: with a table that is constant per
    (level, feature), feature slots identify themselves."""
    net = Net(3, 2, 11, 4, [3, 6, 20])
    cfg = _cfg(net, (-1, -1, -1), 2.0)
    sizes = [(r + 1) ** 3 if (r + 1) ** 3 <= 2048 else 2048 for r in net.level_res]
    table = np.concatenate([np.tile(np.array([10.0 * l, 10.0 * l + 1.0]), s) for l, s in enumerate(sizes)])
    u = oracle.encode(cfg, table, _random_segments(np.random.default_rng(25), 5))
    ref = np.tile(np.array([[10.0 * l + f for l in range(3) for f in range(2)]]), (1, 4))
    assert np.abs(u - ref).max() < 1e-13


# ---------------------------------------------------------------- MLP
def _split_weights(net, W):
    n_in = net.n_samples * net.n_levels * net.n_features
    dims = [(n_in, net.mlp_width)] + [(net.mlp_width, net.mlp_width)] * (net.mlp_hidden - 1) + [(net.mlp_width, net.n_out)]
    mats, o = [], 0
    for fi, fo in dims:
        mats.append(W[o:o + fi * fo].reshape(fo, fi))
        o += fi * fo
    return mats


def test_mlp_matches_library_matmul():
    net = Net(2, 2, 8, 4, [3, 5], mlp_width=32, mlp_hidden=3, n_out=5)
    cfg = _cfg(net)
    rng = np.random.default_rng(31)
    W = rng.normal(size=oracle.n_mlp_params(cfg)) * 0.3
    u = rng.normal(size=(64, 16))
    z = oracle.mlp_forward(cfg, W, u)
    h = u.T
    mats = _split_weights(net, W)
    for M in mats[:-1]:
        h = np.maximum(M @ h, 0.0)
    ref = (mats[-1] @ h).T
    assert np.abs(z - ref).max() < 1e-12


def test_mlp_identity_weights():
    net = Net(2, 2, 8, 2, [3, 5], mlp_width=8, mlp_hidden=2, n_out=5)
    cfg = _cfg(net)
    W = np.concatenate([np.eye(8).reshape(-1), np.eye(8).reshape(-1), np.eye(5, 8).reshape(-1)])
    u = np.random.default_rng(32).normal(size=(10, 8))
    z = oracle.mlp_forward(cfg, W, u)
    assert np.array_equal(z, np.maximum(u, 0.0)[:, :5])


def test_min_abs_preact_matches_library_matmul():
    """The smallest |pre-activation| over every hidden unit of a segment,
    from numpy float64 products of the encoded features, over all hidden
    layers (and never the output layer)."""
    net = Net(2, 2, 8, 2, [3, 5], mlp_width=16, mlp_hidden=3, n_out=5)
    cfg = _cfg(net, (-1, -1, -1), 2.0)
    rng = np.random.default_rng(35)
    table = rng.normal(size=oracle.n_table_params(cfg))
    W = rng.normal(size=oracle.n_mlp_params(cfg)) * 0.4
    segs = _random_segments(rng, 300)
    got = oracle.min_abs_preact(cfg, np.concatenate([table, W]), segs)
    h = oracle.encode(cfg, table, segs).T
    mats = _split_weights(net, W)
    per_layer = []
    for M in mats[:-1]:
        a = M @ h
        per_layer.append(np.abs(a).min(0))
        h = np.maximum(a, 0.0)
    ref = np.min(per_layer, axis=0)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15)
    # every hidden layer can hold the minimum on some segment; the output
    # layer never does (its pre-activations are not ReLU inputs)
    which = np.argmin(per_layer, axis=0)
    assert set(which.tolist()) == {0, 1, 2}
    z = (mats[-1] @ h).T
    assert np.any(np.abs(z).min(1) < got)


def test_layer_amax_identity_network():
    """With W_0 = +-I and W_1 = I the hidden layers carry ReLU(+-u), so the
    per-layer maxima are max|u|, then the largest positive (or negated
    negative) feature twice. The table is shifted negative so that max|u|,
    max u+ and max (-u)+ all differ."""
    net = Net(2, 2, 8, 2, [3, 5], mlp_width=8, mlp_hidden=2, n_out=5)
    cfg = _cfg(net, (-1, -1, -1), 2.0)
    rng = np.random.default_rng(33)
    table = rng.normal(size=oracle.n_table_params(cfg)) - 0.4
    segs = _random_segments(rng, 200)
    u = oracle.encode(cfg, table, segs)
    assert u.max() > 0 and -u.min() > u.max()
    for sign in (1.0, -1.0):
        W = np.concatenate([sign * np.eye(8).reshape(-1), np.eye(8).reshape(-1), np.eye(5, 8).reshape(-1)])
        a = oracle.layer_amax(cfg, np.concatenate([table, W]), segs)
        top = np.maximum(sign * u, 0.0).max()
        assert a.shape == (3,)
        assert a[0] == np.abs(u).max() and a[1] == top and a[2] == top


def test_layer_amax_positive_homogeneity():
    """ReLU(c x) = c ReLU(x) for c > 0: scaling W_1 by 3 triples the maximum
    of layer 2's input only."""
    net = Net(2, 2, 8, 2, [3, 5], mlp_width=16, mlp_hidden=3, n_out=5)
    cfg = _cfg(net, (-1, -1, -1), 2.0)
    rng = np.random.default_rng(34)
    table = rng.normal(size=oracle.n_table_params(cfg))
    W = rng.normal(size=oracle.n_mlp_params(cfg)) * 0.5
    segs = _random_segments(rng, 300)
    a = oracle.layer_amax(cfg, np.concatenate([table, W]), segs)
    W3 = W.copy()
    o = 8 * 16
    W3[o:o + 16 * 16] *= 3.0
    b = oracle.layer_amax(cfg, np.concatenate([table, W3]), segs)
    assert np.all(a > 0)
    assert b[0] == a[0] and b[1] == a[1]
    assert abs(b[2] - 3.0 * a[2]) <= 1e-12 * a[2] and abs(b[3] - 3.0 * a[3]) <= 1e-12 * a[3]


def test_first_hits_hand_cases():
    """The first leaf a ray crosses, the acceptance test and the crossing
    counts on hand-placed boxes (two unit cubes on the x axis, and a copy of
    the first to make a tie that the lower id wins)."""
    boxes = np.array([[0, 0, 0, 1, 1, 1], [2, 0, 0, 3, 1, 1], [0, 0, 0, 1, 1, 1]], dtype=np.float32)
    rays = np.array([[-1, .5, .5, 0, 1, 0, 0, np.inf],     # +x: crosses 0, 2 (tie at t=1) then 1
                     [4, .5, .5, 0, -1, 0, 0, np.inf],     # -x: crosses 1 first
                     [-1, 5, .5, 0, 1, 0, 0, np.inf]],     # misses everything
                    dtype=np.float32)
    u = np.array([0.5, 0.5, 0.0], dtype=np.float32)
    ray, leaf, t0, t1, hits = oracle.first_hits(rays, boxes, u, np.array([1.0, 0.6, 1.0], dtype=np.float32))
    assert ray.tolist() == [0, 1] and leaf.tolist() == [0, 1]
    assert t0.tolist() == [1.0, 1.0] and t1.tolist() == [2.0, 2.0]
    assert hits.tolist() == [2, 2, 2]
    ray, leaf, *_ = oracle.first_hits(rays, boxes, u, np.array([0.5, 0.6, 1.0], dtype=np.float32))
    assert ray.tolist() == [1]  # u = 0.5 is not below an acceptance of 0.5


def test_segment_loss_closed_form_and_mean():
    """At z = 0 each segment's loss is 2 log 2 + h (2 |1/2 - tau| + (1/3)
    sum |n|); at any z the segment losses average to the batch loss."""
    net = Net(1, 2, 8, 1, [3])
    cfg = _cfg(net)
    rng = np.random.default_rng(35)
    lab = _labels(rng, 50)
    z0 = np.zeros((50, 5))
    h, tau, nn = lab[:, 4].astype(np.float64), lab[:, 0].astype(np.float64), lab[:, 1:4].astype(np.float64)
    ref = 2 * np.log(2.0) + h * (2 * np.abs(0.5 - tau) + np.abs(nn).sum(1) / 3.0)
    assert np.abs(oracle.segment_loss(cfg, z0, lab) - ref).max() < 1e-14
    z = rng.normal(size=(50, 5))
    terms, _ = oracle.loss(cfg, z, lab, with_grad=False)
    assert abs(oracle.segment_loss(cfg, z, lab).mean() - terms[0]) < 1e-13


# ---------------------------------------------------------------- loss
def _labels(rng, n, hit_frac=0.5):
    lab = np.zeros((n, 8), dtype=np.float32)
    hit = rng.uniform(size=n) < hit_frac
    lab[:, 0] = np.where(hit, rng.uniform(size=n), 0.0)
    nv = rng.normal(size=(n, 3))
    nv /= np.linalg.norm(nv, axis=1, keepdims=True)
    lab[:, 1:4] = np.where(hit[:, None], nv, 0.0)
    lab[:, 4] = hit
    return lab


def test_loss_closed_form_at_zero():
    """At z = 0: per segment 2 log 2 + h (2 |1/2 - tau| + (1/3) sum |n|), and
    dL/dz = (2 (1/2 - h), 2 h sgn(1/2 - tau) / 4, h sgn(-n) / 3) / B."""
    net = Net(1, 2, 8, 1, [3])
    cfg = _cfg(net)
    rng = np.random.default_rng(41)
    lab = _labels(rng, 257)
    h, tau, n = lab[:, 4].astype(np.float64), lab[:, 0].astype(np.float64), lab[:, 1:4].astype(np.float64)
    terms, dz = oracle.loss(cfg, np.zeros((257, 5)), lab)
    per = 2 * math.log(2.0) + h * (2 * np.abs(0.5 - tau) + np.abs(n).sum(axis=1) / 3.0)
    assert abs(terms[0] - per.mean()) < 1e-14
    assert abs(terms[1] - math.log(2.0)) < 1e-13
    B = 257.0
    assert np.allclose(dz[:, 0], 2 * (0.5 - h) / B, rtol=0, atol=1e-17)
    assert np.allclose(dz[:, 1], h * 2 * np.sign(0.5 - tau) * 0.25 / B, rtol=0, atol=1e-17)
    assert np.allclose(dz[:, 2:5], h[:, None] * np.sign(-n) / (3 * B), rtol=0, atol=1e-17)


def _albedo_labels(rng, n):
    lab = _labels(rng, n)
    lab[:, 5:8] = rng.uniform(0.05, 0.95, size=(n, 3))
    return lab


def test_albedo_loss_closed_forms():
    """With 8 outputs the albedo adds a relative L2 term, (a_hat - a)^2 /
    (a_hat^2 + 0.01) averaged over the channels, masked by the hit label:
    at z = 0 (a_hat = 1/2) it is (1/2 - a)^2 / 0.26 per channel, and it and
    its gradient vanish where a_hat equals the label."""
    net = Net(1, 2, 8, 1, [3], n_out=8)
    cfg = _cfg(net)
    rng = np.random.default_rng(36)
    lab = _albedo_labels(rng, 40)
    l64 = lab.astype(np.float64)
    h, a = l64[:, 4], l64[:, 5:8]
    base = 2 * np.log(2.0) + h * (2 * np.abs(0.5 - l64[:, 0]) + np.abs(l64[:, 1:4]).sum(1) / 3.0)
    ref = base + h * ((0.5 - a) ** 2 / 0.26).mean(1)
    assert np.abs(oracle.segment_loss(cfg, np.zeros((40, 8)), lab) - ref).max() < 1e-13
    terms, _ = oracle.loss(cfg, np.zeros((40, 8)), lab, with_grad=False)
    assert abs(terms[0] - ref.mean()) < 1e-13
    z = rng.normal(size=(40, 8))
    z[:, 5:8] = np.log(a / (1.0 - a))
    _, dz = oracle.loss(cfg, z, lab)
    assert np.abs(dz[:, 5:8]).max() < 1e-15
    w0 = oracle.segment_loss(cfg, z, lab, weights=(2.0, 2.0, 1.0, 0.0))
    assert np.abs(oracle.segment_loss(cfg, z, lab) - w0).max() < 1e-14


def test_albedo_loss_gradient_finite_difference():
    """The relative L2 term's denominator is held constant in the derivative.
    The label enters only the numerator, so central differences of the
    loss in the label direction give -d/d(a_hat) with the denominator
    constant; times the logistic slope sigma'(z) = e^-z / (1 + e^-z)^2 that
    must be the gradient in z. (Differentiating the denominator too would
    differ by (a_hat - a)^2 2 a_hat / (a_hat^2 + 0.01)^2.)"""
    net = Net(1, 2, 8, 1, [3], n_out=8)
    cfg = _cfg(net)
    rng = np.random.default_rng(37)
    lab = _albedo_labels(rng, 30)
    lab[:, 4] = 1.0  # every segment hit: the albedo term is on
    z = rng.normal(size=(30, 8))
    _, dz = oracle.loss(cfg, z, lab)
    h = 1e-6
    checked = 0
    for i in range(30):
        for o in (5, 6, 7):
            lp, lm = lab.copy(), lab.copy()
            lp[i, o] += np.float32(h)
            lm[i, o] -= np.float32(h)
            step = float(lp[i, o]) - float(lm[i, o])
            fd_a = (oracle.loss(cfg, z, lp, with_grad=False)[0][0] - oracle.loss(cfg, z, lm, with_grad=False)[0][0]) / step
            slope = np.exp(-z[i, o]) / (1.0 + np.exp(-z[i, o])) ** 2
            assert abs(-fd_a * slope - dz[i, o]) <= 1e-6 * abs(dz[i, o]) + 1e-10, (i, o, -fd_a * slope, dz[i, o])
            checked += 1
    assert checked == 90 and np.abs(dz[:, 5:8]).max() > 1e-3


def test_loss_gradient_finite_difference():
    """dL/dz against central differences of the loss itself (BCE slope
    sigmoid(z) - h; L1 slopes away from their kinks)."""
    net = Net(1, 2, 8, 1, [3])
    cfg = _cfg(net)
    rng = np.random.default_rng(42)
    n = 64
    lab = _labels(rng, n)
    z = rng.normal(size=(n, 5))
    _, dz = oracle.loss(cfg, z, lab)
    eps = 1e-6
    for i in range(n):
        for o in range(5):
            zp, zm = z.copy(), z.copy()
            zp[i, o] += eps
            zm[i, o] -= eps
            fd = (oracle.loss(cfg, zp, lab, with_grad=False)[0][0] - oracle.loss(cfg, zm, lab, with_grad=False)[0][0]) / (2 * eps)
            assert abs(fd - dz[i, o]) < 1e-8 * max(1.0, abs(dz[i, o])) + 1e-9
    sig = 1 / (1 + np.exp(-z[:, 0]))
    assert np.allclose(dz[:, 0] * n / 2.0, sig - lab[:, 4], atol=1e-13)


# ---------------------------------------------------------------- full gradient
def _small_problem(seed=51, n=96):
    net = Net(3, 2, 9, 4, [3, 8, 21], mlp_width=16, mlp_hidden=2, n_out=5)
    cfg = _cfg(net, (-1.0, -1.0, -1.0), 2.0)
    rng = np.random.default_rng(seed)
    nt, nm = oracle.n_table_params(cfg), oracle.n_mlp_params(cfg)
    params = np.concatenate([rng.normal(0, 0.5, size=nt), rng.normal(0, 0.4, size=nm)])
    segs = _random_segments(rng, n, -0.8, 0.8)
    lab = _labels(rng, n)
    return net, cfg, params, segs, lab


def test_backward_finite_differences():
    """Analytic gradient of the combined loss vs float64 central differences,
    on all MLP weights and on touched table entries. Coordinates whose step
    crosses a kink (ReLU or L1) are detected by two step sizes disagreeing
    and skipped; most coordinates must be checked."""
    net, cfg, params, segs, lab = _small_problem()

    def L(p):
        return oracle.loss(cfg, oracle.forward(cfg, p, segs), lab, with_grad=False)[0][0]

    z = oracle.forward(cfg, params, segs)
    _, dz = oracle.loss(cfg, z, lab)
    g = oracle.backward(cfg, params, segs, dz)
    nt = oracle.n_table_params(cfg)
    rng = np.random.default_rng(52)
    touched = np.nonzero(g[:nt])[0]
    idx = np.concatenate([np.arange(nt, params.size), rng.choice(touched, size=min(300, touched.size), replace=False)])
    checked = 0
    for i in idx:
        fds = []
        for h in (1e-4, 1e-5):
            p1, p2 = params.copy(), params.copy()
            p1[i] += h
            p2[i] -= h
            fds.append((L(p1) - L(p2)) / (2 * h))
        if abs(fds[0] - fds[1]) > 1e-7 * max(1e-3, abs(fds[1])):
            continue
        checked += 1
        assert abs(fds[0] - g[i]) <= 1e-6 * max(abs(g[i]), 1e-4 * np.abs(g).max()), (i, fds, g[i])
    assert checked >= 0.9 * idx.size


def test_backward_sum_over_batch():
    """Gradients of a batch equal the sum of single-segment gradients."""
    net, cfg, params, segs, lab = _small_problem(53, 12)
    z = oracle.forward(cfg, params, segs)
    _, dz = oracle.loss(cfg, z, lab)
    g = oracle.backward(cfg, params, segs, dz)
    acc = np.zeros_like(g)
    for i in range(12):
        acc += oracle.backward(cfg, params, segs[i:i + 1], dz[i:i + 1])
    assert np.abs(acc - g).max() < 1e-14 * max(1.0, np.abs(g).max()) * 100


# ---------------------------------------------------------------- Adam
def test_adam_first_steps_closed_form():
    """Step 1: bias-corrected moments are g and g^2, so the update is
    -lr g / (|g| + eps). Step 2 with g2: m = 0.9*0.1 g + 0.1 g2 over
    (1 - 0.9^2), v likewise with beta2; checked against that hand formula.
    A zero gradient leaves a fresh parameter unchanged."""
    rng = np.random.default_rng(61)
    g = rng.normal(size=1000) * np.logspace(-6, 1, 1000)
    g[:5] = 0.0
    p = rng.normal(size=1000)
    p0 = p.copy()
    m = np.zeros(1000)
    v = np.zeros(1000)
    oracle.adam(p, g, m, v, 1, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8)
    assert np.allclose(p - p0, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    assert np.array_equal(p[:5], p0[:5])
    g2 = rng.normal(size=1000)
    p1 = p.copy()
    oracle.adam(p, g2, m, v, 2, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8)
    mh = (0.9 * 0.1 * g + 0.1 * g2) / (1 - 0.81)
    vh = (0.99 * 0.01 * g * g + 0.01 * g2 * g2) / (1 - 0.99 ** 2)
    assert np.allclose(p - p1, -1e-2 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-10, atol=1e-18)


def test_adam_unscale():
    rng = np.random.default_rng(62)
    g = rng.normal(size=50)
    pa, pb = np.ones(50), np.ones(50)
    ma, va, mb, vb = (np.zeros(50) for _ in range(4))
    oracle.adam(pa, g, ma, va, 1)
    oracle.adam(pb, g * 1024.0, mb, vb, 1, inv_scale=1.0 / 1024.0)
    assert np.array_equal(pa, pb)


# ---------------------------------------------------------------- resolve
def test_resolve_hand_cases():
    """min over hit segments of t0 + sigmoid(z1) (t1 - t0); z0 = 0 is a miss;
    equal t keeps the earlier segment."""
    logit = lambda p: math.log(p / (1 - p))
    offsets = np.array([0, 3, 5, 6, 6], dtype=np.uint64)
    leaf = np.array([7, 3, 9, 1, 2, 4], dtype=np.uint32)
    t0 = np.array([1.0, 1.5, 4.0, 1.0, 1.0, 2.0], dtype=np.float32)
    t1 = np.array([2.0, 3.0, 5.0, 3.0, 2.0, 3.0], dtype=np.float32)
    z = np.zeros((6, 5))
    z[:, 0] = [1.0, 2.0, 3.0, 1.0, 1.0, 0.0]
    z[:, 1] = [logit(0.5), logit(0.1), 0.0, logit(0.25), 0.0, 0.0]
    z[:, 2:5] = np.arange(18).reshape(6, 3)
    out = oracle.resolve(offsets, leaf, t0, t1, z, 5)
    # ray 0: candidates 1.5, 1.65, 4.5 -> segment 0 (leaf 7)
    assert abs(out[0, 0] - 1.5) < 1e-15 and out[0, 4] == 7 and out[0, 5] == 0
    assert np.array_equal(out[0, 1:4], [0, 1, 2])
    # ray 1: 1.0 + 0.25*2 = 1.5 and 1.0 + 0.5*1 = 1.5 -> tie keeps segment 3 (leaf 1)
    assert abs(out[1, 0] - 1.5) < 1e-15 and out[1, 4] == 1
    # ray 2: z0 == 0 -> miss; ray 3: no segments -> miss
    assert out[2, 4] == -1 and out[3, 4] == -1


# ---------------------------------------------------------------- labels (input generator)
def test_labels_bvh_equals_brute_force():
    sc = configs.make_scene(20480, 64)
    p, _ = scene.leaf_probes(sc.boxes, 64, seed=77)
    p = p.astype(np.float64)[:4096]
    a = sc.mesh.closest(p[:, 0:3], p[:, 4:7], p[:, 3], p[:, 7])
    b = sc.mesh.closest(p[:, 0:3], p[:, 4:7], p[:, 3], p[:, 7], brute=True)
    assert a["hit"].mean() > 0.2
    assert np.array_equal(a["tri"], b["tri"]) and np.array_equal(a["t"], b["t"])


def test_labels_sphere_within_sagitta():
    """Amplitude 0: the mesh is the icosphere; hit distances from the origin
    lie between cos(rho) and 1, rho being the largest facet's angular
    circumradius."""
    n = 16
    v, t = scene.icosphere(n)
    mesh = scene.TriangleMesh(v, t)
    rng = np.random.default_rng(78)
    d = rng.normal(size=(2000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.zeros((2000, 3))
    r = mesh.closest(o, d, 0.0, 10.0)
    assert r["hit"].all()
    tv = v[t]
    cen = tv.mean(axis=1)
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    rho = np.arccos(np.clip(np.einsum("tkj,tj->tk", tv, cen), -1, 1)).max()
    assert r["t"].max() <= 1.0 + 1e-12 and r["t"].min() >= math.cos(rho) - 1e-12
    # normals point outward
    assert (np.einsum("ij,ij->i", r["n"], d) > 0).all()


# ---------------------------------------------------------------- queries from inside a leaf (reversed chords)
TAG = oracle.INSIDE_TAG


def test_reverse_traversal_closed_form():
    """+z ray from the centre of the unit cube: the clip rule gives [0, 0.5];
    the reverse rule gives the whole chord [-0.5, 0.5], tagged. A ray from
    outside gets [2, 3] under both rules."""
    box = np.array([[0, 0, 0, 1, 1, 1]], dtype=np.float32)
    rays = np.array([[0.5, 0.5, 0.5, 0, 0, 0, 1, np.inf],
                     [0.5, 0.5, -2.0, 0, 0, 0, 1, np.inf]], dtype=np.float32)
    off, sr, sl, t0, t1 = oracle.traverse(rays, box)
    assert sl.tolist() == [0, 0] and t0.tolist() == [0.0, 2.0] and t1.tolist() == [0.5, 3.0]
    off, sr, sl, t0, t1 = oracle.traverse(rays, box, reverse=True)
    assert sl.tolist() == [TAG, 0] and t0.tolist() == [-0.5, 2.0] and t1.tolist() == [0.5, 3.0]
    # tmin > 0 moves the origin along the ray: from z = 0.5 + 0.25 the chord is unchanged
    r = rays[:1].copy()
    r[0, 3] = 0.25
    _, _, sl, t0, t1 = oracle.traverse(r, box, reverse=True)
    assert sl.tolist() == [TAG] and t0.tolist() == [-0.5] and t1.tolist() == [0.5]


def test_reverse_rule_changes_only_boxes_around_the_origin():
    """Segments of boxes that do not contain the origin are the same under
    both rules; boxes that do get the chord start (entry < tmin) and the tag,
    and the run is still sorted by (t0, tagged id)."""
    rng = np.random.default_rng(31)
    rays, boxes = _random_rays_boxes(rng, 400, 40)
    rays[:, 0:3] = rng.uniform(-0.5, 0.5, size=(400, 3))  # many origins inside boxes
    a = oracle.traverse(rays, boxes)
    b = oracle.traverse(rays, boxes, reverse=True)
    assert np.array_equal(a[0], b[0])
    n_in = 0
    for i, r in enumerate(rays):
        sa = {(int(l), float(x), float(y)) for l, x, y in zip(*(v[a[0][i]:a[0][i + 1]] for v in a[2:]))}
        sb = list(zip(*(v[b[0][i]:b[0][i + 1]] for v in b[2:])))
        assert sorted(sb, key=lambda s: (float(s[1]), int(s[0]))) == sb
        for l, x, y in sb:
            l = int(l)
            if l & TAG:
                n_in += 1
                lo, hi = boxes[l & ~TAG, :3], boxes[l & ~TAG, 3:]
                assert np.all(r[0:3] >= lo) and np.all(r[0:3] <= hi)  # origin in the box
                assert x < r[3] and (l & ~TAG, float(r[3]), float(y)) in sa
                # the chord's entry point lies on the box surface
                p = r[0:3].astype(np.float64) + float(x) * r[4:7].astype(np.float64)
                assert np.min(np.minimum(np.abs(p - lo), np.abs(p - hi))) < 1e-5
            else:
                assert (l, float(x), float(y)) in sa
    assert n_in > 50


def test_reversed_rows_sample_the_chord_backwards():
    """A tagged segment's probe row is the ray (o, -d) over [-t1, -t0]: its
    sample points are the forward chord's in the opposite order."""
    net = Net(2, 2, 10, 4, [4, 8])
    cfg = oracle.make_cfg(net, np.zeros(3, np.float32), np.float32(2.0))
    rays = np.array([[0.7, 0.9, 1.1, 0, 0.3, 0.4, 0.5, np.inf]], dtype=np.float32)
    fwd = oracle.segment_rows(rays, np.array([0]), np.array([-0.8], np.float32), np.array([0.6], np.float32))
    rev = oracle.segment_rows(rays, np.array([0]), np.array([-0.8], np.float32), np.array([0.6], np.float32),
                              np.array([TAG], np.uint32))
    assert rev[0, 3] == np.float32(-0.6) and rev[0, 7] == np.float32(0.8)
    assert np.array_equal(rev[0, 4:7], -rays[0, 4:7])
    xf = oracle.sample_positions(cfg, fwd)[0]
    xr = oracle.sample_positions(cfg, rev)[0]
    assert np.abs(xr - xf[::-1]).max() < 1e-6


def test_resolve_reversed_hand_cases():
    """A tagged segment's hit lies at t1 - sigmoid(z1) (t1 - t0) and counts
    only in front of the origin (t > tmin); the leaf is reported untagged."""
    logit = lambda p: math.log(p / (1 - p))
    offsets = np.array([0, 2, 3, 4], dtype=np.uint64)
    leaf = np.array([5 | TAG, 6, 8 | TAG, 9 | TAG], dtype=np.uint32)
    t0 = np.array([-1.0, 0.5, -1.0, -2.0], dtype=np.float32)
    t1 = np.array([1.0, 3.0, 1.0, 2.0], dtype=np.float32)
    z = np.zeros((4, 5))
    z[:, 0] = 1.0
    z[:, 1] = [logit(0.25), logit(0.5), logit(0.75), logit(0.5)]
    tmin = np.array([0.0, 0.0, 0.0], dtype=np.float32)
    out = oracle.resolve(offsets, leaf, t0, t1, z, 5, tmin)
    # ray 0: tagged 1 - 0.25*2 = 0.5 ahead of 0; the untagged segment gives 1.75 -> 0.5, leaf 5
    assert abs(out[0, 0] - 0.5) < 1e-15 and out[0, 4] == 5 and out[0, 5] == 0
    # ray 1: 1 - 0.75*2 = -0.5 is behind the origin -> miss
    assert out[1, 4] == -1
    # ray 2: 2 - 0.5*4 = 0 is not in front of tmin = 0 -> miss
    assert out[2, 4] == -1


def test_reverse_rule_with_exact_outputs_matches_ground_truth():
    """With network outputs read off the exact labels of each queried
    segment, the reverse rule returns the first surface point in front of the
    origin for secondary rays leaving a surface that crosses the leaf once:
    a square (two triangles) in the middle of a unit box, rays starting just
    above it. Rays pointing down hit it; rays pointing up miss it (the only
    crossing of their chord lies behind the origin)."""
    verts = np.array([[0.1, 0.1, 0.5], [0.9, 0.1, 0.5], [0.9, 0.9, 0.5], [0.1, 0.9, 0.5]])
    tris = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    mesh = scene.TriangleMesh(verts, tris)
    box = np.array([[0, 0, 0, 1, 1, 1]], dtype=np.float32)
    rng = np.random.default_rng(33)
    n = 400
    rays = np.zeros((n, 8), dtype=np.float32)
    rays[:, 0:2] = rng.uniform(0.3, 0.7, size=(n, 2))
    rays[:, 2] = 0.5 + 1e-3
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    off, sr, sl, t0, t1 = oracle.traverse(rays, box, reverse=True)
    assert np.all(sl == TAG)
    rows = oracle.segment_rows(rays, sr, t0, t1, sl)
    lab = scene.probe_labels(mesh, rows)
    tau = np.clip(lab[:, 0].astype(np.float64), 1e-12, 1 - 1e-12)
    z = np.zeros((rows.shape[0], 5))
    z[:, 0] = np.where(lab[:, 4] > 0, 10.0, -10.0)
    z[:, 1] = np.log(tau / (1 - tau))
    z[:, 2:5] = lab[:, 1:4]
    out = oracle.resolve(off, sl, t0, t1, z, 5, rays[:, 3])
    gt = scene.ray_ground_truth(mesh, rays)
    got_hit = out[:, 4] >= 0
    assert np.array_equal(got_hit, gt["hit"]) and 0.2 < gt["hit"].mean() < 0.8
    assert np.abs(out[got_hit, 0] - gt["t"][got_hit]).max() < 1e-6


# ------------------------------------------------------------------ construction: rank and acceptance
def test_node_rank_closed_form():
    """Sec. 5.1: r = 2 log q + log p, q = loss / count, p = hits / rays; a leaf
    without segments, crossings or loss ranks -inf."""
    loss = np.array([2.0, 0.0, 1.0, math.e ** -1.5, 3.0, 5.0])
    count = np.array([4, 0, 2, 1, 3, 1])
    hits = np.array([10, 5, 0, 25, 100, 1])
    r = oracle.node_rank(loss, count, hits, 100)
    assert abs(r[0] - (2 * math.log(0.5) + math.log(0.1))) < 1e-14
    assert r[1] == -math.inf and r[2] == -math.inf
    assert abs(r[3] - (-3.0 + math.log(0.25))) < 1e-14
    assert abs(r[4]) < 1e-14  # q = 1, p = 1
    assert abs(r[5] - (2 * math.log(5.0) + math.log(0.01))) < 1e-13
    assert oracle.node_rank(np.array([0.0]), np.array([3]), np.array([3]), 10)[0] == -math.inf


def test_acceptance_closed_form():
    """Sec. 5.2, read in linear space: max(exp(r - r_max), floor); the worst
    leaf is always trained, -inf takes the floor, no finite rank trains all."""
    r = np.array([-1.0, -3.0, -math.inf, -20.0, -1.0 - math.log(4.0)])
    a = oracle.acceptance(r, 0.005)
    assert a[0] == 1.0 and abs(a[1] - math.exp(-2.0)) < 1e-15
    assert a[2] == 0.005 and a[3] == 0.005 and abs(a[4] - 0.25) < 1e-15
    assert np.all(oracle.acceptance(np.full(3, -math.inf), 0.005) == 1.0)
    # the same leaf order as the ranks (monotone), invariant under a common shift
    rr = np.random.default_rng(3).normal(size=50) * 3
    aa = oracle.acceptance(rr, 0.0)
    assert np.all(np.argsort(rr, kind="stable") == np.argsort(aa, kind="stable"))
    assert np.allclose(oracle.acceptance(rr + 7.5, 0.0), aa, rtol=1e-14)
    # rank of q^2 p: scaling every q by c leaves the acceptance unchanged
    loss = np.random.default_rng(4).uniform(0.1, 2.0, 20)
    cnt = np.random.default_rng(5).integers(1, 50, 20)
    hit = np.random.default_rng(6).integers(1, 90, 20)
    a1 = oracle.acceptance(oracle.node_rank(loss, cnt, hit, 100), 0.0)
    a2 = oracle.acceptance(oracle.node_rank(3.0 * loss, cnt, hit, 100), 0.0)
    assert np.allclose(a1, a2, rtol=1e-13)
    q2p = (loss / cnt) ** 2 * hit
    assert np.allclose(a1, q2p / q2p.max(), rtol=1e-13)
