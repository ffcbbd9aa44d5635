"""FP64 CPU oracle of the N-BVH neural ray query and training step.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library never
does, and it shares no code with it. The arithmetic lives in nbvh_oracle.c
(binary64 except the slab test and the sample positions, which are defined in
binary32 because they decide integers: which leaves are visited and which
hash-grid cell a point falls in).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_nbvh_oracle.so")
_LIB = None
_LOCK = threading.Lock()


def build(force: bool = False) -> str:
    """Compile nbvh_oracle.c with gcc (no FMA contraction, OpenMP)."""
    src = os.path.join(_HERE, "nbvh_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class OcCfg(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("n_features", ctypes.c_int32),
                ("log2_T", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("level_res", ctypes.c_int32 * 32), ("mlp_width", ctypes.c_int32),
                ("mlp_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("scene_lo", ctypes.c_float * 3), ("scene_side", ctypes.c_float)]


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(_SO):
                build()
            L = ctypes.CDLL(_SO)
            P, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
            L.oc_slab_one.argtypes = [P, P, P]
            L.oc_slab_one.restype = ctypes.c_int
            L.oc_traverse_count.argtypes = [P, I, P, I, P]
            L.oc_traverse_fill.argtypes = [P, I, P, I, P, P, P, P, P, ctypes.c_int]
            L.oc_sample_positions.argtypes = [P, P, I, P]
            L.oc_table_params.argtypes = [P]
            L.oc_table_params.restype = I
            L.oc_mlp_params.argtypes = [P]
            L.oc_mlp_params.restype = I
            L.oc_encode.argtypes = [P, P, P, I, P]
            L.oc_mlp_forward.argtypes = [P, P, P, I, P]
            L.oc_loss.argtypes = [P, P, P, I, D, D, D, D, P, P]
            L.oc_segment_loss.argtypes = [P, P, P, I, D, D, D, D, P]
            L.oc_backward.argtypes = [P, P, P, I, P, P]
            L.oc_adam.argtypes = [I, P, P, P, P, I, D, D, D, D, D]
            L.oc_min_abs_preact.argtypes = [P, P, P, I, P]
            L.oc_layer_amax.argtypes = [P, P, P, I, P]
            L.oc_resolve.argtypes = [I, P, P, P, P, P, ctypes.c_int, P, P]
            L.oc_node_rank.argtypes = [I, P, P, P, I, P]
            L.oc_acceptance.argtypes = [I, P, D, P]
            L.oc_num_threads.restype = ctypes.c_int
            _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def make_cfg(net, scene_lo, scene_side) -> OcCfg:
    """net: anything with n_levels, n_features, log2_T, n_samples, level_res,
    mlp_width, mlp_hidden, n_out attributes."""
    c = OcCfg()
    c.n_levels, c.n_features, c.log2_T, c.n_samples = net.n_levels, net.n_features, net.log2_T, net.n_samples
    for i, r in enumerate(net.level_res):
        c.level_res[i] = int(r)
    c.mlp_width, c.mlp_hidden, c.n_out = net.mlp_width, net.mlp_hidden, net.n_out
    for a in range(3):
        c.scene_lo[a] = float(np.float32(scene_lo[a]))
    c.scene_side = float(np.float32(scene_side))
    return c


def n_table_params(cfg: OcCfg) -> int:
    return int(_lib().oc_table_params(ctypes.byref(cfg)))


def n_mlp_params(cfg: OcCfg) -> int:
    return int(_lib().oc_mlp_params(ctypes.byref(cfg)))


def n_in(cfg: OcCfg) -> int:
    return cfg.n_samples * cfg.n_levels * cfg.n_features


def num_threads() -> int:
    return int(_lib().oc_num_threads())


# -- traversal -----------------------------------------------------------------
def slab(ray, box):
    """(hit, t0, t1) of one ray row [o, tmin, d, tmax] against [lo, hi]."""
    out = np.zeros(2, dtype=np.float32)
    h = _lib().oc_slab_one(_p(_c(ray, np.float32)), _p(_c(box, np.float32)), _p(out))
    return bool(h), out[0], out[1]


INSIDE_TAG = 0x80000000


def traverse(rays, boxes, reverse=False):
    """Every-leaf traversal. Returns (offsets uint64 [n+1], seg_ray, seg_leaf
    uint32, seg_t0, seg_t1 float32), each ray's run sorted by (t0, leaf).
    reverse: a leaf around the ray origin gives its whole chord [entry, exit]
    with INSIDE_TAG set in its leaf id (queried backwards)."""
    rays = _c(rays, np.float32)
    boxes = _c(boxes, np.float32)
    n, m = rays.shape[0], boxes.shape[0]
    counts = np.zeros(n, dtype=np.uint32)
    L = _lib()
    L.oc_traverse_count(_p(rays), n, _p(boxes), m, _p(counts))
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=offsets[1:])
    tot = int(offsets[-1])
    sr = np.zeros(tot, dtype=np.uint32)
    sl = np.zeros(tot, dtype=np.uint32)
    t0 = np.zeros(tot, dtype=np.float32)
    t1 = np.zeros(tot, dtype=np.float32)
    L.oc_traverse_fill(_p(rays), n, _p(boxes), m, _p(offsets), _p(sr), _p(sl), _p(t0), _p(t1), int(bool(reverse)))
    return offsets, sr, sl, t0, t1


def segment_rows(rays, seg_ray, seg_t0, seg_t1, seg_leaf=None):
    """[n_seg][8] float32 rows (o, t0, d, t1) for the segments of a traversal.
    A tagged (inside) segment is the chord crossed backwards from its exit:
    the ray (o, -d) over [-t1, -t0], so its samples run from the exit to the
    entry."""
    rays = np.asarray(rays, dtype=np.float32)
    out = np.zeros((seg_ray.shape[0], 8), dtype=np.float32)
    out[:, 0:3] = rays[seg_ray, 0:3]
    out[:, 3] = seg_t0
    out[:, 4:7] = rays[seg_ray, 4:7]
    out[:, 7] = seg_t1
    if seg_leaf is not None:
        inside = (np.asarray(seg_leaf, dtype=np.uint32) & INSIDE_TAG) != 0
        out[inside, 3] = -np.asarray(seg_t1, dtype=np.float32)[inside]
        out[inside, 4:7] = -out[inside, 4:7]
        out[inside, 7] = -np.asarray(seg_t0, dtype=np.float32)[inside]
    return out


# -- encoding and MLP ------------------------------------------------------------
def sample_positions(cfg, segs):
    segs = _c(segs, np.float32)
    x = np.zeros((segs.shape[0], cfg.n_samples, 3), dtype=np.float32)
    _lib().oc_sample_positions(ctypes.byref(cfg), _p(segs), segs.shape[0], _p(x))
    return x


def encode(cfg, table, segs):
    table = _c(table, np.float64)
    segs = _c(segs, np.float32)
    assert table.size >= n_table_params(cfg)
    u = np.zeros((segs.shape[0], n_in(cfg)), dtype=np.float64)
    _lib().oc_encode(ctypes.byref(cfg), _p(table), _p(segs), segs.shape[0], _p(u))
    return u


def mlp_forward(cfg, weights, u):
    W = _c(weights, np.float64)
    u = _c(u, np.float64)
    assert W.size == n_mlp_params(cfg) and u.shape[1] == n_in(cfg)
    z = np.zeros((u.shape[0], cfg.n_out), dtype=np.float64)
    _lib().oc_mlp_forward(ctypes.byref(cfg), _p(W), _p(u), u.shape[0], _p(z))
    return z


def forward(cfg, params, segs):
    """z = MLP(encode(segs)) with params = [table | weights]."""
    params = _c(params, np.float64)
    nt = n_table_params(cfg)
    return mlp_forward(cfg, params[nt:], encode(cfg, params[:nt], segs))


def min_abs_preact(cfg, params, segs):
    """Per segment, the smallest |pre-activation| of any hidden unit."""
    params = _c(params, np.float64)
    segs = _c(segs, np.float32)
    out = np.zeros(segs.shape[0], dtype=np.float64)
    _lib().oc_min_abs_preact(ctypes.byref(cfg), _p(params), _p(segs), segs.shape[0], _p(out))
    return out


def layer_amax(cfg, params, segs):
    """[H + 1]: max |u| over the encoded features, then the largest ReLU
    output of each hidden layer, over the batch."""
    params = _c(params, np.float64)
    segs = _c(segs, np.float32)
    out = np.zeros(cfg.mlp_hidden + 1, dtype=np.float64)
    _lib().oc_layer_amax(ctypes.byref(cfg), _p(params), _p(segs), segs.shape[0], _p(out))
    return out


# -- training ---------------------------------------------------------------------
LOSS_WEIGHTS = (2.0, 2.0, 1.0, 1.0)  # visibility, distance, normal, albedo


def loss(cfg, z, labels, weights=LOSS_WEIGHTS, with_grad=True):
    """Returns (terms [total, bce, dist, normal], dz or None)."""
    z = _c(z, np.float64)
    labels = _c(labels, np.float32)
    out = np.zeros(4, dtype=np.float64)
    dz = np.zeros_like(z) if with_grad else None
    w = tuple(weights) + (1.0,) * (4 - len(weights))
    _lib().oc_loss(ctypes.byref(cfg), _p(z), _p(labels), z.shape[0], float(w[0]), float(w[1]), float(w[2]),
                   float(w[3]), _p(out), _p(dz))
    return out, dz


def segment_loss(cfg, z, labels, weights=LOSS_WEIGHTS):
    """[n] combined loss of each segment (weights applied, no 1/B)."""
    z = _c(z, np.float64)
    labels = _c(labels, np.float32)
    out = np.zeros(z.shape[0], dtype=np.float64)
    w = tuple(weights) + (1.0,) * (4 - len(weights))
    _lib().oc_segment_loss(ctypes.byref(cfg), _p(z), _p(labels), z.shape[0], float(w[0]), float(w[1]),
                           float(w[2]), float(w[3]), _p(out))
    return out


def _first(rays, boxes, u, accept, reverse):
    off, sr, sl, t0, t1 = traverse(rays, boxes, reverse)
    off = off.astype(np.int64)
    has = off[1:] > off[:-1]
    first = off[:-1][has]  # runs are sorted by (t0, leaf): the first entry is the first leaf
    ray = np.nonzero(has)[0]
    tag = sl[first]
    leaf = (tag & ~np.uint32(INSIDE_TAG)).astype(np.int64)
    keep = np.asarray(u, dtype=np.float32)[ray] < np.asarray(accept, dtype=np.float32)[leaf]
    hits = np.bincount((sl & ~np.uint32(INSIDE_TAG)).astype(np.int64), minlength=boxes.shape[0])
    return ray[keep], leaf[keep], tag[keep], t0[first][keep], t1[first][keep], hits


def first_hits(rays, boxes, u, accept, reverse=False):
    """Training-ray selection (Sec. 5.2, "Ray distribution"): for each ray its first crossed leaf
    (smallest t0, ties to the lower id, from the every-leaf traversal), kept
    iff u[r] < accept[leaf] in binary32. Returns (ray indices kept, their
    leaf, t0, t1) in ray order and the number of rays crossing each leaf.
    With reverse, a leaf around the origin reports its chord [entry, exit]."""
    ray, leaf, _, t0, t1, hits = _first(rays, boxes, u, accept, reverse)
    return ray, leaf, t0, t1, hits


def first_hit_probes(rays, boxes, u, accept, reverse=False):
    """The training segments of first_hits as probe rows (o, t0, d, t1), a
    leaf around the origin crossed backwards when reverse is set, and their
    leaf ids, in ray order."""
    ray, leaf, tag, t0, t1, _ = _first(rays, boxes, u, accept, reverse)
    return segment_rows(rays, ray, t0, t1, tag), leaf


def backward(cfg, params, segs, dz):
    params = _c(params, np.float64)
    segs = _c(segs, np.float32)
    dz = _c(dz, np.float64)
    grad = np.zeros(n_table_params(cfg) + n_mlp_params(cfg), dtype=np.float64)
    assert params.size == grad.size
    _lib().oc_backward(ctypes.byref(cfg), _p(params), _p(segs), segs.shape[0], _p(dz), _p(grad))
    return grad


def adam(params, grad, m, v, step, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8, inv_scale=1.0):
    """In-place dense Adam on float64 arrays."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    grad = _c(grad, np.float64)
    _lib().oc_adam(params.size, _p(params), _p(grad), _p(m), _p(v), int(step), lr, beta1, beta2, eps,
                   inv_scale)


def train_step(cfg, params, m, v, step, segs, labels, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8,
               weights=LOSS_WEIGHTS):
    """One full step: forward, loss, backward, Adam (in place). Returns loss terms."""
    z = forward(cfg, params, segs)
    terms, dz = loss(cfg, z, labels, weights)
    g = backward(cfg, params, segs, dz)
    adam(params, g, m, v, step, lr, beta1, beta2, eps)
    return terms


# -- construction ------------------------------------------------------------------
def node_rank(loss_sum, count, hits, n_rays):
    """Sec. 5.1 node error rank r = 2 log q + log p per leaf (-inf where the
    leaf saw no segment, no crossing or zero loss)."""
    loss_sum = _c(loss_sum, np.float64)
    count = _c(count, np.int64)
    hits = _c(hits, np.int64)
    r = np.zeros(loss_sum.shape[0], dtype=np.float64)
    _lib().oc_node_rank(r.shape[0], _p(loss_sum), _p(count), _p(hits), int(n_rays), _p(r))
    return r


def acceptance(r, floor=0.005):
    """Sec. 5.2 per-leaf training-ray acceptance max(exp(r - r_max), floor)."""
    r = _c(r, np.float64)
    a = np.zeros_like(r)
    _lib().oc_acceptance(r.shape[0], _p(r), float(floor), _p(a))
    return a


# -- query -------------------------------------------------------------------------
def resolve(offsets, seg_leaf, seg_t0, seg_t1, z, n_out, ray_tmin=None):
    """Per ray [t, n.xyz, leaf, seg, albedo.rgb]; leaf = seg = -1 on a miss.
    ray_tmin [n] is needed when segments carry INSIDE_TAG (zeros otherwise)."""
    offsets = _c(offsets, np.uint64)
    z = _c(z, np.float64)
    n = offsets.shape[0] - 1
    tmin = _c(np.zeros(n) if ray_tmin is None else ray_tmin, np.float32)
    out = np.zeros((n, 9), dtype=np.float64)
    _lib().oc_resolve(n, _p(offsets), _p(_c(seg_leaf, np.uint32)), _p(_c(seg_t0, np.float32)),
                      _p(_c(seg_t1, np.float32)), _p(z), int(n_out), _p(tmin), _p(out))
    return out


def query(cfg, params, rays, boxes, reverse=False):
    """Full neural ray query: traversal, encode, MLP, resolve. Returns
    (hits [n][9], (offsets, seg_ray, seg_leaf, t0, t1), z). reverse: leaves
    around the ray origin are queried backwards along their chord."""
    tr = traverse(rays, boxes, reverse)
    offsets, sr, sl, t0, t1 = tr
    segs = segment_rows(rays, sr, t0, t1, sl)
    z = forward(cfg, params, segs) if segs.shape[0] else np.zeros((0, cfg.n_out))
    tmin = np.asarray(rays, dtype=np.float32)[:, 3]
    return resolve(offsets, sl, t0, t1, z, cfg.n_out, tmin), tr, z
