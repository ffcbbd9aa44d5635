"""Seeded procedural scenes that stand in for the paper's assets.

Everything here is input preparation on the host: meshes, neural-leaf boxes,
camera rays, probe segments and their classical ground truth. None of it is the
neural ray query itself (no N-BVH traversal, no hash encoding, no MLP); both the
GPU library and the FP64 oracle consume these arrays unchanged.

Shapes follow the paper's workloads: 2^18-probe training batches (Sec. 6,
"Neural model & training"), hash maps of 2^14..2^22 entries, and hundreds to
tens of thousands of neural leaves.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_LIB_LOCK = threading.Lock()

SEED_MESH, SEED_LEAVES, SEED_MLP, SEED_FEATURES, SEED_PROBES = 1, 2, 3, 4, 5
SEED_ALBEDO, SEED_SECONDARY = 6, 7


# --------------------------------------------------------------------------
# native helper (closest-hit labels)
# --------------------------------------------------------------------------
def build_native(force: bool = False) -> str:
    """Compile labels.c into _labels.so next to it (gcc, OpenMP)."""
    src = os.path.join(_HERE, "labels.c")
    out = os.path.join(_HERE, "_labels.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _lib():
    global _LIB
    with _LIB_LOCK:
        if _LIB is None:
            path = os.path.join(_HERE, "_labels.so")
            if not os.path.exists(path):
                build_native()
            lib = ctypes.CDLL(path)
            P = ctypes.c_void_p
            I = ctypes.c_int64
            lib.tb_build.restype = P
            lib.tb_build.argtypes = [P, I, P, I]
            lib.tb_free.argtypes = [P]
            lib.tb_closest.argtypes = [P, P, P, P, P, I, P, P, P, P]
            lib.tb_closest_brute.argtypes = [P, P, I, P, P, P, P, I, P, P, P, P]
            lib.bx_count.argtypes = [P, I, P, P, I, P]
            _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# mesh
# --------------------------------------------------------------------------
def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # faces: vertex triples that are mutual nearest neighbours
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    edge = d[d > 1e-9].min()
    adj = np.abs(d - edge) < 1e-6
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    f = [i, j, k]
                    n = np.cross(v[j] - v[i], v[k] - v[i])
                    if np.dot(n, v[i] + v[j] + v[k]) < 0:
                        f = [i, k, j]
                    faces.append(f)
    assert len(faces) == 20
    return v, np.array(faces, dtype=np.int64)


def icosphere(n: int):
    """Geodesic frequency-n sphere: 10 n^2 + 2 unit vertices, 20 n^2 outward triangles.

    Shared edge and corner points are generated from a canonical (sorted
    corner id) barycentric combination so that neighbouring faces reference
    bit-identical vertices (a watertight indexed mesh).
    """
    V, F = _icosahedron()
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    keep = ii + jj <= n
    ii, jj = ii[keep], jj[keep]
    kk = n - ii - jj
    npf = ii.size  # points per face
    lut = -np.ones((n + 2, n + 2), dtype=np.int64)
    lut[ii, jj] = np.arange(npf)
    # local triangle grid, identical for every face
    ti, tj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m_up = ti + tj <= n - 1
    m_dn = ti + tj <= n - 2
    up = np.stack([lut[ti, tj], lut[ti + 1, tj], lut[ti, tj + 1]], axis=-1)[m_up]
    dn = np.stack([lut[ti + 1, tj], lut[ti + 1, tj + 1], lut[ti, tj + 1]], axis=-1)[m_dn]
    local = np.concatenate([up, dn], 0)
    keys = []
    pos = []
    w = np.stack([ii, jj, kk], axis=1)  # weights of corners F[f][0], F[f][1], F[f][2]
    for f in range(20):
        ids = F[f]
        order = np.argsort(ids)
        ids_s = ids[order]
        w_s = w[:, order]
        # canonical key: nonzero (corner id, weight) pairs sorted by id
        code = np.where(w_s > 0, ids_s[None, :] * 1024 + w_s, 15 * 1024)
        code = np.sort(code, axis=1)
        keys.append(code[:, 0] | (code[:, 1] << 14) | (code[:, 2] << 28))
        p = np.zeros((npf, 3), dtype=np.float64)
        for c in range(3):
            p = p + (w_s[:, c:c + 1] / float(n)) * V[ids_s[c]][None, :]
        pos.append(p)
    keys = np.concatenate(keys, 0)
    pos = np.concatenate(pos, 0)
    uniq, first, inv = np.unique(keys, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    verts = pos[first]
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    tris = np.concatenate([inv[local + f * npf] for f in range(20)], 0)
    # orientation: the local grid keeps the corner order of the outward face,
    # but check and flip per triangle to be safe
    e1 = verts[tris[:, 1]] - verts[tris[:, 0]]
    e2 = verts[tris[:, 2]] - verts[tris[:, 0]]
    cen = verts[tris].mean(axis=1)
    flip = np.einsum("ij,ij->i", np.cross(e1, e2), cen) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    assert tris.shape[0] == 20 * n * n and verts.shape[0] == 10 * n * n + 2
    return verts, tris.astype(np.int32)


def displace(verts: np.ndarray, seed: int = SEED_MESH, amplitude: float = 0.1, n_waves: int = 8):
    """Radial displacement r(u) = 1 + (A/K) sum_k sin(f_k <w_k, u> + phi_k)."""
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(n_waves, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    f = rng.uniform(2.0, 12.0, size=n_waves)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n_waves)
    u = verts / np.linalg.norm(verts, axis=1, keepdims=True)
    r = 1.0 + (amplitude / n_waves) * np.sin(u @ w.T * f[None, :] + ph[None, :]).sum(axis=1)
    return u * r[:, None]


def tessellation_for(n_tris: int) -> int:
    """Icosphere frequency whose 20 n^2 triangle count is nearest n_tris."""
    return max(1, int(round(math.sqrt(n_tris / 20.0))))


# --------------------------------------------------------------------------
# neural leaves: median split of triangle centroids
# --------------------------------------------------------------------------
def median_split_leaves(verts: np.ndarray, tris: np.ndarray, n_leaves: int, pad_rel: float = 1e-4):
    """Split triangle centroids at the median of the widest axis until
    n_leaves groups exist (rounds that split the largest groups first;
    each split orders by (coordinate, triangle id) and cuts at floor(n/2)). Returns (boxes [n][6]
    float32 as lo.xyz, hi.xyz, tri_leaf [n_tris] int32). Each box is the
    triangles' bound padded by pad_rel * scene diagonal per side, rounded
    outward to float32."""
    cen = verts[tris].mean(axis=1)
    groups = [np.arange(tris.shape[0], dtype=np.int64)]
    while len(groups) < n_leaves:
        # one round: split the largest groups (stable by position), as many as
        # still needed; for power-of-two counts every group splits each round
        order = sorted(range(len(groups)), key=lambda i: (-groups[i].size, i))
        todo = set(order[:n_leaves - len(groups)])
        nxt = []
        for i, g in enumerate(groups):
            if i not in todo or g.size < 2:
                nxt.append(g)
                continue
            c = cen[g]
            ax = int(np.argmax(c.max(axis=0) - c.min(axis=0)))
            g = g[np.lexsort((g, c[:, ax]))]
            h = g.size // 2
            nxt += [g[:h], g[h:]]
        if len(nxt) == len(groups):
            break
        groups = nxt
    vlo = verts.min(axis=0)
    vhi = verts.max(axis=0)
    diag = float(np.linalg.norm(vhi - vlo))
    pad = pad_rel * diag
    boxes = np.zeros((len(groups), 6), dtype=np.float32)
    tri_leaf = np.zeros(tris.shape[0], dtype=np.int32)
    for i, g in enumerate(groups):
        p = verts[tris[g]].reshape(-1, 3)
        lo = p.min(axis=0) - pad
        hi = p.max(axis=0) + pad
        lo32 = lo.astype(np.float32)
        hi32 = hi.astype(np.float32)
        lo32 = np.where(lo32.astype(np.float64) > lo, np.nextafter(lo32, np.float32(-np.inf)), lo32)
        hi32 = np.where(hi32.astype(np.float64) < hi, np.nextafter(hi32, np.float32(np.inf)), hi32)
        boxes[i, :3] = lo32
        boxes[i, 3:] = hi32
        tri_leaf[g] = i
    return boxes, tri_leaf


def _padded_box(verts, tris, g, pad):
    p = verts[tris[g]].reshape(-1, 3)
    lo = p.min(axis=0) - pad
    hi = p.max(axis=0) + pad
    lo32 = lo.astype(np.float32)
    hi32 = hi.astype(np.float32)
    lo32 = np.where(lo32.astype(np.float64) > lo, np.nextafter(lo32, np.float32(-np.inf)), lo32)
    hi32 = np.where(hi32.astype(np.float64) < hi, np.nextafter(hi32, np.float32(np.inf)), hi32)
    return lo32, hi32


def base_bvh(verts: np.ndarray, tris: np.ndarray, leaf_tris: int = 16, pad_rel: float = 1e-4):
    """The input geometry's own BVH (the "base BVH" a cut is taken from): the
    same median split as median_split_leaves (widest centroid axis, order by
    (coordinate, triangle id), cut at floor(n/2)), recursed until a node holds
    at most leaf_tris triangles. Node boxes are the triangles' bounds padded
    by pad_rel * scene diagonal and rounded outward to float32, so a child's
    box lies inside its parent's. Returns dict(lo [m][3], hi [m][3] float32,
    left, right [m] int32 (-1 at leaves), n_tris [m] int32); node 0 is the
    root, children follow their parent."""
    cen = verts[tris].mean(axis=1)
    diag = float(np.linalg.norm(verts.max(axis=0) - verts.min(axis=0)))
    pad = pad_rel * diag
    lo, hi, left, right, cnt = [], [], [], [], []

    def new_node(g):
        a, b = _padded_box(verts, tris, g, pad)
        lo.append(a)
        hi.append(b)
        left.append(-1)
        right.append(-1)
        cnt.append(g.size)
        return len(lo) - 1

    stack = [(new_node(np.arange(tris.shape[0], dtype=np.int64)), np.arange(tris.shape[0], dtype=np.int64))]
    while stack:
        node, g = stack.pop()
        if g.size <= leaf_tris:
            continue
        c = cen[g]
        ax = int(np.argmax(c.max(axis=0) - c.min(axis=0)))
        g = g[np.lexsort((g, c[:, ax]))]
        h = g.size // 2
        a, b = g[:h], g[h:]
        left[node] = new_node(a)
        right[node] = new_node(b)
        stack.append((right[node], b))
        stack.append((left[node], a))
    return dict(lo=np.array(lo, dtype=np.float32), hi=np.array(hi, dtype=np.float32),
                left=np.array(left, dtype=np.int32), right=np.array(right, dtype=np.int32),
                n_tris=np.array(cnt, dtype=np.int32))


def scene_cube(boxes: np.ndarray):
    """Normalisation cube: minimum corner of the leaf union and its largest extent (float32)."""
    lo = boxes[:, :3].min(axis=0).astype(np.float32)
    hi = boxes[:, 3:].max(axis=0).astype(np.float32)
    side = np.float32((hi - lo).max())
    return lo, side


# --------------------------------------------------------------------------
# rays
# --------------------------------------------------------------------------
def pinhole_rays(width: int, height: int, eye=(0.0, 0.0, 3.0), fov_deg: float = 45.0, target=(0.0, 0.0, 0.0)):
    """Camera at `eye` looking at `target`, up +y, vertical field of view
    fov_deg, one ray through each pixel centre. Returns [H*W][8] float32 rows
    (o.xyz, tmin, d.xyz, tmax) with tmin = 0 and tmax = +inf."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up0 = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up0)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(fov_deg) / 2.0)
    aspect = width / height
    px = (np.arange(width) + 0.5) / width * 2.0 - 1.0
    py = 1.0 - (np.arange(height) + 0.5) / height * 2.0
    X, Y = np.meshgrid(px * th * aspect, py * th)
    d = fwd[None, None, :] + X[..., None] * right[None, None, :] + Y[..., None] * up[None, None, :]
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    d = d.reshape(-1, 3)
    r = np.zeros((d.shape[0], 8), dtype=np.float32)
    r[:, 0:3] = eye.astype(np.float32)
    r[:, 3] = 0.0
    r[:, 4:7] = d.astype(np.float32)
    r[:, 7] = np.inf
    return r


def _unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def _clip_box64(o, d, lo, hi):
    """Double-precision entry/exit of rays with boxes (input preparation only)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        ta = (lo - o) * inv
        tb = (hi - o) * inv
    zero = d == 0.0
    inside = (o >= lo) & (o <= hi)
    ta = np.where(zero, np.where(inside, -np.inf, np.inf), ta)
    tb = np.where(zero, np.where(inside, np.inf, -np.inf), tb)
    tn = np.minimum(ta, tb).max(axis=1)
    tf = np.maximum(ta, tb).min(axis=1)
    return tn, tf


def leaf_probes(boxes: np.ndarray, per_leaf: int, seed: int = SEED_PROBES, radius_scale: float = 1.5,
                inside_fraction: float = 0.0):
    """BVH-driven probe segments: for each leaf, origins uniform on the sphere
    around the box centre with radius radius_scale * half-diagonal, directions
    uniform on S^2, kept when the ray crosses the box (rejection sampling).
    With inside_fraction > 0, that share of each leaf's probes (the last ones)
    instead starts at a point uniform inside the box, direction uniform on
    S^2, segment [0, exit] (rays that begin inside a leaf, as secondary rays
    leaving a surface do).
    Returns (probes [n_leaves*per_leaf][8] float32 as o.xyz, t0, d.xyz, t1;
    leaf ids [n] int32), leaf-major."""
    rng = np.random.default_rng(seed)
    nl = boxes.shape[0]
    lo = boxes[:, :3].astype(np.float64)
    hi = boxes[:, 3:].astype(np.float64)
    c = 0.5 * (lo + hi)
    R = radius_scale * 0.5 * np.linalg.norm(hi - lo, axis=1)
    out = np.zeros((nl, per_leaf, 8), dtype=np.float32)
    have = np.zeros(nl, dtype=np.int64)
    while True:
        need = np.nonzero(have < per_leaf)[0]
        if need.size == 0:
            break
        m = 8 * per_leaf
        leaf = np.repeat(need, m)
        o = c[leaf] + R[leaf, None] * _unit_vectors(rng, leaf.size)
        d = _unit_vectors(rng, leaf.size)
        tn, tf = _clip_box64(o, d, lo[leaf], hi[leaf])
        ok = (tf >= tn) & (tf > 0.0)
        tn = np.maximum(tn, 0.0)
        # candidates are grouped by leaf: rank accepted ones within their leaf
        acc = np.nonzero(ok)[0]
        la = leaf[acc]
        start = np.searchsorted(la, la, side="left")
        rank = np.arange(acc.size) - start + have[la]
        keep = rank < per_leaf
        s, la, rank = acc[keep], la[keep], rank[keep]
        row = out[la, rank]
        row[:, 0:3] = o[s]
        row[:, 3] = tn[s]
        row[:, 4:7] = d[s]
        row[:, 7] = tf[s]
        out[la, rank] = row
        np.add.at(have, la, 1)
    k = int(round(inside_fraction * per_leaf))
    if k > 0:
        rng2 = np.random.default_rng(seed + 1000)
        leaf = np.repeat(np.arange(nl), k)
        o = lo[leaf] + rng2.uniform(size=(leaf.size, 3)) * (hi - lo)[leaf]
        d = _unit_vectors(rng2, leaf.size)
        _, tf = _clip_box64(o, d, lo[leaf], hi[leaf])
        rows = np.zeros((leaf.size, 8), dtype=np.float32)
        rows[:, 0:3] = o
        rows[:, 4:7] = d
        rows[:, 7] = np.maximum(tf, 0.0)
        out[:, per_leaf - k:] = rows.reshape(nl, k, 8)
    leaf_ids = np.repeat(np.arange(nl, dtype=np.int32), per_leaf)
    return out.reshape(-1, 8), leaf_ids


def surface_probes(verts: np.ndarray, tris: np.ndarray, tri_leaf: np.ndarray, boxes: np.ndarray, per_leaf: int,
                   offset: float, seed: int = SEED_PROBES + 2000):
    """Probe segments that start on the surface inside their leaf, as bounce
    rays do: per leaf, points uniform on the leaf's triangles (area-weighted),
    origin moved `offset` along the triangle's winding-order normal,
    direction cosine-weighted about that normal, segment [0, exit of the
    leaf box]. Origins that the offset moves out of the box are drawn again.
    Returns [n_leaves * per_leaf][8] float32 probes, leaf-major."""
    rng = np.random.default_rng(seed)
    nl = boxes.shape[0]
    lo = boxes[:, :3].astype(np.float64)
    hi = boxes[:, 3:].astype(np.float64)
    v = verts.astype(np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / np.maximum(2.0 * area[:, None], 1e-300)
    order = np.argsort(tri_leaf, kind="stable")
    bounds = np.searchsorted(tri_leaf[order], np.arange(nl + 1))
    out = np.zeros((nl, per_leaf, 8), dtype=np.float32)
    for leaf in range(nl):
        ts = order[bounds[leaf]:bounds[leaf + 1]]
        cdf = np.cumsum(area[ts])
        got = 0
        while got < per_leaf:
            m = 2 * (per_leaf - got)
            t = ts[np.minimum(np.searchsorted(cdf, rng.uniform(0.0, cdf[-1], m)), ts.size - 1)]
            r1, r2 = np.sqrt(rng.uniform(size=m)), rng.uniform(size=m)
            p = (1 - r1)[:, None] * a[t] + (r1 * (1 - r2))[:, None] * b[t] + (r1 * r2)[:, None] * c[t]
            o = p + offset * nrm[t]
            d = cosine_bounces(np.zeros((m, 3)), nrm[t], m, seed=int(rng.integers(1 << 31)))[:, 4:7].astype(np.float64)
            inside = np.all((o >= lo[leaf]) & (o <= hi[leaf]), axis=1)
            _, tf = _clip_box64(o, d, np.broadcast_to(lo[leaf], o.shape), np.broadcast_to(hi[leaf], o.shape))
            ok = np.nonzero(inside & (tf > 0.0))[0][: per_leaf - got]
            rows = out[leaf, got:got + ok.size]
            rows[:, 0:3] = o[ok]
            rows[:, 4:7] = d[ok]
            rows[:, 7] = tf[ok]
            got += ok.size
    return out.reshape(-1, 8)


# --------------------------------------------------------------------------
# ground truth
# --------------------------------------------------------------------------
class TriangleMesh:
    """Indexed mesh with a triangle BVH for double-precision closest hits."""

    def __init__(self, verts: np.ndarray, tris: np.ndarray, albedo: np.ndarray | None = None):
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.albedo = albedo
        self._bvh = _lib().tb_build(_ptr(self.verts), self.verts.shape[0], _ptr(self.tris),
                                    self.tris.shape[0])

    def __del__(self):
        try:
            if self._bvh:
                _lib().tb_free(self._bvh)
                self._bvh = None
        except Exception:
            pass

    def closest(self, o, d, t0, t1, brute: bool = False):
        """Closest hit with t in [t0, t1]. Returns dict(hit, t, tri, u, v, n[, albedo])."""
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        t0 = np.ascontiguousarray(np.broadcast_to(t0, (o.shape[0],)), dtype=np.float64)
        t1 = np.ascontiguousarray(np.broadcast_to(t1, (o.shape[0],)), dtype=np.float64)
        n = o.shape[0]
        t = np.zeros(n)
        tri = np.zeros(n, dtype=np.int64)
        u = np.zeros(n)
        v = np.zeros(n)
        L = _lib()
        if brute:
            L.tb_closest_brute(_ptr(self.verts), _ptr(self.tris), self.tris.shape[0], _ptr(o), _ptr(d),
                               _ptr(t0), _ptr(t1), n, _ptr(t), _ptr(tri), _ptr(u), _ptr(v))
        else:
            L.tb_closest(self._bvh, _ptr(o), _ptr(d), _ptr(t0), _ptr(t1), n, _ptr(t), _ptr(tri),
                         _ptr(u), _ptr(v))
        hit = tri >= 0
        nrm = np.zeros((n, 3))
        if hit.any():
            tv = self.verts[self.tris[tri[hit]]]
            cr = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
            nrm[hit] = cr / np.linalg.norm(cr, axis=1, keepdims=True)
        res = dict(hit=hit, t=np.where(hit, t, 0.0), tri=tri, u=u, v=v, n=nrm)
        if self.albedo is not None:
            alb = np.zeros((n, 3))
            if hit.any():
                ti = self.tris[tri[hit]]
                a0, a1, a2 = (self.albedo[ti[:, k]] for k in range(3))
                uu, vv = u[hit, None], v[hit, None]
                alb[hit] = (1.0 - uu - vv) * a0 + uu * a1 + vv * a2
            res["albedo"] = alb
        return res


def probe_labels(mesh: TriangleMesh, probes: np.ndarray):
    """Labels for probe segments, computed from the float32 probe values:
    [n][8] float32 rows (tau, n.xyz, hit as 0/1, albedo.rgb), where tau is
    the closest hit's distance relative to the segment, (t - t0)/(t1 - t0)
    (0 when t1 == t0), and n the unit geometric normal in winding order."""
    p = probes.astype(np.float64)
    r = mesh.closest(p[:, 0:3], p[:, 4:7], p[:, 3], p[:, 7])
    lab = np.zeros((probes.shape[0], 8), dtype=np.float32)
    span = p[:, 7] - p[:, 3]
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = np.where(span > 0, (r["t"] - p[:, 3]) / np.where(span > 0, span, 1.0), 0.0)
    tau = np.where(r["hit"], np.clip(tau, 0.0, 1.0), 0.0)
    lab[:, 0] = tau
    lab[:, 1:4] = r["n"]
    lab[:, 4] = r["hit"].astype(np.float32)
    if "albedo" in r:
        lab[:, 5:8] = r["albedo"]
    return lab


def ray_ground_truth(mesh: TriangleMesh, rays: np.ndarray):
    """Closest hits of [n][8] rays within [tmin, tmax] (double precision)."""
    p = rays.astype(np.float64)
    return mesh.closest(p[:, 0:3], p[:, 4:7], p[:, 3], p[:, 7])


def cosine_bounces(points: np.ndarray, normals: np.ndarray, count: int, seed: int = SEED_SECONDARY,
                   offset: float = 0.0):
    """Secondary rays: cosine-weighted directions about each normal, origins
    offset along the normal; cycles through the hit points until `count`
    rays exist. Returns [count][8] float32 rays with tmin 0, tmax +inf."""
    rng = np.random.default_rng(seed)
    idx = np.arange(count) % points.shape[0]
    nrm = normals[idx]
    u1 = rng.uniform(size=count)
    u2 = rng.uniform(size=count)
    r = np.sqrt(u1)
    phi = 2.0 * math.pi * u2
    local = np.stack([r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1.0 - u1))], axis=1)
    a = np.where(np.abs(nrm[:, 0:1]) > 0.9, np.array([[0.0, 1.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    t1 = np.cross(nrm, a)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    d = local[:, 0:1] * t1 + local[:, 1:2] * t2 + local[:, 2:3] * nrm
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((count, 8), dtype=np.float32)
    rays[:, 0:3] = points[idx] + offset * nrm
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


def box_crossings(boxes: np.ndarray, rays: np.ndarray) -> np.ndarray:
    """Number of boxes each ray crosses for t >= 0 (double precision; used to
    shape ray sets, not by the neural query)."""
    b = np.ascontiguousarray(boxes, dtype=np.float64)
    o = np.ascontiguousarray(rays[:, 0:3], dtype=np.float64)
    d = np.ascontiguousarray(rays[:, 4:7], dtype=np.float64)
    out = np.zeros(rays.shape[0], dtype=np.int32)
    _lib().bx_count(_ptr(b), b.shape[0], _ptr(o), _ptr(d), o.shape[0], _ptr(out))
    return out


def sphere_rays(center, radius, box_lo, box_hi, n, seed):
    """Origins uniform on a sphere, each aimed at a uniform point of a box."""
    rng = np.random.default_rng(seed)
    o = np.asarray(center, np.float64)[None, :] + radius * _unit_vectors(rng, n)
    tgt = rng.uniform(np.asarray(box_lo, np.float64), np.asarray(box_hi, np.float64), size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n, 8), dtype=np.float32)
    rays[:, 0:3] = o
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


def log_uniform_subsample(counts: np.ndarray, lo: int, hi: int, n_out: int, seed: int) -> np.ndarray:
    """Indices of a subsample whose counts follow P(c) ~ log((c+1)/c) on
    [lo, hi] (log-uniform over the integers), as close as the supply allows."""
    rng = np.random.default_rng(seed)
    cs = np.arange(lo, hi + 1)
    p = np.log((cs + 1.0) / cs)
    p /= p.sum()
    want = np.floor(p * n_out).astype(np.int64)
    want[0] += n_out - want.sum()
    picked = []
    short = 0
    for c, w in zip(cs, want):
        pool = np.nonzero(counts == c)[0]
        take = min(w + short, pool.size)
        short = w + short - take
        picked.append(rng.choice(pool, size=take, replace=False) if take else pool[:0])
    idx = np.concatenate(picked)
    if idx.size < n_out:  # fill from the largest counts available
        rest = np.setdiff1d(np.nonzero((counts >= lo) & (counts <= hi))[0], idx)
        idx = np.concatenate([idx, rng.choice(rest, size=min(n_out - idx.size, rest.size), replace=False)])
    return np.sort(idx)
