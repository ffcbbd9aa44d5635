"""The five seeded workloads (sizes, seeds, and builders for their inputs).

Network hyper-parameters follow the paper's setting (Sec. 6, "Neural model &
training": multiresolution hash grid, ReLU MLP, 2^18-ray batches, Adam at
learning rate 0.01) with the sizes of each workload below. Level resolutions
are N_l = floor(N_min * b^l), handed to both implementations as integers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import scene


@dataclass
class NetConfig:
    n_levels: int
    n_features: int
    log2_T: int
    n_samples: int
    n_min: int
    growth: float
    mlp_width: int
    mlp_hidden: int
    n_out: int
    level_res: list = field(default_factory=list)

    def __post_init__(self):
        if not self.level_res:
            self.level_res = [int(math.floor(self.n_min * self.growth ** l)) for l in range(self.n_levels)]

    @property
    def n_in(self) -> int:
        return self.n_samples * self.n_levels * self.n_features

    def level_sizes(self):
        """Entries per level: (N+1)^3 when that fits in T (dense), else T (hashed)."""
        T = 1 << self.log2_T
        return [(r + 1) ** 3 if (r + 1) ** 3 <= T else T for r in self.level_res]

    def level_dense(self):
        T = 1 << self.log2_T
        return [(r + 1) ** 3 <= T for r in self.level_res]

    @property
    def n_table_params(self) -> int:
        return sum(self.level_sizes()) * self.n_features

    def layer_dims(self):
        """(fan_in, fan_out) of each weight matrix, input layer first."""
        dims = [(self.n_in, self.mlp_width)]
        dims += [(self.mlp_width, self.mlp_width)] * (self.mlp_hidden - 1)
        dims += [(self.mlp_width, self.n_out)]
        return dims

    @property
    def n_mlp_params(self) -> int:
        return sum(a * b for a, b in self.layer_dims())

    @property
    def n_params(self) -> int:
        return self.n_table_params + self.n_mlp_params

    def as_dict(self):
        return dict(n_levels=self.n_levels, n_features=self.n_features, log2_T=self.log2_T,
                    n_samples=self.n_samples, level_res=list(self.level_res), mlp_width=self.mlp_width,
                    mlp_hidden=self.mlp_hidden, n_out=self.n_out)


C1_NET = NetConfig(8, 2, 14, 4, 16, 1.5, 64, 3, 5)
C2_NET = NetConfig(16, 2, 19, 8, 16, 1.38, 128, 4, 5)
C2_NET_S4 = NetConfig(16, 2, 19, 4, 16, 1.38, 128, 4, 5)
C5_NET = NetConfig(16, 4, 22, 4, 16, 1.38, 256, 4, 8)


def init_params(net: NetConfig, feature_init: str = "uniform", feature_scale: float = 1e-4,
                seed_features: int = scene.SEED_FEATURES, seed_mlp: int = scene.SEED_MLP) -> np.ndarray:
    """Flat float32 parameter vector: [hash table | W_0 | ... | W_H].

    Table: level-major, then entry, then feature. Features U(-s, s)
    ("uniform") or N(0, s^2) ("normal"). Each W_k is row-major
    [fan_out][fan_in], Xavier-uniform U(+-sqrt(6/(fan_in+fan_out)))."""
    rng = np.random.default_rng(seed_features)
    if feature_init == "uniform":
        table = rng.uniform(-feature_scale, feature_scale, size=net.n_table_params)
    elif feature_init == "normal":
        table = rng.normal(0.0, feature_scale, size=net.n_table_params)
    else:
        raise ValueError(feature_init)
    rng = np.random.default_rng(seed_mlp)
    ws = []
    for fi, fo in net.layer_dims():
        lim = math.sqrt(6.0 / (fi + fo))
        ws.append(rng.uniform(-lim, lim, size=fi * fo))
    return np.concatenate([table] + ws).astype(np.float32)


@dataclass
class Scene:
    verts: np.ndarray
    tris: np.ndarray
    boxes: np.ndarray
    tri_leaf: np.ndarray
    lo: np.ndarray
    side: np.float32
    mesh: scene.TriangleMesh | None = None

    @property
    def diagonal(self) -> float:
        return float(np.linalg.norm(self.verts.max(axis=0) - self.verts.min(axis=0)))


def make_scene(n_tris: int, n_leaves: int, seed: int = scene.SEED_MESH, amplitude: float = 0.1,
               offset=(0.0, 0.0, 0.0), albedo_seed: int | None = None, with_mesh: bool = True) -> Scene:
    n = scene.tessellation_for(n_tris)
    v, t = scene.icosphere(n)
    v = scene.displace(v, seed=seed, amplitude=amplitude) + np.asarray(offset, dtype=np.float64)
    boxes, tri_leaf = scene.median_split_leaves(v, t, n_leaves)
    lo, side = scene.scene_cube(boxes)
    albedo = None
    if albedo_seed is not None:
        albedo = np.random.default_rng(albedo_seed).uniform(0.0, 1.0, size=(v.shape[0], 3))
    mesh = scene.TriangleMesh(v, t, albedo) if with_mesh else None
    return Scene(v, t, boxes, tri_leaf, lo, side, mesh)


# workload sizes -------------------------------------------------------------
C1 = dict(n_tris=20_480, n_leaves=64, width=256, height=256, net=C1_NET,
          feature_init="uniform", feature_scale=1e-4)
C2 = dict(n_tris=1_003_520, n_leaves=1024, width=1920, height=1080, net=C2_NET,
          feature_init="normal", feature_scale=1e-2)
C3 = dict(C2, batch=1 << 18)
C5 = dict(n_tris=3_996_180, n_leaves=16384, n_rays=1 << 24, net=C5_NET,
          feature_init="normal", feature_scale=1e-2)


def c4_objects():
    """The batched scene: 8 displaced icospheres on a 4 x 2 grid (spacing 3),
    triangle counts log-spaced over 50,000..1,997,120, 256 * 2^floor(5k/7)
    leaves and T = 2^(16 + floor(4k/7)) hash entries for object k, seeds
    100 + k; network otherwise as in the 1920x1080 workload."""
    objs = []
    for k in range(8):
        n_tris = int(round(50_000 * (1_997_120 / 50_000) ** (k / 7)))
        leaves = 256 * 2 ** ((5 * k) // 7)
        log2_T = 16 + (4 * k) // 7
        offset = ((k % 4 - 1.5) * 3.0, (k // 4 - 0.5) * 3.0, 0.0)
        net = NetConfig(16, 2, log2_T, 8, 16, 1.38, 128, 4, 5)
        objs.append(dict(n_tris=n_tris, n_leaves=leaves, seed=100 + k, offset=offset, net=net))
    return objs


def c4_rays(boxes_all: np.ndarray, n_rays: int, seed: int = 107, lo: int = 1, hi: int = 32):
    """Rays from the scene's bounding sphere towards random points of the
    scene box, subsampled so the number of leaf boxes crossed follows a
    log-uniform mix over [lo, hi]."""
    blo = boxes_all[:, :3].min(0).astype(np.float64)
    bhi = boxes_all[:, 3:].max(0).astype(np.float64)
    c = 0.5 * (blo + bhi)
    r = 0.5 * float(np.linalg.norm(bhi - blo)) * 1.05
    cand = scene.sphere_rays(c, r, blo, bhi, 4 * n_rays, seed)
    counts = scene.box_crossings(boxes_all, cand)
    idx = scene.log_uniform_subsample(counts, lo, hi, n_rays, seed + 1)
    return cand[idx], counts[idx]
