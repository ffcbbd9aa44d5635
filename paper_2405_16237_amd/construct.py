"""Error-driven N-BVH construction (Sec. 5.1, "Error-driven construction").

The leaves of the N-BVH are a cut through the base BVH of the input geometry.
The cut starts at the root and grows: the network trains on the current
cut's leaves for a number of steps, then the leaves of largest error rank
r = 2 log q + log p (q: a leaf's mean training loss, p: the fraction of
sampled rays that cross it) are replaced by their two children. Steps and
splits per round grow by user factors until the target leaf count is
reached; a final, longer training round follows.

Training rays are drawn uniformly in the inflated root box with uniform
directions, and each trains only the first leaf it crosses, kept with a
probability that grows with that leaf's rank (Sec. 5.2, "Ray distribution").
The kept probes are grouped by leaf before each training step (a layout
choice: the step's result does not depend on the order beyond rounding).
The paper states it as max(r / r_max, 0.005); with r a sum of logarithms of
numbers below one, r and r_max are negative and that ratio inverts the
order, so the rank is used through exp(r - r_max) = q^2 p / (q^2 p)_max,
which is 1 for the leaf of largest error and monotone in r.

Levels of detail (Sec. 5.3): with lod_interval > 0 the current cut is
registered as a level of detail whenever that many training steps have run
since the last one; each level is an N-BVH view over its cut that shares the
one network. Every training step then picks one of the registered levels or
the current cut uniformly at random and trains on its nodes, each level with
the acceptance probabilities it had when registered.

The driver runs on the host; every per-ray and per-segment step (traversal,
first-hit selection, crossing counts, network, loss, per-leaf sums, ranks,
acceptance probabilities, training) is a library call; the host only orders
the leaves by rank to choose the splits. Labels come from the caller (classical
triangle intersection), as the paper's training data does.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from .nbvh import NBVH, acceptance, node_rank


@dataclass
class Schedule:
    target_leaves: int
    iters: int = 100            # training steps before the first expansion
    iters_growth: float = 1.5   # factor on the steps per round
    splits: int = 1             # leaves split at the first expansion
    splits_growth: float = 1.5  # factor on the splits per round
    final_iters: int = 1000     # the last, longer training round
    rays_per_step: int = 1 << 18  # candidate rays drawn per training step
    stats_rays: int = 1 << 18   # rays drawn to estimate q and p before an expansion
    min_accept: float = 0.005   # acceptance floor of the ray distribution
    inflate: float = 0.5        # the root box grows by this fraction of its extent for sampling
    lod_interval: int = 0       # training steps between registered levels of detail (0: none)


@dataclass
class Cut:
    """Base-BVH nodes whose boxes are the N-BVH leaves (leaf id = position)."""
    nodes: list = field(default_factory=list)

    def boxes(self, base) -> np.ndarray:
        idx = np.asarray(self.nodes, dtype=np.int64)
        return np.concatenate([base["lo"][idx], base["hi"][idx]], axis=1).astype(np.float32)


def choose_splits(cut: Cut, base, r: np.ndarray, k: int) -> list:
    """Positions in the cut of the k splittable leaves of largest rank (ties
    to the lower position)."""
    cand = [i for i, nd in enumerate(cut.nodes) if base["left"][nd] >= 0]
    cand.sort(key=lambda i: (-r[i] if np.isfinite(r[i]) else math.inf, i))
    return sorted(cand[:k])


def expand(cut: Cut, base, positions) -> Cut:
    """Replace the cut nodes at `positions` by their two children (the left
    child takes the parent's place, the right one is appended)."""
    nodes = list(cut.nodes)
    for i in positions:
        nd = nodes[i]
        nodes[i] = int(base["left"][nd])
        nodes.append(int(base["right"][nd]))
    return Cut(nodes)


class Sampler:
    """Uniform rays in the inflated root box (seeded torch generator on the
    device) and their acceptance uniforms."""

    def __init__(self, base, inflate: float, seed: int, device="cuda"):
        lo = base["lo"][0].astype(np.float64)
        hi = base["hi"][0].astype(np.float64)
        ext = hi - lo
        self.lo = torch.tensor(lo - 0.5 * inflate * ext, dtype=torch.float32, device=device)
        self.ext = torch.tensor((1.0 + inflate) * ext, dtype=torch.float32, device=device)
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(seed)
        self.device = device

    def rays(self, n: int):
        o = self.lo + torch.rand((n, 3), generator=self.gen, device=self.device) * self.ext
        d = torch.randn((n, 3), generator=self.gen, device=self.device)
        d = d / d.norm(dim=1, keepdim=True).clamp_min(1e-20)
        r = torch.zeros((n, 8), dtype=torch.float32, device=self.device)
        r[:, 0:3] = o
        r[:, 4:7] = d
        r[:, 7] = float("inf")
        u = torch.rand(n, generator=self.gen, device=self.device)
        return r, u


def construct(net, base, label_fn, schedule: Schedule, scene_lo, scene_side, params=None, precision="bf16",
              seed: int = 11, log=None, lods: list | None = None, **model_kw):
    """Grow a cut of `base` to schedule.target_leaves leaves while training
    the network; returns (model, cut, history). label_fn(probes [k][8]
    float32 numpy) -> labels [k][8] float32 numpy. If `lods` is a list, the
    levels of detail are appended to it as (Cut, NBVH) pairs from coarse to
    fine, the final cut and model last."""
    cut = Cut([0])
    model = NBVH(net, cut.boxes(base), scene_lo, scene_side, precision=precision, **model_kw)
    if params is not None:
        model.set_params(params)
    model.workspace(0, 0, schedule.rays_per_step)
    sampler = Sampler(base, schedule.inflate, seed, model.device)
    accept = torch.ones(1, dtype=torch.float32, device=model.device)
    history = []
    levels = []  # registered levels of detail: (Cut, view, acceptance)
    pick = np.random.default_rng(seed)
    done = [0, 0]  # training steps run, steps at the last registration

    def train(steps):
        losses = []
        for _ in range(steps):
            k = int(pick.integers(len(levels) + 1)) if levels else len(levels)
            tree, acc = (model, accept) if k == len(levels) else (levels[k][1], levels[k][2])
            rays, u = sampler.rays(schedule.rays_per_step)
            probes, leaf = tree.first_hits(rays, u, acc)
            done[0] += 1
            if probes.shape[0] == 0:
                continue
            probes, _ = tree.group_by_leaf(probes, leaf)  # a leaf's probes side by side
            lab = torch.from_numpy(label_fn(probes.cpu().numpy())).to(model.device)
            losses.append(tree.train_step(probes.contiguous(), lab))
        return float(torch.stack(losses)[:, 0].mean()) if losses else float("nan")

    def maybe_register():
        if schedule.lod_interval > 0 and done[0] - done[1] >= schedule.lod_interval:
            done[1] = done[0]
            if not levels or levels[-1][0].nodes != cut.nodes:
                levels.append((Cut(list(cut.nodes)), model.view(cut.boxes(base)), accept.clone()))
                if log:
                    log("level of detail %d: %d leaves" % (len(levels) - 1, len(cut.nodes)))

    def statistics():
        n_leaves = len(cut.nodes)
        hits = torch.zeros(n_leaves, dtype=torch.int32, device=model.device)
        rays, _ = sampler.rays(schedule.stats_rays)
        u0 = torch.zeros(schedule.stats_rays, dtype=torch.float32, device=model.device)  # keep every first hit
        probes, leaf = model.first_hits(rays, u0, torch.ones(n_leaves, device=model.device), leaf_hits=hits)
        loss = torch.zeros(n_leaves, dtype=torch.float32, device=model.device)
        count = torch.zeros(n_leaves, dtype=torch.int32, device=model.device)
        if probes.shape[0]:
            lab = torch.from_numpy(label_fn(probes.cpu().numpy())).to(model.device)
            model.leaf_loss(probes.contiguous(), lab, leaf.contiguous(), loss, count)
        return node_rank(loss, count, hits, schedule.stats_rays)

    iters, splits = float(schedule.iters), float(schedule.splits)
    while len(cut.nodes) < schedule.target_leaves:
        mean_loss = train(int(round(iters)))
        r_dev = statistics()
        accept = acceptance(r_dev, schedule.min_accept)
        r = r_dev.double().cpu().numpy()
        maybe_register()
        k = min(int(round(splits)), schedule.target_leaves - len(cut.nodes))
        pos = choose_splits(cut, base, r, k)
        history.append(dict(leaves=len(cut.nodes), steps=int(round(iters)), loss=mean_loss, split=len(pos)))
        if log:
            log("cut %d leaves, %d steps, mean loss %.4f, splitting %d" % (len(cut.nodes), int(round(iters)),
                                                                           mean_loss, len(pos)))
        if not pos:
            break  # nothing left to split
        cut = expand(cut, base, pos)
        model.rebuild(cut.boxes(base))
        # children start from their parent's rank until the next statistics:
        # the left child keeps the parent's position, the right one is appended
        new_r = torch.cat([r_dev, r_dev[torch.as_tensor(pos, dtype=torch.int64, device=model.device)]])
        accept = acceptance(new_r, schedule.min_accept)
        iters *= schedule.iters_growth
        splits *= schedule.splits_growth
    final = train(schedule.final_iters)
    history.append(dict(leaves=len(cut.nodes), steps=schedule.final_iters, loss=final, split=0))
    if log:
        log("final: %d leaves, %d steps, mean loss %.4f" % (len(cut.nodes), schedule.final_iters, final))
    if lods is not None:
        lods.extend((c, v) for c, v, _ in levels if c.nodes != cut.nodes)
        lods.append((cut, model))
    return model, cut, history
