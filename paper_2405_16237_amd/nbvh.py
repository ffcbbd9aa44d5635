"""Thin Python layer over libnbvh.so: torch tensors for device memory, the
current torch stream for ordering, ctypes for the calls. No compute here."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import check

PRECISIONS = {"fp32": _abi.NBVH_FP32, "bf16": _abi.NBVH_BF16, "fp8": _abi.NBVH_FP8}
INSIDE_RULES = {"clip": _abi.NBVH_INSIDE_CLIP, "reverse": _abi.NBVH_INSIDE_REVERSE}


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_config(net, scene_lo, scene_side, precision="bf16", loss_weights=(2.0, 2.0, 1.0, 1.0), lr=1e-2,
                beta1=0.9, beta2=0.99, eps=1e-8, loss_scale=1024.0, inside="clip") -> _abi.NbvhConfig:
    """net: object with n_levels, n_features, log2_T, n_samples, level_res,
    mlp_width, mlp_hidden, n_out. inside: "clip" or "reverse", how a leaf
    around the ray origin is queried (nbvh_inside_rule)."""
    c = _abi.NbvhConfig()
    c.n_levels, c.n_features, c.log2_T, c.n_samples = net.n_levels, net.n_features, net.log2_T, net.n_samples
    for i, r in enumerate(net.level_res):
        c.level_res[i] = int(r)
    c.mlp_width, c.mlp_hidden, c.n_out = net.mlp_width, net.mlp_hidden, net.n_out
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for a in range(3):
        c.scene_lo[a] = float(np.float32(scene_lo[a]))
    c.scene_side = float(np.float32(scene_side))
    c.w_hit, c.w_t, c.w_normal, c.w_albedo = loss_weights
    c.lr, c.beta1, c.beta2, c.eps, c.loss_scale = lr, beta1, beta2, eps, loss_scale
    c.inside_rule = INSIDE_RULES[inside] if isinstance(inside, str) else int(inside)
    return c


class NBVH:
    """An N-BVH with its network state on one GPU.

    leaf_boxes: [n][6] float32 (lo.xyz, hi.xyz) on the host.
    """

    def __init__(self, net, leaf_boxes, scene_lo, scene_side, precision="bf16", device="cuda", **kw):
        self.lib = _abi.load()
        self.net = net
        self.device = torch.device(device)
        self.cfg = make_config(net, scene_lo, scene_side, precision, **kw)
        self.precision = self.cfg.precision
        self.ctx, self.nodes, self.n_leaves = self._build(leaf_boxes)
        self._owner = None
        nt, nm = ctypes.c_uint64(), ctypes.c_uint64()
        check(self.lib.nbvh_param_count(ctypes.byref(self.cfg), ctypes.byref(nt), ctypes.byref(nm)))
        self.n_table, self.n_mlp = nt.value, nm.value
        offs = (ctypes.c_uint64 * (net.mlp_hidden + 3))()
        check(self.lib.nbvh_param_layout(ctypes.byref(self.cfg), offs))
        self.offsets = [int(o) for o in offs]
        self.n_params = self.offsets[-1]
        dev = self.device
        self.params = torch.zeros(self.n_params, dtype=torch.float32, device=dev)
        self.params_lp = torch.zeros(self.n_params, dtype=torch.bfloat16, device=dev)
        self.adam_m = torch.zeros_like(self.params)
        self.adam_v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.state = torch.zeros(self.lib.nbvh_state_bytes(), dtype=torch.uint8, device=dev)
        self.aux = torch.zeros((self.lib.nbvh_aux_bytes(ctypes.byref(self.cfg)) + 255) // 256 * 256,
                               dtype=torch.uint8, device=dev)
        p = _abi.NbvhParams(_ptr(self.params).value, _ptr(self.params_lp).value, _ptr(self.adam_m).value,
                            _ptr(self.adam_v).value, _ptr(self.grad).value, _ptr(self.state).value,
                            _ptr(self.aux).value)
        check(self.lib.nbvh_bind_params(self.ctx, ctypes.byref(p)))
        check(self.lib.nbvh_reset_optimizer(self.ctx, _stream()))
        self._p = p
        self._ws = None

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.nbvh_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- parameters ---------------------------------------------------------------
    def layer_dims(self):
        n_in = self.net.n_samples * self.net.n_levels * self.net.n_features
        w = self.net.mlp_width
        return [(n_in, w)] + [(w, w)] * (self.net.mlp_hidden - 1) + [(w, self.net.n_out)]

    def set_params(self, flat):
        """flat: unpadded [table | W_0 | ... | W_H] (float32), as nbvh_synth.init_params."""
        flat = torch.as_tensor(np.asarray(flat, dtype=np.float32))
        dev = torch.zeros(self.n_params, dtype=torch.float32)
        dev[: self.n_table] = flat[: self.n_table]
        src = self.n_table
        for k, (fi, fo) in enumerate(self.layer_dims()):
            dst = self.offsets[1 + k]
            dev[dst:dst + fi * fo] = flat[src:src + fi * fo]
            src += fi * fo
        assert src == flat.numel(), (src, flat.numel())
        with torch.no_grad():
            self.params.copy_(dev.to(self.device))
        check(self.lib.nbvh_reset_optimizer(self.ctx, _stream()))

    def get_params(self) -> np.ndarray:
        """Unpadded float32 copy of the master parameters."""
        return self.unpad(self.params)

    def unpad(self, t: torch.Tensor) -> np.ndarray:
        h = t.detach().float().cpu().numpy()
        parts = [h[: self.n_table]]
        for k, (fi, fo) in enumerate(self.layer_dims()):
            o = self.offsets[1 + k]
            parts.append(h[o:o + fi * fo])
        return np.concatenate(parts)

    def sync_shadow(self):
        check(self.lib.nbvh_sync_shadow(self.ctx, _stream()))

    def reset_optimizer(self):
        check(self.lib.nbvh_reset_optimizer(self.ctx, _stream()))

    def calibrate_fp8(self, probes: torch.Tensor):
        """FP8 contexts: per-layer weight and activation scales from the
        calibration segments probes [n][8] float32, then E4M3 weights.
        Needed again after every parameter change."""
        assert probes.is_cuda and probes.dtype == torch.float32 and probes.is_contiguous()
        check(self.lib.nbvh_calibrate_fp8(self.ctx, _ptr(probes), probes.shape[0], _stream()))

    def fp8_scales(self) -> dict:
        """Weight scales sw[k] and activation scales sa[k] (k = 0..mlp_hidden)
        written by the last calibration."""
        n = self.net.mlp_hidden + 1
        off = self.lib.nbvh_aux_bytes(ctypes.byref(self.cfg)) - 4 * 4 * 9
        f = self.aux[off:off + 4 * 4 * 9].view(torch.float32).cpu().numpy()
        return dict(sw=f[:n].copy(), sa=f[9:9 + n].copy(), amax_w=f[18:18 + n].copy(), amax_a=f[27:27 + n].copy())

    # -- workspace ------------------------------------------------------------------
    def workspace(self, max_rays=0, max_segments=0, max_batch=0) -> torch.Tensor:
        need = self.lib.nbvh_workspace_bytes(self.ctx, max_rays, max_segments, max_batch)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def rebuild(self, leaf_boxes):
        """Build the N-BVH over new leaf boxes (for instance a longer cut of a
        base BVH), keeping the network parameters, optimiser moments, device
        state and launch knobs. The hash-grid domain (scene_lo, scene_side)
        is unchanged, so the boxes must stay inside it."""
        tuning = self.get_tuning()
        ctx, nodes, n_leaves = self._build(leaf_boxes)
        check(self.lib.nbvh_bind_params(ctx, ctypes.byref(self._p)))
        old, self.ctx = self.ctx, ctx
        self.lib.nbvh_destroy(old)
        self.nodes, self.n_leaves = nodes, n_leaves
        self.set_tuning(**tuning)

    def view(self, leaf_boxes) -> "NBVH":
        """Another N-BVH over `leaf_boxes` bound to this one's buffers: the
        same hash grid, MLP, optimiser moments, gradient and device state
        (step count, loss scale, flags). This is how several tree cuts share
        one network (levels of detail, Sec. 5.3): a training step through any
        view updates the one set of parameters. Launch knobs are copied. The
        view keeps this object alive. FP8 models have no views: whether their
        E4M3 weights match the parameters is tracked per tree, so a change
        made through one tree could leave another's stale; build an FP8 model
        per tree from the trained parameters instead."""
        if self.cfg.precision == _abi.NBVH_FP8:
            raise ValueError("FP8 models have no views; build one FP8 model per tree from the trained parameters")
        v = NBVH.__new__(NBVH)
        v.lib, v.net, v.device, v.cfg, v.precision = self.lib, self.net, self.device, self.cfg, self.precision
        v.n_table, v.n_mlp, v.offsets, v.n_params = self.n_table, self.n_mlp, self.offsets, self.n_params
        v.params, v.params_lp, v.adam_m, v.adam_v = self.params, self.params_lp, self.adam_m, self.adam_v
        v.grad, v.state, v.aux, v._p = self.grad, self.state, self.aux, self._p
        v._owner = self
        v._ws = None
        v.ctx, v.nodes, v.n_leaves = v._build(leaf_boxes)
        check(v.lib.nbvh_bind_params(v.ctx, ctypes.byref(v._p)))
        v.set_tuning(**self.get_tuning())
        return v

    def _build(self, leaf_boxes):
        """(ctx, nodes, n_leaves) of a fresh N-BVH over leaf_boxes [n][6]."""
        lb = np.ascontiguousarray(leaf_boxes, dtype=np.float32)
        nb = self.lib.nbvh_nodes_bytes(lb.shape[0])
        nodes = torch.empty(nb, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        check(self.lib.nbvh_build(ctypes.byref(self.cfg), lb.ctypes.data_as(ctypes.c_void_p), lb.shape[0],
                                  _ptr(nodes), nb, _stream(), ctypes.byref(ctx)))
        return ctx, nodes, lb.shape[0]

    def tree(self):
        """The node buffer nbvh_build wrote, as host arrays: child boxes
        [n_nodes][2][6] float32 (lo.xyz, hi.xyz) and child indices
        [n_nodes][2] int32 (>= 0 inner node, < 0 leaf ~c, 0x7fffffff none)."""
        raw = self.nodes.cpu().numpy()
        f = raw.view(np.float32).reshape(-1, 16)
        boxes = f[:, :12].reshape(-1, 2, 6).copy()
        children = raw.view(np.int32).reshape(-1, 16)[:, 12:14].copy()
        return boxes, children

    # -- calls --------------------------------------------------------------------
    def first_hits(self, rays: torch.Tensor, u: torch.Tensor, accept: torch.Tensor,
                   leaf_hits: torch.Tensor | None = None):
        """Training-ray selection: (probes [k][8], leaf ids [k] int32) of the
        first leaf each ray crosses, kept where u < accept[leaf]; leaf_hits
        ([n_leaves] int32, optional) counts every leaf crossing."""
        n = rays.shape[0]
        probes = torch.empty((max(n, 1), 8), dtype=torch.float32, device=self.device)
        leaf = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        check(self.lib.nbvh_first_hits(self.ctx, _ptr(rays), n, _ptr(u), _ptr(accept), _ptr(probes), _ptr(leaf),
                                       _ptr(cnt), _ptr(leaf_hits), _stream()))
        k = int(cnt.item())
        return probes[:k], leaf[:k]

    def group_by_leaf(self, probes: torch.Tensor, leaf_ids: torch.Tensor):
        """(probes, leaf ids) reordered by leaf id, stable within a leaf."""
        n = probes.shape[0]
        out = torch.empty_like(probes)
        ids = torch.empty_like(leaf_ids)
        ws = self.workspace(0, 0, n)
        check(self.lib.nbvh_group_by_leaf(self.ctx, _ptr(probes.contiguous()), _ptr(leaf_ids.contiguous()), n, _ptr(out),
                                          _ptr(ids), _ptr(ws), ws.numel(), _stream()))
        return out, ids

    def leaf_loss(self, probes: torch.Tensor, labels: torch.Tensor, leaf_ids: torch.Tensor,
                  leaf_loss: torch.Tensor, leaf_count: torch.Tensor):
        """Adds each segment's combined loss to leaf_loss[leaf] (float32) and
        one to leaf_count[leaf] (int32)."""
        n = probes.shape[0]
        ws = self.workspace(0, 0, n)
        check(self.lib.nbvh_leaf_loss(self.ctx, _ptr(probes), _ptr(labels), _ptr(leaf_ids), n, _ptr(leaf_loss),
                                      _ptr(leaf_count), _ptr(ws), ws.numel(), _stream()))

    def traverse(self, rays: torch.Tensor, seg_capacity: int):
        n = rays.shape[0]
        offsets = torch.empty(n + 1, dtype=torch.int32, device=self.device)
        segs = torch.empty((max(seg_capacity, 1), 4), dtype=torch.int32, device=self.device)
        ws = self.workspace(n, 0, 0)
        check(self.lib.nbvh_traverse(self.ctx, _ptr(rays), n, _ptr(offsets), _ptr(segs), seg_capacity, _ptr(ws),
                                     ws.numel(), _stream()))
        return offsets, segs

    def query(self, rays: torch.Tensor, seg_capacity: int | None = None, hits: torch.Tensor | None = None):
        """rays [n][8] float32 (device). Returns hits [n][8] float32 view:
        t, n.xyz, albedo.rgb, leaf (bits; 0xFFFFFFFF = miss)."""
        n = rays.shape[0]
        if seg_capacity is None:
            seg_capacity = 8 * n + 1024
        if hits is None:
            hits = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        ws = self.workspace(n, seg_capacity, 0)
        check(self.lib.nbvh_query(self.ctx, _ptr(rays), n, _ptr(hits), seg_capacity, _ptr(ws), ws.numel(),
                                  _stream()))
        return hits

    def query_traced(self, rays: torch.Tensor, seg_capacity: int | None = None, z=True, u=False):
        """query() through nbvh_query_traced: returns (hits, offsets [n+1]
        int32, segs [cap][4] int32, z [cap][n_out] or None, u [cap][n_in] or
        None); rows of z and u stay NaN for segments the query did not
        evaluate (early termination)."""
        n = rays.shape[0]
        if seg_capacity is None:
            seg_capacity = 8 * n + 1024
        hits = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        offsets = torch.empty(n + 1, dtype=torch.int32, device=self.device)
        segs = torch.empty((max(seg_capacity, 1), 4), dtype=torch.int32, device=self.device)
        zt = torch.full((max(seg_capacity, 1), self.net.n_out), float("nan"), device=self.device) if z else None
        ut = torch.full((max(seg_capacity, 1), self.net.n_in), float("nan"), device=self.device) if u else None
        tr = _abi.NbvhQueryTrace(_ptr(offsets).value, _ptr(segs).value, _ptr(zt).value if z else None,
                                 _ptr(ut).value if u else None)
        ws = self.workspace(n, seg_capacity, 0)
        check(self.lib.nbvh_query_traced(self.ctx, _ptr(rays), n, _ptr(hits), seg_capacity, _ptr(ws), ws.numel(),
                                         ctypes.byref(tr), _stream()))
        return hits, offsets, segs, zt, ut

    def encode(self, probes: torch.Tensor):
        n = probes.shape[0]
        u = torch.empty((n, self.net.n_samples * self.net.n_levels * self.net.n_features), dtype=torch.float32,
                        device=self.device)
        check(self.lib.nbvh_encode(self.ctx, _ptr(probes), n, _ptr(u), _stream()))
        return u

    def forward(self, probes: torch.Tensor):
        n = probes.shape[0]
        z = torch.empty((n, self.net.n_out), dtype=torch.float32, device=self.device)
        check(self.lib.nbvh_forward(self.ctx, _ptr(probes), n, _ptr(z), None, 0, _stream()))
        return z

    def backward(self, probes: torch.Tensor, dz: torch.Tensor):
        n = probes.shape[0]
        ws = self.workspace(0, 0, n)
        check(self.lib.nbvh_backward(self.ctx, _ptr(probes), n, _ptr(dz.contiguous()), _ptr(ws), ws.numel(),
                                     _stream()))

    def optimizer_step(self):
        check(self.lib.nbvh_optimizer_step(self.ctx, _stream()))

    def train_step(self, probes: torch.Tensor, labels: torch.Tensor, loss: torch.Tensor | None = None):
        n = probes.shape[0]
        ws = self.workspace(0, 0, n)
        if loss is None:
            loss = torch.empty(4, dtype=torch.float32, device=self.device)
        check(self.lib.nbvh_train_step(self.ctx, _ptr(probes), _ptr(labels), n, _ptr(loss), _ptr(ws), ws.numel(),
                                       _stream()))
        return loss

    def loss(self, z: torch.Tensor, labels: torch.Tensor, with_grad=True):
        n = z.shape[0]
        ws = self.workspace(0, 0, n)
        loss = torch.empty(4, dtype=torch.float32, device=self.device)
        dz = torch.empty_like(z) if with_grad else None
        check(self.lib.nbvh_loss(self.ctx, _ptr(z.contiguous()), _ptr(labels), n, _ptr(loss), _ptr(dz), _ptr(ws),
                                 ws.numel(), _stream()))
        return loss, dz

    def query_segments(self, rays: torch.Tensor, offsets: torch.Tensor, segs: torch.Tensor,
                       hits: torch.Tensor | None = None):
        """Evaluation + resolve over a segment queue from traverse()."""
        n = rays.shape[0]
        if hits is None:
            hits = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        ws = self.workspace(n, 0, 0)
        check(self.lib.nbvh_query_segments(self.ctx, _ptr(rays), n, _ptr(offsets), _ptr(segs), _ptr(hits), _ptr(ws),
                                           ws.numel(), _stream()))
        return hits

    def profile_begin(self):
        check(self.lib.nbvh_profile_begin(self.ctx))

    def profile_end(self) -> dict:
        """{group: (total ms, launches)} over the window."""
        p = _abi.NbvhProfile()
        check(self.lib.nbvh_profile_end(self.ctx, ctypes.byref(p)))
        return {name: (p.ms[i], p.calls[i]) for i, name in enumerate(_abi.KERNEL_GROUPS)}

    def get_tuning(self) -> dict:
        t = _abi.NbvhTuning()
        check(self.lib.nbvh_get_tuning(self.ctx, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in _abi.NbvhTuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = _abi.NbvhTuning(**cur)
        check(self.lib.nbvh_set_tuning(self.ctx, ctypes.byref(t)))
        self._ws = None  # the workspace size may depend on the knobs

    def read_state(self) -> dict:
        s = _abi.NbvhStateHost()
        check(self.lib.nbvh_read_state(self.ctx, ctypes.byref(s), _stream()))
        return dict(step=s.step, skipped=s.skipped, loss_scale=s.loss_scale, flags=s.flags,
                    last_loss=list(s.last_loss), last_n_segments=s.last_n_segments, n_evaluated=s.n_evaluated)

    def device_status(self) -> int:
        """The sticky NBVH_FLAG_* bits (synchronises)."""
        f = ctypes.c_uint32()
        check(self.lib.nbvh_device_status(self.ctx, ctypes.byref(f), _stream()))
        return f.value

    def param_bytes(self, which: int) -> int:
        return int(self.lib.nbvh_param_bytes(self.ctx, int(which)))

    def unscaled_grad(self, out: torch.Tensor | None = None, clear: bool = False) -> torch.Tensor:
        """grad / loss scale, computed on the device (out may be self.grad)."""
        if out is None:
            out = torch.empty_like(self.grad)
        check(self.lib.nbvh_unscaled_grad(self.ctx, _ptr(out), 1 if clear else 0, _stream()))
        return out

    def clear_flags(self):
        check(self.lib.nbvh_clear_flags(self.ctx, _stream()))


class NBVHBatch:
    """Several NBVH objects (same network shape) answered together."""

    def __init__(self, models):
        self.lib = _abi.load()
        self.models = list(models)
        n = len(self.models)
        self.device = self.models[0].device
        self.desc = torch.empty(self.lib.nbvh_batch_desc_bytes(n), dtype=torch.uint8, device=self.device)
        arr = (ctypes.c_void_p * n)(*[m.ctx.value for m in self.models])
        b = ctypes.c_void_p()
        check(self.lib.nbvh_batch_create(arr, n, _ptr(self.desc), self.desc.numel(), _stream(), ctypes.byref(b)))
        self.b = b
        self._ws = None

    def __del__(self):
        try:
            if getattr(self, "b", None):
                self.lib.nbvh_batch_destroy(self.b)
                self.b = None
        except Exception:
            pass

    def workspace(self, n_rays, seg_capacity):
        need = self.lib.nbvh_batch_workspace_bytes(self.b, n_rays, seg_capacity)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def query(self, rays: torch.Tensor, seg_capacity: int | None = None, hits: torch.Tensor | None = None):
        """Hits [n][8]; leaf word = (object << 24) | leaf (0xFFFFFFFF = miss)."""
        n = rays.shape[0]
        if seg_capacity is None:
            seg_capacity = 8 * n + 1024
        if hits is None:
            hits = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        ws = self.workspace(n, seg_capacity)
        check(self.lib.nbvh_batch_query(self.b, _ptr(rays), n, _ptr(hits), seg_capacity, _ptr(ws), ws.numel(),
                                        _stream()))
        return hits

    def train_step(self, probes, labels, losses=None, streams=None):
        """One optimiser step per object (batches probes[k], labels[k]).
        streams (optional, one torch stream per object, default priority):
        each object's step is enqueued on its own stream, forked from and
        joined back into the current stream, so the objects' kernels can run
        concurrently (and a HIP graph captured around the call holds them as
        parallel branches). The objects share no buffers."""
        if losses is None:
            losses = torch.empty((len(self.models), 4), dtype=torch.float32, device=self.device)
        if streams is None:
            for k, m in enumerate(self.models):
                m.train_step(probes[k], labels[k], losses[k])
            return losses
        assert len(streams) == len(self.models)
        cur = torch.cuda.current_stream()
        for k, m in enumerate(self.models):
            streams[k].wait_stream(cur)
            with torch.cuda.stream(streams[k]):
                m.train_step(probes[k], labels[k], losses[k])
        for st in streams:
            cur.wait_stream(st)
        return losses


def node_rank(leaf_loss: torch.Tensor, leaf_count: torch.Tensor, leaf_hits: torch.Tensor, n_rays: int) -> torch.Tensor:
    """Per-leaf node error rank 2 log q + log p on the device (nbvh_node_rank)."""
    lib = _abi.load()
    n = leaf_loss.shape[0]
    rank = torch.empty(n, dtype=torch.float32, device=leaf_loss.device)
    check(lib.nbvh_node_rank(_ptr(leaf_loss.contiguous()), _ptr(leaf_count.contiguous()), _ptr(leaf_hits.contiguous()),
                             n, int(n_rays), _ptr(rank), _stream()))
    return rank


def acceptance(rank: torch.Tensor, min_accept: float) -> torch.Tensor:
    """Per-leaf training-ray acceptance max(exp(r - r_max), min_accept) on the
    device (nbvh_acceptance)."""
    lib = _abi.load()
    rank = rank.contiguous().float()
    out = torch.empty_like(rank)
    check(lib.nbvh_acceptance(_ptr(rank), rank.shape[0], float(min_accept), _ptr(out), _stream()))
    return out


def hits_leaf(hits: torch.Tensor) -> torch.Tensor:
    """Leaf ids of hit records (int64; -1 for a miss)."""
    leaf = hits[:, 7].contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    return torch.where(leaf == _abi.NBVH_MISS, torch.full_like(leaf, -1), leaf)
