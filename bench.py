#!/usr/bin/env python3
"""N-BVH neural ray query + training step benchmark on one MI355X.

Default workload ("frame"): 1920x1080 primary camera rays against a
1,003,520-triangle displaced icosphere clustered into 1,024 neural leaves;
hash grid L=16, F=2, T=2^19 (N_min 16, growth 1.38), 8 samples per segment,
MLP 256 -> 4x128 -> 5; training batches of 2^18 probe segments (256 per
leaf) labelled by Moller-Trumbore. The network is first trained (untimed) so
the hit decisions are meaningful; then each timed step is one full query of
the frame plus one training step, in BF16 (the primary path). The same
trained parameters are timed through the FP32 and FP8 paths, and each path's
hit error against the triangle ground truth is reported ("matched hit
error").

--workload secondary: 2^24 cosine-weighted bounce rays from the frame's
primary hits on a 3,996,180-triangle mesh with per-vertex albedo, 16,384
leaves, L=16 F=4 T=2^22, 4 samples, MLP 256 -> 4x256 -> 8.
--workload construct: the error-driven construction (Sec. 5.1) of a 1,024-leaf
cut of the frame mesh's base BVH, timed, with the host's label time apart.
--workload batched: 8 objects of 50,000 .. 1,997,120 triangles with their own
tables (T = 2^16 .. 2^20), 2^22 rays with a log-uniform mix of 1..32 crossed
leaves through one grouped query, and a HIP-graph-captured training step of
2^18 probes per object.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
METRIC = "neural ray queries/s + train segs/s, BF16-MFMA vs FP32, at matched hit error"
TRAFFIC_FILES = {"frame": "traffic_1920x1080_frame_2e18_batch.txt",
                 "secondary": "traffic_2e24_secondary_2e18_batch.txt"}
# kernels behind each library group, as rocprofv3 names them (BF16 instantiations)
TRAFFIC_KERNELS = {
    "query_eval": r"^nbvh::k_query_eval<(bool _Accum|__bf16)",
    "train_tile": r"^nbvh::k_train_tile<(bool _Accum|__bf16)",
    "scatter": r"^nbvh::k_scatter_(hash|lds|pairs)<",
    "scatter_sort": r"^nbvh::k_bin_(count|write)<",
    "scatter_reduce": r"^nbvh::k_bin_reduce<",
    "wgrad": r"k_wgrad",
    "optimizer": r"^nbvh::k_(adam|check_finite)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def hit_error(hits, gt, diag):
    """Hit agreement with the triangle ground truth and depth error over
    agreeing hits (relative to the scene diagonal)."""
    leaf = hits[:, 7].view(np.uint32)
    pred = leaf != 0xFFFFFFFF
    truth = gt["hit"]
    agree = float((pred == truth).mean())
    both = pred & truth
    dep = np.abs(hits[both, 0].astype(np.float64) - gt["t"][both]) / diag
    out = dict(hit_accuracy=agree, hit_error_pct=100.0 * (1.0 - agree),
               depth_err_mean=float(dep.mean()) if both.any() else None,
               depth_err_p99=float(np.quantile(dep, 0.99)) if both.any() else None,
               predicted_hits=int(pred.sum()), true_hits=int(truth.sum()))
    if "albedo" in gt and both.any():
        out["albedo_err_mean"] = float(np.abs(hits[both, 4:7].astype(np.float64) - gt["albedo"][both]).mean())
    return out


class Workload:
    """Inputs of one benchmark workload (all host arrays, seeded)."""
    inside_probes = None  # "surface": inside-starting training probes start on the surface
    tuning = {}  # launch knobs the caller of this workload sets (nbvh_tuning fields)


def parity(torch, m, rays_np, sc, net, params, precision, inside, what):
    """The library's query against the FP64 oracle on a subset of the
    workload's rays, through nbvh_query_traced (the kernels and launch shapes
    the timed query uses): hit-record agreement with the oracle's resolve,
    depth error over agreeing hits (scene diagonals), and the largest logit
    error |dz| / max(1, |z|) over the segments the GPU evaluated. BF16 is
    compared with the oracle run on the BF16-rounded parameters (quantisation
    of the parameters is the format's, not the kernels' error)."""
    import oracle
    rev = inside == "reverse"
    tr = oracle.traverse(rays_np, sc.boxes, rev)
    off, sr, sl, t0, t1 = tr
    n_seg = int(off[-1])
    hits, goff, _, zt, _ = m.query_traced(torch.from_numpy(rays_np).cuda(), n_seg + 64, z=True, u=False)
    torch.cuda.synchronize()
    hits = hits.cpu().numpy()
    zt = zt[:n_seg].cpu().numpy().astype(np.float64)
    same_queue = bool(np.array_equal(goff.cpu().numpy().astype(np.uint32).astype(np.uint64), off))
    pref = params
    if precision == "bf16":
        pref = torch.from_numpy(params).to(torch.bfloat16).float().numpy()
    cfg = oracle.make_cfg(net, sc.lo, sc.side)
    rows = oracle.segment_rows(rays_np, sr, t0, t1, sl)
    z = oracle.forward(cfg, pref.astype(np.float64), rows)
    out = oracle.resolve(off, sl, t0, t1, z, net.n_out, rays_np[:, 3])
    ev = ~np.isnan(zt[:, 0])
    dz = np.abs(zt[ev] - z[ev]) / np.maximum(1.0, np.abs(z[ev]))
    leaf = hits[:, 7].view(np.uint32).astype(np.int64)
    leaf[leaf == 0xFFFFFFFF] = -1
    oleaf = out[:, 4].astype(np.int64)
    both = (leaf >= 0) & (leaf == oleaf)
    dep = np.abs(hits[both, 0].astype(np.float64) - out[both, 0]) / sc.diagonal
    return dict(rays=int(rays_np.shape[0]), sample=what, segments=n_seg, segments_evaluated=int(ev.sum()),
                segment_queue_bitexact=same_queue, leaf_agreement=float((leaf == oleaf).mean()),
                depth_err_mean=float(dep.mean()) if both.any() else None,
                depth_err_p99=float(np.quantile(dep, 0.99)) if both.any() else None,
                max_dz_rel=float(dz.max()) if ev.any() else None,
                oracle_params="BF16-rounded" if precision == "bf16" else "FP32 master")


def node_visits(model, rays_np):
    """Mean nodes a ray's own walk visits (the root, then every inner child
    whose box the ray hits: one node load and two slab tests each), counted
    on the host from the node buffer the library built, with the slab test in
    binary32 as the kernels evaluate it."""
    boxes, children = model.tree()
    o = rays_np[:, 0:3].astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = (np.float32(1.0) / rays_np[:, 4:7]).astype(np.float32)
    neg = np.signbit(rays_np[:, 4:7])
    tmin, tmax = rays_np[:, 3].astype(np.float32), rays_np[:, 7].astype(np.float32)
    ray = np.arange(rays_np.shape[0])
    node = np.zeros_like(ray)
    visits = 0
    while ray.size:
        visits += ray.size
        nxt_r, nxt_n = [], []
        for k in range(2):
            c = children[node, k].astype(np.int64)
            b = boxes[node, k]
            with np.errstate(invalid="ignore"):
                ta = (b[:, 0:3] - o[ray]) * inv[ray]
                tb = (b[:, 3:6] - o[ray]) * inv[ray]
            near = np.where(neg[ray], tb, ta)
            far = np.where(neg[ray], ta, tb)
            tn = np.fmax(tmin[ray], np.fmax.reduce(near, axis=1))
            tf = np.fmin(tmax[ray], np.fmin.reduce(far, axis=1))
            enter = (tn <= tf) & (c >= 0) & (c != 0x7FFFFFFF)
            nxt_r.append(ray[enter])
            nxt_n.append(c[enter])
        ray, node = np.concatenate(nxt_r), np.concatenate(nxt_n)
    return visits / max(1, rays_np.shape[0])


def build_frame(configs, scene, samples=8):
    W = Workload()
    W.name = "frame"
    W.sc = configs.make_scene(1_003_520, 1024)
    W.rays = scene.pinhole_rays(1920, 1080)
    W.gt_idx = None
    W.gt = scene.ray_ground_truth(W.sc.mesh, W.rays)
    W.net = configs.C2_NET if samples == 8 else configs.C2_NET_S4
    W.params0 = configs.init_params(W.net, "normal", 1e-2)
    W.per_leaf = 256
    W.inside_fraction = 0.0
    W.inside = "clip"  # camera rays start outside every leaf
    W.seg_cap_per_ray = 16
    W.describe = ("1920x1080 primary rays on a 1,003,520-triangle displaced icosphere, 1,024 neural leaves; "
                  "hash grid L=16 F=2 T=2^19, %d samples/segment, MLP %d-4x128-5; train batch 2^18 probes"
                  % (samples, samples * 32))
    W.parity_stride = 4
    W.cpu_sample = lambda stride: (W.rays.reshape(1080, 1920, 8)[::stride, ::stride].reshape(-1, 8).copy(),
                                   ("every %dth row and column of the 1920x1080 frame" % stride) if stride > 1 else "the whole 1920x1080 frame")
    return W


def build_secondary(configs, scene, inside="reverse", offset=1e-4, bounce_from="network", inside_probes="surface"):
    W = Workload()
    W.name = "secondary"
    W.sc = configs.make_scene(3_996_180, 16384, albedo_seed=scene.SEED_ALBEDO)
    W.offset = offset * W.sc.diagonal
    W.primary = scene.pinhole_rays(1920, 1080)
    W.bounce_from = bounce_from
    if bounce_from == "mesh":
        g = scene.ray_ground_truth(W.sc.mesh, W.primary)
        hit = g["hit"]
        pts = W.primary[hit, 0:3].astype(np.float64) + g["t"][hit, None] * W.primary[hit, 4:7].astype(np.float64)
        set_bounces(W, scene, pts, g["n"][hit])
    else:
        W.rays = None  # spawned from the trained network's own primary hits (spawn_from_network)
    W.net = configs.C5_NET
    W.params0 = configs.init_params(W.net, "normal", 1e-2)
    W.per_leaf = 16
    W.inside = inside
    W.seg_cap_per_ray = 8
    W.inside_probes = None
    if inside == "reverse":
        # the leaf around each bounce origin is queried backwards along its
        # chord, so training needs only whole chords, as for camera rays
        W.inside_fraction = 0.0
        how = "leaves around the origin queried along the reversed chord; train batch 2^18 whole-chord probes"
    else:
        W.inside_fraction = 0.5  # half the probes start inside their leaf, as the bounce rays do
        if inside_probes == "surface":
            W.inside_probes = "surface"
            how = ("leaves around the origin queried from the origin on; train batch 2^18 probes, half of them "
                   "starting on the surface inside their leaf (offset along the normal, cosine-weighted directions)")
        else:
            how = ("leaves around the origin queried from the origin on; train batch 2^18 probes, half of them "
                   "starting uniformly inside their leaf")
    W.describe = ("2^24 cosine-weighted bounce rays from the 1920x1080 frame's primary hits (%s) on a "
                  "3,996,180-triangle displaced icosphere with per-vertex albedo, 16,384 neural leaves; hash grid "
                  "L=16 F=4 T=2^22, 4 samples/segment, MLP 256-4x256-8 (hit, t, normal, albedo); origins offset by "
                  "%g of the scene diagonal along the normal; "
                  % ("as the trained network predicts them" if bounce_from == "network" else "on the mesh", offset)
                  + how)
    W.parity_stride = 4  # every 256th bounce ray
    W.cpu_sample = lambda stride: (W.rays[::stride * stride * 16].copy(), "every %dth ray" % (stride * stride * 16))
    # the rays come in 24 passes over the primary hits (one bounce per hit and
    # pass): rays leaving one point are 690,000 places apart, so the caller asks
    # the library to evaluate them in the order of their origins
    W.tuning = {"query_order": 1}
    return W


def set_bounces(W, scene, points, normals):
    """2^24 cosine-weighted bounce rays about the given hit points and unit
    normals, and the triangle ground truth of every 16th."""
    W.rays = scene.cosine_bounces(points, normals, 1 << 24, seed=scene.SEED_SECONDARY, offset=W.offset)
    W.gt_idx = np.arange(0, W.rays.shape[0], 16)
    W.gt = scene.ray_ground_truth(W.sc.mesh, W.rays[W.gt_idx])


def self_distance_filter(hits_dev, W, sc):
    """Hit error of the bounce query when predicted hits closer to the ray
    origin than eps (a renderer's ray epsilon; fractions of the scene
    diagonal) are taken as misses. Host-side, on the ground-truth subset."""
    h = hits_dev.cpu().numpy()[W.gt_idx].copy()
    out = {}
    for eps in (1e-3, 3e-3, 1e-2):
        hh = h.copy()
        near = (hh[:, 7].view(np.uint32) != 0xFFFFFFFF) & (hh[:, 0] < eps * sc.diagonal)
        hh[near, 7] = np.uint32(0xFFFFFFFF).view(np.float32)
        e = hit_error(hh, W.gt, sc.diagonal)
        out["%g" % eps] = dict(hit_accuracy=e["hit_accuracy"], predicted_hits=e["predicted_hits"],
                               true_hits=e["true_hits"])
    return out


def spawn_from_network(W, scene, torch, model):
    """Bounce rays from the model's own primary hits, as a renderer spawns
    them: hit point o + t d, the predicted normal normalised and turned to
    face the incoming ray."""
    hits = model.query(torch.from_numpy(W.primary).cuda()).cpu().numpy()
    leaf = hits[:, 7].view(np.uint32)
    hit = leaf != 0xFFFFFFFF
    pr = W.primary[hit].astype(np.float64)
    pts = pr[:, 0:3] + hits[hit, 0:1].astype(np.float64) * pr[:, 4:7]
    n = hits[hit, 1:4].astype(np.float64)
    n /= np.maximum(np.linalg.norm(n, axis=1, keepdims=True), 1e-30)
    n = np.where((n * pr[:, 4:7]).sum(1, keepdims=True) > 0, -n, n)
    set_bounces(W, scene, pts, n)
    return int(hit.sum())


def training_probes(W, scene, seed):
    """One training batch of the workload: whole-chord probes per leaf, and
    for the clip rule on the bounce workload half of each leaf's probes
    starting on the surface inside the leaf."""
    sc = W.sc
    if W.inside_probes != "surface":
        pr, _ = scene.leaf_probes(sc.boxes, W.per_leaf, seed=seed, inside_fraction=W.inside_fraction)
        return pr
    k = int(round(W.inside_fraction * W.per_leaf))
    outer, _ = scene.leaf_probes(sc.boxes, W.per_leaf - k, seed=seed)
    surf = scene.surface_probes(sc.verts, sc.tris, sc.tri_leaf, sc.boxes, k, W.offset, seed=seed + 2000)
    nl = sc.boxes.shape[0]
    return np.concatenate([outer.reshape(nl, -1, 8), surf.reshape(nl, k, 8)], axis=1).reshape(-1, 8)


def timer(torch):
    def time_loop(fn, n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for i in range(n):
            fn(i)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n
    return time_loop


def copy_kernel(torch, mib):
    """Elementwise kernel reading and writing exactly mib MiB (the reference
    dispatch for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log("copy kernel: %d bytes read and %d written per dispatch" % (n * 4, n * 4))


def run_single(args, W, P, torch, configs, scene):
    t0 = time.time()
    sc, net = W.sc, W.net
    batches = []
    for i in range(args.batches):
        pr = training_probes(W, scene, scene.SEED_PROBES + i)
        lb = scene.probe_labels(sc.mesh, pr)
        batches.append((torch.from_numpy(pr).cuda(), torch.from_numpy(lb).cuda()))
    B = batches[0][0].shape[0]
    R = W.rays.shape[0] if W.rays is not None else 1 << 24
    seg_cap = W.seg_cap_per_ray * R
    log("data ready in %.1fs: %d rays, %d triangles, %d leaves, batch %d" %
        (time.time() - t0, R, sc.tris.shape[0], sc.boxes.shape[0], B))

    def accuracy(hits):
        h = hits.cpu().numpy()
        return hit_error(h if W.gt_idx is None else h[W.gt_idx], W.gt, sc.diagonal)

    bf = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1024.0, inside=W.inside)
    bf.set_params(W.params0)
    default_tuning = bf.get_tuning()
    bf.set_tuning(**W.tuning)
    bf.workspace(R, seg_cap, B)
    # levels of detail (Sec. 5.3): a coarser cut of the same median-split
    # hierarchy over the same network, trained on a randomly chosen cut per step
    coarse, coarse_batches, pick = None, [], None
    if args.lod > 0:
        cboxes, _ = scene.median_split_leaves(sc.verts, sc.tris, args.lod)
        coarse = bf.view(cboxes)
        coarse.workspace(R, seg_cap, B)
        for i in range(args.batches):
            pr, _ = scene.leaf_probes(cboxes, max(1, B // args.lod), seed=scene.SEED_PROBES + 50 + i,
                                      inside_fraction=W.inside_fraction)
            coarse_batches.append((torch.from_numpy(pr).cuda(),
                                   torch.from_numpy(scene.probe_labels(sc.mesh, pr)).cuda()))
        pick = np.random.default_rng(12)
    # pre-training (untimed): the trained network of the training workload
    t1 = time.time()
    loss = None
    for i in range(args.pretrain):
        if coarse is not None and pick.integers(2):
            loss = coarse.train_step(*coarse_batches[i % len(coarse_batches)])
            continue
        p, l = batches[i % len(batches)]
        loss = bf.train_step(p, l)
    torch.cuda.synchronize()
    log("pretrain %d steps in %.1fs, loss %s" % (args.pretrain, time.time() - t1,
                                                 None if loss is None else loss.cpu().numpy().round(4).tolist()))
    if W.rays is None:
        t2 = time.time()
        n_hit = spawn_from_network(W, scene, torch, bf)
        log("bounce rays spawned from %d network primary hits in %.1fs (true hit rate %.5f)" %
            (n_hit, time.time() - t2, float(W.gt["hit"].mean())))
    rays = torch.from_numpy(W.rays).cuda()
    hits_bf = torch.empty((R, 8), dtype=torch.float32, device="cuda")

    def run_steps(m, n):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for i in range(n):
            m.query(rays, seg_cap, hits_bf)
            m.train_step(*batches[i % len(batches)])
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    # BF16 primary path: timed steps, then query-only and train-only loops
    run_steps(bf, args.warmup)
    st0 = bf.read_state()
    total_ms = run_steps(bf, args.steps)
    st1 = bf.read_state()
    assert st1["flags"] & 1 == 0, "segment capacity exceeded"
    evaluated = (st1["n_evaluated"] - st0["n_evaluated"]) / max(1, args.steps)
    n_segments = st1["last_n_segments"]
    time_loop = timer(torch)
    q_ms = time_loop(lambda i: bf.query(rays, seg_cap, hits_bf), args.steps)
    t_ms = time_loop(lambda i: bf.train_step(*batches[i % len(batches)]), args.steps)
    q_ms_default = None
    if W.tuning:
        # the same query with the library's default knobs, for comparison
        bf.set_tuning(**{k: default_tuning[k] for k in W.tuning})
        bf.workspace(R, seg_cap, B)
        bf.query(rays, seg_cap, hits_bf)
        q_ms_default = time_loop(lambda i: bf.query(rays, seg_cap, hits_bf), args.steps)
        bf.set_tuning(**W.tuning)
        bf.workspace(R, seg_cap, B)
        bf.query(rays, seg_cap, hits_bf)
        log("query with the default knobs: %.3f ms (with %s: %.3f ms)" % (q_ms_default, W.tuning, q_ms))
    # per-kernel-group device time (HIP events on the launch stream)
    bf.profile_begin()
    run_steps(bf, args.steps)
    prof = bf.profile_end()
    bf.query(rays, seg_cap, hits_bf)
    torch.cuda.synchronize()
    acc_bf = accuracy(hits_bf)
    log("bf16: step %.3f ms (query %.3f, train %.3f), evaluated %.0f / %d segments, hit acc %.4f" %
        (total_ms / args.steps, q_ms, t_ms, evaluated, n_segments, acc_bf["hit_accuracy"]))
    log("profile:", {k: (round(v[0] / max(1, v[1]), 4), v[1]) for k, v in prof.items()})
    trained = bf.get_params()

    # FP32 path with the same trained parameters
    fp32 = None
    if not args.no_fp32:
        fp = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1024.0, inside=W.inside)
        fp.set_params(trained)
        fp.set_tuning(**W.tuning)
        fp.workspace(R, seg_cap, B)
        hits_fp = torch.empty((R, 8), dtype=torch.float32, device="cuda")
        fp.query(rays, seg_cap, hits_fp)
        torch.cuda.synchronize()
        acc_fp = accuracy(hits_fp)
        fq_ms = time_loop(lambda i: fp.query(rays, seg_cap, hits_fp), args.steps)
        ft_ms = time_loop(lambda i: fp.train_step(*batches[i % len(batches)]), args.steps)
        fp32 = dict(query_ms=fq_ms, train_ms=ft_ms, rays_per_s=R / (fq_ms * 1e-3), train_segs_per_s=B / (ft_ms * 1e-3),
                    accuracy=acc_fp)
        log("fp32: query %.3f ms, train %.3f ms, hit acc %.4f" % (fq_ms, ft_ms, acc_fp["hit_accuracy"]))
        del fp, hits_fp

    # FP8 inference option with the same trained parameters: per-layer scales
    # calibrated on 2^16 seeded probe segments
    fp8 = None
    if not args.no_fp8:
        f8 = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp8", inside=W.inside)
        f8.set_params(trained)
        f8.set_tuning(**W.tuning)
        f8.calibrate_fp8(batches[0][0][: 1 << 16].contiguous())
        f8.workspace(R, seg_cap, 0)
        hits_f8 = torch.empty((R, 8), dtype=torch.float32, device="cuda")
        f8.query(rays, seg_cap, hits_f8)
        torch.cuda.synchronize()
        acc_f8 = accuracy(hits_f8)
        f8_ms = time_loop(lambda i: f8.query(rays, seg_cap, hits_f8), args.steps)
        fp8 = dict(query_ms=f8_ms, rays_per_s=R / (f8_ms * 1e-3), accuracy=acc_f8,
                   calibration="2^16 probe segments of the first training batch")
        log("fp8: query %.3f ms, hit acc %.4f" % (f8_ms, acc_f8["hit_accuracy"]))
        del f8, hits_f8

    roofline = rooflines(prof, net, bf.get_tuning(), evaluated, B, R, n_segments, W.name)
    # traversal rate in node visits: visits per ray counted on the parity
    # sample, times the rays of the timed traversal
    tr = roofline["per_kernel"].get("traverse")
    if tr is not None:
        sub, what = W.cpu_sample(W.parity_stride)
        vpr = node_visits(bf, sub)
        tr["node_visits_per_ray"] = round(vpr, 3)
        tr["node_visits_per_s"] = round(vpr * R / (tr["avg_ms"] * 1e-3), 1)
        tr["node_visits_sample"] = what
        log("traversal: %.2f node visits per ray, %.3g visits/s" % (vpr, tr["node_visits_per_s"]))
    roofline["path"] = path_rooflines(net, evaluated, B, R, n_segments,
                                      tr["node_visits_per_ray"] if tr is not None else None, q_ms, t_ms)
    log("path rooflines:", roofline["path"])
    peaks = None
    if not args.no_peaks:
        from paper_2405_16237_amd import peaks as PK
        peaks = PK.measure(torch)
        log("measured ceilings:", {k: {a: round(b, 3) for a, b in v.items()} for k, v in peaks.items()})
        against_ceilings(roofline, peaks, net, evaluated, B, sc_table_bytes(net))

    # parity with the FP64 oracle on a subset of the same rays, trained parameters
    par = None
    if not args.no_parity:
        sub, what = W.cpu_sample(W.parity_stride)
        par = dict(bf16=parity(torch, bf, sub, sc, net, trained, "bf16", W.inside, what))
        log("parity bf16:", par["bf16"])
        if not args.no_fp32:
            fpp = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", inside=W.inside)
            fpp.set_params(trained)
            par["fp32"] = parity(torch, fpp, sub, sc, net, trained, "fp32", W.inside, what)
            log("parity fp32:", par["fp32"])
            del fpp

    lod = None
    if coarse is not None:
        hits_c = torch.empty((R, 8), dtype=torch.float32, device="cuda")
        c0 = coarse.read_state()
        coarse.query(rays, seg_cap, hits_c)
        torch.cuda.synchronize()
        c1 = coarse.read_state()
        acc_c = accuracy(hits_c)
        cq_ms = time_loop(lambda i: coarse.query(rays, seg_cap, hits_c), args.steps)
        lod = dict(coarse_leaves=args.lod, fine_leaves=int(sc.boxes.shape[0]), query_ms=cq_ms,
                   rays_per_s=R / (cq_ms * 1e-3), speedup_vs_fine=q_ms / cq_ms,
                   segments=int(c1["last_n_segments"]), segments_evaluated=int(c1["n_evaluated"] - c0["n_evaluated"]),
                   accuracy=acc_c)
        log("lod: %d leaves, query %.3f ms (%.2fx the %d-leaf cut), hit acc %.4f" %
            (args.lod, cq_ms, q_ms / cq_ms, sc.boxes.shape[0], acc_c["hit_accuracy"]))

    # CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cfg = oracle.make_cfg(net, sc.lo, sc.side)
        params = trained.astype(np.float64)
        stride = 16
        sample, what = W.cpu_sample(stride)
        t2 = time.time()
        oracle.query(cfg, params, sample, sc.boxes, W.inside == "reverse")
        dt = time.time() - t2
        # grow the sample towards the target time
        if dt < args.cpu_seconds / 2 and stride > 1:
            stride = max(1, int(stride / np.sqrt(args.cpu_seconds / max(dt, 1e-3))))
            sample, what = W.cpu_sample(stride)
            t2 = time.time()
            oracle.query(cfg, params, sample, sc.boxes, W.inside == "reverse")
            dt = time.time() - t2
        cpu = dict(value=sample.shape[0] / dt, unit="rays/s", cores=oracle.num_threads(), kind="oracle",
                   sample="%s (%d rays), full query in FP64 (every-leaf traversal, encode, MLP, resolve), %.1f s"
                          % (what, sample.shape[0], dt))
        log("cpu baseline:", cpu)

    return {
        "metric": METRIC,
        "value": R / (q_ms * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": W.describe + ("; the network is also trained on a %d-leaf cut of the same hierarchy, a "
                                      "random cut per step" % args.lod if args.lod else ""),
            "rays": R, "segments": int(n_segments), "segments_evaluated": int(evaluated), "train_batch": B,
            "step": "one full query + one training step (forward, loss, backward, Adam)",
            **({"tuning": W.tuning} if W.tuning else {}),
        },
        "query_ms": q_ms,
        **({"query_ms_default_knobs": q_ms_default} if q_ms_default is not None else {}),
        "train_ms": t_ms,
        "segments_per_s": evaluated / (q_ms * 1e-3),
        "train_segs_per_s": B / (t_ms * 1e-3),
        "accuracy": acc_bf,
        **({"always_miss_accuracy": float(1.0 - W.gt["hit"].mean()),
            "accuracy_ignoring_hits_closer_than": self_distance_filter(hits_bf, W, sc)} if W.name == "secondary"
           else {}),
        "fp32": fp32,
        "fp8": fp8,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": par,
        "ceilings": peaks,
        **({"lod": lod} if lod is not None else {}),
    }


def sc_table_bytes(net):
    """Bytes of the BF16 table shadow the kernels gather from."""
    return net.n_table_params * 2


def _table_class(nbytes):
    """The gather measurement whose table size is nearest above the table's:
    4 MiB (L2 of one die), 32 MiB (Infinity Cache) or 512 MiB (HBM)."""
    return 4 if nbytes <= (4 << 20) else 32 if nbytes <= (64 << 20) else 512


def against_ceilings(roofline, peaks, net, evaluated, B, table_bytes):
    """Adds to each per-kernel roofline the measured ceiling of the unit that
    bounds it and the fraction reached, and matrix-core throughput for the
    fused kernels:
      query_eval / train_tile: table gathers (entry = F x 2 B, one per lane, 8
        lines per wave: rays of a workgroup are neighbours) against the gather
        loop on a table of the same size class;
      scatter: FP32 adds against the LDS 64-bit integer atomic loop (the hash
        route sums a tile's gradients in LDS before its few global atomics);
      scatter_reduce, wgrad, optimizer, traverse: bytes against the streaming
        read of a 1 GiB (HBM) buffer;
      MLP FLOPs (2 per weight and segment forward; forward and input-gradient
        products in the training tile) against the BF16 16x16x32 loop and the
        data-sheet 2.5 PFLOP/s."""
    S, L, F = net.n_samples, net.n_levels, net.n_features
    eb = F * 2
    gkey = "gather_%dMiB_%dB_8lines" % (_table_class(table_bytes), eb)
    mlp = sum(fi * fo for fi, fo in net.layer_dims()) * 2.0
    mf = peaks["mfma_bf16_16x16x32"]["tflops"]
    hbm = peaks["stream_1024MiB"]["gbs"]
    per = roofline["per_kernel"]
    for k, r in per.items():
        if k in ("query_eval", "train_tile"):
            units = (evaluated if k == "query_eval" else B) * S * L * 8
            rate = units / (r["avg_ms"] * 1e-3) / 1e9
            r["ceiling"] = dict(name=gkey, glanes_per_s=round(peaks[gkey]["glanes_per_s"], 2))
            r["gathers_glanes_per_s"] = round(rate, 2)
            r["frac_ceiling"] = round(rate / peaks[gkey]["glanes_per_s"], 4)
            flops = (evaluated if k == "query_eval" else 2 * B) * mlp
            tf = flops / (r["avg_ms"] * 1e-3) / 1e12
            r["mlp"] = dict(tflops=round(tf, 2), frac_peak=round(tf / BF16_PEAK_TFLOPS, 4),
                            ceiling_tflops=round(mf, 1), frac_ceiling=round(tf / mf, 4))
        elif k == "scatter":
            # the hash route sums each tile's corner gradients with LDS integer
            # atomics before few global ones: priced against the LDS loop
            rate = r["algorithmic"] / 4 / (r["avg_ms"] * 1e-3) / 1e9
            c = peaks["lds_atomic_u64"]["gadds_per_s"]
            r["ceiling"] = dict(name="lds_atomic_u64", gadds_per_s=round(c, 2))
            r["frac_ceiling"] = round(rate / c, 4)
        elif r["unit"] == "GB/s":
            r["ceiling"] = dict(name="stream_1024MiB", gbs=round(hbm, 1))
            r["frac_ceiling"] = round(r["achieved"] / hbm, 4)
    dom = roofline["kernel"]
    for key in ("ceiling", "frac_ceiling", "gathers_glanes_per_s", "mlp"):
        if key in per.get(dom, {}):
            roofline[key] = per[dom][key]


def path_rooflines(net, evaluated, B, R, n_segments, visits_per_ray, q_ms, t_ms):
    """Lower bounds of the query and training paths at the data-sheet peaks:
    each stage takes at least its algorithmic bytes over HBM, its MLP FLOPs
    over the BF16 matrix cores and its scalar arithmetic over the FP32 vector
    units (whichever is longest); the stages run one after another, so a
    path's bound is the sum. Algorithmic work per stage:
      traversal: the rays, the segment queue written and read, the counts
        (bytes); 2 slab tests of about 24 operations per node visit (vector);
      evaluation: S*L*8 corners x F x 2 B per evaluated segment; 2 FLOPs per
        weight and evaluated segment;
      training tile: the same gathers and forward FLOPs per probe plus the
        input-gradient products (2x); weight gradient: 2 FLOPs per weight and
        probe; table gradient: one 4-byte read-modify-write per corner,
        feature and level (all levels); Adam: 34 B per parameter.
    `frac` = bound / measured time."""
    S, L, F = net.n_samples, net.n_levels, net.n_features
    mlp = sum(fi * fo for fi, fo in net.layer_dims()) * 2.0
    hbm, mf = HBM_PEAK_GBS * 1e9, BF16_PEAK_TFLOPS * 1e12
    valu_ops = FP32_PEAK_TFLOPS * 1e12 / 4.0  # one 32-bit operation per lane and cycle (the peak counts packed FMAs)

    def bound(nbytes=0.0, flops=0.0, ops=0.0):
        return max(nbytes / hbm, flops / mf, ops / valu_ops) * 1e3

    stages_q = {
        "traverse": bound(nbytes=R * 32 + n_segments * 16 * 2 + R * 12,
                          ops=(visits_per_ray or 0.0) * R * 2 * 24),
        "query_eval": bound(nbytes=evaluated * S * L * 8 * F * 2, flops=evaluated * mlp),
    }
    stages_t = {
        "train_tile": bound(nbytes=B * S * L * 8 * F * 2, flops=3 * B * mlp),
        "wgrad": bound(flops=B * mlp),
        "table_gradient": bound(nbytes=B * S * L * 8 * F * 4 * 2),
        "optimizer": bound(nbytes=(net.n_table_params + net.n_mlp_params) * 34),
    }
    q_bound, t_bound = sum(stages_q.values()), sum(stages_t.values())
    return {
        "query": {"bound_ms": round(q_bound, 4), "measured_ms": round(q_ms, 4), "frac": round(q_bound / q_ms, 4),
                  "stages_ms": {k: round(v, 4) for k, v in stages_q.items()}},
        "train": {"bound_ms": round(t_bound, 4), "measured_ms": round(t_ms, 4), "frac": round(t_bound / t_ms, 4),
                  "stages_ms": {k: round(v, 4) for k, v in stages_t.items()}},
    }


def rooflines(prof, net, tune, evaluated, B, R, n_segments, workload):
    """Per-group rooflines; the dominant group is the one with the most device
    time in the timed step. Algorithmic work per launch:
      query_eval / train_tile: table bytes gathered, S*L*8 corners x F x 2 B;
      scatter routes: one 4-byte read-modify-write per corner and feature of
        the levels each route handles;
      wgrad: the stored BF16 activations and gradients read once (the thin
        GEMMs over the batch stream them; 2 FLOPs per weight and probe are far
        below the matrix cores' rate) plus the split partials written and read;
      optimizer: 34 B per parameter;
      traverse: rays, two passes over the segment queue and the counts."""
    per = {k: (v[0] / max(1, v[1]), v[1], v[0]) for k, v in prof.items() if v[1] > 0}
    c = net
    S, L, F = c.n_samples, c.n_levels, c.n_features
    lds_levels = 0
    if tune["scatter_lds_kb"] > 0:
        acc = 0
        for l, (dense, size) in enumerate(zip(c.level_dense(), c.level_sizes())):
            if not dense or (acc + size * F) * 4 > tune["scatter_lds_kb"] * 1024:
                break
            acc += size * F
            lds_levels = l + 1
    hash_end = min(L, lds_levels + tune["scatter_hash_levels"])
    sorted_levels = L - hash_end if tune["scatter_binned"] else 0
    work = {
        "query_eval": ("hbm", evaluated * S * L * 8 * F * 2, "GB/s"),
        "train_tile": ("hbm", B * S * L * 8 * F * 2, "GB/s"),
        "scatter": ("hbm", B * S * (L - sorted_levels) * 8 * F * 4, "GB/s"),
        "scatter_sort": ("hbm", B * S * sorted_levels * 8 * F * 4, "GB/s"),
        "scatter_reduce": ("hbm", B * S * sorted_levels * 8 * F * 4, "GB/s"),
        "wgrad": ("hbm", B * 2 * sum(fi + (32 if k == len(c.layer_dims()) - 1 else fo)
                                     for k, (fi, fo) in enumerate(c.layer_dims()))
                  + 2 * tune["wgrad_splits"] * c.n_mlp_params * 4, "GB/s"),
        "optimizer": ("hbm", (c.n_table_params + c.n_mlp_params) * 34, "GB/s"),
        "traverse": ("hbm", R * 32 + n_segments * 16 * 2 + R * 12, "GB/s"),
    }

    def roof(group):
        bound, amount, unit = work[group]
        avg_ms = per[group][0]
        if unit == "GB/s":
            achieved, peak = amount / (avg_ms * 1e-3) / 1e9, HBM_PEAK_GBS
        else:
            achieved, peak = amount / (avg_ms * 1e-3) / 1e12, BF16_PEAK_TFLOPS
        return dict(bound=bound, kernel=group, achieved=round(achieved, 2), peak=peak, unit=unit,
                    frac=round(achieved / peak, 4), avg_ms=round(avg_ms, 4), algorithmic=amount)

    dom = max((k for k in per if k in work), key=lambda k: per[k][2])
    roofline = roof(dom)
    # memory traffic per launch from the committed rocprofv3 counter summary of
    # this workload, valid only for the kernel sources it was taken on
    from paper_2405_16237_amd import profiling
    roofline["traffic"] = None
    tr = profiling.read_traffic(os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(workload, "")))
    if tr is not None and tr.get("source_digest") == profiling.source_digest():
        pat = TRAFFIC_KERNELS.get(dom)
        found = [v for k, v in tr["kernels"].items() if pat and re.search(pat, k)]
        if found:
            roofline["traffic"] = sum(v["bytes"] for v in found)
    roofline["per_kernel"] = {k: roof(k) for k in per if k in work}
    return roofline


def run_batched(args, P, torch, configs, scene):
    t0 = time.time()
    objs = []
    for o in configs.c4_objects():
        sc = configs.make_scene(o["n_tris"], o["n_leaves"], seed=o["seed"], offset=o["offset"])
        objs.append((sc, o["net"]))
    boxes_all = np.concatenate([sc.boxes for sc, _ in objs])
    rays_np, counts = configs.c4_rays(boxes_all, 1 << 22)
    gt_idx = np.arange(0, rays_np.shape[0], 16)
    gts = [scene.ray_ground_truth(sc.mesh, rays_np[gt_idx]) for sc, _ in objs]
    gt_t = np.stack([np.where(g["hit"], g["t"], np.inf) for g in gts])
    gt = dict(hit=np.isfinite(gt_t.min(0)), t=gt_t.min(0))
    diag = float(np.linalg.norm(boxes_all[:, 3:].max(0) - boxes_all[:, :3].min(0)))
    batches = []
    for k, (sc, net) in enumerate(objs):
        pr, _ = scene.leaf_probes(sc.boxes, (1 << 18) // sc.boxes.shape[0], seed=scene.SEED_PROBES + 10 * k)
        batches.append((torch.from_numpy(pr).cuda(), torch.from_numpy(scene.probe_labels(sc.mesh, pr)).cuda()))
    rays = torch.from_numpy(rays_np).cuda()
    R = rays.shape[0]
    seg_cap = 8 * R  # per object
    log("data ready in %.1fs: %d rays (%.1f leaves crossed on average), %d objects" %
        (time.time() - t0, R, counts.mean(), len(objs)))
    models = []
    for k, (sc, net) in enumerate(objs):
        m = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1024.0)
        m.set_params(configs.init_params(net, "normal", 1e-2, seed_features=200 + k, seed_mlp=300 + k))
        m.workspace(0, 0, batches[k][0].shape[0])
        models.append(m)
    batch = P.NBVHBatch(models)
    # rays from a sphere around the scene towards random points of its box are
    # incoherent: the caller asks for them to be evaluated in the order of
    # their origins and directions (grouped queries take the first object's)
    tuning = {"query_order": 2}
    models[0].set_tuning(**tuning)
    hits = torch.empty((R, 8), dtype=torch.float32, device="cuda")
    for i in range(args.pretrain):
        for m, (p, l) in zip(models, batches):
            m.train_step(p, l)
    torch.cuda.synchronize()
    # the training step of all objects as one HIP graph: each object's step
    # is a branch of its own (its own stream during capture), so the
    # objects' kernels overlap
    losses = torch.zeros((len(models), 4), dtype=torch.float32, device="cuda")
    obj_streams = [torch.cuda.Stream() for _ in models]
    probes_k = [p for p, _ in batches]
    labels_k = [l for _, l in batches]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.train_step(probes_k, labels_k, losses, streams=None if args.serial_graph else obj_streams)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.train_step(probes_k, labels_k, losses, streams=None if args.serial_graph else obj_streams)
    time_loop = timer(torch)
    for _ in range(args.warmup):
        batch.query(rays, seg_cap, hits)
        g.replay()
    torch.cuda.synchronize()

    def step(i):
        batch.query(rays, seg_cap, hits)
        g.replay()
    step_ms = time_loop(step, args.steps)
    q_ms = time_loop(lambda i: batch.query(rays, seg_cap, hits), args.steps)
    t_ms = time_loop(lambda i: g.replay(), args.steps)
    # the same query in the caller's order, for comparison
    models[0].set_tuning(query_order=0)
    batch.query(rays, seg_cap, hits)
    q_ms_default = time_loop(lambda i: batch.query(rays, seg_cap, hits), args.steps)
    models[0].set_tuning(**tuning)
    batch.query(rays, seg_cap, hits)
    log("grouped query in the caller's order: %.3f ms (with %s: %.3f ms)" % (q_ms_default, tuning, q_ms))
    # per-kernel-group device time over eager steps (the grouped query is
    # recorded by the first object's context, each training step by its own)
    ev0 = [m.read_state()["n_evaluated"] for m in models]
    for m in models:
        m.profile_begin()
    for i in range(args.steps):
        batch.query(rays, seg_cap, hits)
        for k, m in enumerate(models):
            m.train_step(*batches[k], loss=losses[k])
    prof = {}
    for m in models:
        for key, (ms, calls) in m.profile_end().items():
            a = prof.get(key, (0.0, 0))
            prof[key] = (a[0] + ms, a[1] + calls)
    evaluated = sum(m.read_state()["n_evaluated"] - e for m, e in zip(models, ev0)) / max(1, args.steps)
    batch.query(rays, seg_cap, hits)
    torch.cuda.synchronize()
    assert all(m.read_state()["flags"] & 1 == 0 for m in models), "segment capacity exceeded"
    acc = hit_error(hits.cpu().numpy()[gt_idx], gt, diag)
    # grouped launches: one query_eval launch covers every object, the
    # training groups run once per object and step
    n_segments = sum(m.read_state()["last_n_segments"] for m in models)
    net0 = objs[0][1]
    nb_each = batches[0][0].shape[0]
    roofline = rooflines(prof, net0, models[0].get_tuning(), evaluated, nb_each, R, n_segments / len(models),
                         "batched")
    roofline["note"] = ("query_eval: one grouped launch per query over all objects; training groups: per object "
                        "(2^18 probes each), averaged over the objects")
    peaks = None
    if not args.no_peaks:
        from paper_2405_16237_amd import peaks as PK
        peaks = PK.measure(torch)
        against_ceilings(roofline, peaks, net0, evaluated, nb_each,
                         max(sc_table_bytes(net) for _, net in objs))
    # CPU baseline and parity: the oracle's grouped query (every object, the
    # closest hit over objects, ties to the lower object) on every 64th ray
    cpu, par = None, None
    if not (args.no_cpu_baseline and args.no_parity):
        import oracle
        sub_idx = np.arange(0, R, 64)
        sub = rays_np[sub_idx]
        trained = [m.get_params() for m in models]
        t2 = time.time()
        best_t = np.full(sub.shape[0], np.inf)
        best_code = np.full(sub.shape[0], -1, np.int64)
        for k, ((sc, net), prm) in enumerate(zip(objs, trained)):
            out, _, _ = oracle.query(oracle.make_cfg(net, sc.lo, sc.side), prm.astype(np.float64), sub, sc.boxes)
            better = (out[:, 4] >= 0) & (out[:, 0] < best_t)
            best_t[better] = out[better, 0]
            best_code[better] = (k << 24) | out[better, 4].astype(np.int64)
        dt = time.time() - t2
        if not args.no_cpu_baseline:
            cpu = dict(value=sub.shape[0] / dt, unit="rays/s", cores=oracle.num_threads(), kind="oracle",
                       sample="every 64th ray (%d rays) against all 8 objects, full query in FP64, FP32 master "
                              "parameters, %.1f s" % (sub.shape[0], dt))
        if not args.no_parity:
            word = hits.cpu().numpy()[sub_idx, 7].view(np.uint32)
            got = np.where(word == 0xFFFFFFFF, -1, word.astype(np.int64))
            same = (got == best_code) & (best_code >= 0)
            dep = np.abs(hits.cpu().numpy()[sub_idx][same, 0] - best_t[same]) / diag
            par = dict(bf16=dict(rays=int(sub.shape[0]), sample="every 64th ray", leaf_agreement=float((got == best_code).mean()),
                                 depth_err_mean=float(dep.mean()) if same.any() else None,
                                 oracle_params="FP32 master"))
    nb = sum(p.shape[0] for p, _ in batches)
    log("batched: step %.3f ms (query %.3f, train graph %.3f), hit acc %.4f" % (step_ms, q_ms, t_ms,
                                                                               acc["hit_accuracy"]))
    return {
        "metric": METRIC,
        "value": R / (q_ms * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "8 displaced icospheres (50,000..1,997,120 triangles, 256..8,192 leaves, own tables "
                        "T=2^16..2^20, L=16 F=2, 8 samples, MLP 256-4x128-5) queried together by 2^22 rays "
                        "crossing 1..32 leaves (log-uniform); training step of 2^18 probes per object as one "
                        "HIP graph (%s)" % ("objects one after another" if args.serial_graph else
                                            "one parallel branch per object"),
            "rays": R, "objects": len(objs), "train_batch": nb,
            "step": "one grouped query + one graph-captured training step of every object",
            "tuning": tuning,
        },
        "query_ms": q_ms,
        "query_ms_default_knobs": q_ms_default,
        "train_ms": t_ms,
        "segments_per_s": evaluated / (q_ms * 1e-3),
        "train_segs_per_s": nb / (t_ms * 1e-3),
        "accuracy": acc,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": par,
        "ceilings": peaks,
    }


def run_construct(args, P, torch, configs, scene):
    """Error-driven construction (Sec. 5.1) at the frame workload's size: a
    cut of the 1,003,520-triangle mesh's base BVH (16 triangles per node)
    grown to 1,024 leaves while the frame network trains on 2^16 candidate
    rays per step (first leaf only, per-leaf acceptance; 2^18 rays per
    statistics round), then a final training round of --pretrain steps.
    Labels come from the host's Moller-Trumbore (the classical intersection
    the paper's training data comes from); their time is reported apart
    from the library's."""
    from paper_2405_16237_amd import construct as C
    t0 = time.time()
    sc = configs.make_scene(1_003_520, 1024)
    base = scene.base_bvh(sc.verts, sc.tris, leaf_tris=16)
    root = np.concatenate([base["lo"][0], base["hi"][0]])[None, :]
    lo, side = scene.scene_cube(root)
    net = configs.C2_NET
    label_s = [0.0, 0]

    def labels(p):
        t = time.time()
        out = scene.probe_labels(sc.mesh, p)
        label_s[0] += time.time() - t
        label_s[1] += p.shape[0]
        return out

    sched = C.Schedule(target_leaves=1024, iters=30, iters_growth=1.2, splits=16, splits_growth=1.7,
                       final_iters=args.pretrain, rays_per_step=1 << 16, stats_rays=1 << 18)
    prep = time.time() - t0
    torch.cuda.synchronize()
    t1 = time.time()
    model, cut, hist = C.construct(net, base, labels, sched, lo, side,
                                   params=configs.init_params(net, "normal", 1e-2), log=log)
    torch.cuda.synchronize()
    total = time.time() - t1
    rays = scene.pinhole_rays(480, 270)
    gt = scene.ray_ground_truth(sc.mesh, rays)
    acc = hit_error(model.query(torch.from_numpy(rays).cuda()).cpu().numpy(), gt, sc.diagonal)
    steps = sum(h["steps"] for h in hist)
    log("construction: %.1f s (labels %.1f s for %d probes), %d training steps, %d leaves, hit acc %.4f" %
        (total, label_s[0], label_s[1], steps, len(cut.nodes), acc["hit_accuracy"]))
    return {
        "metric": "error-driven N-BVH construction wall time",
        "value": total, "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "config": {"workload": "cut of the base BVH (16 triangles per node) of a 1,003,520-triangle displaced "
                               "icosphere grown to 1,024 leaves; network L=16 F=2 T=2^19, 8 samples, MLP 256-4x128-5; "
                               "2^16 candidate rays per training step, 2^18 per statistics round"},
        "host_labels_s": label_s[0], "labelled_probes": label_s[1], "library_and_driver_s": total - label_s[0],
        "training_steps": steps, "rounds": len(hist), "leaves": len(cut.nodes), "setup_s": prep,
        "accuracy_480x270": acc, "history": hist,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=("frame", "secondary", "batched", "construct"), default="frame")
    ap.add_argument("--pretrain", type=int, default=600, help="untimed BF16 training steps before timing")
    ap.add_argument("--batches", type=int, default=4, help="distinct 2^18-probe batches cycled in training")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--per-leaf", type=int, default=0,
                    help="training probes per leaf (0: the workload's; 32 on the frame workload gives 2^15, one "
                         "GPU's share of a 2^18 batch split over eight)")
    ap.add_argument("--samples", type=int, choices=(8, 4), default=8,
                    help="frame workload: samples per segment (8, n_in = 256; or 4, the literal 128-input MLP)")
    ap.add_argument("--lod", type=int, default=0,
                    help="also train and time a coarser cut of this many leaves over the same network (levels of "
                         "detail); 0 = off")
    ap.add_argument("--inside", choices=("reverse", "clip"), default="reverse",
                    help="secondary workload: how a leaf around a bounce origin is queried")
    ap.add_argument("--bounce-offset", type=float, default=1e-4,
                    help="secondary workload: origin offset along the normal, in scene diagonals")
    ap.add_argument("--bounce-from", choices=("network", "mesh"), default="network",
                    help="secondary workload: spawn the bounces from the trained network's own primary hits (as a "
                         "renderer would) or from the mesh's exact primary hits")
    ap.add_argument("--inside-probes", choices=("surface", "uniform"), default="surface",
                    help="secondary workload with --inside clip: the inside-starting training probes start on the "
                         "surface inside their leaf (as bounce rays do) or uniformly inside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--no-parity", action="store_true", help="skip the comparison with the FP64 oracle")
    ap.add_argument("--no-peaks", action="store_true", help="skip the ceiling micro-benchmarks")
    ap.add_argument("--serial-graph", action="store_true",
                    help="batched workload: capture the objects' training steps one after another instead of as "
                         "parallel graph branches")
    ap.add_argument("--copy-kernel-mib", type=int, default=0,
                    help="first run a plain elementwise copy of this many MiB five times: the reference "
                         "dispatch that scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the query shards by rays and the "
              "training step by probes, but only one GPU is measured here). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2405_16237_amd as P
    from nbvh_synth import configs, scene

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.load()
    if args.copy_kernel_mib > 0:
        copy_kernel(torch, args.copy_kernel_mib)
    if args.workload == "batched":
        out = run_batched(args, P, torch, configs, scene)
    elif args.workload == "construct":
        out = run_construct(args, P, torch, configs, scene)
    else:
        W = build_frame(configs, scene, args.samples) if args.workload == "frame" else build_secondary(configs, scene, args.inside,
                                                                                           args.bounce_offset,
                                                                                           args.bounce_from,
                                                                                           args.inside_probes)
        if args.per_leaf > 0:
            W.per_leaf = args.per_leaf
            W.describe = W.describe.replace("train batch 2^18 probes", "train batch %d probes" % (args.per_leaf * W.sc.boxes.shape[0]))
        out = run_single(args, W, P, torch, configs, scene)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
