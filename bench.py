#!/usr/bin/env python3
"""N-BVH neural ray query + training step benchmark on one MI355X.

Workload: 1920x1080 primary camera rays against a 1,003,520-triangle
displaced icosphere clustered into 1,024 neural leaves; hash grid L=16,
F=2, T=2^19 (N_min 16, growth 1.38), 8 samples per segment, MLP
256 -> 4x128 -> 5; training batches of 2^18 probe segments (256 per leaf)
labelled by Moller-Trumbore. The network is first trained (untimed) so the
hit decisions are meaningful; then each timed step is one full query of the
frame plus one training step, in BF16 (the primary path). The same trained
parameters are timed through the FP32 path, and both paths' hit error
against the triangle ground truth is reported ("matched hit error").

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
METRIC = "neural ray queries/s + train segs/s, BF16-MFMA vs FP32, at matched hit error"


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
    return dict(hit_accuracy=agree, hit_error_pct=100.0 * (1.0 - agree),
                depth_err_mean=float(dep.mean()) if both.any() else None,
                depth_err_p99=float(np.quantile(dep, 0.99)) if both.any() else None,
                predicted_hits=int(pred.sum()), true_hits=int(truth.sum()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pretrain", type=int, default=600, help="untimed BF16 training steps before timing")
    ap.add_argument("--batches", type=int, default=4, help="distinct 2^18-probe batches cycled in training")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--copy-kernel-mib", type=int, default=0,
                    help="first run a plain elementwise copy of this many MiB five times: the reference "
                         "dispatch that scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the query shards by rays and the "
              "training step by probes; see DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2405_16237_amd as P
    from nbvh_synth import configs, scene

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.load()
    if args.copy_kernel_mib > 0:
        # elementwise kernel reading and writing exactly n * 4 bytes
        n = args.copy_kernel_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log("copy kernel: %d bytes read and %d written per dispatch" % (n * 4, n * 4))
        del src, dst
    t0 = time.time()
    sc = configs.make_scene(1_003_520, 1024)
    rays_np = scene.pinhole_rays(1920, 1080)
    gt = scene.ray_ground_truth(sc.mesh, rays_np)
    batches = []
    for i in range(args.batches):
        pr, _ = scene.leaf_probes(sc.boxes, 256, seed=scene.SEED_PROBES + i)
        lb = scene.probe_labels(sc.mesh, pr)
        batches.append((torch.from_numpy(pr).cuda(), torch.from_numpy(lb).cuda()))
    B = batches[0][0].shape[0]
    log("data ready in %.1fs: %d rays, %d triangles, %d leaves, batch %d" %
        (time.time() - t0, rays_np.shape[0], sc.tris.shape[0], sc.boxes.shape[0], B))
    net = configs.C2_NET
    params0 = configs.init_params(net, "normal", 1e-2)
    rays = torch.from_numpy(rays_np).cuda()
    R = rays.shape[0]
    seg_cap = 16 * R

    bf = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1024.0)
    bf.set_params(params0)
    bf.workspace(R, seg_cap, B)
    # pre-training (untimed): the trained network of the training workload
    t1 = time.time()
    loss = None
    for i in range(args.pretrain):
        p, l = batches[i % len(batches)]
        loss = bf.train_step(p, l)
    torch.cuda.synchronize()
    log("pretrain %d steps in %.1fs, loss %s" % (args.pretrain, time.time() - t1,
                                                 None if loss is None else loss.cpu().numpy().round(4).tolist()))

    def run_steps(m, n, timed):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        hits = torch.empty((R, 8), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        qms = 0.0
        ev0.record()
        for i in range(n):
            q0.record()
            m.query(rays, seg_cap, hits)
            q1.record()
            p, l = batches[i % len(batches)]
            m.train_step(p, l)
            if timed:
                q1.synchronize()
                qms += q0.elapsed_time(q1)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1), qms, hits

    # BF16 primary path
    run_steps(bf, args.warmup, False)
    st0 = bf.read_state()
    total_ms, _, _ = run_steps(bf, args.steps, False)
    st1 = bf.read_state()
    evaluated = (st1["n_evaluated"] - st0["n_evaluated"]) / max(1, args.steps)
    n_segments = st1["last_n_segments"]
    # query-only and train-only timing of the same path (separate loops)
    def time_loop(fn, n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for i in range(n):
            fn(i)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    hits_bf = torch.empty((R, 8), dtype=torch.float32, device="cuda")
    q_ms = time_loop(lambda i: bf.query(rays, seg_cap, hits_bf), args.steps)
    t_ms = time_loop(lambda i: bf.train_step(*batches[i % len(batches)]), args.steps)
    # per-kernel device time (HIP events around each kernel group on the launch stream)
    bf.profile_begin()
    run_steps(bf, args.steps, False)
    prof = bf.profile_end()
    torch.cuda.synchronize()
    acc_bf = hit_error(hits_bf.cpu().numpy(), gt, sc.diagonal)
    log("bf16: step %.3f ms (query %.3f, train %.3f), evaluated %.0f / %d segments" %
        (total_ms / args.steps, q_ms, t_ms, evaluated, n_segments))
    log("profile:", {k: (round(v[0] / max(1, v[1]), 4), v[1]) for k, v in prof.items()})

    # FP32 path with the same trained parameters
    fp32 = None
    if not args.no_fp32:
        fp = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1024.0)
        fp.set_params(bf.get_params())
        fp.workspace(R, seg_cap, B)
        hits_fp = torch.empty((R, 8), dtype=torch.float32, device="cuda")
        fp.query(rays, seg_cap, hits_fp)
        torch.cuda.synchronize()
        acc_fp = hit_error(hits_fp.cpu().numpy(), gt, sc.diagonal)
        fq_ms = time_loop(lambda i: fp.query(rays, seg_cap, hits_fp), args.steps)
        fp.set_params(bf.get_params())
        ft_ms = time_loop(lambda i: fp.train_step(*batches[i % len(batches)]), args.steps)
        fp32 = dict(query_ms=fq_ms, train_ms=ft_ms, rays_per_s=R / (fq_ms * 1e-3), train_segs_per_s=B / (ft_ms * 1e-3),
                    accuracy=acc_fp)
        log("fp32: query %.3f ms, train %.3f ms, hit acc %.4f (bf16 %.4f)" %
            (fq_ms, ft_ms, acc_fp["hit_accuracy"], acc_bf["hit_accuracy"]))

    # FP8 inference option with the same trained parameters: per-layer scales
    # calibrated on 2^16 seeded probe segments
    fp8 = None
    if not args.no_fp8:
        f8 = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp8")
        f8.set_params(bf.get_params())
        f8.calibrate_fp8(batches[0][0][: 1 << 16].contiguous())
        f8.workspace(R, seg_cap, 0)
        hits_f8 = torch.empty((R, 8), dtype=torch.float32, device="cuda")
        f8.query(rays, seg_cap, hits_f8)
        torch.cuda.synchronize()
        acc_f8 = hit_error(hits_f8.cpu().numpy(), gt, sc.diagonal)
        f8_ms = time_loop(lambda i: f8.query(rays, seg_cap, hits_f8), args.steps)
        fp8 = dict(query_ms=f8_ms, rays_per_s=R / (f8_ms * 1e-3), accuracy=acc_f8,
                   calibration="2^16 probe segments of the first training batch")
        log("fp8: query %.3f ms, hit acc %.4f (bf16 %.4f)" % (f8_ms, acc_f8["hit_accuracy"], acc_bf["hit_accuracy"]))
        del f8

    # dominant kernel group and its roofline
    per = {k: (v[0] / max(1, v[1]), v[1], v[0]) for k, v in prof.items() if v[1] > 0}
    dom = max(per, key=lambda k: per[k][2])
    avg_ms = per[dom][0]
    c = net
    S, L, F = c.n_samples, c.n_levels, c.n_features
    flops_fwd = 2 * c.n_mlp_params
    work = {
        # bytes of table entries gathered: S*L*8 corners x F features x 2 B (bf16)
        "query_eval": ("hbm", evaluated * S * L * 8 * F * 2, "GB/s"),
        "train_tile": ("hbm", B * S * L * 8 * F * 2, "GB/s"),
        # one 4-byte atomic add per corner and feature
        "scatter": ("hbm", B * S * L * 8 * F * 4, "GB/s"),
        "wgrad": ("mfma", B * flops_fwd, "TFLOP/s"),
        "optimizer": ("hbm", (c.n_table_params + c.n_mlp_params) * 34, "GB/s"),
        "traverse": ("hbm", R * 32 + n_segments * 16 * 2 + R * 12, "GB/s"),
    }
    bound, amount, unit = work.get(dom, ("hbm", 0, "GB/s"))
    if unit == "GB/s":
        achieved = amount / (avg_ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
    else:
        achieved = amount / (avg_ms * 1e-3) / 1e12
        peak = BF16_PEAK_TFLOPS
    roofline = dict(bound=bound, kernel=dom, achieved=round(achieved, 2), peak=peak, unit=unit,
                    frac=round(achieved / peak, 4), traffic=None, avg_ms=round(avg_ms, 4),
                    algorithmic=amount, per_kernel_ms={k: round(v[0], 4) for k, v in per.items()})

    # CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cfg = oracle.make_cfg(net, sc.lo, sc.side)
        params = bf.get_params().astype(np.float64)
        stride = 16
        sample = rays_np.reshape(1080, 1920, 8)[::stride, ::stride].reshape(-1, 8)
        t2 = time.time()
        oracle.query(cfg, params, sample, sc.boxes)
        dt = time.time() - t2
        # grow the sample towards the target time
        if dt < args.cpu_seconds / 4 and stride > 4:
            stride = max(4, int(stride / np.sqrt(args.cpu_seconds / max(dt, 1e-3))))
            sample = rays_np.reshape(1080, 1920, 8)[::stride, ::stride].reshape(-1, 8)
            t2 = time.time()
            oracle.query(cfg, params, sample, sc.boxes)
            dt = time.time() - t2
        cpu = dict(value=sample.shape[0] / dt, unit="rays/s", cores=oracle.num_threads(), kind="oracle",
                   sample="every %dth row and column of the 1920x1080 frame (%d rays), full query in FP64 "
                          "(every-leaf traversal, encode, MLP, resolve), %.1f s" % (stride, sample.shape[0], dt))
        log("cpu baseline:", cpu)

    step_ms = total_ms / args.steps
    out = {
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
            "workload": "1920x1080 primary rays on a 1,003,520-triangle displaced icosphere, 1,024 neural leaves; "
                        "hash grid L=16 F=2 T=2^19, 8 samples/segment, MLP 256-4x128-5; train batch 2^18 probes",
            "rays": R, "segments": int(n_segments), "segments_evaluated": int(evaluated), "train_batch": B,
            "step": "one full-frame query + one training step (forward, loss, backward, Adam)",
        },
        "query_ms": q_ms,
        "train_ms": t_ms,
        "segments_per_s": evaluated / (q_ms * 1e-3),
        "train_segs_per_s": B / (t_ms * 1e-3),
        "accuracy": acc_bf,
        "fp32": fp32,
        "fp8": fp8,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
