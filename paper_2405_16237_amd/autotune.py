"""Launch-shape autotuner for the N-BVH library.

Times candidate knob settings (nbvh_tuning) on the caller's own workload with
HIP events and keeps the fastest. The search runs in stages, each a grid over
a few knobs with the best of the earlier stages applied: for the query, waves
per workgroup x gather unroll x pair loads, then persistent workgroups per CU
x coarse levels in LDS, then how waves walk the tree x the order rays are evaluated in;
for back-propagation, training-tile waves x weight-gradient splits, then the
scatter's LDS budget x hash-aggregated levels x binning. Results can be
cached in a JSON file keyed by the workload signature.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

QUERY_STAGES = [dict(query_waves=(4, 8), query_unroll=(2, 3, 4), query_pairs=(0, 1)),
                dict(query_wgs_per_cu=(0, 1, 2), query_lds_kb=(0, 24, 64)),
                dict(traverse_mode=(0, 1, 2), query_order=(0, 1, 2))]
TRAIN_STAGES = [dict(train_waves=(4, 8), wgrad_splits=(16, 32, 64)),
                dict(scatter_lds_kb=(0, 144), scatter_hash_levels=(0, 4, 8, 12), scatter_binned=(0, 1))]


def _time(fn, reps):
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def signature(model, n_rays, n_probes) -> str:
    net = model.net
    return "L%dF%dT%dS%dW%dH%dO%d_p%d_r%d_b%d_cu%s" % (
        net.n_levels, net.n_features, net.log2_T, net.n_samples, net.mlp_width, net.mlp_hidden, net.n_out,
        model.precision, n_rays, n_probes, torch.cuda.get_device_properties(0).multi_processor_count)


def autotune(model, rays=None, probes=None, reps: int = 3, cache_path: str | None = None, log=None) -> dict:
    """Search the knobs for `model` on `rays` (query) and `probes` (backward),
    apply the best setting to the model and return it with the timings.
    Parameters are not changed (the backward's gradient is discarded)."""
    sig = signature(model, 0 if rays is None else rays.shape[0], 0 if probes is None else probes.shape[0])
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cached = json.load(f)
        if sig in cached:
            model.set_tuning(**cached[sig]["tuning"])
            return cached[sig]
    best = model.get_tuning()
    report = {"signature": sig, "query": [], "train": []}
    if rays is not None:
        seg_cap = 16 * rays.shape[0]
        hits = torch.empty((rays.shape[0], 8), dtype=torch.float32, device=rays.device)
        for space in QUERY_STAGES:
            results = []
            for vals in itertools.product(*space.values()):
                knobs = dict(best, **dict(zip(space.keys(), vals)))
                model.set_tuning(**knobs)
                ms = _time(lambda: model.query(rays, seg_cap, hits), reps)
                results.append((ms, knobs))
                if log:
                    log("query %s: %.3f ms" % (knobs, ms))
            results.sort(key=lambda r: r[0])
            best = dict(results[0][1])
            report["query"] += [(ms, k) for ms, k in results]
        model.set_tuning(**best)
    if probes is not None:
        dz = torch.full((probes.shape[0], model.net.n_out), 1e-3, dtype=torch.float32, device=probes.device)
        for space in TRAIN_STAGES:
            results = []
            for vals in itertools.product(*space.values()):
                knobs = dict(best, **dict(zip(space.keys(), vals)))
                model.set_tuning(**knobs)
                ms = _time(lambda: model.backward(probes, dz), reps)
                results.append((ms, knobs))
                if log:
                    log("backward %s: %.3f ms" % (knobs, ms))
            results.sort(key=lambda r: r[0])
            best = dict(results[0][1])
            report["train"] += [(ms, k) for ms, k in results]
        model.set_tuning(**best)
        model.grad.zero_()
    report["tuning"] = best
    if cache_path:
        cached = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cached = json.load(f)
        cached[sig] = report
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cached, f, indent=1)
    return report
