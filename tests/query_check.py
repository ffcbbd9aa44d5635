"""Helpers for comparing a traced GPU query with the FP64 oracle's query.

Which segments decide a ray's answer, and when that decision is unambiguous
under a stated output tolerance:
  * a segment is predicted hit when its hit logit z0 > 0 (Sec. 5.2,
    "Visibility"); the decision is clear when |z0| exceeds the tolerance on z0;
  * its distance is t = t0 + sigmoid(z1) (t1 - t0) along the queried
    direction (Sec. 5.2, "Intersection point"), mapped back to the ray for a
    reversed inside chord, which also counts only in front of the origin;
  * the ray's answer is the smallest such t; it is clear when no other hit
    segment's t (and, for reversed chords, the origin) lies within the sum of
    the two distance tolerances of the winner's.
The tolerance on z is the caller's (per segment, per output); the distance
tolerance follows from it through sigmoid' <= 1/4.
"""
from __future__ import annotations

import numpy as np

import oracle


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def segment_distance(tr, z, ray_tmin):
    """(t along the ray, valid) for every segment of an oracle traversal, from
    logits z (the oracle's, FP64). valid: predicted hit and, for reversed
    chords, in front of the origin."""
    off, sr, sl, t0, t1 = tr
    t0 = t0.astype(np.float64)
    t1 = t1.astype(np.float64)
    inside = (sl & np.uint32(oracle.INSIDE_TAG)) != 0
    frac = sigmoid(z[:, 1])
    t = np.where(inside, t1 - frac * (t1 - t0), t0 + frac * (t1 - t0))
    valid = z[:, 0] > 0
    valid &= ~inside | (t > ray_tmin[sr].astype(np.float64))
    return t, valid


def clear_rays(tr, z, out, ray_tmin, ztol):
    """Boolean [n_rays]: rays whose answer is unambiguous when every logit may
    move by ztol (same shape as z)."""
    off, sr, sl, t0, t1 = tr
    n = off.shape[0] - 1
    clear = np.ones(n, bool)
    if z.shape[0] == 0:
        return clear
    # hit decisions
    bad = np.abs(z[:, 0]) <= ztol[:, 0]
    t, valid = segment_distance(tr, z, ray_tmin)
    seglen = (t1.astype(np.float64) - t0.astype(np.float64))
    dt = 0.25 * seglen * ztol[:, 1] + 1e-6 * np.maximum(1.0, np.abs(t))
    inside = (sl & np.uint32(oracle.INSIDE_TAG)) != 0
    # a reversed chord's point close to the origin may fall on either side
    bad |= inside & (z[:, 0] > 0) & (np.abs(t - ray_tmin[sr]) <= dt)
    clear[np.unique(sr[bad])] = False
    # distance ties between the winner and any other valid segment of the ray
    win = out[:, 5].astype(np.int64)
    has = win >= 0
    tw = np.full(n, np.nan)
    dtw = np.zeros(n)
    tw[has] = t[win[has]]
    dtw[has] = dt[win[has]]
    idx = np.arange(sr.shape[0])
    other = valid & (idx != win[sr]) & has[sr]
    tie = other & (np.abs(t - tw[sr]) <= dt + dtw[sr])
    clear[np.unique(sr[tie])] = False
    return clear


def output_term_scale(u, W_flat, net):
    """Per segment, the largest magnitude of the sums that produce the logits,
    max_o sum_j |W_H[o, j] h_H[j]| (numpy float64 from the oracle's features):
    the scale a floating-point forward error of the output layer is bounded
    by; it exceeds max|z| where those sums cancel."""
    mats, o = [], 0
    for fi, fo in net.layer_dims():
        mats.append(W_flat[o:o + fi * fo].reshape(fo, fi))
        o += fi * fo
    out = np.empty(u.shape[0])
    for a in range(0, u.shape[0], 16384):
        h = u[a:a + 16384]
        for M in mats[:-1]:
            h = np.maximum(h @ M.T, 0.0)
        out[a:a + 16384] = (np.abs(h) @ np.abs(mats[-1]).T).max(1)
    return out


def leaf_of(hits):
    leaf = hits[:, 7].view(np.uint32).astype(np.int64)
    leaf[leaf == 0xFFFFFFFF] = -1
    return leaf


def evaluated_prefix_ok(off, seg_t0, zt, hits):
    """The segments a ray evaluated are a prefix of its run (at least one),
    and a ray that stopped early has a hit no later than the start of its
    first skipped segment (the early-termination rule). Returns (evaluated
    mask [n_seg], evaluated count per ray)."""
    ev = ~np.isnan(zt[:, 0])
    off = off.astype(np.int64)
    n = off.shape[0] - 1
    total = np.diff(off)
    seg_ray = np.repeat(np.arange(n), total)
    counts = np.bincount(seg_ray[ev], minlength=n)
    pos = np.arange(ev.shape[0]) - off[:-1][seg_ray]
    assert np.array_equal(ev, pos < counts[seg_ray]), "evaluated segments are not a prefix of each run"
    assert np.all(counts[total > 0] >= 1), "a ray with segments evaluated none"
    stopped = np.nonzero(counts < total)[0]
    if stopped.size:
        first_skipped = off[stopped] + counts[stopped]
        assert np.all(leaf_of(hits[stopped]) >= 0), "a ray stopped early without a hit"
        assert np.all(hits[stopped, 0] <= seg_t0[first_skipped]), "a ray stopped before its best hit"
    return ev, counts
