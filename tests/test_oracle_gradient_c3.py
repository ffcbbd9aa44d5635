"""The oracle's analytic gradient at the training workload's network (CPU).

Central differences (h = 1e-4, binary64) of the combined loss on a 1,024-probe
sub-batch of the 2^18-probe training batch (one probe per leaf of the
1,003,520-triangle scene's 1,024 leaves), through the L=16, F=2, T=2^19,
8-sample, 256 -> 4x128 -> 5 network with its seeded N(0, 1e-2) features and
Xavier weights, against the oracle's back-propagation (the definition the GPU
gradients are compared with). Covered: every weight of the output layer W_4,
1,024 sampled weights of each hidden layer's W_0 .. W_3, and 2,000 touched
table entries spread over the levels.

The differences use the oracle's own encoding and per-segment loss; the MLP
between them is replayed in numpy float64 (a textbook product the oracle's MLP
is pinned against), so that a perturbed weight only recomputes the layers
after it. A table entry enters the features linearly, u(theta + h e) =
u(theta) + h u(e), with u(e) the oracle's encoding of the one-hot table e.
A coordinate whose +-h step moves any ReLU pre-activation or any L1 residual
across zero is skipped (the loss has a kink there), as the gradient reading
prescribes: about half of the sampled coordinates of the first three layers
(whose step moves every later pre-activation of the batch) and nearly all
others are checked.
"""
import numpy as np
import pytest

import oracle
from nbvh_synth import configs, scene

pytestmark = pytest.mark.slow

H = 1e-4
REL = 1e-6


def _round_floor(seg_losses, B):
    """Rounding floor of a central difference of the mean loss: per-segment
    loss differences carry a few ulps each, summed over B segments and
    divided by 2hB."""
    return 4.0 * np.sqrt(B) * np.finfo(np.float64).eps * np.abs(seg_losses).max() / (2 * H * B)


@pytest.fixture(scope="module")
def problem():
    net = configs.C2_NET
    sc = configs.make_scene(1_003_520, 1024)
    probes, _ = scene.leaf_probes(sc.boxes, 256)        # the 2^18 batch, leaf-major
    sub = np.ascontiguousarray(probes[::256])            # one probe per leaf
    lab = scene.probe_labels(sc.mesh, sub)
    assert sub.shape[0] == 1024 and lab[:, 4].sum() > 100
    cfg = oracle.make_cfg(net, sc.lo, sc.side)
    params = configs.init_params(net, "normal", 1e-2).astype(np.float64)
    nt = net.n_table_params
    u = oracle.encode(cfg, params[:nt], sub)
    Ws, o = [], nt
    for fi, fo in net.layer_dims():
        Ws.append(params[o:o + fi * fo].reshape(fo, fi))
        o += fi * fo
    z = oracle.forward(cfg, params, sub)
    _, dz = oracle.loss(cfg, z, lab)
    g = oracle.backward(cfg, params, sub, dz)
    return dict(net=net, cfg=cfg, params=params, segs=sub, lab=lab, u=u, Ws=Ws, z=z, g=g, nt=nt)


def _forward(u, Ws):
    """Pre-activations of every hidden layer and the outputs (numpy)."""
    pres, h = [], u
    for W in Ws[:-1]:
        a = h @ W.T
        pres.append(a)
        h = np.maximum(a, 0.0)
    return pres, h @ Ws[-1].T


def _residual_signs(z, lab):
    """Signs of the L1 residuals of hit segments (distance and normal)."""
    tau, n, hit = lab[:, 0], lab[:, 1:4], lab[:, 4] > 0
    sd = np.sign(1.0 / (1.0 + np.exp(-z[..., 1])) - tau)
    sn = np.sign(z[..., 2:5] - n)
    return np.where(hit, sd, 0.0), np.where(hit[:, None], sn, 0.0)


def _segment_losses(cfg, z, lab):
    shp = z.shape[:-1]
    zz = z.reshape(-1, z.shape[-1])
    ll = np.broadcast_to(lab, shp + (lab.shape[1],)).reshape(-1, lab.shape[1])
    return oracle.segment_loss(cfg, zz, ll).reshape(shp)


def test_forward_replay_matches_oracle(problem):
    _, z = _forward(problem["u"], problem["Ws"])
    assert np.abs(z - problem["z"]).max() <= 1e-12 * max(1.0, np.abs(z).max())
    B = problem["segs"].shape[0]
    total = oracle.loss(problem["cfg"], problem["z"], problem["lab"], with_grad=False)[0][0]
    assert abs(_segment_losses(problem["cfg"], problem["z"], problem["lab"]).sum() / B - total) <= 1e-13


def _check_layer(problem, k, coords):
    """Central differences for the weights (i, j) of W_k; returns the number
    of coordinates checked."""
    cfg, lab, Ws, u = problem["cfg"], problem["lab"], problem["Ws"], problem["u"]
    B = u.shape[0]
    Hn = len(Ws) - 1
    pres, z0 = _forward(u, Ws)
    ins = [u] + [np.maximum(a, 0.0) for a in pres]  # input of each layer
    sd0, sn0 = _residual_signs(z0, lab)
    floor = _round_floor(_segment_losses(cfg, z0, lab), B)
    off = problem["nt"] + sum(W.size for W in Ws[:k])
    g = problem["g"][off:off + Ws[k].size].reshape(Ws[k].shape)
    gmax = np.abs(g).max()
    checked = 0
    for c0 in range(0, len(coords), 64):
        ci = coords[c0:c0 + 64]
        I = np.array([c[0] for c in ci])
        J = np.array([c[1] for c in ci])
        C = len(ci)
        losses, smooth = [], np.ones(C, bool)
        for s in (1.0, -1.0):
            d = s * H * ins[k][:, J].T                     # [C, B]: change of unit I's pre-activation
            if k == Hn:
                z = np.broadcast_to(z0, (C,) + z0.shape).copy()
                z[np.arange(C), :, I] += d
            else:
                a_new = pres[k][:, I].T + d                 # [C, B]
                smooth &= ~np.any(np.sign(a_new) != np.sign(pres[k][:, I].T), axis=1)
                dh = np.maximum(a_new, 0.0) - ins[k + 1][:, I].T   # change of h_{k+1}[:, I]
                # rank-one change of the next pre-activation, then the rest in full
                a = pres[k + 1][None] if k + 1 < Hn else None
                if k + 1 < Hn:
                    a = a + dh[:, :, None] * Ws[k + 1][:, I].T[:, None, :]
                    for q in range(k + 1, Hn):
                        smooth &= ~np.any(np.sign(a) != np.sign(pres[q][None]), axis=(1, 2))
                        h = np.maximum(a, 0.0)
                        a = h @ Ws[q + 1].T
                    z = a
                else:
                    z = z0[None] + dh[:, :, None] * Ws[Hn][:, I].T[:, None, :]
            sd, sn = _residual_signs(z, lab)
            smooth &= ~np.any(sd != sd0[None], axis=1) & ~np.any(sn != sn0[None], axis=(1, 2))
            losses.append(_segment_losses(cfg, z, lab))
        fd = (losses[0] - losses[1]).sum(axis=1) / (2 * H * B)
        ref = g[I, J]
        err = np.abs(fd - ref)[smooth]
        bound = REL * np.abs(ref[smooth]) + floor
        assert np.all(err <= bound), (k, float((err / bound).max()))
        checked += int(smooth.sum())
    return checked


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_weights_central_differences(problem, k):
    W = problem["Ws"][k]
    fo, fi = W.shape
    if k == len(problem["Ws"]) - 1:
        coords = [(i, j) for i in range(fo) for j in range(fi)]
    else:
        rng = np.random.default_rng(100 + k)
        flat = rng.choice(fo * fi, size=1024, replace=False)
        coords = [(int(f // fi), int(f % fi)) for f in flat]
    checked = _check_layer(problem, k, coords)
    # a step on an early layer moves every later pre-activation of all 1,024
    # segments, so a fair share of those steps touch some kink and are skipped
    assert checked >= (0.4 if k < 3 else 0.9) * len(coords), (checked, len(coords))


def test_table_central_differences(problem):
    cfg, lab, Ws, u, segs = problem["cfg"], problem["lab"], problem["Ws"], problem["u"], problem["segs"]
    nt, B = problem["nt"], u.shape[0]
    g = problem["g"][:nt]
    gmax = np.abs(g).max()
    touched = np.nonzero(np.abs(g) >= 1e-4 * gmax)[0]
    idx = np.random.default_rng(7).choice(touched, size=2000, replace=False)
    pres0, z0 = _forward(u, Ws)
    sd0, sn0 = _residual_signs(z0, lab)
    floor = _round_floor(_segment_losses(cfg, z0, lab), B)
    onehot = np.zeros(nt)
    checked = 0
    levels = set()
    for e in idx:
        onehot[e] = 1.0
        Je = oracle.encode(cfg, onehot, segs)
        onehot[e] = 0.0
        rows = np.nonzero(np.any(Je != 0.0, axis=1))[0]
        assert rows.size > 0
        ls, smooth = [], True
        for s in (1.0, -1.0):
            pres, z = _forward(u[rows] + s * H * Je[rows], Ws)
            smooth &= all(np.array_equal(np.sign(a), np.sign(p[rows])) for a, p in zip(pres, pres0))
            sd, sn = _residual_signs(z, lab[rows])
            smooth &= np.array_equal(sd, sd0[rows]) and np.array_equal(sn, sn0[rows])
            ls.append(oracle.segment_loss(cfg, z, lab[rows]))
        if not smooth:
            continue
        fd = (ls[0] - ls[1]).sum() / (2 * H * B)
        assert abs(fd - g[e]) <= REL * abs(g[e]) + floor, (int(e), fd, g[e])
        checked += 1
        levels.add(int(np.searchsorted(np.cumsum([0] + configs.C2_NET.level_sizes())[1:] * 2, e, side="right")))
    assert checked >= 0.9 * idx.size, checked
    assert len(levels) >= 12, sorted(levels)
