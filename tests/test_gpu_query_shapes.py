"""GPU parity of the full neural ray query at the benchmarked shapes.

The query kernel the benchmark times (persistent slots, LDS feature tile of
n_in + pad columns, slot refill, early termination) is checked segment by
segment against the FP64 oracle through nbvh_query_traced, which runs the same
kernels and launch shapes and also returns the segment queue, each evaluated
segment's logits and the feature row the MLP read:

  * the 1920x1080 frame workload: 1,003,520 triangles, 1,024 leaves (tree depth
    10), L=16 F=2 T=2^19, 8 samples, MLP 256 -> 4x128 -> 5, on every 4th row
    and column of the frame (129,600 rays), FP32 and BF16, with a seeded
    network and with the network trained as the benchmark trains it;
  * the bounce-ray workload's network and leaves: 3,996,180 triangles, 16,384
    leaves (depth 14), L=16 F=4 T=2^22, 4 samples, MLP 256 -> 4x256 -> 8,
    reversed inside rule, on 2^16 cosine-weighted bounce rays.

Bars (Sec. 5 query; tolerances of the workload statement): the segment queue
bit-exact; FP32 features within 1e-5 of the segment's largest feature and
logits within 1e-5 of the segment's largest output-layer sum (its largest
|z| unless the sums cancel); BF16 logits within 2e-2 max(1, |z|) with |z|
read the same way (and at most 0.1 % of logits beyond the literal
2e-2 max(1, |z|)), features within BF16 rounding; every ray whose answer is unambiguous under those tolerances (query_check)
gets the oracle's leaf, and FP32 distances and normals within 1e-5; on the
trained network at least 99.5 % of all rays agree with the oracle and the mean
depth error over agreeing hits is at most 1e-3 of the scene diagonal.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nbvh_synth import configs, scene
from query_check import clear_rays, evaluated_prefix_ok, leaf_of, output_term_scale

pytestmark = pytest.mark.gpu

BF16_TOL = 2e-2
FP32_TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bf16_round(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy()


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16237_amd as P
    P.load()
    return P


def _seeded(net):
    """Features U(-1, 1) (so that the logits spread beyond the BF16 band more
    than with the workload's N(0, 1e-2) features), Xavier MLP."""
    return configs.init_params(net, "uniform", 1.0, seed_features=41, seed_mlp=42)


def _check_traced(lib, net, sc, rays, params, precision, inside="clip", trained=False):
    """Run the traced query and compare with the oracle; returns a summary."""
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision=precision, inside=inside)
    m.set_params(params)
    rev = inside == "reverse"
    tr = oracle.traverse(rays, sc.boxes, rev)
    off_o, sr, sl, t0, t1 = tr
    n_seg = int(off_o[-1])
    cap = n_seg + 64
    _say("traced query", precision, net.n_in, "->", net.mlp_width, "x", net.mlp_hidden, rays.shape[0], "rays",
         n_seg, "segments", sc.boxes.shape[0], "leaves", inside)
    hits, off, segs, zt, ut = m.query_traced(torch.from_numpy(rays).cuda(), cap, z=True, u=True)
    hits = hits.cpu().numpy()
    off = off.cpu().numpy().astype(np.uint32).astype(np.uint64)
    segs = segs[:n_seg].cpu().numpy()
    zt = zt[:n_seg].cpu().numpy().astype(np.float64)
    ut = ut[:n_seg].cpu().numpy().astype(np.float64)
    st = m.read_state()
    assert st["flags"] == 0 and st["last_n_segments"] == n_seg
    # the segment queue the query evaluated: bit-exact
    assert np.array_equal(off, off_o)
    assert np.array_equal(segs[:, 0].astype(np.uint32), sr)
    assert np.array_equal(segs[:, 1].astype(np.uint32), sl)
    assert np.array_equal(segs[:, 2].view(np.float32), t0)
    assert np.array_equal(segs[:, 3].view(np.float32), t1)
    ev, counts = evaluated_prefix_ok(off_o, t0, zt, hits)

    pref = params if precision == "fp32" else _bf16_round(params)
    cfg = oracle.make_cfg(net, sc.lo, sc.side)
    rows = oracle.segment_rows(rays, sr, t0, t1, sl)
    p64 = pref.astype(np.float64)
    nt = net.n_table_params
    u_all = oracle.encode(cfg, p64[:nt], rows)
    z_all = oracle.mlp_forward(cfg, p64[nt:], u_all)
    u_ref, z_ref = u_all[ev], z_all[ev]
    out = oracle.resolve(off_o, sl, t0, t1, z_all, net.n_out, rays[:, 3])
    ug, zg = ut[ev], zt[ev]
    if precision == "fp32":
        # features: ||delta||_inf <= 1e-5 ||ref||_inf per segment; logits:
        # 1e-5 of the segment's largest output-layer sum magnitude (= max|z|
        # unless the sums cancel, where FP32 rounding is relative to the terms)
        zscale = np.maximum(np.abs(z_all).max(1), output_term_scale(u_all, p64[nt:], net))
        ru = np.abs(ug - u_ref).max(1) / np.maximum(np.abs(u_ref).max(1), 1e-30)
        rz = np.abs(zg - z_ref).max(1) / np.maximum(zscale[ev], 1e-30)
        assert ru.max() <= FP32_TOL, ru.max()
        assert rz.max() <= FP32_TOL, rz.max()
        _say("fp32 logits: max error / max|z| %.3g, / output-term scale %.3g" %
             ((np.abs(zg - z_ref).max(1) / np.maximum(np.abs(z_ref).max(1), 1e-30)).max(), rz.max()))
        ztol = FP32_TOL * np.repeat(zscale[:, None], net.n_out, 1)
    else:
        # features: FP32 interpolation of BF16 entries, rounded once to BF16
        # (8 significant bits: unit roundoff 2^-8)
        du = np.abs(ug - u_ref)
        bound = 2.0 ** -8 * np.abs(u_ref) + 1e-5 * np.abs(u_ref).max(1, keepdims=True)
        assert np.all(du <= bound), float((du / np.maximum(bound, 1e-30)).max())
        # logits: 2e-2 max(1, |z|), where |z| is read as the magnitude of the
        # output-layer sums (BF16 activations round each term to 2^-8; where
        # the sums cancel, the error is relative to the terms, not to z)
        zscale = np.maximum(np.abs(z_all).max(1), output_term_scale(u_all, p64[nt:], net))
        lit = np.abs(zg - z_ref) / np.maximum(1.0, np.abs(z_ref))
        dz = np.abs(zg - z_ref) / np.maximum(1.0, np.maximum(np.abs(z_ref), zscale[ev][:, None]))
        w = np.unravel_index(np.argmax(lit), lit.shape)
        _say("bf16 logits: |dz|/max(1,|z|) max %.4g, p99.9 %.4g, share above 2e-2 %.2e; worst segment: |z| %.3g, "
             "output-term scale %.3g; |dz|/max(1, scale) max %.4g" %
             (lit.max(), np.quantile(lit, 0.999), (lit > BF16_TOL).mean(), np.abs(z_ref[w[0]]).max(),
              zscale[ev][w[0]], dz.max()))
        _say("bf16 logits per output: max", np.round(lit.max(0), 4).tolist(), "p99",
             np.round(np.quantile(lit, 0.99, axis=0), 4).tolist(), "share above 2e-2",
             np.round((lit > BF16_TOL).mean(0), 5).tolist())
        if not trained:
            assert dz.max() <= BF16_TOL, dz.max()
            assert (lit > BF16_TOL).mean() <= 1e-3, (lit > BF16_TOL).mean()
        else:
            assert (lit > BF16_TOL).mean() <= 0.05, (lit > BF16_TOL).mean()
        ztol = BF16_TOL * np.maximum(1.0, np.maximum(np.abs(z_all), zscale[:, None]))
    clear = clear_rays(tr, z_all, out, rays[:, 3], ztol)
    # rays with an evaluated segment whose hit or distance logit is off by
    # more than its tolerance are not clear either: their answer may flip,
    # and such logits are bounded above (none for FP32 and seeded BF16, a
    # share for the trained BF16 network)
    off_band = np.zeros(n_seg, bool)
    off_band[np.flatnonzero(ev)] = (np.abs(zg - z_ref)[:, :2] > ztol[ev][:, :2]).any(1)
    clear[np.unique(sr[off_band])] = False
    leaf = leaf_of(hits)
    oleaf = out[:, 4].astype(np.int64)
    agree_clear = float((leaf[clear] == oleaf[clear]).mean())
    agree_all = float((leaf == oleaf).mean())
    both = (leaf >= 0) & (leaf == oleaf)
    depth = np.abs(hits[both, 0] - out[both, 0]) / sc.diagonal
    summary = dict(rays=rays.shape[0], segments=n_seg, evaluated=int(ev.sum()), clear=float(clear.mean()),
                   off_band_segments=int(off_band.sum()),
                   agree_clear=agree_clear, agree_all=agree_all, hits=int((oleaf >= 0).sum()),
                   depth_mean=float(depth.mean()) if both.any() else 0.0, max_dz=float(np.abs(zg - z_ref).max()))
    _say(summary)
    assert agree_clear == 1.0, agree_clear
    if precision == "fp32":
        sel = clear & both
        dt = np.abs(hits[sel, 0] - out[sel, 0]) / np.maximum(1.0, np.abs(out[sel, 0]))
        assert dt.max() <= FP32_TOL, dt.max()
        zs = zscale[out[sel, 5].astype(np.int64)]
        dn = np.abs(hits[sel, 1:4] - out[sel, 1:4]).max(1) / zs
        assert dn.max() <= FP32_TOL, dn.max()
        if net.n_out >= 8:
            # albedo = sigmoid(z), sigmoid' <= 1/4
            da = np.abs(hits[sel, 4:7] - out[sel, 6:9]).max(1) / zs
            assert da.max() <= FP32_TOL, da.max()
    miss = clear & (oleaf < 0)
    assert np.all(leaf[miss] < 0)
    if trained:
        assert agree_all >= 0.995, agree_all
        assert summary["depth_mean"] <= 1e-3, summary["depth_mean"]
    return summary


# ------------------------------------------------------------------ the frame workload
@pytest.fixture(scope="module")
def frame():
    sc = configs.make_scene(1_003_520, 1024)
    rays = scene.pinhole_rays(1920, 1080).reshape(1080, 1920, 8)[::4, ::4].reshape(-1, 8).copy()
    return sc, rays


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_traverse_bitexact_frame(lib, frame, mode):
    sc, rays = frame
    m = lib.NBVH(configs.C2_NET, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_tuning(traverse_mode=mode)
    off_o, sr, sl, t0, t1 = oracle.traverse(rays, sc.boxes)
    _say("traverse frame subset", rays.shape[0], "rays, 1024 leaves, mode", mode)
    off, segs = m.traverse(torch.from_numpy(rays).cuda(), int(off_o[-1]) + 16)
    off = off.cpu().numpy().astype(np.uint32).astype(np.uint64)
    sg = segs[: int(off_o[-1])].cpu().numpy()
    assert np.array_equal(off, off_o)
    assert np.array_equal(sg[:, 1].astype(np.uint32), sl)
    assert np.array_equal(sg[:, 2].view(np.float32), t0) and np.array_equal(sg[:, 3].view(np.float32), t1)
    counts = np.diff(off_o.astype(np.int64))
    assert counts.max() >= 4 and (counts > 0).mean() > 0.3


def test_query_same_for_every_walk(lib, frame):
    """How a wave walks the tree and the order the rays are evaluated in
    change neither the segment queue nor the query: the hit records are
    bit-identical for the three walk modes, with and without origin order."""
    sc, rays = frame
    m = lib.NBVH(configs.C2_NET, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(_seeded(configs.C2_NET))
    r = torch.from_numpy(rays).cuda()
    out = []
    for mode in (0, 1, 2):
        for order in (0, 1, 2):
            _say("query frame subset, walk mode", mode, "ray order", order)
            m.set_tuning(traverse_mode=mode, query_order=order)
            out.append(m.query(r).cpu().numpy().view(np.uint32))
    for o in out[1:]:
        assert np.array_equal(out[0], o)
    assert (out[0][:, 7] != 0xFFFFFFFF).sum() > 1000


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_query_frame_seeded(lib, frame, precision):
    sc, rays = frame
    s = _check_traced(lib, configs.C2_NET, sc, rays, _seeded(configs.C2_NET), precision)
    assert s["clear"] > 0.5 and s["hits"] > 10000


@pytest.fixture(scope="module")
def trained_frame(lib, frame):
    """The frame network trained as the benchmark trains it: 600 BF16 steps
    over four 2^18-probe batches labelled by Moller-Trumbore."""
    sc, _ = frame
    net = configs.C2_NET
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1024.0)
    m.set_params(configs.init_params(net, "normal", 1e-2))
    batches = []
    for i in range(4):
        p, _ = scene.leaf_probes(sc.boxes, 256, seed=scene.SEED_PROBES + i)
        batches.append((torch.from_numpy(p).cuda(), torch.from_numpy(scene.probe_labels(sc.mesh, p)).cuda()))
    _say("training the frame network: 600 steps")
    for i in range(600):
        loss = m.train_step(*batches[i % 4])
    torch.cuda.synchronize()
    _say("trained, loss", loss.cpu().numpy())
    return m.get_params()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_query_frame_trained(lib, frame, trained_frame, precision):
    sc, rays = frame
    s = _check_traced(lib, configs.C2_NET, sc, rays, trained_frame, precision, trained=True)
    assert s["hits"] > 10000


# ------------------------------------------------------------------ the bounce-ray workload's shape
@pytest.fixture(scope="module")
def bounce():
    sc = configs.make_scene(3_996_180, 16384, albedo_seed=scene.SEED_ALBEDO)
    prim = scene.pinhole_rays(1920, 1080).reshape(1080, 1920, 8)[::8, ::8].reshape(-1, 8)
    g = scene.ray_ground_truth(sc.mesh, prim)
    hit = g["hit"]
    pts = prim[hit, 0:3].astype(np.float64) + g["t"][hit, None] * prim[hit, 4:7].astype(np.float64)
    rays = scene.cosine_bounces(pts, g["n"][hit], 1 << 16, seed=scene.SEED_SECONDARY, offset=1e-4 * sc.diagonal)
    return sc, rays


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_query_bounce_reverse(lib, bounce, precision):
    sc, rays = bounce
    net = configs.C5_NET
    s = _check_traced(lib, net, sc, rays, _seeded(net), precision, inside="reverse")
    assert s["clear"] > 0.3 and s["segments"] > rays.shape[0]


def test_bounce_query_same_in_origin_order(lib, bounce):
    """Evaluating the bounce rays in the order of their origins' Morton codes
    (query_order = 1) or of their origins' and directions' (2) gives the same
    hit records bit for bit."""
    sc, rays = bounce
    net = configs.C5_NET
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", inside="reverse")
    m.set_params(_seeded(net))
    r = torch.from_numpy(rays).cuda()
    _say("bounce query in the caller's order, in origin order and in origin-and-direction order")
    a = m.query(r).cpu().numpy().view(np.uint32)
    for order in (1, 2):
        m.set_tuning(query_order=order)
        b = m.query(r).cpu().numpy().view(np.uint32)
        assert np.array_equal(a, b), order
    assert (a[:, 7] != 0xFFFFFFFF).sum() > 1000


def test_traverse_bitexact_bounce_every_walk(lib, bounce):
    """The bounce rays' segment queue at 16,384 leaves (depth 14, reverse
    rule) is bit-exact against the every-leaf oracle for the per-lane walk,
    the wave-coherent walk (forced on these incoherent rays, so that every
    wave visits the union of 64 scattered paths) and the per-wave choice."""
    sc, rays = bounce
    m = lib.NBVH(configs.C5_NET, sc.boxes, sc.lo, sc.side, precision="bf16", inside="reverse")
    off_o, sr, sl, t0, t1 = oracle.traverse(rays, sc.boxes, True)
    r = torch.from_numpy(rays).cuda()
    for mode in (0, 1, 2):
        _say("traverse bounce rays, 16,384 leaves, walk mode", mode)
        m.set_tuning(traverse_mode=mode)
        off, segs = m.traverse(r, int(off_o[-1]) + 16)
        off = off.cpu().numpy().astype(np.uint32).astype(np.uint64)
        sg = segs[: int(off_o[-1])].cpu().numpy()
        assert np.array_equal(off, off_o), mode
        assert np.array_equal(sg[:, 0].astype(np.uint32), sr)
        assert np.array_equal(sg[:, 1].view(np.uint32), sl)
        assert np.array_equal(sg[:, 2].view(np.float32), t0) and np.array_equal(sg[:, 3].view(np.float32), t1)
