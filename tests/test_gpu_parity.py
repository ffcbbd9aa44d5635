"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs. Sizes span several tiles and ragged tails."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nbvh_synth import configs, scene
from query_check import clear_rays, leaf_of

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16237_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def c1():
    sc = configs.make_scene(20480, 64)
    rays = scene.pinhole_rays(256, 256)
    return sc, rays


def _net(n_levels, n_features, log2_T, n_samples, level_res, width, hidden, n_out=5):
    return configs.NetConfig(n_levels, n_features, log2_T, n_samples, 16, 1.5, width, hidden, n_out, list(level_res))


def _ocfg(net, sc):
    return oracle.make_cfg(net, sc.lo, sc.side)


def _params(net, seed=4, scale=0.5):
    rng = np.random.default_rng(seed)
    p = configs.init_params(net, "uniform", scale, seed_features=seed, seed_mlp=seed + 10)
    return p


def _bf16_round(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy()


def _rel_inf(a, b):
    """per-row ||a - b||_inf / ||b||_inf"""
    num = np.abs(a - b).max(axis=1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-30)
    return num / den


# ------------------------------------------------------------------ traversal
TRAVERSE_MODES = [0, 1, 2]  # per-lane walk, wave-coherent walk, chosen per wave


def _check_traverse(lib, rays_np, boxes, sc_lo, sc_side, net, mode=2):
    m = lib.NBVH(net, boxes, sc_lo, sc_side, precision="fp32")
    m.set_tuning(traverse_mode=mode)
    rays = torch.from_numpy(rays_np).cuda()
    off_o, sr, sl, t0, t1 = oracle.traverse(rays_np, boxes)
    cap = int(off_o[-1]) + 16
    off_g, segs = m.traverse(rays, cap)
    torch.cuda.synchronize()
    off_g = off_g.cpu().numpy().astype(np.uint32)
    assert np.array_equal(off_g.astype(np.uint64), off_o), "segment counts differ"
    sg = segs[: int(off_o[-1])].cpu().numpy()
    assert np.array_equal(sg[:, 0].astype(np.uint32), sr)
    assert np.array_equal(sg[:, 1].astype(np.uint32), sl)
    assert np.array_equal(sg[:, 2].view(np.float32), t0)
    assert np.array_equal(sg[:, 3].view(np.float32), t1)
    st = m.read_state()
    assert st["last_n_segments"] == int(off_o[-1]) and st["flags"] == 0
    return int(off_o[-1])


@pytest.mark.parametrize("mode", TRAVERSE_MODES)
def test_traverse_bitexact_c1(lib, c1, mode):
    sc, rays = c1
    _say("traverse c1: 65536 camera rays, 64 leaves, mode", mode)
    n = _check_traverse(lib, rays, sc.boxes, sc.lo, sc.side, configs.C1_NET, mode)
    assert n > 30000


@pytest.mark.parametrize("mode", TRAVERSE_MODES)
def test_traverse_tiny_scenes(lib, mode):
    rng = np.random.default_rng(5)
    net = configs.C1_NET
    # 1 leaf, 2 overlapping leaves, 7 leaves (ragged tree), with axis-aligned and grazing rays
    for boxes in (np.array([[0, 0, 0, 1, 1, 1]], np.float32),
                  np.array([[0, 0, 0, 1, 1, 1], [0.5, 0.25, 0.5, 1.5, 0.75, 2.0]], np.float32),
                  np.concatenate([rng.uniform(-1, 0, (7, 3)), rng.uniform(0.1, 1, (7, 3))], 1).astype(np.float32)):
        _say("traverse tiny scene with", boxes.shape[0], "leaves, mode", mode)
        n = 3000
        rays = np.zeros((n, 8), np.float32)
        rays[:, 0:3] = rng.uniform(-3, 3, (n, 3))
        d = rng.normal(size=(n, 3))
        k = rng.integers(0, 3, n)
        axis = rng.uniform(size=n) < 0.3
        d[axis] = 0.0
        d[axis, k[axis]] = rng.choice([-1.0, 1.0], axis.sum())
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rays[:, 4:7] = d
        rays[:, 7] = np.where(rng.uniform(size=n) < 0.2, 2.0, np.inf)
        # grazing: origins on box faces/edges, axis directions
        g = rng.integers(0, n, 200)
        rays[g, 0:3] = boxes[0, [0, 4, 2]]
        rays[g, 4:7] = [1.0, 0.0, 0.0]
        _check_traverse(lib, rays, boxes, boxes[:, :3].min(0), np.float32(4.0), net, mode)


@pytest.mark.parametrize("mode", TRAVERSE_MODES)
def test_traverse_many_overlapping_leaves(lib, mode):
    """Rays crossing up to 40 leaves: longer runs than the counting pass
    keeps sorted per ray, so the fill walks the tree again for them."""
    rng = np.random.default_rng(6)
    lo = rng.uniform(-1.0, -0.2, (40, 3))
    hi = rng.uniform(0.2, 1.0, (40, 3))
    boxes = np.concatenate([lo, hi], 1).astype(np.float32)
    n = 4000 + 17
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = rng.uniform(-3, 3, (n, 3))
    d = -rays[:, 0:3] + rng.uniform(-0.3, 0.3, (n, 3))
    rays[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    rays[:, 7] = np.inf
    _say("traverse 40 overlapping leaves, mode", mode)
    total = _check_traverse(lib, rays, boxes, boxes[:, :3].min(0), np.float32(4.0), configs.C1_NET, mode)
    assert total > 20 * n


def test_traverse_capacity_flag(lib, c1):
    sc, rays = c1
    m = lib.NBVH(configs.C1_NET, sc.boxes, sc.lo, sc.side, precision="fp32")
    _say("traverse with too small segment capacity")
    off, segs = m.traverse(torch.from_numpy(rays).cuda(), 100)
    st = m.read_state()
    assert st["flags"] & 1
    off_o, *_ = oracle.traverse(rays[:2000], sc.boxes)
    assert np.array_equal(off.cpu().numpy()[:2001].astype(np.uint64), off_o)


# ------------------------------------------------------------------ encode / forward
NETS = {
    # c1-shaped: 8 levels (2 dense), 4 samples, 64 -> 3x64 -> 5
    "c1": configs.C1_NET,
    # c2-shaped: 16 levels (5 dense), 8 samples, 256 -> 4x128 -> 5
    "c2": configs.C2_NET,
    # F = 4, hashed fine levels, width 32 (smallest tile shapes)
    "f4": _net(8, 4, 12, 4, [4, 6, 9, 14, 21, 32, 48, 72], 32, 2, 8),
    # the secondary-ray workload's network (16 levels, F = 4, 4 samples,
    # 256 -> 4x256 -> 8 with albedo) on a 2^16-entry table
    "c5": configs.NetConfig(16, 4, 16, 4, 16, 1.38, 256, 4, 8),
}


def _probes(sc, n, seed):
    p, _ = scene.leaf_probes(sc.boxes, max(1, n // sc.boxes.shape[0] + 1), seed=seed)
    rng = np.random.default_rng(seed)
    return p[rng.permutation(p.shape[0])[:n]]


@pytest.mark.parametrize("name", ["c1", "c2", "f4", "c5"])
def test_encode_fp32(lib, c1, name):
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_params(params)
    probes = _probes(sc, 3001, 7)
    _say("encode fp32", name, probes.shape)
    u = m.encode(torch.from_numpy(probes).cuda()).cpu().numpy()
    ref = oracle.encode(_ocfg(net, sc), params[: net.n_table_params].astype(np.float64), probes)
    r = _rel_inf(u.astype(np.float64), ref)
    assert r.max() <= 1e-5, r.max()


@pytest.mark.parametrize("name", ["c1", "c2", "f4", "c5"])
def test_encode_bf16_table(lib, c1, name):
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(params)
    probes = _probes(sc, 2000, 8)
    _say("encode bf16", name)
    u = m.encode(torch.from_numpy(probes).cuda()).cpu().numpy()
    ref = oracle.encode(_ocfg(net, sc), _bf16_round(params[: net.n_table_params]).astype(np.float64), probes)
    r = _rel_inf(u.astype(np.float64), ref)
    assert r.max() <= 1e-5, r.max()


@pytest.mark.parametrize("name", ["c1", "c2", "f4", "c5"])
def test_forward_fp32(lib, c1, name):
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_params(params)
    probes = _probes(sc, 1000 + 37, 9)
    _say("forward fp32", name)
    z = m.forward(torch.from_numpy(probes).cuda()).cpu().numpy()
    ref = oracle.forward(_ocfg(net, sc), params.astype(np.float64), probes)
    r = _rel_inf(z.astype(np.float64), ref)
    assert r.max() <= 1e-5, r.max()


@pytest.mark.parametrize("name", ["c1", "c2", "f4", "c5"])
def test_forward_bf16(lib, c1, name):
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(params)
    probes = _probes(sc, 1000 + 37, 10)
    _say("forward bf16", name)
    z = m.forward(torch.from_numpy(probes).cuda()).cpu().numpy().astype(np.float64)
    ref = oracle.forward(_ocfg(net, sc), _bf16_round(params).astype(np.float64), probes)
    err = np.abs(z - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2e-2, err.max()


# ------------------------------------------------------------------ query
def _check_query(lib, net, sc, rays, precision, params):
    """Query through nbvh_query against the oracle's query. A ray is clear
    when no hit decision (|z0| within the tolerance on z) and no distance
    tie between its winner and another hit segment can go either way under
    the output tolerance: FP32 1e-5 of the segment's max |z|, BF16
    2e-2 max(1, |z|)."""
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision=precision)
    m.set_params(params)
    _say("query", precision, rays.shape)
    hits = m.query(torch.from_numpy(rays).cuda()).cpu().numpy()
    leaf = leaf_of(hits)
    pref = params if precision == "fp32" else _bf16_round(params)
    out, tr, z = oracle.query(_ocfg(net, sc), pref.astype(np.float64), rays, sc.boxes)
    if precision == "fp32":
        ztol = 1e-5 * np.repeat(np.abs(z).max(1, keepdims=True), net.n_out, 1)
    else:
        ztol = 2e-2 * np.maximum(1.0, np.abs(z))
    ok = clear_rays(tr, z, out, rays[:, 3], ztol)
    agree = leaf[ok] == out[ok, 4].astype(np.int64)
    return m, hits, out, ok, agree, tr, z


def test_query_fp32_c1(lib, c1):
    sc, rays = c1
    net = configs.C1_NET
    params = _params(net, scale=1.0)
    m, hits, out, ok, agree, tr, z = _check_query(lib, net, sc, rays, "fp32", params)
    assert ok.mean() > 0.9
    assert agree.all(), agree.mean()
    both = ok & (out[:, 4] >= 0)
    same = both & (leaf_of(hits) == out[:, 4].astype(np.int64))
    assert same.sum() > 1000
    dt = np.abs(hits[same, 0] - out[same, 0]) / np.maximum(1.0, np.abs(out[same, 0]))
    assert dt.max() <= 1e-5, dt.max()
    zseg = np.abs(z[out[same, 5].astype(np.int64)]).max(1)  # per-segment ||z||_inf
    dn = np.abs(hits[same, 1:4] - out[same, 1:4]).max(1) / zseg
    assert dn.max() <= 1e-5, dn.max()
    miss = ok & (out[:, 4] < 0)
    assert np.all(hits[miss, 7].view(np.uint32) == 0xFFFFFFFF)


def test_query_bf16_c1(lib, c1):
    sc, rays = c1
    net = configs.C1_NET
    params = _params(net, scale=1.0)
    m, hits, out, ok, agree, tr, z = _check_query(lib, net, sc, rays, "bf16", params)
    assert ok.mean() > 0.5, ok.mean()
    assert agree.all(), agree.mean()
    same = ok & (out[:, 4] >= 0) & (leaf_of(hits) == out[:, 4].astype(np.int64))
    diag = sc.diagonal
    dt = np.abs(hits[same, 0] - out[same, 0])
    assert dt.mean() <= 1e-3 * diag, dt.mean()


# ------------------------------------------------------------------ loss / backward / optimiser
def _clear_of_kinks(net, sc, params, probes, n, margin):
    """The first n probes whose hidden pre-activations (oracle) all stay
    more than `margin` away from 0, where the ReLU mask is decided."""
    keep = oracle.min_abs_preact(_ocfg(net, sc), params.astype(np.float64), probes) > margin
    sel = probes[keep][:n]
    assert sel.shape[0] == n
    return sel


def _labels_for(sc, probes):
    return scene.probe_labels(sc.mesh, probes)


def test_loss_matches_oracle(lib, c1):
    sc, _ = c1
    net = configs.C1_NET
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    probes = _probes(sc, 5000, 11)
    lab = _labels_for(sc, probes)
    rng = np.random.default_rng(12)
    z = rng.normal(size=(5000, 5)).astype(np.float32)
    _say("loss")
    loss, dz = m.loss(torch.from_numpy(z).cuda(), torch.from_numpy(lab).cuda())
    terms, dzo = oracle.loss(_ocfg(net, sc), z.astype(np.float64), lab)
    assert np.allclose(loss.cpu().numpy(), terms, rtol=1e-5, atol=1e-7)
    assert np.abs(dz.cpu().numpy() - dzo).max() <= 1e-5 * np.abs(dzo).max()


@pytest.mark.parametrize("name", ["c1", "c2", "f4", "c5"])
def test_backward_fp32(lib, c1, name):
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1.0)
    m.set_params(params)
    n = 1000 + 37
    probes = _clear_of_kinks(net, sc, params, _probes(sc, 2 * n, 13), n, 1e-4)
    rng = np.random.default_rng(14)
    dz = (rng.normal(size=(n, net.n_out)) / n).astype(np.float32)
    _say("backward fp32", name)
    m.backward(torch.from_numpy(probes).cuda(), torch.from_numpy(dz).cuda())
    g = m.unpad(m.grad)
    ref = oracle.backward(_ocfg(net, sc), params.astype(np.float64), probes, dz.astype(np.float64))
    nt = net.n_table_params
    gw, rw = g[nt:], ref[nt:]
    assert np.abs(gw - rw).max() <= 1e-4 * np.abs(rw).max(), np.abs(gw - rw).max() / np.abs(rw).max()
    gt, rt = g[:nt], ref[:nt]
    assert np.abs(gt - rt).max() <= 1e-5 * np.abs(rt).max(), np.abs(gt - rt).max() / np.abs(rt).max()


SCATTER_PATHS = {
    "pairs": dict(scatter_lds_kb=0, scatter_hash_levels=0, scatter_binned=0),
    "binned": dict(scatter_lds_kb=144, scatter_hash_levels=0, scatter_binned=1),
    # every level through the LDS hash: fine levels overflow the table and
    # take the direct-atomic fallback
    "hash_all": dict(scatter_lds_kb=0, scatter_hash_levels=32, scatter_binned=0),
    "mixed": dict(scatter_lds_kb=144, scatter_hash_levels=4, scatter_binned=1),
}


@pytest.mark.parametrize("path", sorted(SCATTER_PATHS))
@pytest.mark.parametrize("order", ["by_leaf", "shuffled"])
def test_table_gradient_scatter_paths(lib, c1, path, order):
    """Every table-gradient route (LDS levels, per-tile LDS hash, binned
    counting sort, coalesced atomics) gives the oracle's table gradient, with
    probes grouped by leaf (repeated corners) and shuffled."""
    sc, _ = c1
    net = NETS["c2"]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1.0)
    m.set_params(params)
    m.set_tuning(**SCATTER_PATHS[path])
    p, _ = scene.leaf_probes(sc.boxes, 40, seed=17)  # grouped by leaf
    if order == "shuffled":
        p = p[np.random.default_rng(18).permutation(p.shape[0])]
    n = p.shape[0]
    dz = (np.random.default_rng(19).normal(size=(n, net.n_out)) / n).astype(np.float32)
    _say("scatter path", path, order, n)
    m.backward(torch.from_numpy(p).cuda(), torch.from_numpy(dz).cuda())
    g = m.unpad(m.grad)[: net.n_table_params]
    ref = oracle.backward(_ocfg(net, sc), params.astype(np.float64), p, dz.astype(np.float64))[: net.n_table_params]
    assert np.abs(g - ref).max() <= 1e-5 * np.abs(ref).max(), np.abs(g - ref).max() / np.abs(ref).max()


def test_bf16_gradient_records(lib, c1):
    """On the BF16 path the binned levels' contributions travel as 8-byte
    records, each value rounded to a 24-bit float (at most 2^-16 relative).
    Every level binned against every level summed from the FP32 contributions
    (LDS hash, then direct atomics), on the same BF16 forward: the table
    gradients differ only by that rounding and FP32 summation order, far
    inside the BF16 path's own 2e-2 bound."""
    sc, _ = c1
    net = NETS["c2"]
    params = _params(net, scale=1.0)
    p, _ = scene.leaf_probes(sc.boxes, 40, seed=17)
    n = p.shape[0]
    dz = (np.random.default_rng(19).normal(size=(n, net.n_out)) / n).astype(np.float32)
    nt = net.n_table_params
    routes = {"records": dict(scatter_lds_kb=0, scatter_hash_levels=0, scatter_binned=1),
              "fp32 sums": dict(scatter_lds_kb=0, scatter_hash_levels=32, scatter_binned=0)}
    g = {}
    for name, knobs in routes.items():
        m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1024.0)
        m.set_params(params)
        m.set_tuning(**knobs)
        m.backward(torch.from_numpy(p).cuda(), torch.from_numpy(dz).cuda())
        g[name] = m.unpad(m.unscaled_grad())[:nt]
    a, b = g["records"], g["fp32 sums"]
    err = float(np.abs(a - b).max() / np.abs(b).max())
    _say("bf16 table gradient, 8-byte records vs FP32 sums: max |dg| / max |g| = %.3g" % err)
    assert np.abs(b).max() > 0
    assert err <= 2e-4, err


def _blocks(net):
    """(name, slice) of each parameter block of the unpadded layout."""
    out = [("table", slice(0, net.n_table_params))]
    o = net.n_table_params
    for k, (fi, fo) in enumerate(net.layer_dims()):
        out.append(("W%d" % k, slice(o, o + fi * fo)))
        o += fi * fo
    return out


def _check_bf16_grad(lib, net, sc, params, probes, seed, bound):
    """BF16 back-propagation (BF16 activations, weights and gradients on the
    matrix cores, FP32 accumulation) against the oracle's FP64 gradient of the
    BF16-rounded parameters, element by element: |dg| <= bound * max|g| of
    each block (table, W_0 .. W_H)."""
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1024.0)
    m.set_params(params)
    n = probes.shape[0]
    dz = (np.random.default_rng(seed).normal(size=(n, net.n_out)) / n).astype(np.float32)
    m.backward(torch.from_numpy(probes).cuda(), torch.from_numpy(dz).cuda())
    g = m.unpad(m.unscaled_grad())
    ref = oracle.backward(_ocfg(net, sc), _bf16_round(params).astype(np.float64), probes, dz.astype(np.float64))
    worst = {}
    for name, sl in _blocks(net):
        a, b = g[sl], ref[sl]
        worst[name] = float(np.abs(a - b).max() / np.abs(b).max())
    _say("bf16 gradient, worst |dg| / max|g| per block:", worst)
    for name, w in worst.items():
        assert w <= bound, (name, w)


@pytest.mark.parametrize("name", ["c1", "c2", "f4", "c5"])
def test_backward_bf16_active_units(lib, c1, name):
    """Every hidden unit active on every probe (positive features and
    weights), so no ReLU decision depends on rounding: the whole batch's
    gradient is compared element by element."""
    sc, _ = c1
    net = NETS[name]
    params = np.abs(_params(net, scale=1.0)).astype(np.float32)
    params[: net.n_table_params] += np.float32(0.05)
    n = 2048 + 5
    probes = _probes(sc, n, 15)
    assert oracle.min_abs_preact(_ocfg(net, sc), _bf16_round(params).astype(np.float64), probes).min() > 0.05
    _say("backward bf16 (all units active)", name)
    _check_bf16_grad(lib, net, sc, params, probes, 16, 2e-2)


# margin above the largest change BF16 activations make to a hidden
# pre-activation of these networks (about 3.6e-3 at their widths with U(-1, 1)
# features), and the candidate pool that leaves enough probes clear of it
KINK_CLEAR = {"c1": (6e-3, 40000, 1024), "f4": (6e-3, 4000, 1024), "c2": (4e-3, 409600, 160)}


@pytest.mark.parametrize("name", sorted(KINK_CLEAR))
def test_backward_bf16_kink_clear(lib, c1, name):
    """Mixed-sign network: probes whose hidden pre-activations (oracle, BF16
    parameters) all clear 0 by more than BF16 activations can move them, so
    both sides take the same ReLU decisions; gradient element by element."""
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    margin, pool, want = KINK_CLEAR[name]
    cand = _probes(sc, pool, 21)
    keep = oracle.min_abs_preact(_ocfg(net, sc), _bf16_round(params).astype(np.float64), cand) > margin
    probes = cand[keep][:want]
    assert probes.shape[0] >= min(want, 150), probes.shape[0]
    _say("backward bf16 (kink-clear probes)", name, probes.shape[0])
    _check_bf16_grad(lib, net, sc, params, probes, 22, 2e-2)


def test_optimizer_same_gradient(lib, c1):
    """Adam on the GPU vs the oracle's Adam fed the same gradient."""
    sc, _ = c1
    net = configs.C1_NET
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=8.0)
    m.set_params(params)
    rng = np.random.default_rng(17)
    g1 = rng.normal(size=params.size) * np.logspace(-5, 0, params.size)
    g2 = rng.normal(size=params.size)
    p64 = params.astype(np.float64)
    mm, vv = np.zeros_like(p64), np.zeros_like(p64)
    for step, g in ((1, g1), (2, g2)):
        gp = torch.zeros(m.n_params)
        gp_np = gp.numpy()
        gp_np[: m.n_table] = g[: m.n_table] * 8.0
        src = m.n_table
        for k, (fi, fo) in enumerate(m.layer_dims()):
            gp_np[m.offsets[1 + k]: m.offsets[1 + k] + fi * fo] = g[src: src + fi * fo] * 8.0
            src += fi * fo
        m.grad.copy_(gp.cuda())
        _say("optimizer step", step)
        m.optimizer_step()
        oracle.adam(p64, g.astype(np.float32).astype(np.float64) * 8.0, mm, vv, step, 1e-2, 0.9, 0.99, 1e-8, 1.0 / 8.0)
        got = m.get_params()
        assert np.abs(got - p64).max() <= 1e-6, np.abs(got - p64).max()
    assert m.read_state()["step"] == 2
    assert float(m.grad.abs().max()) == 0.0
    lp = m.unpad(m.params_lp.float())
    assert np.array_equal(lp, _bf16_round(m.get_params()))


def test_nonfinite_gradient_skips_step(lib, c1):
    sc, _ = c1
    net = configs.C1_NET
    params = _params(net)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1024.0)
    m.set_params(params)
    g = torch.zeros(m.n_params, device="cuda")
    g[5] = float("inf")
    m.grad.copy_(g)
    _say("non-finite gradient step")
    m.optimizer_step()
    st = m.read_state()
    assert st["skipped"] == 1 and st["step"] == 0 and st["loss_scale"] == 512.0 and (st["flags"] & 2)
    assert np.array_equal(m.get_params(), params)


def _with_albedo(lab, seed):
    """Labels with random albedo on hit segments (the synthetic mesh of these
    tests carries none)."""
    lab = lab.copy()
    alb = np.random.default_rng(seed).uniform(0.05, 0.95, size=(lab.shape[0], 3)).astype(np.float32)
    lab[:, 5:8] = np.where(lab[:, 4:5] > 0, alb, 0.0)
    return lab


def test_loss_with_albedo_matches_oracle(lib, c1):
    """Eight outputs: the relative-L2 albedo term and its gradient."""
    sc, _ = c1
    net = NETS["f4"]
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    probes = _probes(sc, 3000 + 7, 19)
    lab = _with_albedo(_labels_for(sc, probes), 20)
    z = np.random.default_rng(21).normal(size=(probes.shape[0], 8)).astype(np.float32)
    _say("loss with albedo")
    loss, dz = m.loss(torch.from_numpy(z).cuda(), torch.from_numpy(lab).cuda())
    terms, dzo = oracle.loss(_ocfg(net, sc), z.astype(np.float64), lab)
    assert np.allclose(loss.cpu().numpy(), terms, rtol=1e-5, atol=1e-7)
    assert np.abs(dz.cpu().numpy() - dzo).max() <= 1e-5 * np.abs(dzo).max()
    assert np.abs(dzo[:, 5:8]).max() > 0


@pytest.mark.parametrize("name", ["c1", "f4"])
def test_train_step_matches_oracle_fp32(lib, c1, name):
    """One full training step (forward, loss, backward, Adam) in FP32 vs the
    oracle's step; Adam's first update is -lr*sign(g) where |g| >> eps, so
    parameters are compared where the oracle gradient is clear of zero. The
    f4 network has eight outputs, so the albedo term trains too."""
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1.0)
    m.set_params(params)
    n = 4096 + 100
    probes = _clear_of_kinks(net, sc, params, _probes(sc, 2 * n, 18), n, 1e-4)
    lab = _labels_for(sc, probes)
    if net.n_out >= 8:
        lab = _with_albedo(lab, 22)
    _say("train step fp32", name)
    loss = m.train_step(torch.from_numpy(probes).cuda(), torch.from_numpy(lab).cuda()).cpu().numpy()
    cfg = _ocfg(net, sc)
    p64 = params.astype(np.float64)
    z = oracle.forward(cfg, p64, probes)
    terms, dz = oracle.loss(cfg, z, lab)
    g = oracle.backward(cfg, p64, probes, dz)
    assert np.allclose(loss, terms, rtol=1e-5, atol=1e-7), (loss, terms)
    mm, vv = np.zeros_like(p64), np.zeros_like(p64)
    oracle.adam(p64, g, mm, vv, 1)
    got = m.get_params()
    clear = np.abs(g) > 1e-3 * np.abs(g).max()
    assert clear.sum() > 1000
    assert np.abs(got[clear] - p64[clear]).max() <= 1e-6
