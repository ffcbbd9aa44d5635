"""Edge cases through the C ABI: empty inputs, rays that miss everything, a
single-leaf scene, segment-queue overflow, and the largest network shapes
the library accepts (32 levels x 2 features x 8 samples = 512 inputs,
8 hidden layers of 256, 16 outputs)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nbvh_synth import configs, scene

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
    return configs.make_scene(20480, 64)


def test_empty_inputs(lib, c1):
    sc = c1
    m = lib.NBVH(configs.C1_NET, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(configs.init_params(configs.C1_NET))
    none = torch.zeros((0, 8), dtype=torch.float32, device="cuda")
    _say("empty inputs")
    assert m.query(none).shape == (0, 8)
    off, _ = m.traverse(none, 16)
    assert off.cpu().tolist() == [0]
    assert m.forward(none).shape == (0, configs.C1_NET.n_out)
    assert m.encode(none).shape[0] == 0
    p, lf = m.first_hits(none, torch.zeros(0, device="cuda"), torch.ones(64, device="cuda"))
    assert p.shape[0] == 0 and lf.shape[0] == 0
    with pytest.raises(lib.NbvhError):
        m.train_step(none, none)
    batch = lib.NBVHBatch([m])
    assert batch.query(none).shape == (0, 8)
    torch.cuda.synchronize()
    assert m.read_state()["flags"] == 0


def test_rays_that_miss_and_single_leaf(lib, c1):
    sc = c1
    net = configs.C1_NET
    params = configs.init_params(net, "uniform", 1.0, seed_features=30, seed_mlp=31)
    # every ray points away from the scene
    rays = scene.pinhole_rays(64, 64, eye=(0.0, 0.0, 3.0), target=(0.0, 0.0, 6.0))
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_params(params)
    _say("rays that miss every leaf")
    h = m.query(torch.from_numpy(rays).cuda()).cpu().numpy()
    assert np.all(h[:, 7].view(np.uint32) == 0xFFFFFFFF) and np.all(h[:, :7] == 0)
    off, _ = m.traverse(torch.from_numpy(rays).cuda(), 16)
    assert np.all(off.cpu().numpy() == 0)
    # one leaf: the whole scene box
    box = np.concatenate([sc.boxes[:, :3].min(0), sc.boxes[:, 3:].max(0)])[None, :].astype(np.float32)
    m1 = lib.NBVH(net, box, sc.lo, sc.side, precision="fp32")
    m1.set_params(params)
    rays = scene.pinhole_rays(96, 96)
    _say("single leaf query")
    h = m1.query(torch.from_numpy(rays).cuda()).cpu().numpy()
    out, tr, z = oracle.query(oracle.make_cfg(net, sc.lo, sc.side), params.astype(np.float64), rays, box)
    clear = np.ones(rays.shape[0], bool)
    clear[np.unique(tr[1][np.abs(z[:, 0]) <= 1e-4 * np.maximum(1.0, np.abs(z[:, 0]))])] = False
    leaf = h[:, 7].view(np.uint32).astype(np.int64)
    leaf[leaf == 0xFFFFFFFF] = -1
    assert (leaf[clear] == out[clear, 4]).mean() >= 0.999
    hit = clear & (out[:, 4] >= 0)
    assert np.abs(h[hit, 0] - out[hit, 0]).max() <= 1e-5 * max(1.0, np.abs(out[hit, 0]).max())


def test_query_segment_overflow_is_flagged(lib, c1):
    sc = c1
    m = lib.NBVH(configs.C1_NET, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(configs.init_params(configs.C1_NET))
    rays = torch.from_numpy(scene.pinhole_rays(128, 128)).cuda()
    _say("query with a too small segment queue")
    m.query(rays, seg_capacity=100)
    torch.cuda.synchronize()
    assert m.read_state()["flags"] & 1
    m.clear_flags()
    m.query(rays)
    torch.cuda.synchronize()
    assert m.read_state()["flags"] == 0


MAX_NET = configs.NetConfig(32, 2, 14, 8, 4, 1.15, 256, 8, 16)


def test_largest_network_bf16(lib, c1):
    """512 inputs, 8 x 256 hidden, 16 outputs: BF16 forward against the
    oracle on BF16-rounded parameters, and a training step that stays finite."""
    sc = c1
    net = MAX_NET
    assert net.n_in == 512
    params = configs.init_params(net, "uniform", 0.5, seed_features=32, seed_mlp=33)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(params)
    probes, _ = scene.leaf_probes(sc.boxes, 10, seed=34)
    _say("largest network forward", probes.shape)
    z = m.forward(torch.from_numpy(probes).cuda()).cpu().numpy().astype(np.float64)
    pb = torch.from_numpy(params).to(torch.bfloat16).float().numpy().astype(np.float64)
    ref = oracle.forward(oracle.make_cfg(net, sc.lo, sc.side), pb, probes)
    err = np.abs(z - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2e-2, err.max()
    lab = scene.probe_labels(sc.mesh, probes)
    loss = m.train_step(torch.from_numpy(probes).cuda(), torch.from_numpy(lab).cuda())
    torch.cuda.synchronize()
    assert torch.isfinite(loss).all() and m.read_state()["skipped"] == 0


def test_largest_network_fp32_is_refused(lib, c1):
    """In FP32 the 64-row activation tiles of the largest network need more
    than a CU's 160 KiB of LDS: the call fails with a clear error."""
    sc = c1
    m = lib.NBVH(MAX_NET, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_params(configs.init_params(MAX_NET))
    probes, _ = scene.leaf_probes(sc.boxes, 2, seed=35)
    with pytest.raises(lib.NbvhError, match="LDS"):
        m.forward(torch.from_numpy(probes).cuda())


def test_batch_beyond_record_indices_is_refused(lib, c1):
    """The binned table-gradient pass places its records with 32-bit indices:
    a batch that would need more than 2^32 of them is refused before any
    launch, by the training step and by the plain backward pass."""
    from paper_2405_16237_amd import _abi
    sc = c1
    net = configs.C1_NET
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(configs.init_params(net))
    m.set_tuning(scatter_lds_kb=0, scatter_hash_levels=1, scatter_binned=1)
    n = 1 << 25  # x (L - 1) binned levels x S samples x 8 corners > 2^32
    assert n * (net.n_levels - 1) * net.n_samples * 8 > (1 << 32)
    probes = torch.zeros((64, 10), dtype=torch.float32, device="cuda")  # never read
    labels = torch.zeros((64, 5), dtype=torch.float32, device="cuda")
    dz = torch.zeros((64, net.n_out), dtype=torch.float32, device="cuda")
    ws = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    _say("record-index limit", n)
    st = m.lib.nbvh_train_step(m.ctx, probes.data_ptr(), labels.data_ptr(), n, None, ws.data_ptr(), ws.numel(), None)
    assert st == _abi.NBVH_ERR_UNSUPPORTED and "2^32" in m.lib.nbvh_last_error().decode()
    st = m.lib.nbvh_backward(m.ctx, probes.data_ptr(), n, dz.data_ptr(), ws.data_ptr(), ws.numel(), None)
    assert st == _abi.NBVH_ERR_UNSUPPORTED and "2^32" in m.lib.nbvh_last_error().decode()
    torch.cuda.synchronize()
    st = m.read_state()
    assert st["step"] == 0 and st["flags"] == 0


@pytest.mark.parametrize("precision,log2_T,kb", [("bf16", 14, 24), ("fp32", 14, 64), ("fp8", 14, 24),
                                                 ("bf16", 10, 64), ("fp32", 10, 64)])
def test_query_with_levels_staged_in_lds(lib, c1, precision, log2_T, kb):
    """Gathering the table's leading levels from a workgroup's LDS copy gives
    the same hit records, bit for bit, as gathering them from global memory:
    the first (dense) level of a 2^14 table, and every level of a 2^10 table
    (all hashed, the copy ending at the table's end)."""
    sc = c1
    net = configs.NetConfig(8, 2, log2_T, 4, 16, 1.5, 64, 3, 5)
    pb = 4 if precision == "fp32" else 2
    ends = np.cumsum(net.level_sizes()) * net.n_features * pb
    staged = int((ends <= kb * 1024).sum())
    assert staged == (1 if log2_T == 14 else net.n_levels)
    params = configs.init_params(net, "uniform", 1.0, seed_features=36, seed_mlp=37)
    w_out = params.size - net.n_out * net.mlp_width
    params[w_out:w_out + net.mlp_width] *= -1.0  # mostly hits, so t and normals are compared too
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision=precision)
    m.set_params(params)
    if precision == "fp8":
        p, _ = scene.leaf_probes(sc.boxes, 8, seed=38)
        m.calibrate_fp8(torch.from_numpy(p).cuda())
    rays = torch.from_numpy(scene.pinhole_rays(160, 120)).cuda()
    _say("staged levels", precision, log2_T, kb, staged)
    ref = m.query(rays).clone().view(torch.int32)
    assert (ref[:, 7] != -1).sum() > 1000
    m.set_tuning(query_lds_kb=kb)
    got = m.query(rays).view(torch.int32)
    assert torch.equal(got, ref)
    m.set_tuning(query_lds_kb=kb, query_waves=4, query_unroll=3)
    got = m.query(rays).view(torch.int32)
    assert torch.equal(got, ref)


def test_query_lds_kb_is_validated(lib, c1):
    """The LDS budget for staged coarse levels is 0..64 KiB; other values are
    refused and leave the knobs as they were."""
    sc = c1
    m = lib.NBVH(configs.C1_NET, sc.boxes, sc.lo, sc.side, precision="bf16")
    before = m.get_tuning()
    for bad in (-1, 65, 1024):
        with pytest.raises(lib.NbvhError, match="query_lds_kb"):
            m.set_tuning(query_lds_kb=bad)
    assert m.get_tuning() == before
    m.set_tuning(query_lds_kb=64)
    assert m.get_tuning()["query_lds_kb"] == 64


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [64, 2112])
def test_wgrad_splits_cover_the_batch(lib, c1, precision, n):
    """The weight-gradient GEMMs split the batch over wgrad_splits
    workgroups; every split count the tuning accepts must cover every probe
    (65 does not divide a padded batch, 128 and 256 exceed a 64-probe batch's
    32-entry steps), so the gradient equals the default split's and, in FP32,
    the oracle's."""
    sc = c1
    net = configs.C1_NET
    params = configs.init_params(net, "uniform", 0.5)
    p, _ = scene.leaf_probes(sc.boxes, 2 * n // 64 + 1, seed=41)
    # probes whose hidden pre-activations stay clear of the ReLU kink, where
    # FP32 and FP64 could take different 0/1 derivatives
    cfg = oracle.make_cfg(net, sc.lo, sc.side)
    p = p[oracle.min_abs_preact(cfg, params.astype(np.float64), p) > 1e-4][:n]
    assert p.shape[0] == n
    dz = (np.random.default_rng(42).normal(size=(n, net.n_out)) / n).astype(np.float32)
    grads = {}
    for splits in (64, 65, 128, 256):
        m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision=precision, loss_scale=1.0)
        m.set_params(params)
        m.set_tuning(wgrad_splits=splits)
        _say("wgrad splits", precision, n, splits)
        m.backward(torch.from_numpy(p).cuda(), torch.from_numpy(dz).cuda())
        grads[splits] = m.unpad(m.grad)[net.n_table_params:].astype(np.float64)
    ref = grads[64]
    assert np.abs(ref).max() > 0
    for splits in (65, 128, 256):
        err = np.abs(grads[splits] - ref).max() / np.abs(ref).max()
        assert err <= 1e-5, (splits, err)
    if precision == "fp32":
        o = oracle.backward(cfg, params.astype(np.float64), p, dz.astype(np.float64))[net.n_table_params:]
        for splits, g in grads.items():
            kept = np.abs(g - o).max() / np.abs(o).max()
            assert kept <= 1e-4, (splits, kept)


@pytest.mark.parametrize("order", [1, 2])
def test_ray_order_edge_inputs(lib, c1, order):
    """Ray orders on awkward inputs: no rays, one ray, a count that is not a
    multiple of a workgroup, every origin equal (all keys equal: the stable
    sort keeps the caller's order), and origins at infinity (which stretch the
    origins' box; their keys clamp to a cell) all answer as the caller's order
    does, in the single-object and the grouped query."""
    sc = c1
    m = lib.NBVH(configs.C1_NET, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(configs.init_params(configs.C1_NET, "uniform", 1.0, seed_features=71, seed_mlp=72))
    cam = scene.pinhole_rays(128, 96)
    rng = np.random.default_rng(73)
    odd = cam[rng.permutation(cam.shape[0])[:1001]].copy()
    odd[:5, 0:3] = np.array([np.inf, -np.inf, np.inf], np.float32)  # these miss every box
    sets = {"none": cam[:0], "one": cam[6000:6001], "odd": odd, "same origin": cam[:777]}
    batch = lib.NBVHBatch([m])
    for name, rays_np in sets.items():
        _say("ray order", order, name, rays_np.shape[0], "rays")
        rays = torch.from_numpy(np.ascontiguousarray(rays_np)).cuda()
        m.set_tuning(query_order=0)
        ref = m.query(rays).cpu().numpy().view(np.uint32)
        bref = batch.query(rays).cpu().numpy().view(np.uint32)
        m.set_tuning(query_order=order)
        got = m.query(rays).cpu().numpy().view(np.uint32)
        bgot = batch.query(rays).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref) and np.array_equal(bgot, bref), name
    assert m.read_state()["flags"] == 0
