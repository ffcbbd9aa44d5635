"""Error-driven construction through the C ABI: first-hit training-ray
selection and per-leaf losses against the oracle, then a small construction
run (Sec. 5.1) on the 20,480-triangle mesh."""
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


def _box_rays(sc, n, seed):
    """Rays uniform in the 50 %-inflated scene box, uniform directions."""
    rng = np.random.default_rng(seed)
    lo = sc.boxes[:, :3].min(0).astype(np.float64)
    hi = sc.boxes[:, 3:].max(0).astype(np.float64)
    ext = hi - lo
    r = np.zeros((n, 8), dtype=np.float32)
    r[:, 0:3] = lo - 0.25 * ext + rng.uniform(size=(n, 3)) * 1.5 * ext
    d = rng.normal(size=(n, 3))
    r[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    r[:, 7] = np.inf
    return r


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_first_hits_match_oracle(lib, c1, mode):
    sc = c1
    m = lib.NBVH(configs.C1_NET, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_tuning(traverse_mode=mode)
    rays = _box_rays(sc, 50_000 + 33, 71)
    rng = np.random.default_rng(72)
    u = rng.uniform(size=rays.shape[0]).astype(np.float32)
    accept = rng.uniform(0.0, 1.0, size=sc.boxes.shape[0]).astype(np.float32)
    accept[:5] = 1.0
    accept[5:8] = 0.0
    hits = torch.zeros(sc.boxes.shape[0], dtype=torch.int32, device="cuda")
    _say("first hits", rays.shape, "mode", mode)
    probes, leaf = m.first_hits(torch.from_numpy(rays).cuda(), torch.from_numpy(u).cuda(),
                                torch.from_numpy(accept).cuda(), leaf_hits=hits)
    ray, oleaf, t0, t1, ohits = oracle.first_hits(rays, sc.boxes, u, accept)
    assert np.array_equal(hits.cpu().numpy(), ohits)
    p = probes.cpu().numpy()
    lf = leaf.cpu().numpy()
    assert p.shape[0] == ray.size > 1000
    # order is unspecified: sort both by (origin, direction) bits
    key_g = np.lexsort(p.view(np.int32).T[::-1])
    ref = np.zeros((ray.size, 8), dtype=np.float32)
    ref[:, 0:3] = rays[ray, 0:3]
    ref[:, 3] = t0
    ref[:, 4:7] = rays[ray, 4:7]
    ref[:, 7] = t1
    key_o = np.lexsort(ref.view(np.int32).T[::-1])
    assert np.array_equal(p[key_g].view(np.int32), ref[key_o].view(np.int32))
    assert np.array_equal(lf[key_g].astype(np.int64), oleaf[key_o])


def test_leaf_loss_matches_oracle(lib, c1):
    sc = c1
    net = configs.C1_NET
    params = configs.init_params(net, "uniform", 0.5, seed_features=73, seed_mlp=74)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_params(params)
    probes, leaf_ids = scene.leaf_probes(sc.boxes, 40, seed=75)
    labels = scene.probe_labels(sc.mesh, probes)
    n_leaves = sc.boxes.shape[0]
    loss = torch.zeros(n_leaves, dtype=torch.float32, device="cuda")
    count = torch.zeros(n_leaves, dtype=torch.int32, device="cuda")
    _say("leaf loss", probes.shape)
    m.leaf_loss(torch.from_numpy(probes).cuda(), torch.from_numpy(labels).cuda(),
                torch.from_numpy(leaf_ids).cuda(), loss, count)
    cfg = oracle.make_cfg(net, sc.lo, sc.side)
    z = oracle.forward(cfg, params.astype(np.float64), probes)
    seg = oracle.segment_loss(cfg, z, labels)
    ref = np.bincount(leaf_ids, weights=seg, minlength=n_leaves)
    assert np.array_equal(count.cpu().numpy(), np.bincount(leaf_ids, minlength=n_leaves))
    got = loss.double().cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max(), np.abs(got - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("n_leaves", [1, 7, 1024, 16384 + 5])
def test_node_rank_and_acceptance_match_oracle(lib, n_leaves):
    """nbvh_node_rank / nbvh_acceptance (binary32) against the oracle's
    binary64 rank and acceptance on per-leaf sums with empty leaves, leaves
    without crossings and zero losses mixed in."""
    from paper_2405_16237_amd.nbvh import acceptance, node_rank
    rng = np.random.default_rng(n_leaves)
    count = rng.integers(0, 400, n_leaves).astype(np.uint32)
    loss = (rng.uniform(0.0, 3.0, n_leaves) * count).astype(np.float32)
    loss[rng.uniform(size=n_leaves) < 0.05] = 0.0
    hits = rng.integers(0, 5000, n_leaves).astype(np.uint32)
    n_rays = 1 << 18
    _say("node rank and acceptance:", n_leaves, "leaves")
    r = node_rank(torch.from_numpy(loss).cuda(), torch.from_numpy(count).cuda(), torch.from_numpy(hits).cuda(), n_rays)
    a = acceptance(r, 0.005).cpu().numpy().astype(np.float64)
    r = r.cpu().numpy().astype(np.float64)
    ro = oracle.node_rank(loss.astype(np.float64), count.astype(np.int64), hits.astype(np.int64), n_rays)
    ao = oracle.acceptance(ro, 0.005)
    fin = np.isfinite(ro)
    assert np.array_equal(np.isfinite(r), fin)
    assert np.all(r[~fin] == -np.inf)
    if fin.any():
        assert np.abs(r[fin] - ro[fin]).max() <= 2e-6 * max(1.0, np.abs(ro[fin]).max())
    assert np.abs(a - ao).max() <= 2e-6, np.abs(a - ao).max()


def test_construction_grows_cut_and_learns(lib, c1):
    """The cut grows from the root to the target through base-BVH nodes,
    every expansion splits the leaves of largest rank, and the constructed
    N-BVH answers camera rays better than its boxes alone."""
    from paper_2405_16237_amd import construct as C
    sc = c1
    base = scene.base_bvh(sc.verts, sc.tris, leaf_tris=64)
    net = configs.C1_NET
    root = np.concatenate([base["lo"][0], base["hi"][0]])[None, :]
    lo, side = scene.scene_cube(root)
    sched = C.Schedule(target_leaves=32, iters=40, iters_growth=1.3, splits=2, splits_growth=1.6, final_iters=300,
                       rays_per_step=1 << 15, stats_rays=1 << 15)
    model, cut, hist = C.construct(net, base, lambda p: scene.probe_labels(sc.mesh, p), sched, lo, side,
                                   params=configs.init_params(net, "normal", 1e-2), log=_say)
    assert len(cut.nodes) == 32 and len(set(cut.nodes)) == 32
    # the cut is a cut: no node is an ancestor of another, and together they hold every triangle
    parent = np.full(base["lo"].shape[0], -1)
    inner = np.nonzero(base["left"] >= 0)[0]
    parent[base["left"][inner]] = inner
    parent[base["right"][inner]] = inner
    for nd in cut.nodes:
        a = parent[nd]
        while a >= 0:
            assert a not in cut.nodes
            a = parent[a]
    assert base["n_tris"][cut.nodes].sum() == sc.tris.shape[0]
    assert hist[-1]["loss"] < hist[0]["loss"]
    rays = scene.pinhole_rays(256, 256)
    gt = scene.ray_ground_truth(sc.mesh, rays)
    h = model.query(torch.from_numpy(rays).cuda()).cpu().numpy()
    pred = h[:, 7].view(np.uint32) != 0xFFFFFFFF
    acc = float((pred == gt["hit"]).mean())
    off, _ = model.traverse(torch.from_numpy(rays).cuda(), 64 * rays.shape[0])
    off = off.cpu().numpy()
    box_acc = float(((off[1:] > off[:-1]) == gt["hit"]).mean())
    _say("construction: hit accuracy %.4f, boxes alone %.4f, history %s" % (acc, box_acc, hist))
    assert acc > box_acc and acc > 0.9


def test_view_shares_the_network(lib, c1):
    """A view over other leaves answers exactly like a separate model with
    the same parameters on those leaves, and trains the one network."""
    sc = c1
    net = configs.C1_NET
    params = configs.init_params(net, "uniform", 0.5, seed_features=76, seed_mlp=77)
    coarse, _ = scene.median_split_leaves(sc.verts, sc.tris, 8)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_params(params)
    v = m.view(coarse)
    ref = lib.NBVH(net, coarse, sc.lo, sc.side, precision="fp32")
    ref.set_params(params)
    rays = torch.from_numpy(scene.pinhole_rays(128, 128)).cuda()
    _say("view query")
    hv = v.query(rays).cpu().numpy()
    hr = ref.query(rays).cpu().numpy()
    assert np.array_equal(hv.view(np.uint32), hr.view(np.uint32))
    probes, _ = scene.leaf_probes(coarse, 64, seed=78)
    lab = scene.probe_labels(sc.mesh, probes)
    _say("train through the view")
    v.train_step(torch.from_numpy(probes).cuda(), torch.from_numpy(lab).cuda())
    ref.train_step(torch.from_numpy(probes).cuda(), torch.from_numpy(lab).cuda())
    torch.cuda.synchronize()
    assert m.read_state()["step"] == 1 and v.read_state()["step"] == 1
    got, want = m.get_params(), ref.get_params()
    assert not np.array_equal(got, params)
    assert np.abs(got - want).max() <= 1e-6
    with pytest.raises(ValueError):
        lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp8").view(coarse)


def test_lod_view_training_step_matches_oracle(lib, c1):
    """Levels of detail (Sec. 5.3) against the oracle: training rays through
    a coarse cut's view (first leaf of the coarse cut, per-leaf acceptance)
    are the oracle's first hits on that cut, bit for bit; one FP32 training
    step on them through the view moves the shared parameters as the
    oracle's step does, and the fine tree sees the moved parameters."""
    sc = c1
    net = configs.C1_NET
    params = configs.init_params(net, "uniform", 1.0, seed_features=81, seed_mlp=82)
    coarse, _ = scene.median_split_leaves(sc.verts, sc.tris, 16)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1.0)
    m.set_params(params)
    v = m.view(coarse)
    rays = _box_rays(sc, 12_000 + 7, 83)
    rng = np.random.default_rng(84)
    u = rng.uniform(size=rays.shape[0]).astype(np.float32)
    accept = rng.uniform(0.2, 1.0, size=coarse.shape[0]).astype(np.float32)
    _say("first hits through a 16-leaf view")
    probes, leaf = v.first_hits(torch.from_numpy(rays).cuda(), torch.from_numpy(u).cuda(),
                                torch.from_numpy(accept).cuda())
    probes, leaf = v.group_by_leaf(probes, leaf)
    p = probes.cpu().numpy()
    ray, oleaf, t0, t1, _ = oracle.first_hits(rays, coarse, u, accept)
    ref = np.zeros((ray.size, 8), dtype=np.float32)
    ref[:, 0:3], ref[:, 3], ref[:, 4:7], ref[:, 7] = rays[ray, 0:3], t0, rays[ray, 4:7], t1
    assert p.shape[0] == ray.size > 2000
    kg, ko = np.lexsort(p.view(np.int32).T[::-1]), np.lexsort(ref.view(np.int32).T[::-1])
    assert np.array_equal(p[kg].view(np.int32), ref[ko].view(np.int32))
    assert np.array_equal(leaf.cpu().numpy()[kg].astype(np.int64), oleaf[ko])
    lab = scene.probe_labels(sc.mesh, p)
    cfg = oracle.make_cfg(net, sc.lo, sc.side)
    p64 = params.astype(np.float64)
    clear = oracle.min_abs_preact(cfg, p64, p) > 1e-4  # FP32 ReLU decisions equal the oracle's
    assert clear.mean() > 0.5
    p, lab = np.ascontiguousarray(p[clear]), np.ascontiguousarray(lab[clear])
    _say("one training step through the view:", p.shape[0], "probes")
    loss = v.train_step(torch.from_numpy(p).cuda(), torch.from_numpy(lab).cuda()).cpu().numpy()
    mm, vv = np.zeros_like(p64), np.zeros_like(p64)
    z = oracle.forward(cfg, p64, p)
    terms, dz = oracle.loss(cfg, z, lab)
    g = oracle.backward(cfg, p64, p, dz)
    oracle.train_step(cfg, p64, mm, vv, 1, p, lab)
    assert np.allclose(loss, terms, rtol=1e-5, atol=1e-7), (loss, terms)
    got = m.get_params()  # the fine tree's parameters: one buffer
    sel = np.abs(g) > 1e-3 * np.abs(g).max()
    assert sel.sum() > 1000
    assert np.abs(got[sel] - p64[sel]).max() <= 1e-6
    assert m.read_state()["step"] == 1


def test_levels_of_detail(lib, c1):
    """Construction with levels of detail (Sec. 5.3): several cuts of one
    base BVH, coarse to fine, trained together on one network. Every level
    is a cut, answers camera rays well, and the coarser levels cross fewer
    leaves per ray."""
    from paper_2405_16237_amd import construct as C
    sc = c1
    base = scene.base_bvh(sc.verts, sc.tris, leaf_tris=64)
    net = configs.C1_NET
    root = np.concatenate([base["lo"][0], base["hi"][0]])[None, :]
    lo, side = scene.scene_cube(root)
    sched = C.Schedule(target_leaves=48, iters=40, iters_growth=1.3, splits=2, splits_growth=1.6, final_iters=400,
                       rays_per_step=1 << 15, stats_rays=1 << 15, lod_interval=100)
    lods = []
    C.construct(net, base, lambda p: scene.probe_labels(sc.mesh, p), sched, lo, side,
                params=configs.init_params(net, "normal", 1e-2), log=_say, lods=lods)
    sizes = [len(c.nodes) for c, _ in lods]
    _say("level sizes", sizes)
    assert len(lods) >= 3 and sizes == sorted(sizes) and len(set(sizes)) == len(sizes) and sizes[-1] == 48
    rays_np = scene.pinhole_rays(192, 192)
    gt = scene.ray_ground_truth(sc.mesh, rays_np)
    rays = torch.from_numpy(rays_np).cuda()
    segs, accs = [], []
    for c, tree in lods:
        assert base["n_tris"][c.nodes].sum() == sc.tris.shape[0]
        h = tree.query(rays).cpu().numpy()
        accs.append(float(((h[:, 7].view(np.uint32) != 0xFFFFFFFF) == gt["hit"]).mean()))
        torch.cuda.synchronize()
        segs.append(tree.read_state()["last_n_segments"])
    _say("hit accuracy per level", accs, "segments", segs)
    assert min(accs) > 0.85 and accs[-1] > 0.9
    assert segs[0] < segs[-1]


@pytest.mark.parametrize("n_leaves,n,tagged", [(64, 50_033, False), (1024, 70_001, True), (1, 300, False),
                                               (20_000, 4_099, True)])
def test_group_by_leaf_is_a_stable_sort(lib, n_leaves, n, tagged):
    """Grouping probes by leaf is the stable sort by leaf id: compared with
    numpy's stable argsort, bit for bit, for 1, 64, 1,024 and 20,000 leaves
    (one to four 4-bit passes) and batch sizes that are not multiples of 256;
    a bit above the leaf count (the inside tag) is carried along unsorted."""
    rng = np.random.default_rng(n_leaves + n)
    lo = rng.uniform(0.0, 0.9, size=(n_leaves, 3))
    boxes = np.concatenate([lo, lo + rng.uniform(0.01, 0.1, size=(n_leaves, 3))], axis=1).astype(np.float32)
    m = lib.NBVH(configs.C1_NET, boxes, np.zeros(3, np.float32), 1.0, precision="fp32")
    ids = rng.integers(0, n_leaves, size=n).astype(np.uint32)
    if tagged:
        ids[::7] |= np.uint32(0x80000000)
    probes = rng.standard_normal((n, 8)).astype(np.float32)
    _say("group by leaf", n_leaves, n)
    p_out, id_out = m.group_by_leaf(torch.from_numpy(probes).cuda(), torch.from_numpy(ids.view(np.int32)).cuda())
    bits = max(1, int(n_leaves - 1).bit_length())
    key = ids & np.uint32((1 << (4 * ((bits + 3) // 4))) - 1)
    order = np.argsort(key, kind="stable")
    assert np.array_equal(id_out.cpu().numpy().view(np.uint32), ids[order])
    assert np.array_equal(p_out.cpu().numpy().view(np.int32), probes[order].view(np.int32))
    e_p, e_i = m.group_by_leaf(torch.zeros((0, 8), device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert e_p.shape == (0, 8) and e_i.shape == (0,)


def test_backward_does_not_depend_on_probe_order(lib, c1):
    """Grouping a batch by leaf changes its layout only: the gradients of a
    shuffled batch and of the same batch regrouped by nbvh_group_by_leaf agree
    to FP32 summation order (the same per-probe terms, summed in another
    order)."""
    sc = c1
    net = configs.C1_NET
    params = configs.init_params(net, "uniform", 0.5, seed_features=40, seed_mlp=41)
    p, lf = scene.leaf_probes(sc.boxes, 64, seed=42)
    perm = np.random.default_rng(43).permutation(p.shape[0])
    p_s, lf_s = np.ascontiguousarray(p[perm]), np.ascontiguousarray(lf[perm]).astype(np.int32)
    dz = (np.random.default_rng(44).standard_normal((p.shape[0], net.n_out)) * 1e-2).astype(np.float32)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32")
    m.set_params(params)
    _say("backward, shuffled vs regrouped", p.shape)
    g_p, g_ids = m.group_by_leaf(torch.from_numpy(p_s).cuda(), torch.from_numpy(lf_s).cuda())
    order = np.argsort(lf_s, kind="stable")
    assert np.array_equal(g_ids.cpu().numpy(), lf_s[order])
    m.grad.zero_()
    m.backward(torch.from_numpy(p_s).cuda(), torch.from_numpy(dz).cuda())
    g_shuffled = m.grad.double().cpu().numpy()
    m.grad.zero_()
    m.backward(g_p, torch.from_numpy(np.ascontiguousarray(dz[order])).cuda())
    g_grouped = m.grad.double().cpu().numpy()
    scale = np.abs(g_shuffled).max()
    assert scale > 0 and np.count_nonzero(g_shuffled) > 1000
    assert np.abs(g_grouped - g_shuffled).max() <= 1e-4 * scale
