"""FP8 (E4M3) inference through the C ABI: the calibration scales against
their definitions (weight amax exactly, activation amax against the FP64
oracle), and the error of FP8 logits and queries against the oracle.

The FP8 error has no parity bound of its own; it is printed per output and
held to a sanity bound that follows from the format: 3 mantissa bits give a
relative rounding error of at most 2^-4 per stored value, so a layer's
output carries about 2^-4 of its scale, and five layers compound to roughly
10-20 % of the logits' RMS."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from nbvh_synth import configs, scene

pytestmark = pytest.mark.gpu

NETS = {
    "c1": configs.C1_NET,
    # the 16M-ray secondary workload's network (L=16, F=4, 256 -> 4x256 -> 8)
    # with the table cut to T = 2^16 so the oracle stays fast
    "c5": configs.NetConfig(16, 4, 16, 4, 16, 1.38, 256, 4, 8),
}


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


def _params(net, seed=4, scale=0.5):
    return configs.init_params(net, "uniform", scale, seed_features=seed, seed_mlp=seed + 10)


def _probes(sc, n, seed):
    p, _ = scene.leaf_probes(sc.boxes, max(1, n // sc.boxes.shape[0] + 1), seed=seed)
    rng = np.random.default_rng(seed)
    return p[rng.permutation(p.shape[0])[:n]]


def _bf16_table(net, params):
    p = params.copy()
    nt = net.n_table_params
    p[:nt] = torch.from_numpy(p[:nt]).to(torch.bfloat16).float().numpy()
    return p


def _weights(net, params):
    out, o = [], net.n_table_params
    for fi, fo in net.layer_dims():
        out.append(params[o:o + fi * fo])
        o += fi * fo
    return out


def test_fp8_needs_calibration(lib, c1):
    sc, _ = c1
    net = configs.C1_NET
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp8")
    m.set_params(_params(net))
    probes = torch.from_numpy(_probes(sc, 500, 20)).cuda()
    _say("fp8 forward before calibration must fail")
    with pytest.raises(lib.NbvhError):
        m.forward(probes)
    m.calibrate_fp8(probes)
    m.forward(probes)
    m.sync_shadow()
    with pytest.raises(lib.NbvhError):
        m.forward(probes)
    labels = torch.zeros((500, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.NbvhError):
        m.train_step(probes, labels)


@pytest.mark.parametrize("name", ["c1", "c5"])
def test_fp8_calibration_scales(lib, c1, name):
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp8")
    m.set_params(params)
    cal = _probes(sc, 4096 + 17, 21)
    _say("fp8 calibration", name, cal.shape)
    m.calibrate_fp8(torch.from_numpy(cal).cuda())
    s = m.fp8_scales()
    for k, W in enumerate(_weights(net, params)):
        amax = np.float32(np.abs(W).max())
        assert s["amax_w"][k] == amax
        assert s["sw"][k] == np.float32(448.0) / amax
    ref = oracle.layer_amax(oracle.make_cfg(net, sc.lo, sc.side), _bf16_table(net, params).astype(np.float64), cal)
    rel = np.abs(s["amax_a"] - ref) / ref
    _say("activation amax", s["amax_a"], "oracle", ref)
    assert rel.max() <= 1e-4, rel
    assert np.all(s["sa"] == np.float32(448.0) / s["amax_a"].astype(np.float32))


@pytest.mark.parametrize("name", ["c1", "c5"])
def test_fp8_forward_error(lib, c1, name):
    sc, _ = c1
    net = NETS[name]
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp8")
    m.set_params(params)
    m.calibrate_fp8(torch.from_numpy(_probes(sc, 1 << 14, 22)).cuda())
    probes = _probes(sc, 2000 + 45, 23)
    z = m.forward(torch.from_numpy(probes).cuda()).cpu().numpy().astype(np.float64)
    ref = oracle.forward(oracle.make_cfg(net, sc.lo, sc.side), _bf16_table(net, params).astype(np.float64), probes)
    per_out = np.sqrt(((z - ref) ** 2).mean(0)) / np.sqrt((ref ** 2).mean(0))
    total = np.sqrt(((z - ref) ** 2).mean()) / np.sqrt((ref ** 2).mean())
    _say("fp8 %s relative RMS error per output %s, overall %.4f" % (name, np.round(per_out, 4).tolist(), total))
    assert np.all(np.isfinite(z))
    assert total <= 0.25, total


def test_fp8_query_c1(lib, c1):
    sc, rays = c1
    net = configs.C1_NET
    params = _params(net, scale=1.0)
    m = lib.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp8")
    m.set_params(params)
    m.calibrate_fp8(torch.from_numpy(_probes(sc, 1 << 16, 24)).cuda())
    hits = m.query(torch.from_numpy(rays).cuda()).cpu().numpy()
    leaf = hits[:, 7].view(np.uint32).astype(np.int64)
    leaf[leaf == 0xFFFFFFFF] = -1
    out, tr, z = oracle.query(oracle.make_cfg(net, sc.lo, sc.side), _bf16_table(net, params).astype(np.float64),
                              rays, sc.boxes)
    # rays whose every segment's hit logit is clear of the FP8 error band
    band = 0.25 * np.sqrt((z[:, 0] ** 2).mean())
    clear = np.ones(rays.shape[0], bool)
    clear[np.unique(tr[1][np.abs(z[:, 0]) <= band])] = False
    agree = leaf[clear] == out[clear, 4].astype(np.int64)
    _say("fp8 query: %d of %d rays clear of the band, leaf agreement %.5f, overall %.5f"
         % (clear.sum(), clear.size, agree.mean(), (leaf == out[:, 4].astype(np.int64)).mean()))
    assert clear.mean() > 0.5
    assert agree.mean() >= 0.99, agree.mean()
