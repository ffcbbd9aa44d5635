"""torch.autograd wrapper: gradients through the library's backward against
the FP64 oracle gradient and against finite differences of the library's
own forward."""
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
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16237_amd as P
    P.load()
    sc = configs.make_scene(20480, 64)
    net = configs.C1_NET
    params = configs.init_params(net, "uniform", 1.0, seed_features=4, seed_mlp=14)
    cfg = oracle.make_cfg(net, sc.lo, sc.side)
    p, _ = scene.leaf_probes(sc.boxes, 40, seed=31)
    keep = oracle.min_abs_preact(cfg, params.astype(np.float64), p) > 1e-4
    probes = p[keep][:1500]
    return P, sc, net, params, cfg, probes


def test_autograd_matches_oracle_gradient(setup):
    P, sc, net, params, cfg, probes = setup
    m = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1.0)
    m.set_params(params)
    pt = torch.from_numpy(probes).cuda()
    rng = np.random.default_rng(32)
    wz = rng.normal(size=(probes.shape[0], net.n_out)).astype(np.float32) / probes.shape[0]
    _say("autograd backward fp32")
    z = P.nbvh_forward(m, pt)
    loss = (z * torch.from_numpy(wz).cuda()).sum()
    loss.backward()
    g = m.unpad(m.params.grad)
    ref = oracle.backward(cfg, params.astype(np.float64), probes, wz.astype(np.float64))
    nt = net.n_table_params
    assert np.abs(g[nt:] - ref[nt:]).max() <= 1e-4 * np.abs(ref[nt:]).max()
    assert np.abs(g[:nt] - ref[:nt]).max() <= 1e-5 * np.abs(ref[:nt]).max()
    # a second backward through a fresh graph gives the same gradient up to
    # the summation order of the FP32 atomics (the library's accumulation
    # buffer is cleared in between, nothing carries over)
    m.params.grad = None
    z2 = P.nbvh_forward(m, pt)
    (z2 * torch.from_numpy(wz).cuda()).sum().backward()
    g2 = m.unpad(m.params.grad)
    assert np.abs(g2 - g).max() <= 1e-6 * np.abs(g).max()


def test_autograd_finite_differences(setup):
    """Central differences of the library's own FP32 forward on the
    coordinates with the largest gradients."""
    P, sc, net, params, cfg, probes = setup
    m = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="fp32", loss_scale=1.0)
    m.set_params(params)
    pt = torch.from_numpy(probes).cuda()
    rng = np.random.default_rng(33)
    wz = torch.from_numpy(rng.normal(size=(probes.shape[0], net.n_out)).astype(np.float32)).cuda()

    def L():
        with torch.no_grad():
            return float((m.forward(pt).double() * wz.double()).sum())

    z = P.nbvh_forward(m, pt)
    (z * wz).sum().backward()
    g = m.params.grad.detach().clone()
    nt = m.n_table
    gw = g[m.offsets[1]:].abs()
    gt = g[:nt].abs()
    idx = torch.cat([torch.topk(gw, 12).indices + m.offsets[1], torch.topk(gt, 12).indices]).cpu().numpy()
    _say("finite differences on", len(idx), "coordinates")

    def fd(i, h):
        with torch.no_grad():
            old = float(m.params[i])
            m.params[i] = old + h
            lp = L()
            m.params[i] = old - h
            lm = L()
            m.params[i] = old
        return (lp - lm) / (2 * h)

    checked = 0
    for i in idx:
        a, b = fd(i, 1e-3), fd(i, 2e-3)
        gi = float(g[i])
        if abs(a - b) > 1e-2 * abs(gi) + 1e-3:
            continue  # a ReLU kink inside the step: the two differences disagree
        assert abs(a - gi) <= 2e-2 * abs(gi) + 1e-3, (int(i), a, b, gi)
        checked += 1
    assert checked >= 0.75 * len(idx), checked


def test_autograd_bf16_trains(setup):
    """A torch optimiser driving the library through the wrapper lowers the
    combined loss (BF16 path)."""
    P, sc, net, params, cfg, probes = setup
    m = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16", loss_scale=1.0)
    m.set_params(configs.init_params(net, "uniform", 1e-4))
    p, _ = scene.leaf_probes(sc.boxes, 256, seed=34)
    lab = torch.from_numpy(scene.probe_labels(sc.mesh, p)).cuda()
    pt = torch.from_numpy(p).cuda()
    opt = torch.optim.Adam([m.params], lr=1e-2, betas=(0.9, 0.99), eps=1e-8)
    first = last = None
    _say("autograd training bf16")
    for it in range(60):
        opt.zero_grad()
        z = P.nbvh_forward(m, pt)
        loss, dz = m.loss(z.detach(), lab)
        z.backward(dz)
        opt.step()
        if it == 0:
            first = float(loss[0])
        last = float(loss[0])
    assert last < 0.7 * first, (first, last)
