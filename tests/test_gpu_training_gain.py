"""What the trained network gains over the method without it.

The 1,003,520-triangle scene with 1,024 neural leaves and the L=16, F=2,
T=2^19, 8-sample, 256-4x128-5 network is trained for 2,000 steps on 2^18-probe
batches labelled by triangle intersection (the paper trains in 2^18-ray
batches with Adam at learning rate 0.01). On camera rays it must beat both
network-free answers against the triangle ground truth:
  - box-only: hit at the entry of the first leaf box the ray crosses;
  - untrained: the network at its initial parameters.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nbvh_synth import configs, scene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _score(pred_hit, pred_t, gt, diag):
    acc = float((pred_hit == gt["hit"]).mean())
    both = pred_hit & gt["hit"]
    dep = float(np.abs(pred_t[both] - gt["t"][both]).mean() / diag)
    return acc, dep


def test_training_gain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16237_amd as P
    P.load()
    sc = configs.make_scene(1_003_520, 1024)
    rays_np = scene.pinhole_rays(480, 270)
    gt = scene.ray_ground_truth(sc.mesh, rays_np)
    rays = torch.from_numpy(rays_np).cuda()
    batches = []
    for i in range(4):
        p, _ = scene.leaf_probes(sc.boxes, 256, seed=scene.SEED_PROBES + 10 + i)
        batches.append((torch.from_numpy(p).cuda(), torch.from_numpy(scene.probe_labels(sc.mesh, p)).cuda()))
    net = configs.C2_NET
    m = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(configs.init_params(net, "normal", 1e-2))
    diag = sc.diagonal

    # untrained network
    h0 = m.query(rays).cpu().numpy()
    leaf0 = h0[:, 7].view(np.uint32)
    untrained = _score(leaf0 != 0xFFFFFFFF, h0[:, 0].astype(np.float64), gt, diag)
    # box-only: first segment's entry
    off, segs = m.traverse(rays, 16 * rays.shape[0])
    off = off.cpu().numpy().astype(np.int64)
    segs = segs.cpu().numpy()
    has = off[1:] > off[:-1]
    t_box = np.zeros(rays.shape[0])
    t_box[has] = segs[off[:-1][has], 2].view(np.float32)
    box_only = _score(has, t_box, gt, diag)

    _say("training 2000 steps")
    for it in range(2000):
        m.train_step(*batches[it % 4])
    torch.cuda.synchronize()
    st = m.read_state()
    assert st["step"] == 2000 and st["skipped"] == 0
    h = m.query(rays).cpu().numpy()
    leaf = h[:, 7].view(np.uint32)
    trained = _score(leaf != 0xFFFFFFFF, h[:, 0].astype(np.float64), gt, diag)
    _say("hit accuracy / depth error (fraction of diagonal): trained %s, box-only %s, untrained %s"
         % (trained, box_only, untrained))
    assert trained[0] > box_only[0] and trained[0] > untrained[0]
    assert trained[1] < box_only[1] and trained[1] < untrained[1]
    assert trained[0] > 0.98
