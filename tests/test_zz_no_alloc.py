"""The no-allocation query (nbvh_query_noalloc, workspace in a library-owned
static device buffer) against nbvh_query with a caller workspace: the same
kernels, so the hit records are bit-identical; two calls in a row, the second
smaller, a query too large for the buffer refused before any launch, and a
query in origin order (whose sort also lives in the buffer)."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from nbvh_synth import configs, scene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_query_noalloc_matches_query():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_16237_amd as P
    from paper_2405_16237_amd import _abi
    P.load()
    lib = _abi.load()
    sc = configs.make_scene(20480, 64)
    net = configs.C1_NET
    m = P.NBVH(net, sc.boxes, sc.lo, sc.side, precision="bf16")
    m.set_params(configs.init_params(net, "uniform", 1.0, seed_features=61, seed_mlp=62))
    rays_all = scene.pinhole_rays(256, 256)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n in (65536, 20011):
        rays = torch.from_numpy(rays_all[-n:].copy()).cuda()
        cap = 8 * n + 1024
        _say("no-allocation query:", n, "rays, capacity", cap)
        ref = m.query(rays, cap).cpu().numpy()
        got = torch.full((n, 8), float("nan"), device="cuda")
        st = lib.nbvh_query_noalloc(m.ctx, ctypes.c_void_p(rays.data_ptr()), n, ctypes.c_void_p(got.data_ptr()), cap,
                                    stream)
        assert st == _abi.NBVH_OK, lib.nbvh_last_error().decode()
        got = got.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        assert m.read_state()["flags"] == 0
    # beyond the 64 MiB buffer: refused, nothing written
    n = 1 << 20
    big = torch.zeros((n, 8), device="cuda")
    out = torch.full((n, 8), 7.0, device="cuda")
    _say("no-allocation query: oversize request")
    st = lib.nbvh_query_noalloc(m.ctx, ctypes.c_void_p(big.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), 8 * n,
                                stream)
    assert st == _abi.NBVH_ERR_CAPACITY
    assert "64" in lib.nbvh_last_error().decode() or "scratch" in lib.nbvh_last_error().decode()
    torch.cuda.synchronize()
    assert float(out.min()) == 7.0 and float(out.max()) == 7.0
    # with the rays evaluated in origin order the scratch also holds the sort
    m.set_tuning(query_order=1)
    n = 20011
    rays = torch.from_numpy(rays_all[:n].copy()).cuda()
    _say("no-allocation query in origin order:", n, "rays")
    ref = m.query(rays, 8 * n + 1024).cpu().numpy()
    got = torch.full((n, 8), float("nan"), device="cuda")
    st = lib.nbvh_query_noalloc(m.ctx, ctypes.c_void_p(rays.data_ptr()), n, ctypes.c_void_p(got.data_ptr()),
                                8 * n + 1024, stream)
    assert st == _abi.NBVH_OK, lib.nbvh_last_error().decode()
    assert np.array_equal(got.cpu().numpy().view(np.uint32), ref.view(np.uint32))
