"""The C-ABI library loads and exports every entry point include/nbvh.h
declares; host-only calls (no GPU work) behave. CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def abi():
    from paper_2405_16237_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2405_16237_amd import build
        build.build()
    _abi.load()
    return _abi


def _declared():
    src = open(os.path.join(ROOT, "include", "nbvh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbvh_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(abi):
    L = abi.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(abi.EXPORTS) == names


def _cfg(abi, **kw):
    from nbvh_synth import configs
    from paper_2405_16237_amd.nbvh import make_config
    net = kw.pop("net", configs.C2_NET)
    c = make_config(net, np.zeros(3, np.float32), np.float32(2.0), **kw)
    return c


def test_param_counts_match_generator(abi):
    from nbvh_synth import configs
    L = abi.load()
    for net in (configs.C1_NET, configs.C2_NET, configs.C5_NET):
        c = _cfg(abi, net=net)
        nt, nm = ctypes.c_uint64(), ctypes.c_uint64()
        assert L.nbvh_param_count(ctypes.byref(c), ctypes.byref(nt), ctypes.byref(nm)) == 0
        assert nt.value == net.n_table_params and nm.value == net.n_mlp_params
        offs = (ctypes.c_uint64 * (net.mlp_hidden + 3))()
        assert L.nbvh_param_layout(ctypes.byref(c), offs) == 0
        assert offs[1] >= nt.value and all(o % 64 == 0 for o in offs[1:-1])
        for k, (fi, fo) in enumerate(net.layer_dims()):
            assert offs[2 + k] >= offs[1 + k] + fi * fo


def test_invalid_configs_rejected(abi):
    L = abi.load()
    nt, nm = ctypes.c_uint64(), ctypes.c_uint64()
    for field, val in (("n_features", 3), ("mlp_width", 48), ("n_out", 4), ("log2_T", 0), ("mlp_hidden", 0),
                       ("n_samples", 0), ("scene_side", 0.0), ("n_levels", 33)):
        c = _cfg(abi)
        setattr(c, field, val)
        st = L.nbvh_param_count(ctypes.byref(c), ctypes.byref(nt), ctypes.byref(nm))
        assert st in (abi.NBVH_ERR_INVALID_ARG, abi.NBVH_ERR_UNSUPPORTED), field
        assert L.nbvh_last_error().decode()
    c = _cfg(abi)
    c.n_samples = 3  # 3*16*2 = 96 inputs: fine; 5*16*2 = 160: fine; odd widths are not
    assert L.nbvh_param_count(ctypes.byref(c), ctypes.byref(nt), ctypes.byref(nm)) == 0


def test_sizes(abi):
    L = abi.load()
    assert L.nbvh_nodes_bytes(1) == 64 and L.nbvh_nodes_bytes(1024) == 1023 * 64
    assert L.nbvh_state_bytes() >= 64
    c = _cfg(abi)
    assert L.nbvh_aux_bytes(ctypes.byref(c)) > 0
    assert L.nbvh_version().decode().startswith("nbvh")


def test_null_arguments_rejected_before_any_gpu_work(abi):
    L = abi.load()
    c = _cfg(abi)
    out = ctypes.c_void_p()
    assert L.nbvh_build(ctypes.byref(c), None, 0, None, 0, None, ctypes.byref(out)) == abi.NBVH_ERR_INVALID_ARG
    assert L.nbvh_query(None, None, 0, None, 0, None, 0, None) == abi.NBVH_ERR_INVALID_ARG
    assert L.nbvh_train_step(None, None, None, 0, None, None, 0, None) == abi.NBVH_ERR_INVALID_ARG


def test_profile_groups_match_header(abi):
    src = open(os.path.join(ROOT, "include", "nbvh.h")).read()
    n = int(re.search(r"NBVH_K_COUNT\s*=\s*(\d+)", src).group(1))
    assert abi.NBVH_K_COUNT == n == len(abi.KERNEL_GROUPS)
    ids = re.findall(r"NBVH_K_([A-Z_]+)\s*=\s*(\d+)", src)
    names = {int(v): k.lower() for k, v in ids if k != "COUNT"}
    assert [names[i] for i in range(n)] == abi.KERNEL_GROUPS
