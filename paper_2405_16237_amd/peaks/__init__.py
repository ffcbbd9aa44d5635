"""Measured ceilings of the units the N-BVH kernels are bound by (scattered
table gathers, streaming reads per cache level, FP32 and LDS atomics, the
matrix cores), from the loops in peaks.hip. Used by bench.py to state each
kernel's roofline fraction against what the hardware delivers for that
access pattern, next to the data-sheet peak."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbvh_peaks.so")
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libnbvh_peaks.so is not built (%s); run paper_2405_16237_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, U64, U32, I, D = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
        L.peaks_gather.argtypes = [P, U64, I, I, U32, I, P, P]
        L.peaks_stream.argtypes = [P, U64, I, U32, P, P]
        L.peaks_atomic_f32.argtypes = [P, U64, I, U32, I, P]
        L.peaks_lds_atomic.argtypes = [U32, I, P, P]
        L.peaks_mfma.argtypes = [I, U32, I, P, ctypes.POINTER(D), P]
        for f in (L.peaks_gather, L.peaks_stream, L.peaks_atomic_f32, L.peaks_lds_atomic, L.peaks_mfma):
            f.restype = D
        _lib = L
    return _lib


def _ok(ms, what):
    if ms <= 0:
        raise RuntimeError("peak loop %s failed (%g)" % (what, ms))
    return ms


def measure(torch, n_cu: int = 256, repeat: int = 3) -> dict:
    """Best of `repeat` runs of each loop. Rates: gathers in G lane-loads/s
    and GB/s of entry bytes, streams in GB/s, atomics in G adds/s, matrix
    cores in TFLOP/s."""
    L = load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    grid = n_cu * 16
    sink = torch.zeros(grid * 256 * 2, dtype=torch.int32, device="cuda")
    sp = ctypes.c_void_p(sink.data_ptr())
    out = {}

    def best(fn):
        return min(fn() for _ in range(repeat))

    big = torch.randint(0, 1 << 30, ((1 << 30) // 4,), dtype=torch.int32, device="cuda")  # 1 GiB
    bp = ctypes.c_void_p(big.data_ptr())
    iters = 64
    for mb in (4, 32, 512):
        for eb in (4, 8):
            for lines in ((1, 2, 4, 8, 16, 64) if (mb == 32 and eb == 4) else (8, 64)):
                ms = best(lambda: _ok(L.peaks_gather(bp, mb << 20, eb, lines, grid, iters, sp, s), "gather"))
                n = grid * 256 * iters * 8
                out["gather_%dMiB_%dB_%dlines" % (mb, eb, lines)] = dict(
                    glanes_per_s=n / (ms * 1e-3) / 1e9, gbs=n * eb / (ms * 1e-3) / 1e9,
                    lanes_per_cu_cycle=n / (ms * 1e-3) / (n_cu * 2.4e9))
    for mb, reps in ((2, 200), (128, 8), (1024, 2)):
        ms = best(lambda: _ok(L.peaks_stream(bp, mb << 20, reps, grid, sp, s), "stream"))
        out["stream_%dMiB" % mb] = dict(gbs=(mb << 20) * reps / (ms * 1e-3) / 1e9)
    del big
    grad = torch.zeros(1 << 23, dtype=torch.float32, device="cuda")  # 32 MiB, a gradient-sized buffer
    for run in (1, 4):
        ms = best(lambda: _ok(L.peaks_atomic_f32(ctypes.c_void_p(grad.data_ptr()), grad.numel(), run, grid, 16, s),
                              "atomic"))
        n = grid * 256 * 16 * 4
        out["atomic_f32_32MiB_run%d" % run] = dict(gadds_per_s=n / (ms * 1e-3) / 1e9)
    del grad
    ms = best(lambda: _ok(L.peaks_lds_atomic(grid, 64, sp, s), "lds atomic"))
    out["lds_atomic_u64"] = dict(gadds_per_s=grid * 256 * 64 * 4 / (ms * 1e-3) / 1e9)
    names = ("mfma_bf16_16x16x32", "mfma_bf16_32x32x16", "mfma_fp8_16x16x32", "mfma_fp8_16x16x128")
    for kind, name in enumerate(names):
        fl = ctypes.c_double()
        ms = best(lambda: _ok(L.peaks_mfma(kind, grid, 2048, sp, ctypes.byref(fl), s), "mfma"))
        out[name] = dict(tflops=fl.value / (ms * 1e-3) / 1e12)
    return out
