"""Binding of include/stein_icp_peaks.h: device ceilings measured on the
device itself (a streaming copy, unpacked FP32 fused multiply-adds, 32x32x16
FP16 / BF16 matrix-core products). Argument marshalling only: the probes are
kernels of libstein_icp.so, timed here with HIP events on the stream they are
launched on."""
import ctypes as C

import torch

from . import stein_icp as S

PEAK_COPY, PEAK_FMA32, PEAK_MFMA_F16, PEAK_MFMA_BF16 = 0, 1, 2, 3

EXPORTS = ["stein_icp_peak_probe", "stein_icp_peak_work", "stein_icp_device_info"]

_bound = False


def lib():
    global _bound
    L = S.lib()
    if not _bound:
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.stein_icp_peak_probe.argtypes = [C.c_int, vp, vp, i64, i32, C.c_float, C.c_float, vp]
        L.stein_icp_peak_probe.restype = C.c_int
        L.stein_icp_peak_work.argtypes = [C.c_int, i64, i32]
        L.stein_icp_peak_work.restype = C.c_double
        L.stein_icp_device_info.argtypes = [C.POINTER(i32)] * 4 + [C.c_char_p, i32]
        L.stein_icp_device_info.restype = C.c_int
        _bound = True
    return L


def peak_probe(kind, inp, out, n, iters=1, b=1.0, c=1.0, stream=None):
    """Enqueue one probe (stein_icp_peak_probe) on `stream` (default: torch's
    current stream)."""
    rc = lib().stein_icp_peak_probe(kind, S._ptr(inp) if inp is not None else None, S._ptr(out), n, iters, b, c,
                                    S._stream(stream))
    S._check("stein_icp_peak_probe", rc)


def peak_work(kind, n, iters=1):
    return lib().stein_icp_peak_work(kind, n, iters)


def device_info():
    v = [C.c_int32() for _ in range(4)]
    arch = C.create_string_buffer(128)
    S._check("stein_icp_device_info", lib().stein_icp_device_info(*[C.byref(x) for x in v], arch, 128))
    return {"compute_units": v[0].value, "lds_bytes_per_cu": v[1].value, "wave_size": v[2].value,
            "clock_mhz": v[3].value / 1000.0, "arch": arch.value.decode()}


def _time(fn, reps):
    s = torch.cuda.current_stream()
    fn()   # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    return best


def measure(copy_mib=1024, reps=5):
    """Best of `reps` timed calls of each probe, as rates: HBM GB/s of the
    copy, TFLOP/s of the FMA and matrix-core loops."""
    dev = torch.device("cuda")
    info = device_info()
    out = {"device": info}
    n4 = copy_mib * (1 << 20) // 16
    a = torch.empty(n4 * 4, dtype=torch.float32, device=dev).uniform_()
    b = torch.empty_like(a)
    t = _time(lambda: peak_probe(PEAK_COPY, a, b, n4), reps)
    out["hbm_copy_gbps"] = peak_work(PEAK_COPY, n4) / t / 1e9
    del a, b
    waves = info["compute_units"] * 4 * 8    # eight wavefronts per SIMD
    lanes = waves * 64
    res = torch.empty(lanes, dtype=torch.float32, device=dev)
    iters = 4096
    t = _time(lambda: peak_probe(PEAK_FMA32, None, res, lanes, iters, 1.0, 1.0), reps)
    out["fp32_fma_tflops"] = peak_work(PEAK_FMA32, lanes, iters) / t / 1e12
    # operands of ones (FP16 0x3C00, BF16 0x3F80): nonzero data, exact sums
    for kind, key, one in ((PEAK_MFMA_F16, "mfma_f16_tflops", 0x3C00), (PEAK_MFMA_BF16, "mfma_bf16_tflops", 0x3F80)):
        frag = torch.full((128 * 4,), one | (one << 16), dtype=torch.int32, device=dev)
        t = _time(lambda: peak_probe(kind, frag, res, lanes, iters), reps)
        out[key] = peak_work(kind, lanes, iters) / t / 1e12
    return out
