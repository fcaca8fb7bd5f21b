"""ctypes binding of libstein_icp.so (C ABI in include/stein_icp.h).

Argument marshalling only: tensors are passed as raw device pointers and the
current HIP stream of torch is passed as the stream; every step of the
iteration runs in the library's HIP kernels. The functions keep the C names.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstein_icp.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE = 0, -1, -2, -3, -4
NN_FP32, NN_BF16_RERANK, NN_F16_RERANK = 0, 1, 2
OPT_ADAM, OPT_SGD = 0, 1
BW_MEDIAN, BW_FIXED = 0, 1
PRIOR_UNIFORM, PRIOR_GAUSS_VONMISES = 0, 1
METRIC_POINT, METRIC_PLANE = 0, 1


class SteinICPError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


class stein_icp_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("num_particles", C.c_int32),
        ("batch_size", C.c_int32),
        ("schedule_rows", C.c_int32),
        ("lr", C.c_double),
        ("beta1", C.c_double),
        ("beta2", C.c_double),
        ("eps", C.c_double),
        ("seed", C.c_uint64),
        ("init_half_trans", C.c_double),
        ("init_half_rot", C.c_double),
        ("init_centre", C.c_double * 6),
        ("nn_mode", C.c_int32),
        ("optimizer", C.c_int32),
        ("bandwidth_mode", C.c_int32),
        ("prior_mode", C.c_int32),
        ("fixed_h_trans", C.c_double),
        ("fixed_h_rot", C.c_double),
        ("prior_mu", C.c_double * 6),
        ("prior_var_trans", C.c_double * 3),
        ("prior_kappa_rot", C.c_double * 3),
        ("n_scale", C.c_int64),
        ("use_graph", C.c_int32),
        ("autotune", C.c_int32),
        ("metric", C.c_int32),
        ("normal_k", C.c_int32),
    ]


EXPORTS = [
    "stein_icp_default_config", "stein_icp_init", "stein_icp_batch_init", "stein_icp_step",
    "stein_icp_particles", "stein_icp_get_state", "stein_icp_set_state",
    "stein_icp_particles_f32", "stein_icp_set_particles_f32",
    "stein_icp_get_diagnostics", "stein_icp_shape", "stein_icp_nn_tiling", "stein_icp_set_nn_tiling",
    "stein_icp_stage_times", "stein_icp_time_nn", "stein_icp_nn_rescans",
    "stein_icp_destroy",
    "stein_icp_last_error", "stein_icp_nn", "stein_icp_nn_noalloc", "stein_icp_screen_values",
    "stein_icp_make_schedule",
    "stein_icp_make_init",
    "stein_icp_knn", "stein_icp_normals", "stein_icp_get_normals", "stein_icp_posterior_scores",
]

_lib = None


def lib():
    """Load the library; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2106_03287_amd/csrc/build.py`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, u64, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_double
    cfgp = C.POINTER(stein_icp_config)
    L.stein_icp_default_config.argtypes = [cfgp]
    L.stein_icp_default_config.restype = None
    L.stein_icp_init.argtypes = [C.POINTER(vp), cfgp, vp, i64, vp, i64, vp, vp, vp]
    L.stein_icp_batch_init.argtypes = [C.POINTER(vp), cfgp, i32, C.POINTER(vp), C.POINTER(i64),
                                       C.POINTER(vp), C.POINTER(i64), vp, C.POINTER(vp), vp]
    L.stein_icp_step.argtypes = [vp, i32, vp]
    L.stein_icp_particles.argtypes = [vp, vp, vp]
    L.stein_icp_get_state.argtypes = [vp, vp, vp, vp, C.POINTER(i64), vp]
    L.stein_icp_particles_f32.argtypes = [vp, vp, vp]
    L.stein_icp_set_particles_f32.argtypes = [vp, vp, vp]
    L.stein_icp_set_state.argtypes = [vp, vp, vp, vp, i64, vp]
    L.stein_icp_get_diagnostics.argtypes = [vp, vp, vp, vp, vp, vp]
    L.stein_icp_shape.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.stein_icp_nn_tiling.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                      C.POINTER(i32), C.POINTER(i32), C.POINTER(dbl)]
    L.stein_icp_set_nn_tiling.argtypes = [vp, i32, i32, i32, i32, vp]
    L.stein_icp_stage_times.argtypes = [vp, i32, C.POINTER(dbl), vp]
    L.stein_icp_time_nn.argtypes = [vp, i32, C.POINTER(dbl), vp]
    L.stein_icp_nn_rescans.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), vp]
    L.stein_icp_destroy.argtypes = [vp]
    L.stein_icp_destroy.restype = None
    L.stein_icp_last_error.argtypes = []
    L.stein_icp_last_error.restype = C.c_char_p
    L.stein_icp_nn.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp]
    L.stein_icp_nn_noalloc.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp]
    L.stein_icp_screen_values.argtypes = [vp, i64, vp, i64, i32, vp, vp, C.POINTER(i32), vp]
    L.stein_icp_knn.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp]
    L.stein_icp_normals.argtypes = [vp, i64, i32, vp, vp, vp]
    L.stein_icp_get_normals.argtypes = [vp, vp, vp]
    L.stein_icp_posterior_scores.argtypes = [vp, i64, vp, i64, vp, vp]
    L.stein_icp_make_schedule.argtypes = [u64, i64, i32, i32, vp]
    L.stein_icp_make_init.argtypes = [u64, i32, dbl, dbl, vp, vp]
    for name in EXPORTS:
        if name not in ("stein_icp_default_config", "stein_icp_destroy", "stein_icp_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    cfg = stein_icp_config()
    L.stein_icp_default_config(C.byref(cfg))
    if cfg.struct_size != C.sizeof(stein_icp_config):
        raise ImportError("stein_icp_config layout differs between library and binding")
    return L


def _check(fn, rc):
    if rc != OK:
        raise SteinICPError(fn, rc, lib().stein_icp_last_error().decode())


def _ptr(t):
    """Device (or host, for host helpers) address of a contiguous tensor/array."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(t.data_ptr())
    return C.c_void_p(t.ctypes.data)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, shape=None, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {shape}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


# ----------------------------------------------------------------- C names

def stein_icp_default_config(**overrides) -> stein_icp_config:
    cfg = stein_icp_config()
    lib().stein_icp_default_config(C.byref(cfg))
    for k, v in overrides.items():
        if k in ("init_centre", "prior_mu", "prior_var_trans", "prior_kappa_rot"):
            arr = getattr(cfg, k)
            for i, x in enumerate(v):
                arr[i] = float(x)
        else:
            setattr(cfg, k, v)
    return cfg


def stein_icp_init(cfg, src, ref, init_particles=None, schedule=None, stream=None):
    import torch
    _need(src, torch.float32, (src.shape[0], 3), "src")
    _need(ref, torch.float32, (ref.shape[0], 3), "ref")
    if init_particles is not None:
        _need(init_particles, torch.float64, (cfg.num_particles, 6), "init_particles")
    if schedule is not None:
        _need(schedule, torch.int32, (cfg.schedule_rows, cfg.batch_size), "schedule")
    ctx = C.c_void_p()
    rc = lib().stein_icp_init(C.byref(ctx), C.byref(cfg), _ptr(src), src.shape[0], _ptr(ref),
                              ref.shape[0], _ptr(init_particles), _ptr(schedule), _stream(stream))
    _check("stein_icp_init", rc)
    return ctx


def stein_icp_batch_init(cfg, srcs, refs, init_particles=None, schedules=None, stream=None):
    import torch
    P = len(srcs)
    if len(refs) != P or (schedules is not None and len(schedules) != P):
        raise ValueError("srcs, refs and schedules need one entry per pair")
    for s, r in zip(srcs, refs):
        _need(s, torch.float32, (s.shape[0], 3), "src")
        _need(r, torch.float32, (r.shape[0], 3), "ref")
    if init_particles is not None:
        _need(init_particles, torch.float64, (P, cfg.num_particles, 6), "init_particles")
    sp = (C.c_void_p * P)(*[s.data_ptr() for s in srcs])
    rp = (C.c_void_p * P)(*[r.data_ptr() for r in refs])
    ns = (C.c_int64 * P)(*[s.shape[0] for s in srcs])
    nr = (C.c_int64 * P)(*[r.shape[0] for r in refs])
    schp = None
    if schedules is not None:
        for s in schedules:
            _need(s, torch.int32, (cfg.schedule_rows, cfg.batch_size), "schedule")
        schp = (C.c_void_p * P)(*[s.data_ptr() for s in schedules])
    ctx = C.c_void_p()
    rc = lib().stein_icp_batch_init(C.byref(ctx), C.byref(cfg), P, sp, ns, rp, nr,
                                    _ptr(init_particles), schp, _stream(stream))
    _check("stein_icp_batch_init", rc)
    return ctx


def stein_icp_step(ctx, n_iters, stream=None):
    _check("stein_icp_step", lib().stein_icp_step(ctx, int(n_iters), _stream(stream)))


def stein_icp_shape(ctx):
    P, K, m = C.c_int32(), C.c_int32(), C.c_int32()
    _check("stein_icp_shape", lib().stein_icp_shape(ctx, C.byref(P), C.byref(K), C.byref(m)))
    return P.value, K.value, m.value


def stein_icp_particles(ctx, out=None, stream=None):
    import torch
    P, K, _ = stein_icp_shape(ctx)
    if out is None:
        out = torch.empty((P, K, 6), dtype=torch.float64, device="cuda")
    _need(out, torch.float64, None, "out")
    if out.numel() != P * K * 6:
        raise ValueError("out must hold n_pairs * K * 6 values")
    _check("stein_icp_particles", lib().stein_icp_particles(ctx, _ptr(out), _stream(stream)))
    return out


def stein_icp_get_state(ctx, stream=None):
    import torch
    P, K, _ = stein_icp_shape(ctx)
    th, mo, ve = (torch.empty((P, K, 6), dtype=torch.float64, device="cuda") for _ in range(3))
    t = C.c_int64()
    _check("stein_icp_get_state", lib().stein_icp_get_state(ctx, _ptr(th), _ptr(mo), _ptr(ve),
                                                            C.byref(t), _stream(stream)))
    return th, mo, ve, t.value


def stein_icp_set_state(ctx, theta, mom=None, vel=None, t=0, stream=None):
    import torch
    P, K, _ = stein_icp_shape(ctx)
    for x, nm in ((theta, "theta"), (mom, "mom"), (vel, "vel")):
        if x is not None:
            _need(x, torch.float64, None, nm)
            if x.numel() != P * K * 6:
                raise ValueError(f"{nm} must hold n_pairs * K * 6 values")
    _check("stein_icp_set_state", lib().stein_icp_set_state(ctx, _ptr(theta), _ptr(mom), _ptr(vel),
                                                            int(t), _stream(stream)))


def stein_icp_particles_f32(ctx, stream=None):
    """Particles rounded to FP32, (P, K, 6) float32 on the device."""
    import torch
    P, K, _ = stein_icp_shape(ctx)
    out = torch.empty((P, K, 6), dtype=torch.float32, device="cuda")
    _check("stein_icp_particles_f32", lib().stein_icp_particles_f32(ctx, _ptr(out), _stream(stream)))
    return out


def stein_icp_set_particles_f32(ctx, theta, stream=None):
    """Start again from FP32 particles (P * K * 6 float32 on the device)."""
    import torch
    P, K, _ = stein_icp_shape(ctx)
    _need(theta, torch.float32, None, "theta")
    if theta.numel() != P * K * 6:
        raise ValueError("theta must hold n_pairs * K * 6 values")
    _check("stein_icp_set_particles_f32", lib().stein_icp_set_particles_f32(ctx, _ptr(theta), _stream(stream)))


def stein_icp_get_diagnostics(ctx, stream=None):
    import torch
    P, K, m = stein_icp_shape(ctx)
    gbar = torch.empty((P, K, 6), dtype=torch.float64, device="cuda")
    phi = torch.empty((P, K, 6), dtype=torch.float64, device="cuda")
    h = torch.empty((P, 2), dtype=torch.float64, device="cuda")
    match = torch.empty((P, K, m), dtype=torch.int32, device="cuda")
    _check("stein_icp_get_diagnostics",
           lib().stein_icp_get_diagnostics(ctx, _ptr(gbar), _ptr(phi), _ptr(h), _ptr(match),
                                           _stream(stream)))
    return {"gbar": gbar, "phi": phi, "h": h, "match": match}


def stein_icp_nn_tiling(ctx):
    q, w, ch, nch, per = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    ms = C.c_double()
    _check("stein_icp_nn_tiling", lib().stein_icp_nn_tiling(ctx, C.byref(q), C.byref(w), C.byref(ch),
                                                            C.byref(nch), C.byref(per), C.byref(ms)))
    return {"queries_per_lane": q.value, "waves": w.value, "chunk": ch.value, "chunks": nch.value,
            "persist": per.value, "tuned_ms": ms.value}


def stein_icp_set_nn_tiling(ctx, queries_per_lane, waves, chunk, persist=0, stream=None):
    _check("stein_icp_set_nn_tiling", lib().stein_icp_set_nn_tiling(
        ctx, int(queries_per_lane), int(waves), int(chunk), int(persist), _stream(stream)))


def stein_icp_stage_times(ctx, n_iters, stream=None):
    """Summed ms per stage over n_iters profiled iterations."""
    out = (C.c_double * 3)()
    _check("stein_icp_stage_times", lib().stein_icp_stage_times(ctx, int(n_iters), out,
                                                                _stream(stream)))
    return {"nn": out[0], "grad_bandwidth": out[1], "phi_update": out[2]}


def stein_icp_time_nn(ctx, n_launches, stream=None):
    """Mean ms of the nearest-neighbour kernel over back-to-back launches."""
    ms = C.c_double()
    _check("stein_icp_time_nn", lib().stein_icp_time_nn(ctx, int(n_launches), C.byref(ms),
                                                        _stream(stream)))
    return ms.value


def stein_icp_nn_rescans(ctx, stream=None):
    """(failed certificates, certificates) of the BF16 screen since init."""
    r, n = C.c_int64(), C.c_int64()
    _check("stein_icp_nn_rescans", lib().stein_icp_nn_rescans(ctx, C.byref(r), C.byref(n), _stream(stream)))
    return r.value, n.value


def stein_icp_destroy(ctx):
    if ctx:
        lib().stein_icp_destroy(ctx)


def stein_icp_last_error():
    return lib().stein_icp_last_error().decode()


def stein_icp_nn(q, ref, mode=NN_FP32, stream=None):
    import torch
    _need(q, torch.float32, (q.shape[0], 3), "q")
    _need(ref, torch.float32, (ref.shape[0], 3), "ref")
    idx = torch.empty(q.shape[0], dtype=torch.int32, device=q.device)
    d2 = torch.empty(q.shape[0], dtype=torch.float32, device=q.device)
    _check("stein_icp_nn", lib().stein_icp_nn(_ptr(q), q.shape[0], _ptr(ref), ref.shape[0],
                                              int(mode), _ptr(idx), _ptr(d2), _stream(stream)))
    return idx, d2


def stein_icp_nn_noalloc(q, ref, mode=NN_FP32, idx=None, d2=None, stream=None):
    """stein_icp_nn on the library's own scratch (no device allocation in the
    library); idx / d2 may be given (int32 / float32, nq each) to write into."""
    import torch
    _need(q, torch.float32, (q.shape[0], 3), "q")
    _need(ref, torch.float32, (ref.shape[0], 3), "ref")
    if idx is None:
        idx = torch.empty(q.shape[0], dtype=torch.int32, device=q.device)
    if d2 is None:
        d2 = torch.empty(q.shape[0], dtype=torch.float32, device=q.device)
    _need(idx, torch.int32, (q.shape[0],), "idx")
    _need(d2, torch.float32, (q.shape[0],), "d2")
    _check("stein_icp_nn_noalloc", lib().stein_icp_nn_noalloc(_ptr(q), q.shape[0], _ptr(ref), ref.shape[0],
                                                              int(mode), _ptr(idx), _ptr(d2), _stream(stream)))
    return idx, d2


def stein_icp_screen_values(q, ref, mode=NN_F16_RERANK, stream=None):
    """(values (nq, M) float32 on the device, centre (4,) and scale exponent)
    of a matrix-core screen's raw screened distances."""
    import torch
    _need(q, torch.float32, (q.shape[0], 3), "q")
    _need(ref, torch.float32, (ref.shape[0], 3), "ref")
    vals = torch.empty((q.shape[0], ref.shape[0]), dtype=torch.float32, device=q.device)
    centre = (C.c_float * 4)()
    e = C.c_int32()
    _check("stein_icp_screen_values", lib().stein_icp_screen_values(
        _ptr(q), q.shape[0], _ptr(ref), ref.shape[0], int(mode), _ptr(vals), centre, C.byref(e), _stream(stream)))
    return vals, np.array(centre[:], dtype=np.float32), e.value


def stein_icp_knn(q, ref, k, stream=None):
    import torch
    _need(q, torch.float32, (q.shape[0], 3), "q")
    _need(ref, torch.float32, (ref.shape[0], 3), "ref")
    idx = torch.empty((q.shape[0], k), dtype=torch.int32, device=q.device)
    d2 = torch.empty((q.shape[0], k), dtype=torch.float32, device=q.device)
    _check("stein_icp_knn", lib().stein_icp_knn(_ptr(q), q.shape[0], _ptr(ref), ref.shape[0], int(k),
                                                _ptr(idx), _ptr(d2), _stream(stream)))
    return idx, d2


def stein_icp_normals(ref, k, eig=False, stream=None):
    import torch
    _need(ref, torch.float32, (ref.shape[0], 3), "ref")
    n = torch.empty((ref.shape[0], 3), dtype=torch.float64, device=ref.device)
    w = torch.empty((ref.shape[0], 3), dtype=torch.float64, device=ref.device) if eig else None
    _check("stein_icp_normals", lib().stein_icp_normals(_ptr(ref), ref.shape[0], int(k), _ptr(n), _ptr(w),
                                                        _stream(stream)))
    return (n, w) if eig else n


def stein_icp_get_normals(ctx, n_total, stream=None):
    import torch
    out = torch.empty((n_total, 3), dtype=torch.float64, device="cuda")
    _check("stein_icp_get_normals", lib().stein_icp_get_normals(ctx, _ptr(out), _stream(stream)))
    return out


def stein_icp_posterior_scores(a, b):
    """KL (translation, rotation) and per-coordinate OVL of pose samples a
    against reference samples b (host FP64 arrays n x 6)."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 6)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1, 6)
    kl, ovl = np.empty(2), np.empty(6)
    _check("stein_icp_posterior_scores",
           lib().stein_icp_posterior_scores(_ptr(a), len(a), _ptr(b), len(b), _ptr(kl), _ptr(ovl)))
    return kl, ovl


def stein_icp_make_schedule(seed, n_src, m, rows):
    import numpy as np
    out = np.empty((rows, m), dtype=np.int32)
    _check("stein_icp_make_schedule",
           lib().stein_icp_make_schedule(int(seed), int(n_src), int(m), int(rows), _ptr(out)))
    return out


def stein_icp_make_init(seed, K, half_trans, half_rot, centre=None):
    import numpy as np
    out = np.empty((K, 6), dtype=np.float64)
    c = None if centre is None else np.ascontiguousarray(centre, dtype=np.float64)
    _check("stein_icp_make_init", lib().stein_icp_make_init(int(seed), int(K), float(half_trans),
                                                            float(half_rot), _ptr(c), _ptr(out)))
    return out


class SteinICP:
    """Owns one context; methods forward to the C calls above."""

    def __init__(self, cfg, src, ref, init_particles=None, schedule=None, stream=None):
        self.cfg = cfg
        self.ctx = stein_icp_init(cfg, src, ref, init_particles, schedule, stream)

    @classmethod
    def batch(cls, cfg, srcs, refs, init_particles=None, schedules=None, stream=None):
        self = cls.__new__(cls)
        self.cfg = cfg
        self.ctx = stein_icp_batch_init(cfg, srcs, refs, init_particles, schedules, stream)
        return self

    def step(self, n_iters, stream=None):
        stein_icp_step(self.ctx, n_iters, stream)

    def particles(self, out=None, stream=None):
        return stein_icp_particles(self.ctx, out, stream)

    def particles_f32(self):
        return stein_icp_particles_f32(self.ctx)

    def set_particles_f32(self, theta):
        stein_icp_set_particles_f32(self.ctx, theta)

    def get_state(self):
        return stein_icp_get_state(self.ctx)

    def set_state(self, theta, mom=None, vel=None, t=0):
        stein_icp_set_state(self.ctx, theta, mom, vel, t)

    def diagnostics(self):
        return stein_icp_get_diagnostics(self.ctx)

    def tiling(self):
        return stein_icp_nn_tiling(self.ctx)

    def set_tiling(self, queries_per_lane, waves, chunk, persist=0):
        stein_icp_set_nn_tiling(self.ctx, queries_per_lane, waves, chunk, persist)

    def stage_times(self, n_iters):
        return stein_icp_stage_times(self.ctx, n_iters)

    def normals(self, n_total):
        return stein_icp_get_normals(self.ctx, n_total)

    def time_nn(self, n_launches):
        return stein_icp_time_nn(self.ctx, n_launches)

    def nn_rescans(self):
        return stein_icp_nn_rescans(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            stein_icp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
