"""ctypes binding of include/stein_icp_proposal.h (the learned initial-particle
proposal). Argument marshalling only: every step runs in the library's
kernels. Tensors are torch CUDA (HIP) tensors; the library must be built."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import stein_icp as S
from .stein_icp import _check, _need, _ptr, _stream

MAX_POINTS = 4096
MAX_PARTICLES = 1024
MAX_SCALES = 4


class stein_icp_proposal_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint64),
        ("num_particles", C.c_int32),
        ("points", C.c_int32),
        ("max_batch", C.c_int32),
        ("n_loss_scales", C.c_int32),
        ("loss_sigma", (C.c_double * 6) * MAX_SCALES),
    ]


EXPORTS = [
    "stein_icp_proposal_default_config", "stein_icp_proposal_param_count", "stein_icp_proposal_create",
    "stein_icp_proposal_destroy", "stein_icp_proposal_set_params", "stein_icp_proposal_get_params",
    "stein_icp_proposal_prepare", "stein_icp_proposal_forward", "stein_icp_proposal_loss",
    "stein_icp_proposal_adam", "stein_icp_proposal_mmd", "stein_icp_propose", "stein_icp_gemm_bf16",
    "stein_icp_proposal_read_weights", "stein_icp_proposal_load",
]

_ready = False


def lib():
    """The shared library with the proposal entry points typed."""
    global _ready
    L = S.lib()
    if _ready:
        return L
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    cfgp = C.POINTER(stein_icp_proposal_config)
    L.stein_icp_proposal_default_config.argtypes = [cfgp]
    L.stein_icp_proposal_param_count.argtypes = [i32, C.POINTER(i64)]
    L.stein_icp_proposal_create.argtypes = [C.POINTER(vp), cfgp]
    L.stein_icp_proposal_destroy.argtypes = [vp]
    L.stein_icp_proposal_set_params.argtypes = [vp, vp, vp]
    L.stein_icp_proposal_get_params.argtypes = [vp, vp, vp]
    L.stein_icp_proposal_prepare.argtypes = [vp, vp, i64, vp, vp]
    L.stein_icp_proposal_forward.argtypes = [vp, vp, i32, vp, vp, vp]
    L.stein_icp_proposal_loss.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.stein_icp_proposal_adam.argtypes = [vp, dbl, dbl, dbl, dbl, vp]
    L.stein_icp_proposal_mmd.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp]
    L.stein_icp_propose.argtypes = [vp, vp, i64, vp, i64, vp, C.POINTER(i32), vp]
    L.stein_icp_gemm_bf16.argtypes = [i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i32, i32, i32,
                                      vp, vp]
    L.stein_icp_proposal_read_weights.argtypes = [C.c_char_p, vp, i64, C.POINTER(i64), C.POINTER(i32)]
    L.stein_icp_proposal_load.argtypes = [C.POINTER(vp), C.c_char_p]
    for name in EXPORTS:
        getattr(L, name).restype = C.c_int
    cfg = stein_icp_proposal_config()
    _check("stein_icp_proposal_default_config", L.stein_icp_proposal_default_config(C.byref(cfg)))
    if cfg.struct_size != C.sizeof(stein_icp_proposal_config):
        raise ImportError("stein_icp_proposal_config layout differs between library and binding")
    _ready = True
    return L


# ----------------------------------------------------------------- C names
def stein_icp_proposal_default_config(**overrides) -> stein_icp_proposal_config:
    cfg = stein_icp_proposal_config()
    _check("stein_icp_proposal_default_config", lib().stein_icp_proposal_default_config(C.byref(cfg)))
    for k, v in overrides.items():
        if k == "loss_sigma":
            v = np.asarray(v, dtype=np.float64).reshape(-1, 6)
            cfg.n_loss_scales = len(v)
            for s in range(MAX_SCALES):
                for d in range(6):
                    cfg.loss_sigma[s][d] = float(v[s, d]) if s < len(v) else 0.0
        else:
            setattr(cfg, k, v)
    return cfg


def stein_icp_proposal_param_count(num_particles: int) -> int:
    n = C.c_int64()
    _check("stein_icp_proposal_param_count", lib().stein_icp_proposal_param_count(int(num_particles), C.byref(n)))
    return n.value


def stein_icp_proposal_create(cfg):
    m = C.c_void_p()
    _check("stein_icp_proposal_create", lib().stein_icp_proposal_create(C.byref(m), C.byref(cfg)))
    return m


def stein_icp_proposal_destroy(model):
    _check("stein_icp_proposal_destroy", lib().stein_icp_proposal_destroy(model))


def stein_icp_proposal_set_params(model, params, stream=None):
    _check("stein_icp_proposal_set_params", lib().stein_icp_proposal_set_params(model, _ptr(params),
                                                                                _stream(stream)))


def stein_icp_proposal_get_params(model, params, stream=None):
    _check("stein_icp_proposal_get_params", lib().stein_icp_proposal_get_params(model, _ptr(params),
                                                                                _stream(stream)))


def stein_icp_proposal_prepare(model, xyz, out, stream=None):
    _check("stein_icp_proposal_prepare", lib().stein_icp_proposal_prepare(model, _ptr(xyz), xyz.shape[0],
                                                                          _ptr(out), _stream(stream)))


def stein_icp_proposal_forward(model, clouds, particles, nonfinite=None, stream=None):
    _check("stein_icp_proposal_forward", lib().stein_icp_proposal_forward(
        model, _ptr(clouds), clouds.shape[0], _ptr(particles), _ptr(nonfinite), _stream(stream)))


def stein_icp_proposal_loss(model, clouds, targets, loss, grad=None, stream=None):
    _check("stein_icp_proposal_loss", lib().stein_icp_proposal_loss(
        model, _ptr(clouds), _ptr(targets), clouds.shape[0], _ptr(loss), _ptr(grad), _stream(stream)))


def stein_icp_proposal_adam(model, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check("stein_icp_proposal_adam", lib().stein_icp_proposal_adam(model, float(lr), float(beta1), float(beta2),
                                                                    float(eps), _stream(stream)))


def stein_icp_proposal_mmd(X, Y, sigma, out=None, stream=None):
    """Set distance per pair of sets: X, Y (B, K, 6) float64 CUDA tensors."""
    import torch
    _need(X, torch.float64, what="X")
    _need(Y, torch.float64, tuple(X.shape), "Y")
    sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(-1, 6))
    if out is None:
        out = torch.empty(X.shape[0], dtype=torch.float64, device=X.device)
    _check("stein_icp_proposal_mmd", lib().stein_icp_proposal_mmd(
        _ptr(X), _ptr(Y), X.shape[0], X.shape[1], len(sig), sig.ctypes.data_as(C.c_void_p), _ptr(out),
        _stream(stream)))
    return out


def stein_icp_propose(model, src, ref, particles, stream=None) -> bool:
    """Fill `particles` (K, 6) float64; returns True when the uniform draw
    should be used instead (non-finite network output)."""
    fb = C.c_int32(0)
    _check("stein_icp_propose", lib().stein_icp_propose(model, _ptr(src), src.shape[0], _ptr(ref), ref.shape[0],
                                                        _ptr(particles), C.byref(fb), _stream(stream)))
    return bool(fb.value)


def stein_icp_gemm_bf16(A, B, C_out, ta=0, tb=0, bias=None, relu=0, accumulate=0, splits=1, workspace=None,
                        stream=None):
    """C_out (M x N) = op(A) op(B) (+ bias) (relu) (+ C_out); 2-D float32 CUDA tensors."""
    M, N = C_out.shape
    K = A.shape[0] if ta else A.shape[1]
    _check("stein_icp_gemm_bf16", lib().stein_icp_gemm_bf16(
        int(ta), int(tb), M, N, K, _ptr(A), A.shape[1], _ptr(B), B.shape[1], _ptr(C_out), C_out.shape[1],
        _ptr(bias), int(relu), int(accumulate), int(splits), _ptr(workspace), _stream(stream)))


def stein_icp_proposal_read_weights(path):
    """(parameters as a host float32 array, K) of a weight file, read and
    checked by the library (no device needed)."""
    n, K = C.c_int64(), C.c_int32()
    b = os.fsencode(path)
    _check("stein_icp_proposal_read_weights",
           lib().stein_icp_proposal_read_weights(b, None, 0, C.byref(n), C.byref(K)))
    out = np.empty(n.value, dtype=np.float32)
    _check("stein_icp_proposal_read_weights",
           lib().stein_icp_proposal_read_weights(b, out.ctypes.data, n.value, C.byref(n), C.byref(K)))
    return out, K.value


def stein_icp_proposal_load(path):
    """A model created by the library from a weight file (default config with
    the file's K)."""
    m = C.c_void_p()
    _check("stein_icp_proposal_load", lib().stein_icp_proposal_load(C.byref(m), os.fsencode(path)))
    return m


# ------------------------------------------------------------------ wrapper
class Proposal:
    """A proposal model: forward, training steps and the one-pair proposal."""

    def __init__(self, cfg=None, params=None):
        import torch
        self.cfg = cfg if cfg is not None else stein_icp_proposal_default_config()
        self.K = self.cfg.num_particles
        self.P = self.cfg.points
        self.n_params = stein_icp_proposal_param_count(self.K)
        self.model = stein_icp_proposal_create(self.cfg)
        if params is not None:
            self.set_params(params)
        self._torch = torch

    @classmethod
    def load(cls, path):
        """The model the library loads from a weight file (default config,
        K from the file)."""
        import torch
        self = cls.__new__(cls)
        _, K = stein_icp_proposal_read_weights(path)
        self.cfg = stein_icp_proposal_default_config(num_particles=K)
        self.K, self.P = K, self.cfg.points
        self.n_params = stein_icp_proposal_param_count(K)
        self.model = stein_icp_proposal_load(path)
        self._torch = torch
        return self

    def set_params(self, params):
        import torch
        p = torch.as_tensor(np.asarray(params, dtype=np.float32) if not isinstance(params, torch.Tensor)
                            else params, dtype=torch.float32).to("cuda").contiguous()
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.numel()}")
        stein_icp_proposal_set_params(self.model, p)
        torch.cuda.current_stream().synchronize()

    def params(self):
        p = self._torch.empty(self.n_params, dtype=self._torch.float32, device="cuda")
        stein_icp_proposal_get_params(self.model, p)
        return p

    def prepare(self, xyz, out=None):
        if out is None:
            out = self._torch.empty(self.P, 3, dtype=self._torch.float32, device="cuda")
        stein_icp_proposal_prepare(self.model, xyz, out)
        return out

    def forward(self, clouds):
        """clouds (B, 2, P, 3) float32 -> (particles (B, K, 6) float64, nonfinite (B,) int32)."""
        B = clouds.shape[0]
        out = self._torch.empty(B, self.K, 6, dtype=self._torch.float64, device="cuda")
        bad = self._torch.empty(B, dtype=self._torch.int32, device="cuda")
        stein_icp_proposal_forward(self.model, clouds, out, bad)
        return out, bad

    def loss(self, clouds, targets, grad=False):
        B = clouds.shape[0]
        loss = self._torch.empty(B, dtype=self._torch.float64, device="cuda")
        g = self._torch.empty(self.n_params, dtype=self._torch.float32, device="cuda") if grad else None
        stein_icp_proposal_loss(self.model, clouds, targets, loss, g)
        return (loss, g) if grad else loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        stein_icp_proposal_adam(self.model, lr, beta1, beta2, eps)

    def propose(self, src, ref):
        """(particles (K, 6) float64, used_fallback)."""
        out = self._torch.empty(self.K, 6, dtype=self._torch.float64, device="cuda")
        fb = stein_icp_propose(self.model, src, ref, out)
        return out, fb

    def close(self):
        if getattr(self, "model", None) is not None and self.model.value:
            stein_icp_proposal_destroy(self.model)
            self.model = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_params(K: int, seed: int = 0, head_scale: float = 0.01) -> np.ndarray:
    """Seeded He-uniform initial weights (zero biases); the last layer is
    scaled by `head_scale` so the first proposals sit near the origin."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = [("W", 3, 64), ("b", 64), ("W", 64, 128), ("b", 128), ("W", 128, 256), ("b", 256),
              ("W", 512, 256), ("b", 256), ("W", 256, 6 * K), ("b", 6 * K)]
    out = []
    for i, b in enumerate(blocks):
        if b[0] == "W":
            lim = np.sqrt(6.0 / b[1])
            w = rng.uniform(-lim, lim, size=(b[1], b[2]))
            if i == 8:
                w *= head_scale
            out.append(w.reshape(-1))
        else:
            out.append(np.zeros(b[1]))
    return np.concatenate(out).astype(np.float32)
