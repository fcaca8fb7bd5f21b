"""Python face of the Stein-ICP oracle (plain FP64 C, see stein_icp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg. The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stein_icp_oracle.c")
_LIB = os.path.join(_HERE, "libstein_icp_oracle.so")

# x86-64 with FMA3 is assumed for the host (fmaf in hardware; glibc's
# software fallback gives the same correctly rounded result, only slower).
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-mfma"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libstein_icp_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Config(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("m", C.c_int32), ("N", C.c_int64), ("M", C.c_int64),
        ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
        ("optimizer", C.c_int32), ("bandwidth", C.c_int32),
        ("h_fixed_trans", C.c_double), ("h_fixed_rot", C.c_double),
        ("prior", C.c_int32), ("pad_", C.c_int32),
        ("prior_mu", C.c_double * 6), ("prior_var_trans", C.c_double * 3),
        ("prior_kappa_rot", C.c_double * 3),
        ("metric", C.c_int32), ("pad2_", C.c_int32),
    ]


ADAM, SGD = 0, 1
BW_MEDIAN, BW_FIXED = 0, 1
POINT, PLANE = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp, fp, ip = C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        cfg = C.POINTER(Config)
        L.or_rotation.argtypes = [dp, dp, dp]
        L.or_transform.argtypes = [dp, dp, fp, dp]
        L.or_dist2_f32.argtypes = [fp, fp]
        L.or_dist2_f32.restype = C.c_float
        L.or_nn_f32.argtypes = [fp, C.c_int64, fp, C.c_int64, ip, fp]
        L.or_icp_cost.argtypes = [dp, fp, fp, ip, C.c_int32, ip]
        L.or_icp_cost.restype = C.c_double
        L.or_icp_gradient.argtypes = [dp, fp, fp, ip, C.c_int32, ip, dp]
        L.or_prior_grad.argtypes = [cfg, dp, dp]
        L.or_median.argtypes = [dp, C.c_int64]
        L.or_median.restype = C.c_double
        L.or_svgd_phi.argtypes = [cfg, dp, dp, dp, dp]
        L.or_update.argtypes = [cfg, C.c_int64, dp, dp, dp, dp]
        L.or_knn_f32.argtypes = [fp, C.c_int64, fp, C.c_int64, C.c_int32, ip, fp]
        L.or_normals.argtypes = [fp, C.c_int64, C.c_int32, dp, dp]
        L.or_plane_cost.argtypes = [dp, fp, fp, dp, ip, C.c_int32, ip]
        L.or_plane_cost.restype = C.c_double
        L.or_plane_gradient.argtypes = [dp, fp, fp, dp, ip, C.c_int32, ip, dp]
        L.or_step.argtypes = [cfg, fp, fp, dp, ip, dp, dp, dp, lp, dp, dp, dp, ip]
        L.or_run.argtypes = [cfg, fp, fp, dp, ip, C.c_int32, C.c_int32, dp, dp, dp, lp]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def make_config(K, m, N, M, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8,
                optimizer=ADAM, bandwidth=BW_MEDIAN, h_fixed=(1.0, 1.0),
                prior=None, metric=POINT) -> Config:
    c = Config()
    c.K, c.m, c.N, c.M = int(K), int(m), int(N), int(M)
    c.lr, c.beta1, c.beta2, c.eps = lr, beta1, beta2, eps
    c.optimizer, c.bandwidth = optimizer, bandwidth
    c.h_fixed_trans, c.h_fixed_rot = h_fixed
    c.metric = metric
    if prior is not None:
        c.prior = 1
        for i, v in enumerate(prior["mu"]):
            c.prior_mu[i] = v
        for i, v in enumerate(prior["var_trans"]):
            c.prior_var_trans[i] = v
        for i, v in enumerate(prior["kappa_rot"]):
            c.prior_kappa_rot[i] = v
    return c


def rotation(theta):
    th = _f64(theta)
    R = np.zeros(9)
    dR = np.zeros(27)
    lib().or_rotation(_p(th, C.c_double), _p(R, C.c_double), _p(dR, C.c_double))
    return R.reshape(3, 3), dR.reshape(3, 3, 3)


def transform(theta, s):
    """FP64 transform of FP32 points by one pose (N x 3 -> N x 3 float64)."""
    R, _ = rotation(theta)
    Rf = _f64(R.reshape(9))
    u = _f64(np.asarray(theta)[:3])
    s = _f32(s).reshape(-1, 3)
    out = np.empty((len(s), 3))
    q = np.zeros(3)
    for i in range(len(s)):
        lib().or_transform(_p(Rf, C.c_double), _p(u, C.c_double), _p(s[i], C.c_float),
                           _p(q, C.c_double))
        out[i] = q
    return out


def dist2_f32(q, r):
    q, r = _f32(q), _f32(r)
    return float(lib().or_dist2_f32(_p(q, C.c_float), _p(r, C.c_float)))


def nn_f32(q, ref):
    q, ref = _f32(q).reshape(-1, 3), _f32(ref).reshape(-1, 3)
    idx = np.empty(len(q), dtype=np.int32)
    d2 = np.empty(len(q), dtype=np.float32)
    lib().or_nn_f32(_p(q, C.c_float), len(q), _p(ref, C.c_float), len(ref),
                    _p(idx, C.c_int32), _p(d2, C.c_float))
    return idx, d2


def icp_cost(theta, src, ref, batch, match):
    th, src, ref = _f64(theta), _f32(src), _f32(ref)
    batch, match = _i32(batch), _i32(match)
    return lib().or_icp_cost(_p(th, C.c_double), _p(src, C.c_float), _p(ref, C.c_float),
                             _p(batch, C.c_int32), len(batch), _p(match, C.c_int32))


def icp_gradient(theta, src, ref, batch, match):
    th, src, ref = _f64(theta), _f32(src), _f32(ref)
    batch, match = _i32(batch), _i32(match)
    g = np.zeros(6)
    lib().or_icp_gradient(_p(th, C.c_double), _p(src, C.c_float), _p(ref, C.c_float),
                          _p(batch, C.c_int32), len(batch), _p(match, C.c_int32),
                          _p(g, C.c_double))
    return g


def knn_f32(q, ref, k):
    """k nearest references per query, ascending (distance, index); -1 / inf
    beyond the reference count."""
    q, ref = _f32(q).reshape(-1, 3), _f32(ref).reshape(-1, 3)
    idx = np.empty((len(q), k), dtype=np.int32)
    d2 = np.empty((len(q), k), dtype=np.float32)
    lib().or_knn_f32(_p(q, C.c_float), len(q), _p(ref, C.c_float), len(ref), int(k),
                     _p(idx, C.c_int32), _p(d2, C.c_float))
    return idx, d2


def normals(ref, k):
    """Unit normals (M x 3, zero where undefined) and the neighbourhood
    covariance eigenvalues (M x 3, ascending)."""
    ref = _f32(ref).reshape(-1, 3)
    n = np.empty((len(ref), 3))
    w = np.empty((len(ref), 3))
    lib().or_normals(_p(ref, C.c_float), len(ref), int(k), _p(n, C.c_double), _p(w, C.c_double))
    return n, w


def plane_cost(theta, src, ref, nrm, batch, match):
    th, src, ref, nrm = _f64(theta), _f32(src), _f32(ref), _f64(nrm)
    batch, match = _i32(batch), _i32(match)
    return lib().or_plane_cost(_p(th, C.c_double), _p(src, C.c_float), _p(ref, C.c_float),
                               _p(nrm, C.c_double), _p(batch, C.c_int32), len(batch), _p(match, C.c_int32))


def plane_gradient(theta, src, ref, nrm, batch, match):
    th, src, ref, nrm = _f64(theta), _f32(src), _f32(ref), _f64(nrm)
    batch, match = _i32(batch), _i32(match)
    g = np.zeros(6)
    lib().or_plane_gradient(_p(th, C.c_double), _p(src, C.c_float), _p(ref, C.c_float),
                            _p(nrm, C.c_double), _p(batch, C.c_int32), len(batch), _p(match, C.c_int32),
                            _p(g, C.c_double))
    return g


def _normals_arg(cfg, nrm, M):
    if cfg.metric != PLANE:
        return None, None
    if nrm is None:
        raise ValueError("the point-to-plane metric needs the reference normals")
    nrm = _f64(nrm).reshape(-1, 3)
    if len(nrm) != M:
        raise ValueError("one normal per reference point")
    return nrm, _p(nrm, C.c_double)


def prior_grad(cfg: Config, theta):
    th = _f64(theta)
    out = np.zeros(6)
    lib().or_prior_grad(C.byref(cfg), _p(th, C.c_double), _p(out, C.c_double))
    return out


def median(vals):
    v = _f64(vals)
    return lib().or_median(_p(v, C.c_double), len(v))


def svgd_phi(cfg: Config, theta, G):
    th, G = _f64(theta), _f64(G)
    phi = np.zeros_like(th)
    h = np.zeros(2)
    lib().or_svgd_phi(C.byref(cfg), _p(th, C.c_double), _p(G, C.c_double),
                      _p(phi, C.c_double), _p(h, C.c_double))
    return phi, h


def update(cfg: Config, t, theta, mom, vel, phi):
    """In-place update; returns (theta, mom, vel)."""
    th, mo, ve, ph = _f64(theta).copy(), _f64(mom).copy(), _f64(vel).copy(), _f64(phi)
    lib().or_update(C.byref(cfg), int(t), _p(th, C.c_double), _p(mo, C.c_double),
                    _p(ve, C.c_double), _p(ph, C.c_double))
    return th, mo, ve


class State:
    """Particles, Adam moments and the step count."""

    def __init__(self, theta, mom=None, vel=None, t=0):
        self.theta = _f64(theta).copy()
        self.mom = np.zeros_like(self.theta) if mom is None else _f64(mom).copy()
        self.vel = np.zeros_like(self.theta) if vel is None else _f64(vel).copy()
        self.t = np.array([t], dtype=np.int64)

    def copy(self):
        return State(self.theta, self.mom, self.vel, int(self.t[0]))


def step(cfg: Config, src, ref, batch, state: State, normals=None):
    """One iteration in place; returns diagnostics dict (gbar, phi, h, match).
    normals: M x 3, for the point-to-plane metric."""
    src, ref, batch = _f32(src), _f32(ref), _i32(batch)
    keep, nptr = _normals_arg(cfg, normals, len(ref) // 3 if ref.ndim == 1 else len(ref))
    K, m = cfg.K, cfg.m
    gbar = np.zeros((K, 6))
    phi = np.zeros((K, 6))
    h = np.zeros(2)
    match = np.zeros((K, m), dtype=np.int32)
    lib().or_step(C.byref(cfg), _p(src, C.c_float), _p(ref, C.c_float), nptr, _p(batch, C.c_int32),
                  _p(state.theta, C.c_double), _p(state.mom, C.c_double),
                  _p(state.vel, C.c_double), _p(state.t, C.c_int64),
                  _p(gbar, C.c_double), _p(phi, C.c_double), _p(h, C.c_double),
                  _p(match, C.c_int32))
    return {"gbar": gbar, "phi": phi, "h": h, "match": match}


def run(cfg: Config, src, ref, schedule, T, state: State, normals=None):
    """T iterations in place (iteration with step count t uses row t mod rows).
    normals: M x 3, for the point-to-plane metric."""
    src, ref, schedule = _f32(src), _f32(ref), _i32(schedule)
    keep, nptr = _normals_arg(cfg, normals, len(ref) // 3 if ref.ndim == 1 else len(ref))
    lib().or_run(C.byref(cfg), _p(src, C.c_float), _p(ref, C.c_float), nptr,
                 _p(schedule, C.c_int32), schedule.shape[0], int(T),
                 _p(state.theta, C.c_double), _p(state.mom, C.c_double),
                 _p(state.vel, C.c_double), _p(state.t, C.c_int64))
    return state
