"""Oracle of the learned initial-particle proposal (plain NumPy, FP64).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg. The product path never imports it.

What it computes (the network is not from the paper; it seeds the particle
set that Stein ICP otherwise draws uniformly, Sec. V):

* network: per point h1 = relu(x W1 + b1) (3 -> 64), h2 = relu(h1 W2 + b2)
  (64 -> 128), h3 = relu(h2 W3 + b3) (128 -> 256); per cloud the maximum of
  h3 over its points (first maximum on ties); per pair
  z = relu([f_src, f_ref] W4 + b4) (512 -> 256), y = z W5 + b5 (256 -> 6K),
  read as K row-major particles.
* precision: with ``bf16=True`` every operand of every matrix product is
  first rounded to FP32 and then to BF16 (round to nearest even), the way the
  network's matrix-core products consume their FP32 inputs; the products
  and everything else are evaluated in FP64. ``bf16=False`` gives the plain
  FP64 network (used by the finite-difference pins).
* set loss: the biased MMD^2 estimate between the predicted set X and the
  target set Y (K x 6 each) with a sum of Gaussian kernels over widths
  sigma_s (angle differences wrapped to [-pi, pi]); the batch loss is the
  mean over pairs.
* backward: the dense chain rule through the above, layer by layer over
  every point: the gradient of a pooled feature goes to the point that won
  it (a scatter into an all-points gradient of the last per-point layer),
  then back through each ReLU and matrix product. With ``bf16=True`` every
  matrix product of the backward pass, like those of the forward pass,
  rounds both of its operands to BF16 first; the bias gradients are plain
  column sums.
* Adam with bias correction.

Pins (tests/test_proposal_oracle.py): BF16 rounding against torch's
conversion; a hand-built network whose output has a closed form; gradients
against central finite differences of the FP64 network; the BF16 gradients
against torch autograd of the same network built from a matrix product that
rounds its operands (forward and backward) to BF16; MMD^2 closed form at
K = 1, zero on identical sets, positive otherwise, invariant under particle
permutation and 2 pi angle shifts; Adam's first steps in closed form.
"""
from __future__ import annotations

import numpy as np

F1, F2, F3, FCAT, FZ = 64, 128, 256, 512, 256


# ------------------------------------------------------------------ rounding
def bf16_round(x) -> np.ndarray:
    """Round to FP32 (nearest even), then to BF16 (nearest even); FP64 out."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    finite = (b & 0x7F800000) != 0x7F800000
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    r = np.where(finite, r, b & 0xFFFF0000)
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def matmul(A, B, bf16: bool = True) -> np.ndarray:
    """A @ B in FP64, operands rounded to BF16 first when ``bf16``."""
    if bf16:
        A, B = bf16_round(A), bf16_round(B)
    return np.asarray(A, np.float64) @ np.asarray(B, np.float64)


# ----------------------------------------------------------------- parameters
def param_count(K: int) -> int:
    return sum(int(np.prod(s)) for _, s in layout(K).values())


def layout(K: int) -> dict:
    """Offsets and shapes of the parameter blocks in the flat vector."""
    shapes = [("W1", (3, F1)), ("b1", (F1,)), ("W2", (F1, F2)), ("b2", (F2,)),
              ("W3", (F2, F3)), ("b3", (F3,)), ("W4", (FCAT, FZ)), ("b4", (FZ,)),
              ("W5", (FZ, 6 * K)), ("b5", (6 * K,))]
    out, o = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = (o, shp)
        o += n
    return out


def unpack(params, K: int) -> dict:
    L = layout(K)
    p = np.asarray(params, dtype=np.float64)
    return {k: p[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in L.items()}


def pack(blocks: dict, K: int) -> np.ndarray:
    L = layout(K)
    out = np.zeros(param_count(K), dtype=np.float64)
    for k, (o, s) in L.items():
        out[o:o + int(np.prod(s))] = np.asarray(blocks[k], np.float64).reshape(-1)
    return out


# -------------------------------------------------------------------- network
def subsample(xyz, P: int) -> np.ndarray:
    """Network input of a cloud: point p takes cloud point floor(p n / P)."""
    xyz = np.asarray(xyz)
    n = len(xyz)
    idx = (np.arange(P, dtype=np.int64) * n) // P
    return xyz[idx]


def forward(params, clouds, K: int, bf16: bool = True) -> dict:
    """clouds: (B, 2, P, 3) with source then reference per pair. Returns the
    activations, the pooled features, the winning points and Y (B, K, 6)."""
    w = unpack(params, K)
    X = np.asarray(clouds, dtype=np.float64)
    B, two, P, _ = X.shape
    assert two == 2
    x = X.reshape(B * 2 * P, 3)
    relu = lambda a: np.maximum(a, 0.0)
    H1 = relu(matmul(x, w["W1"], bf16) + w["b1"])
    H2 = relu(matmul(H1, w["W2"], bf16) + w["b2"])
    H3 = relu(matmul(H2, w["W3"], bf16) + w["b3"])
    H3c = H3.reshape(B * 2, P, F3)
    arg = np.argmax(H3c, axis=1)                       # first maximum
    pooled = np.take_along_axis(H3c, arg[:, None, :], axis=1)[:, 0, :]
    Fcat = pooled.reshape(B, 2 * F3)                   # [source | reference]
    Z = relu(matmul(Fcat, w["W4"], bf16) + w["b4"])
    Y = matmul(Z, w["W5"], bf16) + w["b5"]
    return {"x": x, "H1": H1, "H2": H2, "H3": H3, "arg": arg, "F": Fcat, "Z": Z,
            "Y": Y.reshape(B, K, 6), "B": B, "P": P}


def pool_margin(cache: dict) -> float:
    """Smallest gap between the largest and second-largest value of any pooled
    feature whose maximum is positive (how far every max-pool decision that
    carries gradient is from a tie; a feature that is 0 at every point passes
    no gradient through the ReLU, whichever point wins)."""
    H3c = cache["H3"].reshape(cache["B"] * 2, cache["P"], F3)
    if cache["P"] < 2:
        return np.inf
    s = np.sort(H3c, axis=1)
    gap = s[:, -1, :] - s[:, -2, :]
    live = s[:, -1, :] > 0
    return float(np.min(gap[live])) if live.any() else np.inf


# ------------------------------------------------------------------ set loss
def _diff(u, v):
    d = np.asarray(u, np.float64) - np.asarray(v, np.float64)
    d = d.copy()
    d[..., 3:] = d[..., 3:] - np.rint(d[..., 3:] / (2 * np.pi)) * (2 * np.pi)
    return d


def kernel(u, v, sigma) -> np.ndarray:
    """k(u_i, v_j) = sum_s exp(-1/2 |(u_i - v_j) / sigma_s|^2), wrapped angles;
    u (n, 6), v (m, 6), sigma (S, 6) -> (n, m)."""
    d = _diff(np.asarray(u)[:, None, :], np.asarray(v)[None, :, :])
    out = np.zeros(d.shape[:2])
    for s in np.atleast_2d(sigma):
        out += np.exp(-0.5 * np.sum((d / s) ** 2, axis=-1))
    return out


def mmd2(X, Y, sigma) -> float:
    """Biased MMD^2 between particle sets X and Y (K x 6 each)."""
    K = len(X)
    return float((kernel(X, X, sigma).sum() + kernel(Y, Y, sigma).sum()
                  - 2.0 * kernel(X, Y, sigma).sum()) / (K * K))


def mmd2_grad(X, Y, sigma) -> np.ndarray:
    """d mmd2(X, Y) / dX: (2 / K^2) sum_j [grad_u k(x_i, x_j) - grad_u k(x_i, y_j)]
    with grad_u exp(-1/2 |d / s|^2) = -exp(...) d / s^2."""
    K = len(X)

    def grad_u(U, V):
        d = _diff(np.asarray(U)[:, None, :], np.asarray(V)[None, :, :])
        g = np.zeros(d.shape)
        for s in np.atleast_2d(sigma):
            e = np.exp(-0.5 * np.sum((d / s) ** 2, axis=-1))
            g += -e[..., None] * d / (s * s)
        return g.sum(axis=1)

    return 2.0 / (K * K) * (grad_u(X, X) - grad_u(X, Y))


# ------------------------------------------------------------------ backward
def loss_and_grad(params, clouds, targets, K: int, sigma, bf16: bool = True):
    """Per-pair losses L_b and the gradient of mean_b L_b (flat FP64)."""
    w = unpack(params, K)
    c = forward(params, clouds, K, bf16)
    B, P = c["B"], c["P"]
    T = np.asarray(targets, np.float64)
    losses = np.array([mmd2(c["Y"][b], T[b], sigma) for b in range(B)])
    dY = np.stack([mmd2_grad(c["Y"][b], T[b], sigma) for b in range(B)]) / B
    dY = dY.reshape(B, 6 * K)
    g = {}
    # head
    g["W5"] = matmul(c["Z"].T, dY, bf16)
    g["b5"] = dY.sum(axis=0)
    dZ = matmul(dY, w["W5"].T, bf16) * (c["Z"] > 0)
    g["W4"] = matmul(c["F"].T, dZ, bf16)
    g["b4"] = dZ.sum(axis=0)
    dF = matmul(dZ, w["W4"].T, bf16)
    # max-pool: pooled feature f of cloud cl is the value of point arg[cl, f],
    # so its gradient lands on that point's row of the last layer's output
    npts = B * 2 * P
    dH3 = np.zeros((npts, F3))
    win = np.arange(B * 2)[:, None] * P + c["arg"]                 # (clouds, F3) point rows
    dH3[win.reshape(-1), np.tile(np.arange(F3), B * 2)] = dF.reshape(B * 2, F3).reshape(-1)
    dA3 = dH3 * (c["H3"] > 0)
    g["W3"] = matmul(c["H2"].T, dA3, bf16)
    g["b3"] = dA3.sum(axis=0)
    dA2 = matmul(dA3, w["W3"].T, bf16) * (c["H2"] > 0)
    g["W2"] = matmul(c["H1"].T, dA2, bf16)
    g["b2"] = dA2.sum(axis=0)
    dA1 = matmul(dA2, w["W2"].T, bf16) * (c["H1"] > 0)
    g["W1"] = matmul(c["x"].T, dA1, bf16)
    g["b1"] = dA1.sum(axis=0)
    return losses, pack(g, K), c


def loss_only(params, clouds, targets, K: int, sigma, bf16: bool = False) -> float:
    c = forward(params, clouds, K, bf16)
    T = np.asarray(targets, np.float64)
    return float(np.mean([mmd2(c["Y"][b], T[b], sigma) for b in range(c["B"])]))


# --------------------------------------------------------------------- Adam
def adam(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One bias-corrected Adam step (t = step number after the increment)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return w, m, v
