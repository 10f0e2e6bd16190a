"""Learned starting guess for the SCC power series, in float64.

Test infrastructure only (see the package docstring).

The paper starts every SCC's series from P_0 = W'_C (Sec. 4.3.2) and notes
that a previous ranking could serve as the initial rank (Sec. 7).  Here a
small network predicts, per SCC vertex, the logarithm of its rank relative to
the component's mean weight, from four local quantities.  The prediction R_0
is only a starting point: the series is then run on the residual
    r_0 = W'_C + c A_CC^T R_0 - R_0,     R = R_0 + sum_k (c A_CC^T)^k r_0,
which converges to the same R_C = (I - c A_CC^T)^{-1} W'_C (Def. 3.5,
Sec. 4.3) whatever R_0 is.  The guess is kept for a component only when
||r_0||_1 < ||c A_CC^T W'_C||_1, the norm of the first term the plain start
would add; otherwise the component falls back to the plain series.

Features of an SCC vertex v (s_C = ||W'_C||_1 / |C|, loops ignored,
repeated edges counted):
    f0 = log(1 + in-degree of v)
    f1 = log(1 + out-degree of v)
    f2 = log(1 + (W'_v - W_v) / s_C)       rank flowing in from higher levels
    f3 = log(1 + R1_v / s_C),  R1 = W'_C + c A_CC^T W'_C   (one series step)
Target: t_v = log(R_v / s_C).  Prediction: R_0,v = s_C exp(y_v).

Network: 4 -> 64 -> 64 -> 1, GELU (exact, with erf) after the two hidden
layers.  Parameters in one flat vector, in this order: W1 [64 x 4] row-major,
b1 [64], W2 [64 x 64] row-major, b2 [64], W3 [1 x 64], b3 [1]; 4545 values.
Training minimises the mean squared error of y against t with Adam (Kingma
and Ba, 2015: bias-corrected first and second moment estimates).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H = 64
N_IN = 4
SHAPES = [("W1", (H, N_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (1, H)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Views of the flat parameter vector, in the documented order."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        fan_in = shape[1] if len(shape) == 2 else (N_IN if name == "b1" else H)
        b = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, size=int(np.prod(shape))))
    return np.concatenate(parts)


def gelu(x):
    """x * Phi(x) with the exact normal CDF."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, X, keep=False):
    """y [B] for features X [B, 4]; with keep, also the intermediate values."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(z2)
    y = (h2 @ P["W3"].T)[:, 0] + P["b3"][0]
    if keep:
        return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)
    return y


def loss_and_grad(theta, X, t):
    """L = mean_i (y_i - t_i)^2 and dL/dtheta by the chain rule."""
    P = unpack(theta)
    y, c = forward(theta, X, keep=True)
    B = len(y)
    d = y - np.asarray(t, dtype=np.float64)
    L = float(np.mean(d * d))
    dy = 2.0 * d / B                       # [B]
    gW3 = dy @ c["h2"]                     # [64]
    gb3 = dy.sum()
    dh2 = dy[:, None] * P["W3"][0][None, :]
    dz2 = dh2 * gelu_grad(c["z2"])
    gW2 = dz2.T @ c["h1"]
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ P["W2"]
    dz1 = dh1 * gelu_grad(c["z1"])
    gW1 = dz1.T @ c["X"]
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), [gb3]])
    return L, g


class Adam:
    """Adam with bias correction; the state is two moment vectors and a step count."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.beta1 * self.m + (1.0 - self.beta1) * g
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * g * g
        mhat = self.m / (1.0 - self.beta1 ** self.t)
        vhat = self.v / (1.0 - self.beta2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def in_degree(n, row_ptr, col):
    """In-degree without self-loops, duplicates counted."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    keep = src != col
    return np.bincount(col[keep], minlength=n).astype(np.int64)


def scc_features(Vs, Wp, W, local, nc, sub, c, indeg, outdeg):
    """Features [len(Vs), 4] and the per-component scale s_C for the SCC
    vertices Vs of one level (local: component index of each, sub: A^T
    restricted to Vs, block diagonal)."""
    size = np.bincount(local, minlength=nc).astype(np.float64)
    s = np.bincount(local, weights=Wp, minlength=nc) / np.maximum(size, 1.0)
    sv = s[local]
    safe = np.where(sv > 0, sv, 1.0)
    R1 = Wp + c * (sub @ Wp)
    F = np.stack([np.log1p(indeg[Vs].astype(np.float64)), np.log1p(outdeg[Vs].astype(np.float64)),
                  np.log1p((Wp - W[Vs]) / safe), np.log1p(R1 / safe)], axis=1)
    return F, s, R1


GELU_LIPSCHITZ = 1.1289  # max over x of |d/dx x Phi(x)| (at x = +-sqrt(2))


def forward_bf16_bound(theta, X, u=2.0 ** -8):
    """First-order bound on |y_computed - y| when every matrix-product operand
    (weights, features, hidden activations) is rounded to bfloat16 (unit
    roundoff u) and products are summed exactly: per layer, rounding both
    factors of each product adds at most 2u |W||h|, an input error e adds
    |W| e, and GELU multiplies errors by at most GELU_LIPSCHITZ."""
    P = unpack(theta)
    Xs = np.asarray(X, dtype=np.float64)
    _, c = forward(theta, Xs, keep=True)
    X = np.abs(Xs)
    aW1, aW2, aW3 = np.abs(P["W1"]), np.abs(P["W2"]), np.abs(P["W3"][0])
    e1 = 2 * u * (X @ aW1.T)
    eh1 = GELU_LIPSCHITZ * e1
    h1 = np.abs(c["h1"])
    e2 = 2 * u * (h1 @ aW2.T) + eh1 @ aW2.T
    eh2 = GELU_LIPSCHITZ * e2
    h2 = np.abs(c["h2"])
    return 2 * u * (h2 @ aW3) + eh2 @ aW3


def to_bf16(a):
    """Round to bfloat16 (nearest even) through the float32 bit pattern."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    """The network with every matrix-product operand rounded to bfloat16 and
    everything else (sums, biases, GELU) in float64: the arithmetic a
    BF16-operand, wide-accumulator implementation performs, up to the order of
    its sums."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = gelu(to_bf16(X) @ to_bf16(P["W1"]).T + P["b1"])
    h2 = gelu(to_bf16(h1) @ to_bf16(P["W2"]).T + P["b2"])
    return to_bf16(h2) @ to_bf16(P["W3"][0]) + P["b3"][0]


GELU_CURVATURE = 0.7979  # max over x of |d^2/dx^2 x Phi(x)| = |phi(x) (2 - x^2)| (at x = 0: 2 / sqrt(2 pi))


def loss_and_grad_bf16(theta, X, t):
    """loss_and_grad with every matrix-product operand of the forward and the
    backward pass rounded to bfloat16 (products summed in float64, everything
    else exact): the arithmetic a BF16-operand, wide-accumulator gradient
    performs, up to the order of its sums."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    b = to_bf16
    z1 = b(X) @ b(P["W1"]).T + P["b1"]
    h1 = gelu(z1)
    z2 = b(h1) @ b(P["W2"]).T + P["b2"]
    h2 = gelu(z2)
    y = b(h2) @ b(P["W3"][0]) + P["b3"][0]
    B = len(y)
    d = y - np.asarray(t, dtype=np.float64)
    L = float(np.mean(d * d))
    dy = 2.0 * d / B
    gW3 = b(dy) @ b(h2)
    gb3 = dy.sum()
    dh2 = b(dy)[:, None] * b(P["W3"][0])[None, :]
    dz2 = dh2 * gelu_grad(z2)
    gW2 = b(dz2).T @ b(h1)
    gb2 = dz2.sum(axis=0)
    dh1 = b(dz2) @ b(P["W2"])
    dz1 = dh1 * gelu_grad(z1)
    gW1 = b(dz1).T @ b(X)
    gb1 = dz1.sum(axis=0)
    return L, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), [gb3]])


def grad_bf16_bound(theta, X, t, u=2.0 ** -8):
    """First-order bound, entry by entry, on |g_computed - g| for the gradient
    of the mean squared error when every matrix-product operand of the forward
    and backward passes is rounded to bfloat16 (unit roundoff u) and products
    are summed exactly.  Errors are carried through the chain rule as absolute
    bounds: a product of a (error ea) and b (error eb), both rounded, is off by
    at most ea |b| + |a| eb + 2u |a| |b|; an elementwise factor GELU'(z) adds
    |dh| GELU_CURVATURE e_z.  Also returns the magnitude gradient (the same
    sums over absolute values), which bounds float32 accumulation error when
    scaled by the accumulation depth times 2^-24."""
    P = unpack(theta)
    Xs = np.asarray(X, dtype=np.float64)
    y, c = forward(theta, Xs, keep=True)
    B = len(y)
    aX = np.abs(Xs)
    aW1, aW2, aW3 = np.abs(P["W1"]), np.abs(P["W2"]), np.abs(P["W3"][0])
    z1, h1, z2, h2 = c["z1"], np.abs(c["h1"]), c["z2"], np.abs(c["h2"])
    # forward
    e_z1 = 2 * u * (aX @ aW1.T)
    e_h1 = GELU_LIPSCHITZ * e_z1
    e_z2 = 2 * u * (h1 @ aW2.T) + e_h1 @ aW2.T
    e_h2 = GELU_LIPSCHITZ * e_z2
    e_y = 2 * u * (h2 @ aW3) + e_h2 @ aW3
    # backward
    d = y - np.asarray(t, dtype=np.float64)
    dy = np.abs(2.0 * d / B)
    e_dy = 2.0 * e_y / B
    e_gW3 = e_dy @ h2 + dy @ e_h2 + 2 * u * (dy @ h2)
    e_gb3 = e_dy.sum()
    dh2 = dy[:, None] * aW3[None, :]
    e_dh2 = e_dy[:, None] * aW3[None, :] + 2 * u * dh2
    gp2 = np.abs(gelu_grad(z2))
    dz2 = dh2 * gp2
    e_dz2 = e_dh2 * gp2 + dh2 * GELU_CURVATURE * e_z2
    e_gW2 = e_dz2.T @ h1 + dz2.T @ e_h1 + 2 * u * (dz2.T @ h1)
    e_gb2 = e_dz2.sum(axis=0)
    dh1 = dz2 @ aW2
    e_dh1 = e_dz2 @ aW2 + 2 * u * dh1
    gp1 = np.abs(gelu_grad(z1))
    dz1 = dh1 * gp1
    e_dz1 = e_dh1 * gp1 + dh1 * GELU_CURVATURE * e_z1
    e_gW1 = e_dz1.T @ aX + 2 * u * (dz1.T @ aX)
    e_gb1 = e_dz1.sum(axis=0)
    bound = np.concatenate([e_gW1.ravel(), e_gb1, e_gW2.ravel(), e_gb2, e_gW3.ravel(), [e_gb3]])
    mag = np.concatenate([(dz1.T @ aX).ravel(), dz1.sum(axis=0), (dz2.T @ h1).ravel(), dz2.sum(axis=0),
                          dy @ h2, [dy.sum()]])
    return bound, mag
