"""Oracle for the subpixel stage (TEST INFRASTRUCTURE ONLY; never imported by
the product path, shares no code with the GPU library).

Classical estimator (Photon Subpixel Resolution section, Fig. f): the centroid
of the hit's 3x3 signal with pixels within noise zeroed -- momentum over
droplet, Dx = sum(s*dx)/sum(s) and likewise Dy -- followed by the
linearization the paper calls for ("the centroids require linearization to
yield actual positions"), done here with the empirical cumulative distribution
of centroids on hits with uniformly distributed impact points (eta
correction).

Learned estimator: a 25-64-64-2 ReLU network on the 5x5 patch scaled by
1/photon_adu.  The GPU runs its matrix products in bfloat16 with float32
accumulation; `mlp_forward` / `mlp_backward` round the same operands to
bfloat16 (round to nearest even) so that GPU and oracle differ only by float32
summation order.  With bf16=False they are the plain float64 definitions that
the tests compare against finite differences.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
N_IN, N_H, N_OUT = 25, 64, 2
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 5954


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    a = np.ascontiguousarray(x, dtype=F32)
    b = a.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(F32).reshape(a.shape)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n]).reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name]).reshape(-1) for name, _ in SHAPES])


def init_params(seed):
    """He-uniform weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name[0] == "W":
            lim = np.sqrt(6.0 / shape[0])
            p[name] = rng.uniform(-lim, lim, size=shape).astype(F32)
        else:
            p[name] = np.zeros(shape, F32)
    return pack(p)


def mlp_forward(theta, patches, photon_adu=150.0, bf16_ops=True):
    """patches [B,5,5] -> (y [B,2], cache)."""
    p = unpack(theta)
    r = (lambda a: bf16(a)) if bf16_ops else (lambda a: np.asarray(a, np.float64))
    dt = F32 if bf16_ops else np.float64
    x = np.asarray(patches, dt).reshape(len(patches), N_IN) * dt(1.0 / photon_adu)
    xb = r(x)
    z1 = xb.astype(dt) @ r(p["W1"]).astype(dt) + p["b1"].astype(dt)
    h1 = np.maximum(z1, 0)
    h1b = r(h1)
    z2 = h1b.astype(dt) @ r(p["W2"]).astype(dt) + p["b2"].astype(dt)
    h2 = np.maximum(z2, 0)
    h2b = r(h2)
    y = h2b.astype(dt) @ r(p["W3"]).astype(dt) + p["b3"].astype(dt)
    return y, dict(xb=xb, z1=z1, h1b=h1b, z2=z2, h2b=h2b, p=p)


def mlp_loss(y, target):
    """L = sum((y - t)^2) / (2 B)."""
    d = np.asarray(y, np.float64) - np.asarray(target, np.float64)
    return float(np.sum(d * d) / (2 * len(y)))


def mlp_backward(theta, patches, target, photon_adu=150.0, bf16_ops=True):
    """Gradient of mlp_loss with respect to the packed parameters."""
    y, c = mlp_forward(theta, patches, photon_adu, bf16_ops)
    p = c["p"]
    r = (lambda a: bf16(a)) if bf16_ops else (lambda a: np.asarray(a, np.float64))
    dt = F32 if bf16_ops else np.float64
    B = len(y)
    dy = (y.astype(dt) - np.asarray(target, dt)) * dt(1.0 / B)
    dyb = r(dy)
    g = {}
    g["W3"] = c["h2b"].astype(dt).T @ dyb.astype(dt)
    g["b3"] = dy.sum(axis=0)
    dh2 = (dyb.astype(dt) @ r(p["W3"]).astype(dt).T) * (c["z2"] > 0)
    dh2b = r(dh2)
    g["W2"] = c["h1b"].astype(dt).T @ dh2b.astype(dt)
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2b.astype(dt) @ r(p["W2"]).astype(dt).T) * (c["z1"] > 0)
    dh1b = r(dh1)
    g["W1"] = c["xb"].astype(dt).T @ dh1b.astype(dt)
    g["b1"] = dh1.sum(axis=0)
    return pack(g), mlp_loss(y, target)


def adam(theta, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (float32), step counted from 1."""
    m = (F32(b1) * m + F32(1 - b1) * grad).astype(F32)
    v = (F32(b2) * v + F32(1 - b2) * grad * grad).astype(F32)
    mh = m / F32(1 - b1 ** step)
    vh = v / F32(1 - b2 ** step)
    theta = (theta - F32(lr) * mh / (np.sqrt(vh) + F32(eps))).astype(F32)
    return theta, m, v


# ---------------------------------------------------------------------------
# classical estimator
# ---------------------------------------------------------------------------
def centroid(patches, t_nb):
    """Masked 3x3 centroid (dy, dx) of each 5x5 patch, float32, fixed order:
    rows top to bottom, columns left to right.  0 where the masked sum is 0."""
    P = np.asarray(patches, F32)
    n = len(P)
    s = np.zeros(n, F32)
    sy = np.zeros(n, F32)
    sx = np.zeros(n, F32)
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            v = P[:, 2 + dr, 2 + dc]
            m = np.where(v > F32(t_nb), v, F32(0))
            s = (s + m).astype(F32)
            sy = (sy + m * F32(dr)).astype(F32)
            sx = (sx + m * F32(dc)).astype(F32)
    with np.errstate(invalid="ignore", divide="ignore"):
        cy = np.where(s > 0, sy / np.where(s > 0, s, F32(1)), F32(0)).astype(F32)
        cx = np.where(s > 0, sx / np.where(s > 0, s, F32(1)), F32(0)).astype(F32)
    return np.stack([cy, cx], axis=1)


def eta_bin_pos(c, nbins):
    """Position of centroid coordinates on [-1, 1] in units of bins, in
    float32: (clamp(c, -1, 1) + 1) * 0.5 * nbins.  The bin of c is
    min(floor(pos), nbins - 1); float32 takes this integer decision on both
    sides."""
    c = np.clip(np.asarray(c, F32), F32(-1), F32(1))
    return ((c + F32(1)) * F32(0.5) * F32(nbins)).astype(F32)


def eta_table(centroids, nbins=1023):
    """Per axis, the empirical CDF of the centroid coordinate at the nbins + 1
    bin edges: table[a][b] = (number of centroids in bins < b) / n, float32
    (quotient formed in float64).  An odd nbins puts 0 inside a bin."""
    c = np.asarray(centroids)
    out = np.empty((2, nbins + 1), F32)
    for a in range(2):
        b = np.minimum(np.floor(eta_bin_pos(c[:, a], nbins)).astype(np.int64), nbins - 1)
        h = np.bincount(b, minlength=nbins)
        out[a, 0] = 0.0
        out[a, 1:] = (np.cumsum(h) / float(len(b))).astype(F32)
    return out


def eta_apply(centroids, table):
    """Position = CDF(c) - 1/2 with the CDF linear between table edges, in
    float32: t = bin position, i = min(floor(t), nbins - 1), f = t - i,
    table[i] (1 - f) + table[i + 1] f - 0.5 evaluated left to right."""
    nb = table.shape[1] - 1
    c = np.asarray(centroids)
    out = np.empty((len(c), 2), F32)
    for a in range(2):
        t = eta_bin_pos(c[:, a], nb)
        i = np.minimum(np.floor(t).astype(np.int64), nb - 1)
        f = (t - i.astype(F32)).astype(F32)
        lo = (table[a, i] * (F32(1) - f)).astype(F32)
        hi = (table[a, i + 1] * f).astype(F32)
        out[:, a] = ((lo + hi).astype(F32) - F32(0.5)).astype(F32)
    return out
