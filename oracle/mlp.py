"""CPU oracle of the learned edge heuristic -- TEST INFRASTRUCTURE ONLY.

A small MLP scores each candidate edge (i, r -> j) from local geometry; its
score sigma(z) replaces eta = 1/d in the random proportional rule (Section 2,
Eq. 1).  This module is the reference the GPU kernels are checked against:
plain numpy, FP64 arithmetic on the same BF16-rounded operands.

Features (8 per candidate slot), each computed with exactly rounded FP64
operations from integers and rounded once to FP32 (then to BF16 for the
network), so both sides obtain the same bits:
  0  d_ij / max(d_i0, 1)          distance over the nearest-candidate distance
  1  d_ij / max(d_i,k-1, 1)       distance over the k-th candidate distance
  2  r / (k - 1)                  candidate rank
  3  rev / (k - 1), or 1          rank of i in j's list (1 when absent)
  4  cos(angle)                   between the edge i->j and the direction from
  5  sin(angle)                   i to the centroid of i's candidates (1, 0 if undefined)
  6  d_i,k-1 / mean_i d_i,k-1     local radius at i (density), instance-normalised
  7  d_j,k-1 / mean_i d_i,k-1     the same at j

Network (parameters theta in FP32; W1, W2, W3 used as BF16):
  a1 = W1b x + b1, h1 = relu(a1), h1b = bf16(h1)          (64)
  a2 = W2b h1b + b2, h2 = relu(a2), h2b = bf16(h2)        (64)
  z  = W3b . h2b + b3,  score = sigmoid(z)
Loss: mean over edges of w_e * BCE(sigmoid(z_e), y_e), w = pos_weight for y = 1.
Backward, with BF16 rounding where the GPU feeds matrix cores:
  g = w (sigmoid(z) - y) / E
  dW3 = sum_e g h2b, db3 = sum_e g
  d2 = (W3b g) * [a2 > 0],  dW2 = sum_e bf16(d2) h1b^T,  db2 = sum_e d2
  d1 = (W2b^T bf16(d2)) * [a1 > 0],  dW1 = sum_e bf16(d1) x^T,  db1 = sum_e d1
"""
from __future__ import annotations

import numpy as np

F, H = 8, 64
# offsets of the parameter blocks in the flat FP32 master vector
OFF = {"W1": 0, "b1": 512, "W2": 576, "b2": 4672, "W3": 4736, "b3": 4800}
NPARAM = 4801


def bf16(a) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) from FP32; returned as float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), np.float32(np.nan), out)


def bf16_bits(a) -> np.ndarray:
    return (bf16(a).view(np.uint32) >> 16).astype(np.uint16)


def unpack(theta):
    t = np.asarray(theta, dtype=np.float32)
    return dict(W1=t[0:512].reshape(H, F), b1=t[512:576], W2=t[576:4672].reshape(H, H),
                b2=t[4672:4736], W3=t[4736:4800], b3=t[4800])


def init_theta(seed: int) -> np.ndarray:
    """He-style initial weights from a seeded generator (test inputs, not method arithmetic)."""
    rng = np.random.default_rng(seed)
    t = np.zeros(NPARAM, np.float32)
    t[0:512] = rng.normal(0, np.sqrt(2.0 / F), 512)
    t[576:4672] = rng.normal(0, np.sqrt(2.0 / H), H * H)
    t[4736:4800] = rng.normal(0, np.sqrt(1.0 / H), H)
    return t


# ---------------------------------------------------------------- features
def features(xy, nn, nnd, rev) -> np.ndarray:
    """FP32 features [n, k, 8] (exactly rounded FP64 operations, one rounding to FP32)."""
    xy = np.asarray(xy, np.int64)
    nn = np.asarray(nn, np.int64)
    nnd = np.asarray(nnd, np.int64)
    rev = np.asarray(rev, np.int64)
    n, k = nn.shape
    x, y = xy[:, 0], xy[:, 1]
    d = nnd.astype(np.float64)
    d0 = np.maximum(nnd[:, :1], 1).astype(np.float64)
    dk = np.maximum(nnd[:, k - 1:k], 1).astype(np.float64)
    out = np.empty((n, k, F), np.float32)
    out[..., 0] = (d / d0).astype(np.float32)
    out[..., 1] = (d / dk).astype(np.float32)
    km1 = float(k - 1) if k > 1 else 1.0
    r = np.broadcast_to(np.arange(k, dtype=np.float64), (n, k))
    out[..., 2] = (r / km1).astype(np.float32) if k > 1 else np.float32(0.0)
    out[..., 3] = np.where(rev >= 0, (rev.astype(np.float64) / km1), 1.0).astype(np.float32)
    ex = (x[nn] - x[:, None]).astype(np.float64)
    ey = (y[nn] - y[:, None]).astype(np.float64)
    cx = (x[nn] - x[:, None]).sum(1).astype(np.float64)[:, None]
    cy = (y[nn] - y[:, None]).sum(1).astype(np.float64)[:, None]
    dot = ex * cx + ey * cy
    crs = ex * cy - ey * cx
    ne = np.sqrt(ex * ex + ey * ey)
    nc = np.sqrt(cx * cx + cy * cy)
    den = ne * nc
    ok = den > 0
    safe = np.where(ok, den, 1.0)
    out[..., 4] = np.where(ok, dot / safe, 1.0).astype(np.float32)
    out[..., 5] = np.where(ok, crs / safe, 0.0).astype(np.float32)
    rk = nnd[:, k - 1]
    mean = float(int(rk.sum())) / float(n)
    if mean > 0:
        out[..., 6] = (rk.astype(np.float64)[:, None] / mean).astype(np.float32)
        out[..., 7] = (rk[nn].astype(np.float64) / mean).astype(np.float32)
    else:
        out[..., 6] = 1.0
        out[..., 7] = 1.0
    return out


# ---------------------------------------------------------------- network
def near_bf16_step(v, delta):
    """True where moving v by up to `delta` could change relu-then-BF16 of it:
    a BF16 rounding midpoint or 0 lies within delta, or delta spans a BF16 step."""
    v = np.asarray(v, np.float64)
    delta = np.asarray(delta, np.float64)
    a = np.abs(v).astype(np.float32)
    u = a.view(np.uint32).astype(np.int64)
    lo = ((u >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    step = (((u >> 16) + 1) << 16).astype(np.uint32).view(np.float32).astype(np.float64) - lo
    off = np.abs(np.abs(v) - (lo + 0.5 * step))         # distance to the midpoint of v's step
    return (off <= delta) | (step - off <= delta) | (np.abs(v) <= delta) | (delta >= 0.25 * step)


def forward(theta, X, quantize=True, want_cache=False):
    """Logits z [E] for FP32 features X [E, 8]; FP64 arithmetic.
    With quantize, operands are BF16 as on the matrix cores."""
    P = unpack(theta)
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float32))
    W1, W2, W3 = (q(P[w]).astype(np.float64) for w in ("W1", "W2", "W3"))
    b1, b2, b3 = P["b1"].astype(np.float64), P["b2"].astype(np.float64), float(P["b3"])
    xb = q(X).astype(np.float64)                                   # [E, 8]
    a1 = xb @ W1.T + b1                                            # [E, 64]
    s1 = np.abs(xb) @ np.abs(W1).T + np.abs(b1)
    h1 = np.maximum(a1, 0.0)
    h1b = (q(h1.astype(np.float32)) if quantize else h1).astype(np.float64)
    a2 = h1b @ W2.T + b2
    s2 = np.abs(h1b) @ np.abs(W2).T + np.abs(b2)
    h2 = np.maximum(a2, 0.0)
    h2b = (q(h2.astype(np.float32)) if quantize else h2).astype(np.float64)
    z = h2b @ W3 + b3
    if not want_cache:
        return z
    return z, dict(xb=xb, a1=a1, s1=s1, h1b=h1b, a2=a2, s2=s2, h2b=h2b, W1=W1, W2=W2, W3=W3,
                   b3=b3)


# Worst-case relative error of an FP32 sum of K exact products plus a bias,
# in any order: (K + 1) 2^-24 of the sum of magnitudes, taken with a factor 2
# of margin (K = 8, 64, 64 for the three layers).
GAMMA1, GAMMA2 = 2.0**-20, 2.0**-17


def forward_bound(theta, X):
    """(z, dz, flip) for an implementation that forms the same BF16 operands
    but accumulates in FP32 in another order: |z_impl - z| <= dz.  A hidden
    value whose FP32 error could cross a BF16 rounding point (or 0) may round
    differently; `flip` marks the edges where that is possible, and dz then
    carries the propagated change (one BF16 step, 2^-7 relative at most)."""
    z, c = forward(theta, X, True, want_cache=True)
    aW2, aW3 = np.abs(c["W2"]), np.abs(c["W3"])
    d1 = GAMMA1 * c["s1"]
    n1 = near_bf16_step(c["a1"], d1)
    dh1 = np.where(n1, d1 + 2.0**-7 * (np.abs(c["a1"]) + d1), 0.0)
    d2 = GAMMA2 * (c["s2"] + dh1 @ aW2.T) + dh1 @ aW2.T
    n2 = near_bf16_step(c["a2"], d2)
    dh2 = np.where(n2, d2 + 2.0**-7 * (np.abs(c["a2"]) + d2), 0.0)
    Sz = np.abs(c["h2b"]) @ aW3 + abs(c["b3"])
    dz = GAMMA2 * (Sz + dh2 @ aW3) + dh2 @ aW3
    return z, dz, n1.any(1) | n2.any(1)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-np.asarray(z, np.float64)))


def loss(theta, X, y, pos_weight, quantize=True):
    z = forward(theta, X, quantize)
    y = np.asarray(y, np.float64)
    w = np.where(y > 0.5, pos_weight, 1.0)
    # BCE with logits: log(1 + exp(z)) - y z
    return float(np.mean(w * (np.logaddexp(0.0, z) - y * z)))


def backward(theta, X, y, pos_weight, quantize=True):
    """(loss, grad [NPARAM] float64) of the weighted mean BCE."""
    z, c = forward(theta, X, quantize, want_cache=True)
    y = np.asarray(y, np.float64)
    E = len(y)
    w = np.where(y > 0.5, pos_weight, 1.0)
    L = float(np.mean(w * (np.logaddexp(0.0, z) - y * z)))
    g = w * (sigmoid(z) - y) / E                                   # [E]
    q = (lambda a: bf16(a.astype(np.float32)).astype(np.float64)) if quantize else (lambda a: a)
    grad = np.zeros(NPARAM, np.float64)
    grad[OFF["W3"]:OFF["W3"] + H] = g @ c["h2b"]
    grad[OFF["b3"]] = g.sum()
    d2 = (g[:, None] * c["W3"][None, :]) * (c["a2"] > 0)          # [E, 64]
    grad[OFF["W2"]:OFF["W2"] + H * H] = (q(d2).T @ c["h1b"]).ravel()
    grad[OFF["b2"]:OFF["b2"] + H] = d2.sum(0)
    d1 = (q(d2) @ c["W2"]) * (c["a1"] > 0)                        # [E, 64]
    grad[OFF["W1"]:OFF["W1"] + H * F] = (q(d1).T @ c["xb"]).ravel()
    grad[OFF["b1"]:OFF["b1"] + H] = d1.sum(0)
    return L, grad


def labels_from_tour(nn, tour) -> np.ndarray:
    """y[i, r] = 1 when the edge {i, nn[i][r]} is an edge of the closed tour."""
    nn = np.asarray(nn)
    n, k = nn.shape
    t = np.asarray(tour, np.int64)
    nxt = np.empty(n, np.int64)
    prv = np.empty(n, np.int64)
    nxt[t] = np.roll(t, -1)
    prv[t] = np.roll(t, 1)
    return ((nn == nxt[:, None]) | (nn == prv[:, None])).astype(np.uint8)


def backward_scale(theta, X, y, pos_weight):
    """S_p = sum over edges of |term| for every gradient entry p: the gradient
    formulas of `backward` with every factor replaced by its absolute value.
    Scales the error bound of an FP32-accumulated gradient."""
    z, c = forward(theta, X, True, want_cache=True)
    y = np.asarray(y, np.float64)
    E = len(y)
    w = np.where(y > 0.5, pos_weight, 1.0)
    g = np.abs(w * (sigmoid(z) - y) / E)
    aW2, aW3 = np.abs(c["W2"]), np.abs(c["W3"])
    S = np.zeros(NPARAM, np.float64)
    S[OFF["W3"]:OFF["W3"] + H] = g @ c["h2b"]
    S[OFF["b3"]] = g.sum()
    d2 = (g[:, None] * aW3[None, :]) * (c["a2"] > 0)
    S[OFF["W2"]:OFF["W2"] + H * H] = (d2.T @ c["h1b"]).ravel()
    S[OFF["b2"]:OFF["b2"] + H] = d2.sum(0)
    d1 = (d2 @ aW2) * (c["a1"] > 0)
    S[OFF["W1"]:OFF["W1"] + H * F] = (d1.T @ np.abs(c["xb"])).ravel()
    S[OFF["b1"]:OFF["b1"] + H] = d1.sum(0)
    return S


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) in FP32: moments, bias
    corrections, parameter step.  beta1 and beta2 are FP32 values, used as
    such in the moments and (powers in FP64, rounded once) in the bias
    corrections.  Returns new (theta, m, v)."""
    f = np.float32
    t, m, v, g = (np.asarray(a, f) for a in (theta, m, v, grad))
    b1, b2 = f(beta1), f(beta2)
    m = b1 * m + (f(1) - b1) * g
    v = b2 * v + (f(1) - b2) * (g * g)
    c1 = f(1.0 - float(b1) ** step)
    c2 = f(1.0 - float(b2) ** step)
    mh = m / c1
    vh = v / c2
    t = t - f(lr) * mh / (np.sqrt(vh) + f(eps))
    return t.astype(f), m.astype(f), v.astype(f)
