"""FP64 reference of the learned warm start (per-sample features and the MLP
that maps them to initial dual values).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: only ``tests/``, the
smoke check and the CPU-baseline leg of ``bench.py`` use it; it shares no
code with the HIP library.

The warm start is not part of the paper's method: the paper's solver starts
from zero duals (Algorithm 1).  The dual problem of Eq. 4 is invariant under
(alpha + t 1, beta - t 1) when the marginals have equal mass, so the targets
the network learns are gauge-fixed (a.alpha = b.beta).

Features of a sample (all distances squared and multiplied by the cost scale
s, the factor that normalises the cost of Sec. 2.1):
  * the feature vector times sqrt(s);
  * the distance to its own centroid: a source sample's class centroid; a
    target sample's pseudo-class centroid, where the pseudo-class of a target
    is the class of its nearest source centroid and the pseudo-class centroid
    is the mean of the targets that share it;
  * the least distance to the other side's centroids (target pseudo-class
    centroids for a source sample, source class centroids for a target);
  * the fraction of its side's samples in its (pseudo-)class;
  * side (0 source, 1 target), log gamma, log mu, log n_src, log n_tgt.

The network: Linear(d_in, w) - GELU - Linear(w, w) - GELU - Linear(w, 1),
GELU(z) = z Phi(z) with the exact normal CDF.  Parameters are one flat
vector: W1 [d_in, w] (row = input), b1 [w], W2 [w, w], b2 [w], w3 [w], b3.
With ``bf16=True`` every operand of the three products is rounded to
bfloat16 (round to nearest even, from its float32 value), the precision the
device network multiplies in; sums stay exact here.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

LOG_MU_FLOOR = 1e-8


# ---------------------------------------------------------------- rounding
def bf16_round(x):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- features
def features(xs, xt, labels, n_groups, scale, gamma, mu):
    """Feature rows of one instance: (F_src [n, d+8], F_tgt [m, d+8],
    pseudo_labels [m])."""
    xs = np.asarray(xs, dtype=np.float64)
    xt = np.asarray(xt, dtype=np.float64)
    labels = np.asarray(labels)
    n, d = xs.shape
    m = xt.shape[0]
    s = float(scale)
    present = np.array([l for l in range(n_groups) if np.any(labels == l)])
    cs = np.stack([xs[labels == l].mean(0) for l in present])           # source class centroids
    d_ts = ((xt[:, None, :] - cs[None, :, :]) ** 2).sum(-1)             # [m, classes]
    pk = np.argmin(d_ts, axis=1)                                         # first minimum: smallest label
    pseudo = present[pk]
    tp = np.unique(pseudo)
    ct_ = {l: xt[pseudo == l].mean(0) for l in tp}                        # target pseudo-class centroids
    ctm = np.stack([ct_[l] for l in tp])
    logs = [math.log(gamma), math.log(max(mu, LOG_MU_FLOOR)), math.log(n), math.log(m)]

    Fs = np.zeros((n, d + 8))
    for i in range(n):
        l = labels[i]
        own = ((xs[i] - cs[np.searchsorted(present, l)]) ** 2).sum() * s
        other = ((xs[i][None, :] - ctm) ** 2).sum(-1).min() * s
        frac = np.count_nonzero(labels == l) / n
        Fs[i, :d] = xs[i] * math.sqrt(s)
        Fs[i, d:] = [own, other, frac, 0.0] + logs
    Ft = np.zeros((m, d + 8))
    for j in range(m):
        l = pseudo[j]
        own = ((xt[j] - ct_[l]) ** 2).sum() * s
        other = d_ts[j].min() * s
        frac = np.count_nonzero(pseudo == l) / m
        Ft[j, :d] = xt[j] * math.sqrt(s)
        Ft[j, d:] = [own, other, frac, 1.0] + logs
    return Fs, Ft, pseudo


def gauge_fix(alpha, beta, a=None, b=None):
    """(alpha - t, beta + t) with t chosen so that a.alpha = b.beta; the
    objective of Eq. 4 is unchanged when sum a = sum b."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    a = np.full(alpha.size, 1.0 / alpha.size) if a is None else np.asarray(a, np.float64)
    b = np.full(beta.size, 1.0 / beta.size) if b is None else np.asarray(b, np.float64)
    t = (a @ alpha - b @ beta) / (a.sum() + b.sum())
    return alpha - t, beta + t


# ---------------------------------------------------------------- network
def n_params(d_in, w):
    return d_in * w + w + w * w + w + w + 1


def unpack(p, d_in, w):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + d_in * w].reshape(d_in, w); o += d_in * w
    b1 = p[o:o + w]; o += w
    W2 = p[o:o + w * w].reshape(w, w); o += w * w
    b2 = p[o:o + w]; o += w
    w3 = p[o:o + w]; o += w
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def init_params(d_in, w, seed):
    """He-style initial parameters drawn from a seeded generator (input to
    both the device network and this reference)."""
    r = np.random.default_rng(seed)
    W1 = r.standard_normal((d_in, w)) * math.sqrt(2.0 / d_in)
    W2 = r.standard_normal((w, w)) * math.sqrt(2.0 / w)
    w3 = r.standard_normal(w) * math.sqrt(1.0 / w)
    p = np.concatenate([W1.ravel(), np.zeros(w), W2.ravel(), np.zeros(w), w3, [0.0]])
    return p.astype(np.float32)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _r(x, on):
    return bf16_round(x) if on else np.asarray(x, dtype=np.float64)


def forward(p, F, d_in, w, bf16=False):
    """Network output [N] and the intermediate values (Z1, H1, Z2, H2)."""
    W1, b1, W2, b2, w3, b3 = unpack(p, d_in, w)
    F = np.asarray(F, dtype=np.float64)
    Z1 = _r(F, bf16) @ _r(W1, bf16) + b1
    H1 = gelu(Z1)
    Z2 = _r(H1, bf16) @ _r(W2, bf16) + b2
    H2 = gelu(Z2)
    out = _r(H2, bf16) @ _r(w3, bf16) + b3
    return out, (Z1, H1, Z2, H2)


def loss_grad(p, F, y, d_in, w, bf16=False):
    """Mean squared error over the N rows and its gradient (flat, same
    layout as the parameters).  With bf16 the operands of every product of
    the backward pass are rounded as in the forward pass."""
    W1, b1, W2, b2, w3, b3 = unpack(p, d_in, w)
    F = np.asarray(F, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N = F.shape[0]
    out, (Z1, H1, Z2, H2) = forward(p, F, d_in, w, bf16)
    e = out - y
    loss = float(e @ e) / N
    dout = 2.0 * e / N
    dw3 = _r(H2, bf16).T @ dout
    db3 = dout.sum()
    dZ2 = np.outer(dout, _r(w3, bf16)) * gelu_grad(Z2)
    dW2 = _r(H1, bf16).T @ _r(dZ2, bf16)
    db2 = dZ2.sum(0)
    dZ1 = (_r(dZ2, bf16) @ _r(W2, bf16).T) * gelu_grad(Z1)
    dW1 = _r(F, bf16).T @ _r(dZ1, bf16)
    db1 = dZ1.sum(0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])
    return loss, g


def adam_step(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma and Ba): bias-corrected first and second moments."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
