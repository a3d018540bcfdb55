"""Seeded synthetic inputs for group-sparse smooth-dual OT.

This module only draws random numbers: labelled source features, unlabelled
target features, class labels and the regularisation parameters.  It holds
none of the method's arithmetic (no cost matrix, no dual, no plan), so both
the FP64 oracle and the HIP path can consume the same draws without sharing
any computation.

Every generator returns a dict with float32 features ``xs`` [n_src, d],
``xt`` [n_tgt, d], int32 ``labels`` [n_src] in [0, n_groups), and the
scalars ``gamma``, ``mu``, ``n_groups``.  Naming: ``n_src`` rows are the
labelled source samples (the paper's m), ``n_tgt`` columns the unlabelled
target samples (the paper's n).

Workloads (the paper's datasets are not available; these stand in for them):
  * ``gaussian4_2d``      - 4 isotropic classes in 2-D, target rotated and
                            shifted (small CPU-sized problem).
  * ``blobs``             - many Gaussian blobs in d dims, target = same blobs
                            under a random orthogonal rotation plus a shift
                            (digit-recognition-sized stand-in, 10 classes).
  * ``zipf_blobs``        - 100 classes with Zipf(1.1) sizes (many-class
                            stand-in, the face-recognition setting has 68).
  * ``batch_instances``   - uneven instances with Dirichlet class shares
                            (object-recognition instance sizes 157..1123).
  * ``paper_synthetic``   - the paper's synthetic set: class l has mean
                            (5l, -5) in the source and (5l, 5) in the target,
                            unit normal noise, g samples per class (Sec.
                            Experiment, "Datasets").
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian4_2d",
    "blobs",
    "zipf_sizes",
    "zipf_blobs",
    "batch_instances",
    "instance_from_generator",
    "paper_synthetic",
    "random_duals",
]


def _rng(*seed):
    return np.random.default_rng(list(seed))


def gaussian4_2d(seed: int = 1, per_class: int = 50, radius: float = 3.0,
                 sigma: float = 0.5, gamma: float = 1.0, mu: float = 0.1):
    """Four 2-D Gaussian classes, means on a circle at angles 2*pi*k/4.

    Target: the same mixture (``per_class`` per class, fresh noise) rotated
    by 30 degrees about the origin and shifted by (1, 1)."""
    r = _rng(seed)
    L = 4
    ang = 2 * np.pi * np.arange(L) / L
    means = radius * np.stack([np.cos(ang), np.sin(ang)], 1)
    labels = np.repeat(np.arange(L), per_class)
    xs = means[labels] + sigma * r.standard_normal((labels.size, 2))
    tl = np.repeat(np.arange(L), per_class)
    xt0 = means[tl] + sigma * r.standard_normal((tl.size, 2))
    th = np.deg2rad(30.0)
    rot = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    xt = xt0 @ rot.T + np.array([1.0, 1.0])
    return dict(xs=xs.astype(np.float32), xt=xt.astype(np.float32),
                labels=labels.astype(np.int32), n_groups=L,
                gamma=float(gamma), mu=float(mu))


def _haar_rotation(r, d):
    q, rr = np.linalg.qr(r.standard_normal((d, d)))
    return q * np.sign(np.diag(rr))[None, :]


def _even_sizes(n, L):
    base = np.full(L, n // L)
    base[: n % L] += 1
    return base


def blobs(seed: int = 2, n_src: int = 4096, n_tgt: int = 4096, d: int = 64,
          n_groups: int = 10, mean_var: float = 4.0, shift_var: float = 0.5,
          gamma: float = 0.1, mu: float = 0.1, sizes=None):
    """Gaussian blobs: class means ~ N(0, mean_var I), unit-variance noise.

    Target = the same blobs (class shares as in the source, fresh noise)
    under one Haar-random orthogonal rotation plus one global shift drawn
    from N(0, shift_var I).  Class sizes default to as-even-as-possible."""
    r = _rng(seed)
    L = n_groups
    src_sizes = _even_sizes(n_src, L) if sizes is None else np.asarray(sizes)
    tgt_sizes = _even_sizes(n_tgt, L) if sizes is None or n_tgt != n_src else np.asarray(sizes)
    means = np.sqrt(mean_var) * r.standard_normal((L, d))
    labels = np.repeat(np.arange(L), src_sizes)
    xs = means[labels] + r.standard_normal((labels.size, d))
    tl = np.repeat(np.arange(L), tgt_sizes)
    rot = _haar_rotation(r, d)
    shift = np.sqrt(shift_var) * r.standard_normal(d)
    xt = (means[tl] + r.standard_normal((tl.size, d))) @ rot.T + shift
    # shuffle both sides so that neither the labels nor the target blobs
    # arrive sorted (the library must group and cluster by itself)
    ps = r.permutation(labels.size)
    pt = r.permutation(tl.size)
    return dict(xs=xs[ps].astype(np.float32), xt=xt[pt].astype(np.float32),
                labels=labels[ps].astype(np.int32), n_groups=L,
                gamma=float(gamma), mu=float(mu))


def zipf_sizes(n: int, L: int, s: float = 1.1, floor: int = 32):
    """Class sizes proportional to k^-s (k = 1..L), at least ``floor`` each;
    the rounding remainder goes to the largest class."""
    w = np.arange(1, L + 1, dtype=np.float64) ** (-s)
    sz = np.maximum(np.floor(n * w / w.sum()).astype(np.int64), floor)
    sz[0] += n - sz.sum()
    assert sz.min() >= floor and sz.sum() == n
    return sz


def zipf_blobs(seed: int = 3, n_src: int = 32768, n_tgt: int = 32768, d: int = 256,
               n_groups: int = 100, noise: float = 0.3, shift_sd: float = 0.3,
               gamma: float = 0.05, mu: float = 0.5):
    """Many classes with Zipf(1.1) sizes; means ~ N(0, I), noise 0.3 N(0, I).

    Target: the same class means with the same Zipf shares, fresh noise,
    plus one global shift drawn from N(0, shift_sd^2 I)."""
    r = _rng(seed)
    L = n_groups
    means = r.standard_normal((L, d))
    ss = zipf_sizes(n_src, L)
    ts = zipf_sizes(n_tgt, L)
    labels = np.repeat(np.arange(L), ss)
    xs = means[labels] + noise * r.standard_normal((n_src, d))
    tl = np.repeat(np.arange(L), ts)
    xt = means[tl] + noise * r.standard_normal((n_tgt, d)) + shift_sd * r.standard_normal(d)
    ps = r.permutation(n_src)
    pt = r.permutation(n_tgt)
    return dict(xs=xs[ps].astype(np.float32), xt=xt[pt].astype(np.float32),
                labels=labels[ps].astype(np.int32), n_groups=L,
                gamma=float(gamma), mu=float(mu))


def instance_from_generator(seed_pair, n_lo=64, n_hi=2048, d=64, L_lo=2, L_hi=31,
                            gamma_lo=0.05, gamma_hi=1.0, mu_lo=0.01, mu_hi=1.0):
    """One uneven instance: n, m ~ U[n_lo, n_hi], class count ~ U[L_lo, L_hi],
    class shares ~ Dirichlet(1) (so some classes may be empty), blob features
    as in ``blobs``; gamma and mu log-uniform in their ranges."""
    r = _rng(*seed_pair)
    n = int(r.integers(n_lo, n_hi + 1))
    m = int(r.integers(n_lo, n_hi + 1))
    L = int(r.integers(L_lo, L_hi + 1))
    share = r.dirichlet(np.ones(L))
    ssz = r.multinomial(n, share)
    tsz = r.multinomial(m, share)
    gamma = float(np.exp(r.uniform(np.log(gamma_lo), np.log(gamma_hi))))
    mu = float(np.exp(r.uniform(np.log(mu_lo), np.log(mu_hi))))
    means = 2.0 * r.standard_normal((L, d))
    labels = np.repeat(np.arange(L), ssz)
    xs = means[labels] + r.standard_normal((n, d))
    tl = np.repeat(np.arange(L), tsz)
    rot = _haar_rotation(r, d)
    shift = np.sqrt(0.5) * r.standard_normal(d)
    xt = (means[tl] + r.standard_normal((m, d))) @ rot.T + shift
    ps = r.permutation(n)
    pt = r.permutation(m)
    return dict(xs=xs[ps].astype(np.float32), xt=xt[pt].astype(np.float32),
                labels=labels[ps].astype(np.int32), n_groups=L,
                gamma=gamma, mu=mu)


def batch_instances(seed: int = 4, count: int = 256, **kw):
    """``count`` independent uneven instances; instance i uses seed (seed, i)."""
    return [instance_from_generator((seed, i), **kw) for i in range(count)]


def paper_synthetic(n_classes: int, g: int = 10, seed: int = 7,
                    gamma: float = 1.0, mu: float = 0.1):
    """The paper's synthetic dataset: g samples per class in 2-D, class l
    (l = 1..|L|) centred at (5l, -5) in the source and (5l, 5) in the target,
    standard normal noise; n_src = n_tgt = |L| g.  Target labels only place
    the points and are not returned."""
    r = _rng(seed, n_classes, g)
    l = np.repeat(np.arange(n_classes), g)
    cs = np.stack([5.0 * (l + 1), np.full(l.size, -5.0)], 1)
    ct = np.stack([5.0 * (l + 1), np.full(l.size, 5.0)], 1)
    xs = cs + r.standard_normal(cs.shape)
    xt = ct + r.standard_normal(ct.shape)
    return dict(xs=xs.astype(np.float32), xt=xt.astype(np.float32),
                labels=l.astype(np.int32), n_groups=n_classes,
                gamma=float(gamma), mu=float(mu))


def random_duals(seed, n_src, n_tgt, scale=0.5, offset=0.0):
    """Random dual points (alpha, beta) in float32 for gradient parity checks."""
    r = _rng(seed, n_src, n_tgt)
    a = (offset + scale * r.standard_normal(n_src)).astype(np.float32)
    b = (offset + scale * r.standard_normal(n_tgt)).astype(np.float32)
    return a, b
