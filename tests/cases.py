"""Seeded problem instances shared by the GPU tests: features from ``synth``,
costs from the oracle's double-precision definition rounded to float32 (the
same float32 cost is the input of both sides)."""
import numpy as np

import oracle
import synth


def with_cost(inst, normalize=True):
    """float32 normalised cost C32 and the oracle Problem reading C32 upcast."""
    C, _ = oracle.cost_normalized(inst["xs"], inst["xt"]) if normalize else (
        oracle.cost_sqeuclid(inst["xs"], inst["xt"]), 1.0)
    C32 = C.astype(np.float32)
    P = oracle.Problem(C32.astype(np.float64), inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    return C32, P


def ragged(seed, ns, nt, sizes, gamma=0.3, mu=0.4, d=5):
    """Uneven groups given by ``sizes`` (zeros allowed: empty labels)."""
    rng = np.random.default_rng(seed)
    labels = rng.permutation(np.repeat(np.arange(len(sizes)), sizes)).astype(np.int32)
    assert labels.size == ns
    means = 2.0 * rng.standard_normal((len(sizes), d))
    xs = (means[labels] + rng.standard_normal((ns, d))).astype(np.float32)
    xt = (means[rng.integers(0, len(sizes), nt)] + rng.standard_normal((nt, d)) + 0.3).astype(np.float32)
    return dict(xs=xs, xt=xt, labels=labels, n_groups=len(sizes), gamma=gamma, mu=mu)


def dual_point(P, seed, spread=0.3, level=None):
    """A point where a fair share of the blocks is active: alpha around the
    typical cost plus noise."""
    rng = np.random.default_rng(seed)
    if level is None:
        level = 0.5 * float(np.median(P.C))
    a = (level + spread * rng.standard_normal(P.ns)).astype(np.float32)
    b = (level * 0.5 + spread * rng.standard_normal(P.nt)).astype(np.float32)
    return a, b
