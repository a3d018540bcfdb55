"""Pins of the FP64 warm-start reference (features, network, Adam), each
against something other than the reference itself: worked examples by hand,
textbook values of the normal CDF, central finite differences, autograd of
an independent library (torch on the CPU, float64), closed forms."""
import math

import numpy as np
import pytest

import oracle
from oracle import warmstart as W


def test_bf16_round_worked_values():
    one = 1.0
    cases = [
        (one, one),
        (one + 2.0 ** -8, one),                        # halfway, even neighbour is 1
        (one + 3 * 2.0 ** -8, one + 2.0 ** -6),         # halfway, even neighbour is 1 + 2^-6
        (one + 2.0 ** -8 + 2.0 ** -20, one + 2.0 ** -7),  # just above halfway
        (-(one + 2.0 ** -8 + 2.0 ** -20), -(one + 2.0 ** -7)),
        (3.0, 3.0),
        (0.1, 0.10009765625),                           # 0x3DCD
        (0.0, 0.0),
    ]
    got = W.bf16_round([c[0] for c in cases])
    np.testing.assert_array_equal(got, [c[1] for c in cases])
    x = np.random.default_rng(0).standard_normal(1000)
    r = W.bf16_round(x)
    np.testing.assert_array_equal(W.bf16_round(r), r)           # idempotent
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))


def test_gelu_textbook_values():
    phi1 = 0.8413447460685429                                  # standard normal CDF at 1
    np.testing.assert_allclose(W.gelu(np.array([0.0, 1.0, -1.0])), [0.0, phi1, -(1 - phi1)],
                               rtol=0, atol=1e-15)
    z = np.linspace(-6, 6, 97)
    h = 1e-6
    fd = (W.gelu(z + h) - W.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(W.gelu_grad(z), fd, rtol=0, atol=1e-8)
    assert abs(W.gelu(40.0) - 40.0) < 1e-12 and abs(W.gelu(-40.0)) < 1e-12


def _tiny(seed=1, d_in=5, w=6, N=7):
    r = np.random.default_rng(seed)
    p = r.standard_normal(W.n_params(d_in, w)) * 0.7
    F = r.standard_normal((N, d_in))
    y = r.standard_normal(N)
    return p, F, y, d_in, w


def test_network_gradient_matches_central_differences():
    p, F, y, d_in, w = _tiny()
    loss, g = W.loss_grad(p, F, y, d_in, w)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (W.loss_grad(p + e, F, y, d_in, w)[0] - W.loss_grad(p - e, F, y, d_in, w)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_network_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p, F, y, d_in, w = _tiny(seed=3, d_in=4, w=9, N=11)
    loss, g = W.loss_grad(p, F, y, d_in, w)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = pt[o:o + d_in * w].reshape(d_in, w); o += d_in * w
    b1 = pt[o:o + w]; o += w
    W2 = pt[o:o + w * w].reshape(w, w); o += w * w
    b2 = pt[o:o + w]; o += w
    w3 = pt[o:o + w]; o += w
    b3 = pt[o]
    Ft = torch.tensor(F, dtype=torch.float64)
    gelu = torch.nn.functional.gelu
    out = gelu(gelu(Ft @ W1 + b1) @ W2 + b2) @ w3 + b3
    lt = ((out - torch.tensor(y, dtype=torch.float64)) ** 2).mean()
    lt.backward()
    assert abs(lt.item() - loss) <= 1e-14 * max(1.0, loss)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_forward_rounds_only_product_operands():
    p, F, y, d_in, w = _tiny(seed=4)
    out_r, _ = W.forward(p, F, d_in, w, bf16=True)
    # the same network fed pre-rounded weights and inputs: the first product
    # is then identical, later ones round activations the same way
    W1, b1, W2, b2, w3, b3 = W.unpack(p, d_in, w)
    Z1 = W.bf16_round(F) @ W.bf16_round(W1) + b1
    Z2 = W.bf16_round(W.gelu(Z1)) @ W.bf16_round(W2) + b2
    out = W.bf16_round(W.gelu(Z2)) @ W.bf16_round(w3) + b3
    np.testing.assert_array_equal(out_r, out)
    out_x, _ = W.forward(p, F, d_in, w, bf16=False)
    assert np.max(np.abs(out_r - out_x)) < 0.05 * np.max(np.abs(out_x))


def test_adam_first_step_closed_form():
    p = np.array([0.5, -1.0, 2.0])
    g = np.array([0.3, -4.0, 1e-3])
    q, m, v = W.adam_step(p, np.zeros(3), np.zeros(3), g, step=1, lr=0.01)
    # bias correction makes the first step lr * g / (|g| + eps)
    np.testing.assert_allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def test_features_worked_example():
    # 1-D: source class 0 at {0, 2} (centroid 1), class 1 at {10}; targets
    # 1.5 -> class 0, 9, 11, 12 -> class 1 (pseudo-centroids 1.5 and 32/3)
    xs = np.array([[0.0], [10.0], [2.0]])
    labels = np.array([0, 1, 0])
    xt = np.array([[1.5], [9.0], [11.0], [12.0]])
    s = 0.5
    Fs, Ft, pseudo = W.features(xs, xt, labels, 2, s, gamma=0.25, mu=0.5)
    np.testing.assert_array_equal(pseudo, [0, 1, 1, 1])
    logs = [math.log(0.25), math.log(0.5), math.log(3), math.log(4)]
    c1 = 32.0 / 3.0
    exp_s = [
        [0.0, 0.5, 2.25 * s, 2 / 3, 0.0],
        [10 * math.sqrt(s), 0.0, (10 - c1) ** 2 * s, 1 / 3, 0.0],
        [2 * math.sqrt(s), 0.5, 0.25 * s, 2 / 3, 0.0],
    ]
    exp_t = [
        [1.5 * math.sqrt(s), 0.0, 0.25 * s, 1 / 4, 1.0],
        [9 * math.sqrt(s), (9 - c1) ** 2 * s, 1.0 * s, 3 / 4, 1.0],
        [11 * math.sqrt(s), (11 - c1) ** 2 * s, 1.0 * s, 3 / 4, 1.0],
        [12 * math.sqrt(s), (12 - c1) ** 2 * s, 4.0 * s, 3 / 4, 1.0],
    ]
    np.testing.assert_allclose(Fs, [r + logs for r in exp_s], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(Ft, [r + logs for r in exp_t], rtol=1e-14, atol=1e-14)


def test_gauge_fix_keeps_the_objective():
    r = np.random.default_rng(5)
    C = r.random((6, 5))
    labels = np.array([0, 1, 1, 2, 0, 2], dtype=np.int32)
    P = oracle.Problem(C, labels, 3, 0.4, 0.3)
    al, be = r.standard_normal(6), r.standard_normal(5)
    fa, fb = W.gauge_fix(al, be)
    assert abs(fa.mean() - fb.mean()) < 1e-15
    assert abs(oracle.dual_obj(P, al, be) - oracle.dual_obj(P, fa, fb)) < 1e-14
