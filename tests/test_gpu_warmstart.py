"""Learned warm start on the device against the FP64 reference
(oracle.warmstart): features, network forward, loss gradient, Adam, and the
solver started from the prediction (same optimum as the cold start)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import warmstart as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _prob(inst, O):
    return dict(labels=_dev(inst["labels"]), n_groups=inst["n_groups"], gamma=inst["gamma"], mu=inst["mu"],
                x_src=_dev(inst["xs"]), x_tgt=_dev(inst["xt"]), cost_mode=O.OT_GS_COST_MATERIALIZE,
                cost_scale=0.0)


def test_features_match_oracle():
    O = _O()
    insts = [synth.instance_from_generator((90, i), n_lo=40, n_hi=300, d=16) for i in range(4)]
    probs = [_prob(i, O) for i in insts]
    h = O.Handle(probs)
    scales = h.cost_scale()
    d = 16
    tn = sum(i["xs"].shape[0] for i in insts)
    tm = sum(i["xt"].shape[0] for i in insts)
    F = torch.empty((tn + tm, d + 8), dtype=torch.float32, device="cuda")
    O.features(probs, scales, F)
    torch.cuda.synchronize()
    F = F.cpu().numpy().astype(np.float64)
    os_, ot_ = 0, tn
    for inst, s in zip(insts, scales):
        Fs, Ft, _ = W.features(inst["xs"], inst["xt"], inst["labels"], inst["n_groups"], s,
                               inst["gamma"], inst["mu"])
        n, m = Fs.shape[0], Ft.shape[0]
        for got, ref in ((F[os_:os_ + n], Fs), (F[ot_:ot_ + m], Ft)):
            np.testing.assert_allclose(got, ref, rtol=2e-5, atol=2e-6)
        os_ += n
        ot_ += m
    # scale: 1 / max of the float32 cost the handle normalised
    for inst, s in zip(insts, scales):
        cmax = oracle.cost_sqeuclid(inst["xs"], inst["xt"]).max()
        assert abs(s * cmax - 1.0) < 1e-5


def _net_case(seed=0, N=300, d_in=24, w=256):
    r = np.random.default_rng(seed)
    p = W.init_params(d_in, w, seed)
    p[d_in * w:d_in * w + w] = 0.1 * r.standard_normal(w)            # nonzero biases
    F = r.standard_normal((N, d_in)).astype(np.float32)
    y = r.standard_normal(N).astype(np.float32)
    return p, F, y, d_in, w


def test_forward_matches_oracle():
    O = _O()
    p, F, y, d_in, w = _net_case()
    M = O.Mlp(d_in, w, max_rows=128)        # several row batches (300 rows)
    M.set_params(_dev(p))
    out = M.forward(_dev(F)).cpu().numpy()
    ref, (Z1, H1, Z2, H2) = W.forward(p, F, d_in, w, bf16=True)
    _, _, _, _, w3, b3 = W.unpack(p, d_in, w)
    # float32 accumulation, and an activation that rounds to the other
    # bfloat16 neighbour, move a product by at most 2^-8 of its absolute sum
    S = np.abs(W.bf16_round(H2)) @ np.abs(W.bf16_round(w3)) + abs(b3)
    assert np.all(np.abs(out - ref) <= 2.0 ** -6 * S + 1e-6), np.max(np.abs(out - ref) / S)
    assert np.median(np.abs(out - ref) / S) < 1e-5


def test_loss_gradient_matches_oracle():
    O = _O()
    p, F, y, d_in, w = _net_case(seed=1, N=5000)     # two split-K partials (4096 rows each)
    M = O.Mlp(d_in, w, max_rows=5000)
    M.set_params(_dev(p))
    loss, g = M.loss_grad(_dev(F), _dev(y))
    loss, g = float(loss.cpu()[0]), g.cpu().numpy().astype(np.float64)
    rl, rg = W.loss_grad(p, F, y, d_in, w, bf16=True)
    assert abs(loss - rl) <= 1e-5 * rl
    o = 0
    for name, size in (("W1", d_in * w), ("b1", w), ("W2", w * w), ("b2", w), ("w3", w), ("b3", 1)):
        a, b = g[o:o + size], rg[o:o + size]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel < 5e-3, (name, rel)
        assert np.max(np.abs(a - b)) <= 2e-2 * np.max(np.abs(b)) + 1e-9, name
        o += size
    # the unrounded network's gradient (pinned by finite differences) is close too
    _, xg = W.loss_grad(p, F, y, d_in, w, bf16=False)
    assert np.linalg.norm(g - xg) / np.linalg.norm(xg) < 3e-2


def test_adam_step_matches_oracle():
    O = _O()
    p, F, y, d_in, w = _net_case(seed=2, N=700)
    M = O.Mlp(d_in, w, max_rows=1024)
    M.set_params(_dev(p))
    _, g = M.loss_grad(_dev(F), _dev(y))
    g = g.cpu().numpy().astype(np.float64)
    M.set_params(_dev(p))
    lr = 1e-3
    M.train(_dev(F), _dev(y), batch=700, epochs=1, lr=lr)
    got = M.get_params().cpu().numpy().astype(np.float64)
    ref, _, _ = W.adam_step(p.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1, lr)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-7)


def test_training_reduces_the_loss():
    O = _O()
    r = np.random.default_rng(3)
    d_in, w, N = 12, 256, 4096
    F = r.standard_normal((N, d_in)).astype(np.float32)
    y = (np.sin(F[:, 0]) + 0.5 * F[:, 1] * F[:, 2]).astype(np.float32)
    M = O.Mlp(d_in, w, max_rows=512)
    M.set_params(_dev(W.init_params(d_in, w, 3)))
    steps = 40 * (N // 512)
    tr = torch.zeros(steps, dtype=torch.float64, device="cuda")
    M.train(_dev(F), _dev(y), batch=512, epochs=40, lr=2e-3, loss_trace=tr)
    t = tr.cpu().numpy()
    assert np.all(np.isfinite(t))
    assert t[-8:].mean() < 0.1 * t[:8].mean(), (t[:8].mean(), t[-8:].mean())


def _cold_duals(h, count, iters):
    a, b, info, _ = h.solve(max_iter=iters, use_screen=1)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), info


def test_warm_start_reaches_the_cold_optimum():
    """Train on converged duals of small instances, then start held-out
    instances from the prediction: same optimum (1e-6 relative), fewer
    iterations on most instances."""
    O = _O()
    d = 16
    kw = dict(n_lo=48, n_hi=256, d=d)
    train = [synth.instance_from_generator((91, i), **kw) for i in range(96)]
    held = [synth.instance_from_generator((92, i), **kw) for i in range(24)]
    tp = [_prob(i, O) for i in train]
    ht = O.Handle(tp)
    a, b, _ = _cold_duals(ht, len(train), 3000)
    ys, yt, os_, ot_ = [], [], 0, 0
    for inst in train:
        n, m = inst["xs"].shape[0], inst["xt"].shape[0]
        fa, fb = W.gauge_fix(a[os_:os_ + n], b[ot_:ot_ + m])
        ys.append(fa)
        yt.append(fb)
        os_ += n
        ot_ += m
    y = np.concatenate(ys + yt).astype(np.float32)
    F = torch.empty((y.size, d + 8), dtype=torch.float32, device="cuda")
    O.features(tp, ht.cost_scale(), F)
    perm = np.random.default_rng(0).permutation(y.size)
    Fp = F[_dev(perm.astype(np.int64))].contiguous()
    yp = _dev(y[perm])
    M = O.Mlp(d + 8, 256, max_rows=1024)
    M.set_params(_dev(W.init_params(d + 8, 256, 7)))
    M.train(Fp, yp, batch=1024, epochs=60, lr=1e-3)

    hp = [_prob(i, O) for i in held]
    hh = O.Handle(hp)
    K = 3000
    tr_c = torch.full((len(held) * (K + 1),), float("nan"), dtype=torch.float64, device="cuda")
    hh.solve(max_iter=K, use_screen=1, obj_trace=tr_c)
    a0, b0 = hh.warm_start(M, hp)
    tr_w = torch.full((len(held) * (K + 1),), float("nan"), dtype=torch.float64, device="cuda")
    _, _, info_w, _ = hh.solve(a0, b0, max_iter=K, use_screen=1, init_user=1, obj_trace=tr_w)
    torch.cuda.synchronize()
    tc = tr_c.cpu().numpy().reshape(len(held), K + 1)
    tw = tr_w.cpu().numpy().reshape(len(held), K + 1)
    gains = []
    for k in range(len(held)):
        dstar = max(np.nanmax(tc[k]), np.nanmax(tw[k]))
        best_w = np.nanmax(tw[k])
        assert (dstar - best_w) <= 1e-6 * abs(dstar), (k, dstar, best_w)
        ic = np.nonzero((dstar - tc[k]) <= 1e-6 * abs(dstar))[0][0]
        iw = np.nonzero((dstar - tw[k]) <= 1e-6 * abs(dstar))[0][0]
        gains.append(ic - iw)
    assert np.median(gains) > 0, gains
