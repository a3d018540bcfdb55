"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (the same layout, row buckets and
autotuned tile variants), through the C ABI.

* blobs 4096 x 4096 (d = 64, 10 classes): the whole gradient and D against
  the FP64 oracle, at a point of the oracle's own L-BFGS trajectory and at a
  seeded point with many active blocks; screened == dense bit for bit.
* blobs 16384 x 16384 (1 GiB cost; whole-group tiles of 56 loads per lane):
  the same at a seeded point.
* Zipf 32768 x 32768, d = 256, 100 classes, cost on the fly: integer
  features make every float32 step of the tile cost exact, so the oracle
  reads the same cost.  The oracle evaluates sub-problems that fix sampled
  outputs exactly: all rows and a sample of target columns give grad_beta
  there, whole (small) groups and all columns give grad_alpha of their rows.
  The two gradient blocks sum to the same total (1 - sum T) at any size, and
  screened == dense bit for bit.
* 256 uneven instances in one batched handle: sampled instances in full
  against the oracle; screened == dense bit for bit over the whole batch.

Costs of the materialized workloads are formed on the host in float64
(squared distances, divided by the maximum), rounded once to float32 and
given to both sides."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)
    sys.stdout.flush()


def host_cost32(xs, xt):
    """float32(||x - y||^2 / max) from float64 sums (input preparation)."""
    xs = xs.astype(np.float64)
    xt = xt.astype(np.float64)
    C = xs @ xt.T
    C *= -2.0
    C += (xs * xs).sum(1)[:, None]
    C += (xt * xt).sum(1)[None, :]
    np.maximum(C, 0.0, out=C)
    C /= C.max()
    return C.astype(np.float32)


def given_handle(C32, labels, L, gamma, mu):
    O = _O()
    return O.Handle([dict(labels=_dev(labels), n_groups=L, gamma=gamma, mu=mu, cost=_dev(C32),
                          cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN)])


def seeded_point(ns, nt, level, seed, spread=0.3):
    rng = np.random.default_rng(seed)
    a = (level + spread * rng.standard_normal(ns)).astype(np.float32)
    b = (0.5 * level + spread * rng.standard_normal(nt)).astype(np.float32)
    return a, b


def evaluate(h, a32, b32, mode):
    al, be = _dev(a32), _dev(b32)
    ga, gb = torch.empty_like(al), torch.empty_like(be)
    obj = torch.empty(h.count, dtype=torch.float64, device="cuda")
    h.dual_grad(al, be, ga, gb, obj, mode=mode)
    torch.cuda.synchronize()
    return ga.cpu().numpy(), gb.cpu().numpy(), obj.cpu().numpy()


def mass_bounds(a, b, oa, ob):
    """1e-6 plus 4e-6 times the row / column plan mass (T >= 0, so the mass
    of row i is a_i - grad_alpha_i): float32 sums of O(1) entries cannot meet
    a flat 1e-6 at points far from the optimum."""
    return 1e-6 + 4e-6 * (np.abs(a - oa) + np.abs(a)), 1e-6 + 4e-6 * (np.abs(b - ob) + np.abs(b))


def check_full(P, a32, b32, ga, gb, D, traj):
    oa, ob, oD = oracle.dual_grad(P, a32.astype(np.float64), b32.astype(np.float64))
    assert abs(D - oD) <= 1e-5 * max(1.0, abs(oD)), (D, oD)
    if traj:
        np.testing.assert_allclose(ga, oa, rtol=0, atol=1e-6)
        np.testing.assert_allclose(gb, ob, rtol=0, atol=1e-6)
    else:
        # the point is not trivial: many rows and columns carry plan mass
        assert np.mean(P.a - oa > 0) > 0.1 and np.mean(P.b - ob > 0) > 0.1
        ra, rb = mass_bounds(P.a, P.b, oa, ob)
        assert np.all(np.abs(ga - oa) <= ra), np.max(np.abs(ga - oa) / ra)
        assert np.all(np.abs(gb - ob) <= rb), np.max(np.abs(gb - ob) / rb)


def screened_equals_dense(h, a32, b32, seed):
    O = _O()
    evaluate(h, a32, b32, O.OT_GS_SNAPSHOT)
    rng = np.random.default_rng(seed)
    for eps in (1e-5, 1e-3):
        a2 = (a32 + eps * rng.standard_normal(a32.size)).astype(np.float32)
        b2 = (b32 + eps * rng.standard_normal(b32.size)).astype(np.float32)
        d = evaluate(h, a2, b2, O.OT_GS_DENSE)
        s = evaluate(h, a2, b2, O.OT_GS_SCREENED)
        for x, y in zip(d, s):
            np.testing.assert_array_equal(x, y)


def test_blobs_4096():
    O = _O()
    inst = synth.blobs(seed=2, n_src=4096, n_tgt=4096, d=64, n_groups=10, gamma=0.1, mu=0.1)
    C32 = host_cost32(inst["xs"], inst["xt"])
    P = oracle.Problem(C32, inst["labels"], 10, 0.1, 0.1)
    _say("blobs 4096: handle, autotune")
    h = given_handle(C32, inst["labels"], 10, 0.1, 0.1)
    h.autotune(repeats=3)
    r = oracle.solve(P, max_iter=8)
    a32, b32 = r["alpha"].astype(np.float32), r["beta"].astype(np.float32)
    _say("blobs 4096: trajectory point")
    ga, gb, D = evaluate(h, a32, b32, O.OT_GS_DENSE)
    check_full(P, a32, b32, ga, gb, D[0], traj=True)
    level = 0.5 * float(np.median(C32[::7, ::5]))
    a32, b32 = seeded_point(4096, 4096, level, 21)
    _say("blobs 4096: seeded point")
    ga, gb, D = evaluate(h, a32, b32, O.OT_GS_DENSE)
    check_full(P, a32, b32, ga, gb, D[0], traj=False)
    _say("blobs 4096: screened vs dense")
    screened_equals_dense(h, a32, b32, 22)
    h.close()


def test_blobs_16384():
    O = _O()
    n = 16384
    inst = synth.blobs(seed=2, n_src=n, n_tgt=n, d=64, n_groups=10, gamma=0.1, mu=0.1)
    C32 = host_cost32(inst["xs"], inst["xt"])
    _say("blobs 16384: handle, autotune")
    h = given_handle(C32, inst["labels"], 10, 0.1, 0.1)
    assert h.get_tile_config(11)["n_tiles"] == 10 * (n // 32)   # every tile in the R = 56 bucket
    h.autotune(repeats=2)
    level = 0.5 * float(np.median(C32[::97, ::89]))
    a32, b32 = seeded_point(n, n, level, 31)
    _say("blobs 16384: dense evaluation")
    ga, gb, D = evaluate(h, a32, b32, O.OT_GS_DENSE)
    P = oracle.Problem(C32, inst["labels"], 10, 0.1, 0.1)
    del C32
    check_full(P, a32, b32, ga, gb, D[0], traj=False)
    del P
    _say("blobs 16384: screened vs dense")
    screened_equals_dense(h, a32, b32, 32)
    h.close()


def int_zipf(n, L, d, seed, lo=-4, hi=4):
    """Integer features with Zipf(1.1) class sizes (floor 32): every float32
    step of |x|^2 + |y|^2 - 2 x.y is exact (|values| < 2^24)."""
    rng = np.random.default_rng(seed)
    sizes = synth.zipf_sizes(n, L)
    labels = rng.permutation(np.repeat(np.arange(L), sizes)).astype(np.int32)
    means = rng.integers(lo, hi + 1, (L, d))
    xs = np.clip(means[labels] + rng.integers(-1, 2, (n, d)), lo, hi).astype(np.float32)
    xt = np.clip(means[rng.integers(0, L, n)] + rng.integers(-1, 2, (n, d)), lo, hi).astype(np.float32)
    return xs, xt, labels, sizes


def exact_cost(xs, xt, scale):
    """||x - y||^2 * scale for integer features (exact in float64)."""
    xs = xs.astype(np.float64)
    xt = xt.astype(np.float64)
    return ((xs * xs).sum(1)[:, None] + (xt * xt).sum(1)[None, :] - 2.0 * (xs @ xt.T)) * scale


def test_zipf_32768_onthefly():
    O = _O()
    n, L, d, gamma, mu = 32768, 100, 256, 0.05, 0.5
    xs, xt, labels, sizes = int_zipf(n, L, d, seed=41)
    scale = 2.0 ** -14          # a power of two: scaling is exact too
    _say("zipf 32768 on the fly: handle, autotune")
    h = _O().Handle([dict(labels=_dev(labels), n_groups=L, gamma=gamma, mu=mu, x_src=_dev(xs),
                          x_tgt=_dev(xt), cost_mode=O.OT_GS_COST_ONTHEFLY, cost_scale=scale)])
    h.autotune(repeats=2)
    rng = np.random.default_rng(42)
    J = np.sort(rng.choice(n, 64, replace=False))
    CJ = exact_cost(xs, xt[J], scale)
    level = 0.5 * float(np.median(CJ))
    a32, b32 = seeded_point(n, n, level, 43)
    _say("zipf 32768 on the fly: dense evaluation")
    ga, gb, D = evaluate(h, a32, b32, O.OT_GS_DENSE)
    a = np.full(n, 1.0 / n)
    b = np.full(n, 1.0 / n)
    # sampled columns: all rows, every group
    PJ = oracle.Problem(CJ, labels, L, gamma, mu, a=a, b=b[J])
    _, obJ, _ = oracle.dual_grad(PJ, a32.astype(np.float64), b32[J].astype(np.float64))
    assert np.mean(b[J] - obJ > 0) > 0.1
    _, rb = mass_bounds(a, b[J], a, obJ)
    assert np.all(np.abs(gb[J] - obJ) <= rb), np.max(np.abs(gb[J] - obJ) / rb)
    # whole groups and every column: the three smallest, and the largest of at
    # most 4096 rows (evaluated in 1024-row chunks)
    chunked = max((g for g in range(L) if 1024 < sizes[g] <= 4096), key=lambda g: sizes[g])
    for g in list(np.argsort(sizes)[:3]) + [chunked]:
        I = np.nonzero(labels == g)[0]
        CI = exact_cost(xs[I], xt, scale)
        PI = oracle.Problem(CI, np.zeros(I.size, np.int32), 1, gamma, mu, a=a[I], b=b)
        oaI, _, _ = oracle.dual_grad(PI, a32[I].astype(np.float64), b32.astype(np.float64))
        assert np.mean(a[I] - oaI > 0) > 0.1, g
        ra, _ = mass_bounds(a[I], b, oaI, b)
        assert np.all(np.abs(ga[I] - oaI) <= ra), (g, np.max(np.abs(ga[I] - oaI) / ra))
    # both blocks sum to 1 - sum T
    sa, sb = float(np.sum(ga, dtype=np.float64)), float(np.sum(gb, dtype=np.float64))
    assert abs(sa - sb) <= 1e-4 * max(1.0, abs(sa)), (sa, sb)
    assert np.isfinite(D[0])
    _say("zipf 32768 on the fly: screened vs dense")
    screened_equals_dense(h, a32, b32, 44)
    h.close()


def test_batch_256():
    O = _O()
    insts = synth.batch_instances(seed=4, count=256)
    costs = [host_cost32(i["xs"], i["xt"]) for i in insts]
    probs = [dict(labels=_dev(i["labels"]), n_groups=i["n_groups"], gamma=i["gamma"], mu=i["mu"],
                  cost=_dev(C), cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN) for i, C in zip(insts, costs)]
    _say("batch 256: handle, autotune")
    h = O.Handle(probs)
    h.autotune(repeats=2)
    pts = [seeded_point(C.shape[0], C.shape[1], 0.5 * float(np.median(C[::3, ::3])), 500 + k)
           for k, C in enumerate(costs)]
    a32 = np.concatenate([p[0] for p in pts])
    b32 = np.concatenate([p[1] for p in pts])
    _say("batch 256: dense evaluation")
    ga, gb, D = evaluate(h, a32, b32, O.OT_GS_DENSE)
    offa = np.concatenate([[0], np.cumsum([C.shape[0] for C in costs])])
    offb = np.concatenate([[0], np.cumsum([C.shape[1] for C in costs])])
    for k in (0, 1, 37, 100, 128, 199, 254, 255):
        i = insts[k]
        P = oracle.Problem(costs[k], i["labels"], i["n_groups"], i["gamma"], i["mu"])
        check_full(P, a32[offa[k]:offa[k + 1]], b32[offb[k]:offb[k + 1]],
                   ga[offa[k]:offa[k + 1]], gb[offb[k]:offb[k + 1]], D[k], traj=False)
    _say("batch 256: screened vs dense")
    screened_equals_dense(h, a32, b32, 501)
    h.close()
