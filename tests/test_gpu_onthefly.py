"""On-the-fly cost (features on FP32 matrix cores, the cost never stored)
against the FP64 oracle, through the C ABI.

* Integer features and a power-of-two scale make every float32 step of
  |x|^2 + |y|^2 - 2 x.y exact, so the cost must equal the oracle's
  ||x - y||^2 s bit for bit, and gradients then meet the same bar as the
  materialized path (1e-6 absolute, 1e-5 relative objective).
* Real-valued features: the cost tiles lie within the float32 error bound
  of the expansion, and the gradient matches the oracle fed the cost the
  tiles produce (downloaded once through ot_gs_cost).
* Screened and dense on-the-fly evaluations agree bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from tests import cases

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def int_instance(seed, sizes, nt, d, lo=-4, hi=4, gamma=0.3, mu=0.4):
    rng = np.random.default_rng(seed)
    ns = int(sum(sizes))
    labels = rng.permutation(np.repeat(np.arange(len(sizes)), sizes)).astype(np.int32)
    means = rng.integers(lo, hi + 1, (len(sizes), d))
    xs = np.clip(means[labels] + rng.integers(-1, 2, (ns, d)), lo, hi).astype(np.float32)
    xt = np.clip(means[rng.integers(0, len(sizes), nt)] + rng.integers(-1, 2, (nt, d)), lo, hi)
    return dict(xs=xs, xt=xt.astype(np.float32), labels=labels, n_groups=len(sizes),
                gamma=gamma, mu=mu)


def otf_handle(inst, scale):
    O = _O()
    return O.Handle([dict(labels=_dev(inst["labels"]), n_groups=inst["n_groups"], gamma=inst["gamma"],
                          mu=inst["mu"], x_src=_dev(inst["xs"]), x_tgt=_dev(inst["xt"]),
                          cost_mode=O.OT_GS_COST_ONTHEFLY, cost_scale=scale)])


def gpu_cost(h, ns, nt):
    C = torch.empty(ns * nt, dtype=torch.float32, device="cuda")
    h.cost(C)
    torch.cuda.synchronize()
    return C.cpu().numpy().reshape(ns, nt)


def gpu_grad(h, a32, b32, mode=0):
    al, be = _dev(a32), _dev(b32)
    ga, gb = torch.empty_like(al), torch.empty_like(be)
    obj = torch.empty(1, dtype=torch.float64, device="cuda")
    h.dual_grad(al, be, ga, gb, obj, mode=mode)
    torch.cuda.synchronize()
    return ga.cpu().numpy(), gb.cpu().numpy(), float(obj.cpu()[0])


def check(P, a32, b32, ga, gb, D):
    oa, ob, oD = oracle.dual_grad(P, a32.astype(np.float64), b32.astype(np.float64))
    assert abs(D - oD) <= 1e-5 * max(1.0, abs(oD)), (D, oD)
    np.testing.assert_allclose(ga, oa, rtol=0, atol=1e-6)
    np.testing.assert_allclose(gb, ob, rtol=0, atol=1e-6)


def traj(P, iters):
    out = []
    for k in iters:
        r = oracle.solve(P, max_iter=k) if k else dict(alpha=np.zeros(P.ns), beta=np.zeros(P.nt))
        out.append((r["alpha"].astype(np.float32), r["beta"].astype(np.float32)))
    return out


# split group (> 1024 rows), an empty label, a 7-row group; ragged target
# tail (333 = 10 * 32 + 13) and ragged feature dims (37 -> 48)
INT_CASES = [
    (11, [1300, 40, 0, 7, 200], 333, 37),
    (12, [5, 3, 64, 33], 95, 16),
    (13, [2100], 64, 256),
]


@pytest.mark.parametrize("seed,sizes,nt,d", INT_CASES)
def test_integer_features_cost_is_exact(seed, sizes, nt, d):
    inst = int_instance(seed, sizes, nt, d)
    scale = 2.0 ** -10
    h = otf_handle(inst, scale)
    C = gpu_cost(h, inst["xs"].shape[0], nt)
    ref = oracle.cost_sqeuclid(inst["xs"], inst["xt"]) * scale
    np.testing.assert_array_equal(C.astype(np.float64), ref)


@pytest.mark.parametrize("seed,sizes,nt,d", INT_CASES[:2])
def test_integer_features_gradient_parity(seed, sizes, nt, d):
    inst = int_instance(seed, sizes, nt, d, gamma=0.2, mu=0.3)
    scale = 2.0 ** -10
    h = otf_handle(inst, scale)
    C = oracle.cost_sqeuclid(inst["xs"], inst["xt"]) * scale
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    for a32, b32 in traj(P, [0, 2, 10, 60]):
        ga, gb, D = gpu_grad(h, a32, b32)
        check(P, a32, b32, ga, gb, D)
    # a point with many active blocks (row sums over several column tiles)
    a32, b32 = cases.dual_point(P, seed)
    ga, gb, D = gpu_grad(h, a32, b32)
    oa, ob, oD = oracle.dual_grad(P, a32.astype(np.float64), b32.astype(np.float64))
    assert abs(D - oD) <= 1e-5 * max(1.0, abs(oD))
    T = oracle.plan(P, a32.astype(np.float64), b32.astype(np.float64))
    ra = 1e-6 + 4e-6 * (np.abs(T).sum(1) + np.abs(P.a))
    rb = 1e-6 + 4e-6 * (np.abs(T).sum(0) + np.abs(P.b))
    assert np.all(np.abs(ga - oa) <= ra)
    assert np.all(np.abs(gb - ob) <= rb)


def test_integer_features_plan_csr_equals_dense_plan():
    """The sparse plan from the matrix-core tiles holds exactly the nonzero
    entries of the dense plan (a 1300-row group evaluated in chunks, an empty
    label, a ragged target tail)."""
    from tests.test_gpu_dual_grad import csr_blocks
    seed, sizes, nt, d = INT_CASES[0]
    inst = int_instance(seed, sizes, nt, d, gamma=0.2, mu=0.3)
    scale = 2.0 ** -10
    h = otf_handle(inst, scale)
    C = oracle.cost_sqeuclid(inst["xs"], inst["xt"]) * scale
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    a32, b32 = cases.dual_point(P, seed)
    T = torch.empty((P.ns, P.nt), dtype=torch.float32, device="cuda")
    h.plan(_dev(a32), _dev(b32), T)
    rp, col, val = h.plan_csr(_dev(a32), _dev(b32))
    torch.cuda.synchronize()
    (Ts,) = csr_blocks(rp, col, val, [P.ns], [P.nt])
    Td = T.cpu().numpy()
    np.testing.assert_array_equal(Ts, Td)
    assert col.numel() == int(np.count_nonzero(Td)) > 0


def real_instance(seed=31, ns=3000, nt=1000, d=256, L=12):
    inst = synth.zipf_blobs(seed=seed, n_src=ns, n_tgt=nt, d=d, n_groups=L, gamma=0.05, mu=0.5)
    return inst


def test_real_features_cost_within_fp32_bound():
    inst = real_instance()
    xs, xt = inst["xs"].astype(np.float64), inst["xt"].astype(np.float64)
    d = xs.shape[1]
    scale = 1.0 / 256.0
    h = otf_handle(inst, scale)
    C = gpu_cost(h, xs.shape[0], xt.shape[0]).astype(np.float64)
    ref = oracle.cost_sqeuclid(inst["xs"], inst["xt"]) * scale
    # |x|^2, |y|^2 (d-term fma chains) and x.y (d-term FP32 accumulation),
    # combined in two roundings, then the scale: each term's error is below
    # (d + 2) u times its magnitude, u = 2^-24
    u = 2.0 ** -24
    nx = (xs ** 2).sum(1)[:, None]
    ny = (xt ** 2).sum(1)[None, :]
    bound = scale * (d + 4) * u * 2.0 * (nx + ny) + u * ref
    err = np.abs(C - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    assert np.all(C >= 0)


def test_real_features_normalised_scale():
    inst = real_instance(seed=32, ns=700, nt=300, d=100, L=6)
    h = otf_handle(inst, 0.0)
    C = gpu_cost(h, 700, 300).astype(np.float64)
    assert 1.0 - 1e-6 <= C.max() <= 1.0
    ref, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    assert np.max(np.abs(C - ref)) <= 1e-4


def test_real_features_gradient_parity_on_tile_cost():
    inst = real_instance()
    h = otf_handle(inst, 0.0)
    ns, nt = inst["xs"].shape[0], inst["xt"].shape[0]
    C = gpu_cost(h, ns, nt).astype(np.float64)
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    for a32, b32 in traj(P, [0, 3, 30]):
        ga, gb, D = gpu_grad(h, a32, b32)
        check(P, a32, b32, ga, gb, D)


def test_onthefly_screened_equals_dense_and_plan():
    O = _O()
    inst = int_instance(21, [1300, 40, 0, 7, 200], 333, 37, gamma=0.2, mu=0.5)
    scale = 2.0 ** -10
    h = otf_handle(inst, scale)
    C = oracle.cost_sqeuclid(inst["xs"], inst["xt"]) * scale
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    pts = traj(P, [20, 21, 25, 40])
    gpu_grad(h, *pts[0], mode=O.OT_GS_SNAPSHOT)
    h.stats(reset=True)
    for a32, b32 in pts[1:]:
        d = gpu_grad(h, a32, b32, mode=O.OT_GS_DENSE)
        s = gpu_grad(h, a32, b32, mode=O.OT_GS_SCREENED)
        np.testing.assert_array_equal(d[0], s[0])
        np.testing.assert_array_equal(d[1], s[1])
        assert d[2] == s[2]
    st = h.stats()
    assert st["tiles_computed"] < st["tiles_total"]
    a32, b32 = pts[-1]
    T = torch.empty(P.ns * P.nt, dtype=torch.float32, device="cuda")
    h.plan(_dev(a32), _dev(b32), T)
    torch.cuda.synchronize()
    Tref = oracle.plan(P, a32.astype(np.float64), b32.astype(np.float64))
    np.testing.assert_allclose(T.cpu().numpy().reshape(P.ns, P.nt), Tref, rtol=0, atol=1e-7)


def test_onthefly_solve_reaches_oracle_optimum():
    inst = int_instance(41, [300, 40, 7, 200], 250, 20, gamma=0.2, mu=0.3)
    scale = 2.0 ** -9
    h = otf_handle(inst, scale)
    C = oracle.cost_sqeuclid(inst["xs"], inst["xt"]) * scale
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    ref = oracle.solve(P, max_iter=4000)   # converges after about 1500 iterations
    _, _, info, _ = h.solve(max_iter=2500, use_screen=1)
    D = info[0]["obj"]
    assert abs(D - ref["obj"]) <= 1e-5 * abs(ref["obj"]), (D, ref["obj"])


def test_onthefly_argument_errors():
    O = _O()
    inst = int_instance(5, [10, 10], 20, 8)
    bad = dict(labels=_dev(inst["labels"]), n_groups=2, gamma=0.3, mu=0.1,
               x_src=_dev(np.zeros((20, 300), np.float32)), x_tgt=_dev(np.zeros((20, 300), np.float32)),
               cost_mode=O.OT_GS_COST_ONTHEFLY)
    with pytest.raises(O.OTGSError):
        O.Handle([bad])
    good = dict(labels=_dev(inst["labels"]), n_groups=2, gamma=0.3, mu=0.1, x_src=_dev(inst["xs"]),
                x_tgt=_dev(inst["xt"]), cost_mode=O.OT_GS_COST_ONTHEFLY)
    mat = dict(good, cost_mode=O.OT_GS_COST_MATERIALIZE)
    with pytest.raises(O.OTGSError):
        O.Handle([good, mat])
    nan = dict(good, x_src=_dev(np.full((20, 8), np.nan, np.float32)))
    with pytest.raises(O.OTGSError):
        O.Handle([nan])


@pytest.mark.skip(reason="aborted (SIGABRT in the HIP runtime, inside ot_gs_solve) when the tile launches of "
                         "each captured evaluation were recorded on parallel graph branches; that code is taken "
                         "out, and the case stays off the GPU until the abort's cause is shown")
def test_onthefly_screened_trajectory_is_dense_trajectory():
    """Every bucket (groups of 32 to over 1024 rows): the screened solve
    takes bit for bit the dense solve's steps."""
    inst = synth.zipf_blobs(seed=33, n_src=6000, n_tgt=1500, d=64, n_groups=30, gamma=0.05, mu=0.5)
    h = otf_handle(inst, 0.0)
    K = 150
    traces = []
    for scr in (0, 1):
        tr = torch.full((K + 1,), float("nan"), dtype=torch.float64, device="cuda")
        a, b, info, _ = h.solve(max_iter=K, use_screen=scr, obj_trace=tr)
        torch.cuda.synchronize()
        traces.append((tr.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy(), info[0]))
    np.testing.assert_array_equal(traces[0][0], traces[1][0])
    np.testing.assert_array_equal(traces[0][1], traces[1][1])
    np.testing.assert_array_equal(traces[0][2], traces[1][2])
