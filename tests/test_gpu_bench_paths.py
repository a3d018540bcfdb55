"""Parity of the paths the measured workloads run, through the C ABI.

- the cost the library builds from features (COST_MATERIALIZE, scale 1/max C
  formed on the device), read back and compared with the FP64 definition
  c_ij = ||x_i - y_j||^2 / max C (Sec. 2.1), then gradients and objective on
  that handle against the oracle on the FP64 cost at trajectory points;
- non-uniform marginals a, b (Eq. 4);
- the corners of the experiments' (gamma, rho) grid (Sec. 5.2), gamma = 1e-3
  and 1e3, on the paper's synthetic set;
- ties z = mu gamma exactly and one float32 step either side (a block is zero
  iff z <= mu gamma, Eq. 5), and duplicated points (c_ij = 0);
- a batched screened solve whose instances end in a failed line search right
  after a snapshot evaluation: screened evaluations afterwards still equal
  dense ones bit for bit (Theorem 2 needs z~ exact at alpha~, beta~).
"""
import numpy as np
import pytest

import oracle
import synth
from tests import cases
from tests.test_gpu_dual_grad import _dev, check_parity, gpu_grad, make_handle, trajectory_points

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24   # unit roundoff of float32


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def materialized_handle(inst, **extra):
    O = _O()
    p = dict(labels=_dev(inst["labels"]), n_groups=inst["n_groups"], gamma=inst["gamma"], mu=inst["mu"],
             x_src=_dev(inst["xs"]), x_tgt=_dev(inst["xt"]), cost_mode=O.OT_GS_COST_MATERIALIZE,
             cost_scale=0.0)
    p.update(extra)
    return O.Handle([p])


def read_cost(h, ns, nt):
    C = torch.empty((ns, nt), dtype=torch.float32, device="cuda")
    h.cost(C)
    torch.cuda.synchronize()
    return C.cpu().numpy().astype(np.float64)


def cost_bound(C64):
    """|C_dev - C| for the compensated float32 sum (within ~1 rounding of the
    exact cost of the float32 features), the max taken over those values,
    the scale 1/max rounded to float32 and the product rounded: each step at
    most one rounding relative to the value, so 4 u relative bounds it."""
    return 4.0 * U32 * C64 + 2.0 ** -149


def test_materialized_cost_blobs4096_matches_fp64_definition():
    """The blobs 4096 x 4096 handle exactly as the benchmark builds it."""
    inst = synth.blobs(seed=2, n_src=4096, n_tgt=4096, d=64, n_groups=10, gamma=0.1, mu=0.1)
    h = materialized_handle(inst)
    Cd = read_cost(h, 4096, 4096)
    C64, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    err = np.abs(Cd - C64)
    assert np.all(err <= cost_bound(C64)), float(np.max(err / np.maximum(C64, 1e-30)) / U32)
    assert Cd.max() == 1.0


def test_materialized_blobs4096_gradient_matches_fp64_oracle():
    """Gradients at 1e-6 absolute and D at 1e-5 relative against the oracle
    on the FP64 cost, at points of the oracle's own L-BFGS trajectory; the
    screened evaluation after a snapshot equals the dense one bit for bit."""
    O = _O()
    inst = synth.blobs(seed=2, n_src=4096, n_tgt=4096, d=64, n_groups=10, gamma=0.1, mu=0.1)
    h = materialized_handle(inst)
    C64, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    P = oracle.Problem(C64, inst["labels"], 10, 0.1, 0.1)
    for a32, b32 in trajectory_points(P, [6, 30]):
        ga, gb, D = gpu_grad(h, a32, b32, mode=O.OT_GS_SNAPSHOT)
        check_parity(P, a32, b32, ga, gb, D[0])
        s = gpu_grad(h, a32, b32, mode=O.OT_GS_SCREENED)
        for x, y in zip((ga, gb, D), s):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("seed,sizes,nt", [(90, [40, 0, 300, 17], 211), (91, [2500, 60], 97)])
def test_materialized_ragged_with_duplicates(seed, sizes, nt):
    """Built cost on ragged shapes (an empty label, a split group); some
    targets duplicate source points, so their cost is exactly 0."""
    inst = cases.ragged(seed, sum(sizes), nt, sizes)
    xt = inst["xt"].copy()
    xt[: min(9, nt)] = inst["xs"][: min(9, nt)]
    inst["xt"] = xt
    h = materialized_handle(inst)
    Cd = read_cost(h, sum(sizes), nt)
    C64, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    assert np.all(np.abs(Cd - C64) <= cost_bound(C64))
    for j in range(min(9, nt)):
        assert Cd[j, j] == 0.0
    P = oracle.Problem(C64, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    for a32, b32 in trajectory_points(P, [3, 20]):
        ga, gb, D = gpu_grad(h, a32, b32)
        check_parity(P, a32, b32, ga, gb, D[0])


def test_nonuniform_marginals():
    """a, b non-uniform (positive, equal total mass in float32): gradients
    a - T1 and b - T^T 1 and D = a.alpha + b.beta - sum psi."""
    O = _O()
    inst = cases.ragged(92, 700, 333, [200, 0, 450, 50], gamma=0.2, mu=0.3)
    C32, P0 = cases.with_cost(inst)
    r = np.random.default_rng(92)
    a = r.uniform(0.2, 1.8, P0.ns)
    b = r.uniform(0.2, 1.8, P0.nt)
    a32 = (a / a.sum()).astype(np.float32)
    b32 = (b / b.sum()).astype(np.float32)
    P = oracle.Problem(C32.astype(np.float64), inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"],
                       a=a32.astype(np.float64), b=b32.astype(np.float64))
    h = make_handle(C32, P, a=_dev(a32), b=_dev(b32))
    for al, be in trajectory_points(P, [0, 4, 40]):
        ga, gb, D = gpu_grad(h, al, be)
        check_parity(P, al, be, ga, gb, D[0])
        s = gpu_grad(h, al, be, mode=O.OT_GS_SNAPSHOT)
        for x, y in zip((ga, gb, D), s):
            np.testing.assert_array_equal(x, y)
    # the device solve reaches the oracle's optimum with these marginals
    ref = oracle.solve(P, max_iter=4000, gtol=1e-11)
    _, _, info, _ = h.solve(max_iter=3000, use_screen=1)
    assert abs(info[0]["obj"] - ref["obj"]) <= 1e-6 * abs(ref["obj"]), (info[0], ref["obj"])


def fp32_bound(P, a32, b32):
    """Bound on the gradient error of a float32 evaluation at (a32, b32)
    beyond the 1e-6 bar: each f_ij = alpha_i + beta_j - c_ij carries at most
    e = 2u (max|alpha| + max|beta| + max c) of rounding; a group block's map
    f_[l] -> t_[l] (the gradient of the 1/gamma-smooth psi_l) is
    (1/gamma)-Lipschitz, so a column's block sum moves by at most g_l e / gamma
    and one entry by (1 + sqrt(g_l)) e / gamma.  Blocks count where they are
    active or within sqrt(g_l) e of the threshold (they may switch)."""
    e = 2 * U32 * (np.abs(a32).max() + np.abs(b32).max() + P.C.max())
    Z, _, _ = oracle.group_norms(P, a32.astype(np.float64), b32.astype(np.float64))
    g = P.group_sizes().astype(np.float64)
    act = Z > (P.mu * P.gamma - np.sqrt(g)[:, None] * e)          # [L, nt]
    col = (act * g[:, None]).sum(0) * e / P.gamma
    row = (act[P.labels] * (1 + np.sqrt(g[P.labels]))[:, None]).sum(1) * e / P.gamma
    return 1e-6 + row, 1e-6 + col


@pytest.mark.parametrize("gamma,rho", [(1e-3, 0.2), (1e-3, 0.8), (1e3, 0.2), (1e3, 0.8)])
def test_rho_grid_corners(gamma, rho):
    """The corners of the experiments' grid (Sec. 5.2) on the paper's
    synthetic set with 10 classes of 10 samples: gradients at trajectory
    points (at gamma = 1e3 within 1e-6; at gamma = 1e-3 the float32 rounding
    of f is amplified by 1/gamma, so within the derived bound above), and
    screened == dense along the device solve, which reaches the FP64
    optimum."""
    O = _O()
    g_, m_ = oracle.rho_form(gamma, rho)
    inst = synth.paper_synthetic(10, g=10, gamma=g_, mu=m_)
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    for a32, b32 in trajectory_points(P, [1, 10, 60]):
        ga, gb, D = gpu_grad(h, a32, b32)
        oa, ob, oD = oracle.dual_grad(P, a32.astype(np.float64), b32.astype(np.float64))
        assert abs(D[0] - oD) <= 1e-5 * max(1.0, abs(oD)), (D[0], oD)
        ra, rb = fp32_bound(P, a32, b32)
        assert np.all(np.abs(ga - oa) <= ra), np.max(np.abs(ga - oa) / ra)
        assert np.all(np.abs(gb - ob) <= rb), np.max(np.abs(gb - ob) / rb)
    K = 3000
    runs = []
    for scr in (0, 1):
        tr = torch.full((K + 1,), float("nan"), dtype=torch.float64, device="cuda")
        a, b, info, _ = h.solve(max_iter=K, use_screen=scr, obj_trace=tr)
        torch.cuda.synchronize()
        runs.append((a.cpu().numpy(), b.cpu().numpy(), tr.cpu().numpy(), info[0]))
    np.testing.assert_array_equal(runs[0][2], runs[1][2])
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    ref = oracle.solve(P, max_iter=20000, gtol=1e-12)
    # Table 1's corner gamma = 1e3, rho = 0.8 sits at D* >= gamma rho / sqrt(g) = 252.98
    gap = (ref["obj"] - runs[0][3]["obj"]) / abs(ref["obj"])
    print(f"gamma={gamma} rho={rho}: D*={ref['obj']!r} device {runs[0][3]} rel gap {gap:.3e}")
    assert abs(gap) <= (1e-6 if gamma >= 1 else 1e-4), (runs[0][3], ref["obj"])


def test_ties_at_the_threshold():
    """z = mu gamma exactly gives a zero block; one float32 step above gives
    a nonzero one, one below zero again (Eq. 5 with the zero case z <= mu
    gamma).  mu gamma = 0.125 is exact in both precisions, and each tested
    block has a single positive entry, so z equals that entry exactly on
    both sides.  Screened evaluations after a snapshot agree bit for bit."""
    O = _O()
    thr = np.float32(0.125)
    up = np.nextafter(thr, np.float32(1))
    dn = np.nextafter(thr, np.float32(0))
    # rows 0..2 each alone in its group; rows 3, 4 share group 3 with a
    # negative partner; column 0 is a duplicate of every source point (c = 0)
    labels = np.array([0, 1, 2, 3, 3], np.int32)
    C32 = np.array([[0, .5, .25], [0, .5, .25], [0, .5, .25], [0, .5, .25], [.9, .5, .25]], np.float32)
    P = oracle.Problem(C32.astype(np.float64), labels, 4, 0.5, 0.25)
    assert P.mu * P.gamma == 0.125
    h = make_handle(C32, P)
    a32 = np.array([thr, up, dn, up, 0.0], np.float32)
    b32 = np.zeros(3, np.float32)
    for mode in (O.OT_GS_DENSE, O.OT_GS_SNAPSHOT, O.OT_GS_SCREENED):
        ga, gb, D = gpu_grad(h, a32, b32, mode=mode)
        oa, ob, oD = oracle.dual_grad(P, a32.astype(np.float64), b32.astype(np.float64))
        # rows 0 and 2: zero blocks, the gradient is exactly the marginal
        assert ga[0] == np.float32(0.2) and ga[2] == np.float32(0.2)
        assert oa[0] == 0.2 and oa[2] == 0.2
        # rows 1 and 3: z one step above the threshold, a tiny transport
        assert ga[1] < np.float32(0.2) and ga[3] < np.float32(0.2) and oa[1] < 0.2 and oa[3] < 0.2
        np.testing.assert_allclose(ga, oa, rtol=0, atol=1e-6)
        np.testing.assert_allclose(gb, ob, rtol=0, atol=1e-6)
        assert abs(D[0] - oD) <= 1e-5 * max(1.0, abs(oD))


def test_batched_snapshot_kept_after_failed_line_search():
    """Every instance ends its solve in a failed line search (two trials per
    search) while each accepted step refreshes the snapshot (r = 1), so the
    last evaluation of most instances is a snapshot trial at a point the
    solve rejects.  The snapshot must describe that point: screened
    evaluations at new points afterwards equal dense ones bit for bit."""
    O = _O()
    insts = [cases.ragged(95 + i, n, m, s, gamma=0.1, mu=0.5) for i, (n, m, s) in
             enumerate([(300, 200, [100, 150, 50]), (64, 700, [32, 32]), (900, 90, [500, 0, 400]),
                        (130, 130, [60, 70])])]
    probs, Ps = [], []
    for inst in insts:
        C32, P = cases.with_cost(inst)
        probs.append(dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                          cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN))
        Ps.append(P)
    h = O.Handle(probs)
    a, b, info, _ = h.solve(max_iter=400, use_screen=1, refresh=1, max_ls=2)
    torch.cuda.synchronize()
    assert sum(x["status"] == O.OT_GS_LINESEARCH for x in info) >= 2, info
    an, bn = a.cpu().numpy(), b.cpu().numpy()
    rng = np.random.default_rng(3)
    for eps in (0.0, 1e-4, 3e-3, 3e-2):
        a2 = (an + eps * rng.standard_normal(an.size)).astype(np.float32)
        b2 = (bn + eps * rng.standard_normal(bn.size)).astype(np.float32)
        s = gpu_grad(h, a2, b2, mode=O.OT_GS_SCREENED)
        d = gpu_grad(h, a2, b2, mode=O.OT_GS_DENSE)
        for x, y in zip(d, s):
            np.testing.assert_array_equal(x, y)
