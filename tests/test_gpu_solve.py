"""Device L-BFGS (Algorithm 1 around the screened gradient) against the FP64
oracle: converged objective within 1e-5 relative, marginals and duality gap
at the GPU's final point checked by the oracle, screened == dense
trajectories bit for bit, batched == single instances."""
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


def handle_for(C32, P):
    O = _O()
    return O.Handle([dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                          cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN)])


def run(h, max_iter, **kw):
    tr = torch.full((h.count * (max_iter + 1),), float("nan"), dtype=torch.float64, device="cuda")
    a, b, info, rc = h.solve(obj_trace=tr, max_iter=max_iter, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), info, tr.cpu().numpy().reshape(h.count, max_iter + 1), rc


def test_solve_small_matches_oracle_optimum():
    inst = synth.gaussian4_2d()
    C32, P = cases.with_cost(inst)
    ref = oracle.solve(P, max_iter=3000, gtol=1e-11)
    h = handle_for(C32, P)
    a, b, info, tr, rc = run(h, 600, use_screen=0)
    D = info[0]["obj"]
    assert abs(D - ref["obj"]) <= 1e-5 * abs(ref["obj"]), (D, ref["obj"])
    # the oracle at the GPU's final point: objective, marginals, duality gap
    ga, gb, oD, T = oracle.dual_grad(P, a.astype(np.float64), b.astype(np.float64), want_plan=True)
    assert abs(oD - D) <= 1e-5 * abs(oD)
    assert np.abs(ga).max() < 1e-4 and np.abs(gb).max() < 1e-4
    # primal-dual gap: equals -(alpha.grad_alpha + beta.grad_beta) and closes
    # to the level the float32 solve leaves in the gradient
    gap = oracle.primal(P, T) - oD
    assert abs(gap + (a.astype(np.float64) @ ga + b.astype(np.float64) @ gb)) < 1e-10
    # the float32 line search stops once objective changes fall under the
    # float32 rounding of psi (about 1e-7 |D|); the gap left there is
    # |alpha.grad_alpha + beta.grad_beta|, a few 1e-4 |D| at most
    assert abs(gap) < 1e-3 * abs(ref["obj"])
    # the trace is nondecreasing (every accepted step satisfies sufficient increase)
    t = tr[0][~np.isnan(tr[0])]
    assert np.all(np.diff(t) >= -1e-12 * abs(t[-1]))


# (2600, 2): 1300-row whole groups; (4400, 2): split groups; (4000, 2000)
# and (8000, 4000): 44000 and 88000 group tiles, where the screen takes two
# and four passes of tiles per block
@pytest.mark.parametrize("n_src,n_groups", [(800, 5), (2600, 2), (4400, 2), (4000, 2000), (8000, 4000)])
def test_screened_trajectory_is_bitwise_dense(n_src, n_groups):
    inst = synth.blobs(seed=12, n_src=n_src, n_tgt=700, d=8, n_groups=n_groups, gamma=0.1, mu=0.3)
    C32, P = cases.with_cost(inst)
    h = handle_for(C32, P)
    ad, bd, infod, trd, _ = run(h, 120, use_screen=0)
    h.stats(reset=True)
    as_, bs_, infos, trs, _ = run(h, 120, use_screen=1)
    st = h.stats()
    np.testing.assert_array_equal(trd, trs)
    np.testing.assert_array_equal(ad, as_)
    np.testing.assert_array_equal(bd, bs_)
    assert infod[0]["evals"] == infos[0]["evals"]
    assert st["tiles_computed"] < st["tiles_total"] and st["refreshes"] >= 1
    # the ablation without the set N follows the same path too
    al, bl, infol, trl, _ = run(h, 120, use_screen=1, use_lower=0)
    np.testing.assert_array_equal(trd, trl)


def test_batched_solve_equals_single_solves():
    O = _O()
    insts = [cases.ragged(60 + i, n, m, s, gamma=g, mu=mu) for i, (n, m, s, g, mu) in enumerate(
        [(120, 90, [60, 60], 0.2, 0.3), (700, 50, [600, 100], 0.5, 0.1), (40, 200, [10, 10, 20], 0.1, 1.0)])]
    probs, singles = [], []
    for inst in insts:
        C32, P = cases.with_cost(inst)
        pr = dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                  cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN)
        probs.append(pr)
        singles.append((O.Handle([pr]), P))
    hb = O.Handle(probs)
    ab, bb, infob, trb, _ = run(hb, 80, use_screen=1)
    oa = ob = 0
    for i, (h, P) in enumerate(singles):
        a, b, info, tr, _ = run(h, 80, use_screen=1)
        np.testing.assert_array_equal(tr[0], trb[i])
        np.testing.assert_array_equal(a, ab[oa:oa + P.ns])
        np.testing.assert_array_equal(b, bb[ob:ob + P.nt])
        assert info[0]["evals"] == infob[i]["evals"]
        oa += P.ns
        ob += P.nt


def test_batched_solve_with_long_vectors_equals_single_solves():
    """Batches whose vectors total at least 32768 elements form the L-BFGS
    dots with one wavefront per vector block over all history slots, single
    solves with one per (block, slot): the trajectories agree bit for bit."""
    O = _O()
    shapes = [(1700, 1500), (1400, 1900), (2000, 1300), (1600, 1600), (1800, 1700), (1500, 2000),
              (1900, 1400), (1300, 2100), (1650, 1550), (1750, 1450), (1550, 1800)]
    assert sum(n + m for n, m in shapes) >= 32768 + 32 * len(shapes)
    probs, keep = [], {}
    for i, (n, m) in enumerate(shapes):
        L = 3 + i % 5
        sizes = [n // L] * (L - 1) + [n - (n // L) * (L - 1)]
        inst = cases.ragged(90 + i, n, m, sizes, gamma=0.2 + 0.05 * i, mu=0.1 + 0.03 * i)
        C32, P = cases.with_cost(inst)
        probs.append(dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                          cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN))
        if i in (0, 5, 10):
            keep[i] = P
    hb = O.Handle(probs)
    ab, bb, infob, trb, _ = run(hb, 60, use_screen=1)
    oa = np.concatenate([[0], np.cumsum([n for n, _ in shapes])])
    ob = np.concatenate([[0], np.cumsum([m for _, m in shapes])])
    for i, P in keep.items():
        a, b, info, tr, _ = run(O.Handle([probs[i]]), 60, use_screen=1)
        np.testing.assert_array_equal(tr[0], trb[i])
        np.testing.assert_array_equal(a, ab[oa[i]:oa[i + 1]])
        np.testing.assert_array_equal(b, bb[ob[i]:ob[i + 1]])
        assert info[0]["evals"] == infob[i]["evals"]


def test_user_start_at_the_optimum_stays_there():
    inst = cases.ragged(70, 150, 120, [50, 100], gamma=0.3, mu=0.2)
    C32, P = cases.with_cost(inst)
    ref = oracle.solve(P, max_iter=3000, gtol=1e-11)
    h = handle_for(C32, P)
    a0 = _dev(ref["alpha"].astype(np.float32))
    b0 = _dev(ref["beta"].astype(np.float32))
    a, b, info, rc = h.solve(a0, b0, max_iter=50, init_user=1, use_screen=1, gtol=1e-5)
    assert info[0]["iters"] <= 5
    assert abs(info[0]["obj"] - ref["obj"]) <= 1e-5 * abs(ref["obj"])


def test_graph_replay_equals_direct_launches():
    """The solver's recorded steps, replayed many times, give bit for bit the
    trajectory of direct launches (batched, screened, with refreshes)."""
    O = _O()
    insts = [synth.instance_from_generator((77, i), n_lo=40, n_hi=400, d=8) for i in range(6)]
    probs = [dict(labels=_dev(i["labels"]), n_groups=i["n_groups"], gamma=i["gamma"], mu=i["mu"],
                  x_src=_dev(i["xs"]), x_tgt=_dev(i["xt"]), cost_mode=O.OT_GS_COST_MATERIALIZE,
                  cost_scale=0.0) for i in insts]
    h = O.Handle(probs)
    res = []
    for g in (0, 1, 1):
        a, b, info, tr, rc = run(h, 300, use_screen=1, use_graph=g)
        res.append((a, b, tr, [x["evals"] for x in info]))
    for r in res[1:]:
        np.testing.assert_array_equal(res[0][0], r[0])
        np.testing.assert_array_equal(res[0][1], r[1])
        np.testing.assert_array_equal(res[0][2], r[2])
        assert res[0][3] == r[3]
