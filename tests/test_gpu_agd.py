"""The accelerated-ascent solver on the device (OT_GS_SOLVER_AGD) against the
oracle's accelerated ascent and the FP64 optimum:

- its first accepted objectives follow the oracle's run of the same method
  (same steps, float32 against float64 vectors);
- it reaches the oracle's optimum within the float32 floor, with accepted
  objectives that never decrease;
- screened (with and without N) and dense solves follow the same trajectory
  bit for bit (the screening composes with this solver too, Theorem 1);
- a batch of instances gives each instance's single-handle trajectory.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import cases
from tests.test_gpu_solve import handle_for

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run_agd(h, max_iter, **kw):
    O = _O()
    tr = torch.full((h.count * (max_iter + 1),), float("nan"), dtype=torch.float64, device="cuda")
    a, b, info, rc = h.solve(obj_trace=tr, max_iter=max_iter, solver=O.OT_GS_SOLVER_AGD, max_ls=60, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), info, tr.cpu().numpy().reshape(h.count, max_iter + 1), rc


def _instance(seed=31, n_src=300, n_tgt=260, n_groups=5, gamma=0.1, mu=0.3):
    inst = synth.blobs(seed=seed, n_src=n_src, n_tgt=n_tgt, d=8, n_groups=n_groups, gamma=gamma, mu=mu)
    return cases.with_cost(inst)


def test_first_steps_follow_the_oracle():
    C32, P = _instance()
    ref = oracle.agd_solve(P, max_iter=30, max_bt=60)
    h = handle_for(C32, P)
    _, _, info, tr, _ = run_agd(h, 30, use_screen=0)
    t = tr[0][:31]
    # float32 points against float64 ones: the objectives agree to the
    # float32 rounding of a step (a few 1e-7 of D per step, accumulating)
    np.testing.assert_allclose(t, ref["trace"][:31], rtol=2e-5, atol=1e-7)


@pytest.mark.parametrize("gamma,mu", [(0.1, 0.3), (1.0, 0.1), (0.02, 1.0)])
def test_reaches_the_optimum(gamma, mu):
    C32, P = _instance(gamma=gamma, mu=mu)
    ref = oracle.solve(P, max_iter=5000, gtol=1e-12)
    h = handle_for(C32, P)
    a, b, info, tr, _ = run_agd(h, 6000, use_screen=1)
    t = tr[0][~np.isnan(tr[0])]
    assert np.all(np.diff(t) >= 0.0)
    D = info[0]["obj"]
    assert abs(D - ref["obj"]) <= 1e-5 * abs(ref["obj"]), (D, ref["obj"], info)
    # the oracle at the device's final point agrees with the device's D
    _, _, oD = oracle.dual_grad(P, a.astype(np.float64), b.astype(np.float64))
    assert abs(oD - D) <= 1e-5 * abs(oD)


@pytest.mark.parametrize("n_src,n_groups,use_lower", [(800, 5, 1), (800, 5, 0), (2600, 2, 1), (700, 300, 1)])
def test_screened_trajectory_is_bitwise_dense(n_src, n_groups, use_lower):
    inst = synth.blobs(seed=12, n_src=n_src, n_tgt=700, d=8, n_groups=n_groups, gamma=0.1, mu=0.5)
    C32, P = cases.with_cost(inst)
    h = handle_for(C32, P)
    ad, bd, infod, trd, _ = run_agd(h, 150, use_screen=0)
    h.stats(reset=True)
    as_, bs_, infos, trs, _ = run_agd(h, 150, use_screen=1, use_lower=use_lower, refresh=5)
    st = h.stats()
    np.testing.assert_array_equal(trd, trs)
    np.testing.assert_array_equal(ad, as_)
    np.testing.assert_array_equal(bd, bs_)
    assert infod[0]["evals"] == infos[0]["evals"] and infod[0]["iters"] == infos[0]["iters"]
    assert st["tiles_computed"] < st["tiles_total"] and st["refreshes"] >= 1


def test_batched_equals_single():
    O = _O()
    insts = [synth.blobs(seed=40 + i, n_src=200 + 90 * i, n_tgt=150 + 70 * i, d=8, n_groups=3 + i,
                         gamma=0.1 * (i + 1), mu=0.3) for i in range(3)]
    Cs = [cases.with_cost(x) for x in insts]
    probs = [dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32), cost_scale=1.0,
                  cost_mode=O.OT_GS_COST_GIVEN) for C32, P in Cs]
    hb = O.Handle(probs)
    ab, bb, infob, trb, _ = run_agd(hb, 200, use_screen=1)
    ro = co = 0
    for k, (C32, P) in enumerate(Cs):
        a1, b1, info1, tr1, _ = run_agd(handle_for(C32, P), 200, use_screen=1)
        np.testing.assert_array_equal(trb[k], tr1[0])
        np.testing.assert_array_equal(ab[ro:ro + P.ns], a1)
        np.testing.assert_array_equal(bb[co:co + P.nt], b1)
        assert infob[k] == info1[0]
        ro += P.ns
        co += P.nt


def test_options_are_checked():
    O = _O()
    C32, P = _instance()
    h = handle_for(C32, P)
    with pytest.raises(O.OTGSError) as e:
        h.solve(max_iter=5, solver=O.OT_GS_SOLVER_AGD, use_screen=1, verify=1)
    assert e.value.code == O.OT_GS_EINVAL
    with pytest.raises(O.OTGSError) as e:
        h.solve(max_iter=5, solver=7)
    assert e.value.code == O.OT_GS_EINVAL




def test_onthefly_cost_screened_equals_dense_and_follows_the_oracle():
    """Cost recomputed on the matrix cores (integer features, power-of-two
    scale: the cost is exact): screened and dense accelerated ascent follow
    the same trajectory, and the first steps follow the oracle's."""
    from tests.test_gpu_onthefly import int_instance, otf_handle
    inst = int_instance(41, [300, 40, 7, 200], 250, 20, gamma=0.2, mu=0.3)
    scale = 2.0 ** -9
    h = otf_handle(inst, scale)
    ad, bd, infod, trd, _ = run_agd(h, 300, use_screen=0)
    as_, bs_, infos, trs, _ = run_agd(h, 300, use_screen=1, refresh=5)
    np.testing.assert_array_equal(trd, trs)
    np.testing.assert_array_equal(ad, as_)
    np.testing.assert_array_equal(bd, bs_)
    C = oracle.cost_sqeuclid(inst["xs"], inst["xt"]) * scale
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    ref = oracle.agd_solve(P, max_iter=30, max_bt=60)
    np.testing.assert_allclose(trd[0][:31], ref["trace"][:31], rtol=2e-5, atol=1e-7)
