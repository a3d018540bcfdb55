"""Pins for the oracle's second solver, accelerated gradient ascent on the
dual with Algorithm 1's screening around it (the screening does not depend
on the solver: Theorem 1 and the remark after it in Sec. 3.4).  The paper
fixes no such solver, so the pins come from what the mathematics fixes:

- the optimum value: closed forms (one target, one source, constant cost)
  and the L-BFGS optimum on random problems, including uneven groups and
  non-uniform marginals (D is concave, its maximum value is unique);
- the step rule: every accepted objective is at least the previous one
  (the function-value restart), and at the final point the marginal
  conditions grad D = a - T1, b - T^T 1 = 0 hold to 1e-6;
- the momentum: with it the ascent reaches 1e-6 of the optimum in fewer
  accepted steps than without it (a wrong extrapolation coefficient or sign
  loses that);
- the screening: it follows the dense trajectory, bit for bit while N is
  empty (skipped blocks are exact zeros, Lemma 2) and up to the rounding
  of Algorithm 2's summation order once N holds blocks.
"""
import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import rand_problem


def _agd(P, **kw):
    kw.setdefault("max_iter", 20000)
    kw.setdefault("gtol", 1e-11)
    return oracle.agd_solve(P, **kw)


def test_agd_closed_form_single_target():
    P = rand_problem(10, 8, 1, 3, gamma=0.7, mu=0.3, sizes=[3, 1, 4])
    r = _agd(P)
    grp = sum(np.linalg.norm(P.a[P.labels == l]) for l in range(3))
    ref = P.a @ P.C[:, 0] + P.gamma * (0.5 * P.a @ P.a + P.mu * grp)
    assert abs(r["obj"] - ref) < 1e-10


def test_agd_closed_form_single_source():
    P = rand_problem(11, 1, 9, 1, gamma=0.7, mu=0.3)
    r = _agd(P)
    ref = P.b @ P.C[0] + P.gamma * np.sum(0.5 * P.b ** 2 + P.mu * P.b)
    assert abs(r["obj"] - ref) < 1e-10


def test_agd_closed_form_constant_cost():
    ns, nt, c = 8, 6, 0.37
    labels = np.array([0, 0, 0, 1, 2, 2, 2, 2])
    P = oracle.Problem(np.full((ns, nt), c), labels, 3, 0.7, 0.3)
    r = _agd(P)
    g = np.bincount(labels)
    ref = c + P.gamma * (1 / (2 * ns * nt) + P.mu * np.sqrt(g).sum() / ns)
    assert abs(r["obj"] - ref) < 1e-10


def _nonuniform(seed, ns, nt, L, gamma, mu):
    P = rand_problem(seed, ns, nt, L, gamma=gamma, mu=mu)
    rng = np.random.default_rng(seed + 100)
    a = rng.random(ns) + 0.2
    b = rng.random(nt) + 0.2
    return oracle.Problem(P.C, P.labels, L, gamma, mu, a=a / a.sum(), b=b / b.sum())


@pytest.mark.parametrize("case", [
    (20, 60, 50, 4, 0.5, 0.3, False), (21, 45, 70, 6, 0.1, 0.1, False),
    (22, 50, 40, 3, 0.05, 1.0, True), (23, 30, 80, 5, 1.0, 0.0, True)])
def test_agd_reaches_the_lbfgs_optimum(case):
    seed, ns, nt, L, gamma, mu, nonuni = case
    P = _nonuniform(seed, ns, nt, L, gamma, mu) if nonuni else rand_problem(seed, ns, nt, L, gamma, mu)
    ref = oracle.solve(P, max_iter=5000, gtol=1e-12)
    r = _agd(P)
    assert abs(r["obj"] - ref["obj"]) <= 1e-10 * abs(ref["obj"])
    # accepted objectives never decrease
    assert np.all(np.diff(r["trace"]) >= 0.0)
    # the point is optimal: its gradient a - T1, b - T^T 1 vanishes
    ga, gb, D = oracle.dual_grad(P, r["alpha"], r["beta"])
    assert D == r["obj"]
    assert max(np.abs(ga).max(), np.abs(gb).max()) <= 1e-6


@pytest.mark.parametrize("seed,gamma,mu", [(30, 0.1, 0.1), (31, 0.05, 0.5), (32, 0.5, 0.3)])
def test_momentum_accelerates(seed, gamma, mu):
    P = rand_problem(seed, 60, 50, 4, gamma=gamma, mu=mu)
    ref = oracle.solve(P, max_iter=5000, gtol=1e-12)

    def steps_to(r, tol=1e-6):
        rel = (ref["obj"] - r["trace"]) / abs(ref["obj"])
        hit = np.nonzero(rel <= tol)[0]
        return hit[0] if hit.size else np.inf
    fast = steps_to(oracle.agd_solve(P, max_iter=20000))
    slow = steps_to(oracle.agd_solve(P, max_iter=20000, momentum=False))
    assert fast < np.inf and fast < 0.5 * slow, (fast, slow)


@pytest.mark.parametrize("use_lower", [True, False])
@pytest.mark.parametrize("sizes", [[14] * 5, [1] * 20 + [2] * 20])
def test_screened_agd_follows_the_dense_trajectory(use_lower, sizes):
    # groups of 14 rows (N stays empty: the lower bound never clears mu
    # gamma a step away) and groups of one or two rows (N fills)
    P = rand_problem(41, sum(sizes), 50, len(sizes), gamma=0.2, mu=0.2 if sizes[0] == 1 else 0.8,
                     sizes=sizes)
    d = oracle.agd_solve(P, max_iter=600)
    s = oracle.agd_solve(P, max_iter=600, use_screen=True, r=7, use_lower=use_lower)
    if s["s_i"] == 0:
        np.testing.assert_array_equal(d["trace"], s["trace"])
        np.testing.assert_array_equal(d["alpha"], s["alpha"])
        np.testing.assert_array_equal(d["beta"], s["beta"])
    else:
        # Algorithm 2 adds the blocks in N first: the same sums in another
        # order, equal up to rounding (near the optimum, where D is flat, the
        # points then drift apart by more than the objectives do)
        np.testing.assert_allclose(s["trace"], d["trace"], rtol=1e-12, atol=0)
    # the upper bound skipped checked pairs, and only the lower bound puts
    # pairs in N
    assert s["s_u"] < s["s_n"]
    assert (s["s_i"] > 0) == (use_lower and sizes[0] == 1)
