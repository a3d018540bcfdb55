"""Pins for the FP64 oracle: each test checks the oracle against something other
than itself (a definition solved numerically, a closed form, an invariant, a
library routine or a value printed in the paper), chosen so that a dropped
term, a wrong sign or index or a transposed operand fails at least one."""
import math
import os

import numpy as np
import pytest
import scipy.optimize as so
from scipy.spatial.distance import cdist

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_problem(seed, ns, nt, L, gamma=0.5, mu=0.3, d=3, sizes=None):
    rng = np.random.default_rng(seed)
    xs = rng.standard_normal((ns, d))
    xt = rng.standard_normal((nt, d)) + 0.4
    if sizes is None:
        labels = rng.integers(0, L, ns)
    else:
        labels = rng.permutation(np.repeat(np.arange(L), sizes))
    C, _ = oracle.cost_normalized(xs, xt)
    return oracle.Problem(C, labels, L, gamma, mu)


def Psi(t, labels, L, gamma, mu):
    """Regulariser of one column, Eq. 3."""
    grp = sum(np.linalg.norm(t[labels == l]) for l in range(L))
    return gamma * (0.5 * t @ t + mu * grp)


# --------------------------------------------------------------- psi and grad psi

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_psi_is_the_conjugate_of_the_regulariser(seed):
    """psi(f) = sup_{g >= 0} f.g - Psi(g) (Sec. 2.3): solve the sup numerically
    (smoothed group norm, bound-constrained L-BFGS-B) and compare the value
    and maximiser with the oracle's objective and plan on a 1-column problem."""
    ns, L, gamma, mu = 9, 3, 0.7, 0.4
    P = rand_problem(seed, ns, 1, L, gamma, mu)
    rng = np.random.default_rng(100 + seed)
    f = 0.8 * rng.standard_normal(ns)
    alpha = f + P.C[:, 0]            # beta = 0 so that f = alpha - c
    beta = np.zeros(1)
    _, _, D, T = oracle.dual_grad(P, alpha, beta, want_plan=True)
    psi_oracle = P.a @ alpha - D

    eps = 1e-10

    def negobj(g):
        val, grad = -f @ g, -f.copy()
        val += gamma * 0.5 * g @ g
        grad += gamma * g
        for l in range(L):
            m = P.labels == l
            nrm = math.sqrt(g[m] @ g[m] + eps * eps)
            val += gamma * mu * nrm
            grad[m] += gamma * mu * g[m] / nrm
        return val, grad

    best = None
    for start in (np.maximum(f, 0) / gamma, np.full(ns, 0.1), np.zeros(ns) + 1e-3):
        res = so.minimize(negobj, start, jac=True, method="L-BFGS-B",
                          bounds=[(0, None)] * ns, options=dict(ftol=1e-15, gtol=1e-13, maxiter=5000))
        if best is None or res.fun < best.fun:
            best = res
    assert abs(psi_oracle - (-best.fun)) < 1e-7
    np.testing.assert_allclose(T[:, 0], best.x, atol=2e-5)


@pytest.mark.parametrize("seed", [3, 4])
def test_plan_satisfies_kkt_of_the_sup(seed):
    """The plan column t = grad psi(f) satisfies the optimality conditions of
    max_{g>=0} f.g - Psi(g): on a nonzero group, f_i - gamma t_i - gamma mu
    t_i/||t_[l]|| = 0 where t_i > 0 and <= 0 where t_i = 0; a zero group has
    ||[f_[l]]_+|| <= gamma mu."""
    ns, nt, L, gamma, mu = 12, 4, 3, 0.3, 0.5
    P = rand_problem(seed, ns, nt, L, gamma, mu)
    rng = np.random.default_rng(seed)
    alpha = 0.6 + 0.3 * rng.standard_normal(ns)
    beta = 0.3 * rng.standard_normal(nt)
    T = oracle.plan(P, alpha, beta)
    nz = 0
    for j in range(nt):
        f = alpha + beta[j] - P.C[:, j]
        for l in range(L):
            m = P.labels == l
            t = T[m, j]
            if np.all(t == 0):
                assert np.linalg.norm(np.maximum(f[m], 0)) <= gamma * mu + 1e-12
            else:
                nz += 1
                nrm = np.linalg.norm(t)
                r = f[m] - gamma * t - gamma * mu * t / nrm
                assert np.all(np.abs(r[t > 0]) < 1e-12)
                assert np.all(r[t == 0] <= 1e-12)
    assert nz > 0


def test_mu_zero_reduces_to_squared_l2_smooth_ot():
    """With mu = 0 the regulariser is gamma/2 ||t||^2, whose conjugate over
    t >= 0 is ||[f]_+||^2 / (2 gamma) with gradient [f]_+ / gamma."""
    P = rand_problem(5, 15, 11, 4, gamma=0.25, mu=0.0)
    rng = np.random.default_rng(5)
    alpha = 0.5 + 0.2 * rng.standard_normal(P.ns)
    beta = 0.2 * rng.standard_normal(P.nt)
    ga, gb, D, T = oracle.dual_grad(P, alpha, beta, want_plan=True)
    F = alpha[:, None] + beta[None, :] - P.C
    Tref = np.maximum(F, 0) / P.gamma
    np.testing.assert_allclose(T, Tref, rtol=1e-13, atol=1e-15)
    Dref = P.a @ alpha + P.b @ beta - (np.maximum(F, 0) ** 2).sum() / (2 * P.gamma)
    assert abs(D - Dref) < 1e-13
    np.testing.assert_allclose(ga, P.a - Tref.sum(1), atol=1e-14)
    np.testing.assert_allclose(gb, P.b - Tref.sum(0), atol=1e-14)


# --------------------------------------------------------------- gradient of D

@pytest.mark.parametrize("seed", [6, 7])
def test_gradient_matches_central_differences(seed):
    P = rand_problem(seed, 14, 10, 3, gamma=0.4, mu=0.2, sizes=[6, 5, 3])
    rng = np.random.default_rng(seed)
    alpha = 0.5 + 0.3 * rng.standard_normal(P.ns)
    beta = 0.3 * rng.standard_normal(P.nt)
    ga, gb, _ = oracle.dual_grad(P, alpha, beta)
    h = 1e-6
    for i in range(P.ns):
        e = np.zeros(P.ns); e[i] = h
        fd = (oracle.dual_obj(P, alpha + e, beta) - oracle.dual_obj(P, alpha - e, beta)) / (2 * h)
        assert abs(fd - ga[i]) < 1e-7 * max(1.0, abs(ga[i]))
    for j in range(P.nt):
        e = np.zeros(P.nt); e[j] = h
        fd = (oracle.dual_obj(P, alpha, beta + e) - oracle.dual_obj(P, alpha, beta - e)) / (2 * h)
        assert abs(fd - gb[j]) < 1e-7 * max(1.0, abs(gb[j]))


def test_duality_gap_identity_and_mass_balance():
    """Fenchel-Young gives P(T(alpha,beta)) - D(alpha,beta) =
    -(alpha.grad_alpha + beta.grad_beta) at every point, and both gradient
    blocks sum to 1 - sum(T)."""
    P = rand_problem(8, 20, 16, 5, gamma=0.3, mu=0.6)
    rng = np.random.default_rng(8)
    for k in range(3):
        alpha = 0.4 + 0.3 * rng.standard_normal(P.ns)
        beta = 0.3 * rng.standard_normal(P.nt)
        ga, gb, D, T = oracle.dual_grad(P, alpha, beta, want_plan=True)
        gap = oracle.primal(P, T) - D
        assert abs(gap + (alpha @ ga + beta @ gb)) < 1e-12
        assert abs(ga.sum() - (1 - T.sum())) < 1e-13
        assert abs(gb.sum() - (1 - T.sum())) < 1e-13
        # the plan written out agrees with the gradient it implies
        np.testing.assert_allclose(ga, P.a - T.sum(1), atol=1e-15)


def test_empty_group_contributes_nothing():
    P = rand_problem(9, 12, 7, 3, sizes=[5, 7, 0])
    rng = np.random.default_rng(9)
    alpha = 0.5 + 0.3 * rng.standard_normal(P.ns)
    beta = 0.3 * rng.standard_normal(P.nt)
    P2 = oracle.Problem(P.C, P.labels, 2, P.gamma, P.mu)   # the empty label removed
    r1, r2 = oracle.dual_grad(P, alpha, beta), oracle.dual_grad(P2, alpha, beta)
    for x, y in zip(r1, r2):
        np.testing.assert_array_equal(x, y)


# --------------------------------------------------------------- whole solver

def _converge(P, **kw):
    r = oracle.solve(P, max_iter=kw.pop("max_iter", 3000), gtol=1e-11, **kw)
    return r


def test_closed_form_single_target():
    """n_tgt = 1: the only feasible plan is T = a, so D* = a.c +
    gamma(||a||^2/2 + mu sum_l ||a_[l]||)."""
    P = rand_problem(10, 8, 1, 3, gamma=0.7, mu=0.3, sizes=[3, 1, 4])
    r = _converge(P)
    grp = sum(np.linalg.norm(P.a[P.labels == l]) for l in range(3))
    ref = P.a @ P.C[:, 0] + P.gamma * (0.5 * P.a @ P.a + P.mu * grp)
    assert abs(r["obj"] - ref) < 1e-10


def test_closed_form_single_source():
    """n_src = 1: T = b^T, each column's only group has one entry, so
    D* = b.c + gamma sum_j (b_j^2/2 + mu b_j)."""
    P = rand_problem(11, 1, 9, 1, gamma=0.7, mu=0.3)
    r = _converge(P)
    ref = P.b @ P.C[0] + P.gamma * np.sum(0.5 * P.b ** 2 + P.mu * P.b)
    assert abs(r["obj"] - ref) < 1e-10


def test_closed_form_constant_cost():
    """Constant C = c with uniform marginals: the uniform plan is optimal and
    D* = c + gamma (1/(2 n_src n_tgt) + mu sum_l sqrt(g_l) / n_src)."""
    ns, nt, c = 8, 6, 0.37
    labels = np.array([0, 0, 0, 1, 2, 2, 2, 2])
    P = oracle.Problem(np.full((ns, nt), c), labels, 3, 0.7, 0.3)
    r = _converge(P)
    g = np.bincount(labels)
    ref = c + P.gamma * (1 / (2 * ns * nt) + P.mu * np.sqrt(g).sum() / ns)
    assert abs(r["obj"] - ref) < 1e-10


@pytest.mark.parametrize("seed,ns,nt,L", [(12, 3, 3, 2), (13, 2, 3, 1), (14, 3, 2, 2)])
def test_brute_force_tiny(seed, ns, nt, L):
    """On instances of at most 3 x 3, a derivative-free Nelder-Mead ascent of
    D and an SLSQP solve of the primal (Eqs. 2-3) over the transportation
    polytope both reach the oracle's D* (strong duality)."""
    P = rand_problem(seed, ns, nt, L, gamma=0.6, mu=0.5)
    r = _converge(P)

    def negD(x):
        return -oracle.dual_obj(P, x[:ns], x[ns:])
    nm = so.minimize(negD, np.zeros(ns + nt), method="Nelder-Mead",
                     options=dict(xatol=1e-12, fatol=1e-15, maxiter=200000, maxfev=200000))
    assert abs(-nm.fun - r["obj"]) < 1e-9

    def primal(t):
        T = t.reshape(ns, nt)
        val = (T * P.C).sum()
        for j in range(nt):
            val += Psi(T[:, j], P.labels, L, P.gamma, P.mu)
        return val
    cons = [dict(type="eq", fun=lambda t: t.reshape(ns, nt).sum(1) - P.a),
            dict(type="eq", fun=lambda t: t.reshape(ns, nt).sum(0)[:-1] - P.b[:-1])]
    sq = so.minimize(primal, np.outer(P.a, P.b).ravel(), method="SLSQP", constraints=cons,
                     bounds=[(0, None)] * (ns * nt), options=dict(ftol=1e-14, maxiter=2000))
    assert abs(sq.fun - r["obj"]) < 1e-6


def test_scipy_lbfgsb_reaches_the_same_optimum():
    P = rand_problem(15, 30, 25, 4, gamma=0.3, mu=0.4)
    r = _converge(P)

    def fg(x):
        ga, gb, D = oracle.dual_grad(P, x[:P.ns], x[P.ns:])
        return -D, -np.concatenate([ga, gb])
    sp = so.minimize(fg, np.zeros(P.ns + P.nt), jac=True, method="L-BFGS-B",
                     options=dict(ftol=1e-16, gtol=1e-12, maxiter=20000, maxcor=20))
    assert abs(-sp.fun - r["obj"]) < 1e-10 * abs(r["obj"])
    # optimal plans coincide (the primal is strongly convex) and are feasible
    T1 = oracle.plan(P, r["alpha"], r["beta"])
    T2 = oracle.plan(P, sp.x[:P.ns], sp.x[P.ns:])
    np.testing.assert_allclose(T1, T2, atol=1e-7)
    # marginals hold up to the final gradient (grad_alpha = a - T1), and the
    # primal-dual gap closes
    assert r["gnorm_inf"] < 1e-7
    np.testing.assert_allclose(T1.sum(1), P.a, atol=1.01 * r["gnorm_inf"])
    np.testing.assert_allclose(T1.sum(0), P.b, atol=1.01 * r["gnorm_inf"])
    assert abs(oracle.primal(P, T1) - r["obj"]) < 1e-8


# --------------------------------------------------------------- bounds

def _snap_and_move(P, seed, scale_move=0.05):
    rng = np.random.default_rng(seed)
    a_s = 0.5 + 0.3 * rng.standard_normal(P.ns)
    b_s = 0.3 * rng.standard_normal(P.nt)
    a = a_s + scale_move * rng.standard_normal(P.ns)
    b = b_s + scale_move * rng.standard_normal(P.nt)
    return a_s, b_s, a, b


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("move", [0.0, 0.01, 0.2])
def test_bounds_sandwich_the_group_norm(seed, move):
    """Lemmas 1 and 4: z_lower <= z <= z_upper for any snapshot and any point."""
    P = rand_problem(20 + seed, 17, 13, 4, sizes=[6, 5, 4, 2])
    a_s, b_s, a, b = _snap_and_move(P, seed, move)
    Zs, Os, Ks = oracle.group_norms(P, a_s, b_s)
    Z, _, _ = oracle.group_norms(P, a, b)
    up = oracle.upper_bound(P, a, b, a_s, b_s, Zs)
    lo = oracle.lower_bound(P, a, b, a_s, b_s, Ks, Os)
    assert np.all(lo <= Z + 1e-12)
    assert np.all(Z <= up + 1e-12)
    if move == 0.0:
        # Theorem 3: no error when the point is the snapshot
        np.testing.assert_array_equal(up, Z)


def test_upper_bound_terms_are_tight_for_pure_shifts():
    """Eq. 6 is exact when the group block of f is a positive constant vector
    and the move is a nonnegative shift of beta_j: z grows by exactly
    sqrt(g_l) dbeta_j (the triangle inequality holds with equality for
    parallel vectors)."""
    rng = np.random.default_rng(30)
    labels = np.array([0, 0, 0, 0, 0, 0, 1, 1, 1, 1])
    crow = rng.uniform(0, 1, (2, 6))
    C = crow[labels]                             # rows equal within a group
    P = oracle.Problem(C, labels, 2, 0.5, 0.3)
    a_s = np.full(P.ns, 2.0)                     # f > 0 and constant per group
    b_s = np.zeros(P.nt)
    Zs, _, _ = oracle.group_norms(P, a_s, b_s)
    b = b_s + np.linspace(0.0, 0.3, P.nt)
    Z, _, _ = oracle.group_norms(P, a_s, b)
    up = oracle.upper_bound(P, a_s, b, a_s, b_s, Zs)
    np.testing.assert_allclose(up, Z, rtol=1e-14)
    # and it is strict for a shift of alpha that is not constant in the group
    a = a_s.copy(); a[0] += 0.5
    Z2, _, _ = oracle.group_norms(P, a, b_s)
    up2 = oracle.upper_bound(P, a, b_s, a_s, b_s, Zs)
    assert np.all(up2[0] > Z2[0]) and np.all(up2[1] == Z2[1])


def test_lower_bound_error_at_the_snapshot():
    """Theorem 4 and Corollary 1: at the snapshot the lower bound misses z by
    exactly | ||f+|| + ||f-|| - ||f|| |, which is zero for single-signed
    groups."""
    P = rand_problem(31, 16, 9, 3, sizes=[7, 5, 4])
    rng = np.random.default_rng(31)
    a = 0.5 + 0.3 * rng.standard_normal(P.ns)
    b = 0.3 * rng.standard_normal(P.nt)
    a[P.labels == 0] = 3.0                      # group 0 all positive
    a[P.labels == 1] = -3.0                     # group 1 all negative
    Z, O, K = oracle.group_norms(P, a, b)
    lo = oracle.lower_bound(P, a, b, a, b, K, O)
    np.testing.assert_allclose(Z - lo, np.abs(Z + O - K), atol=1e-14)
    np.testing.assert_allclose(lo[0], Z[0], rtol=1e-14)
    np.testing.assert_allclose(lo[1], Z[1], atol=1e-14)


# --------------------------------------------------------------- Algorithms 1-2

def test_algorithm2_equals_the_dense_gradient():
    """Theorem 2 at the level of one evaluation: with any snapshot and any
    set N, Algorithm 2 returns the dense gradient and objective."""
    P = rand_problem(40, 40, 30, 5, gamma=0.2, mu=0.8)
    rng = np.random.default_rng(40)
    a_s, b_s = 0.3 * rng.standard_normal(P.ns), 0.3 * rng.standard_normal(P.nt)
    S = oracle.ScreenState(P, a_s, b_s)
    for k in range(4):
        a = a_s + 0.05 * rng.standard_normal(P.ns)
        b = b_s + 0.05 * rng.standard_normal(P.nt)
        if k == 2:
            S.extract(a, b)
        ga, gb, D = oracle.dual_grad(P, a, b)
        ga2, gb2, D2 = oracle.gradpsi(P, S, a, b)
        np.testing.assert_allclose(ga2, ga, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(gb2, gb, rtol=1e-13, atol=1e-15)
        assert abs(D - D2) <= 1e-14 * max(1, abs(D))
    c = S.counters
    assert c["s_n"] + c["s_i"] == 4 * P.L * P.nt
    assert c["s_u"] <= c["s_n"]


# --------------------------------------------------------------- set N (Eq. 8)

def test_extraction_is_sound():
    """Lemma 5: every block put in N by Eq. 8 has z > mu gamma at the point of
    extraction (its gradient is nonzero).  Snapshots near the point make N
    large; the check would fail for an N holding every block, since many
    blocks there have z <= mu gamma."""
    P = rand_problem(45, 60, 50, 4, gamma=0.2, mu=0.4)
    rng = np.random.default_rng(45)
    a = 0.4 + 0.3 * rng.standard_normal(P.ns)
    b = 0.3 * rng.standard_normal(P.nt)
    Z, _, _ = oracle.group_norms(P, a, b)
    thr = P.mu * P.gamma
    assert 0 < np.count_nonzero(Z > thr) < Z.size
    sizes = []
    for eps in (0.0, 1e-4, 1e-3, 1e-2, 5e-2):
        S = oracle.ScreenState(P, a + eps * rng.standard_normal(P.ns), b + eps * rng.standard_normal(P.nt))
        S.extract(a, b)
        N = S.inN.astype(bool)
        assert np.all(Z[N] > thr)
        sizes.append(int(N.sum()))
    # close snapshots extract most active blocks, far ones fewer
    assert sizes[0] > 0 and sizes[0] >= sizes[-1]


def test_extraction_is_exact_for_single_signed_blocks_at_the_snapshot():
    """Corollary 1: at the snapshot (no change in alpha, beta) the lower
    bound equals z for a block whose f has one sign, so N is exactly
    {z > mu gamma} there.  One-row groups make every block single-signed;
    one block sits exactly at z = mu gamma (0.125, exact in binary) and must
    stay out of N (Eq. 8 is strict)."""
    ns, nt = 6, 5
    labels = np.arange(ns, dtype=np.int32)
    C = np.tile(np.linspace(0.0, 0.5, nt), (ns, 1))
    P = oracle.Problem(C, labels, ns, 0.5, 0.25)
    thr = P.mu * P.gamma
    assert thr == 0.125
    a = np.array([0.125, 0.3, 0.1, 0.7, 0.2, 0.0])
    b = np.zeros(nt)
    Z, O, K = oracle.group_norms(P, a, b)
    assert Z[0, 0] == thr
    S = oracle.ScreenState(P, a, b)
    S.extract(a, b)
    np.testing.assert_array_equal(S.inN.astype(bool), Z > thr)
    assert not S.inN[0, 0]


def test_extraction_against_a_far_snapshot_is_empty():
    """Eq. 7 subtracts ||alpha - alpha~|| restricted to the group from
    k~ = ||f~||; once that change exceeds every k~, no lower bound is
    positive and N is empty, although many blocks have z > mu gamma at the
    point itself.  (Bounds taken against the point itself instead of the
    snapshot would put those blocks in N.)"""
    P = rand_problem(46, 40, 30, 3, gamma=0.2, mu=0.3)
    rng = np.random.default_rng(46)
    a = 0.5 + 0.2 * rng.standard_normal(P.ns)
    b = 0.2 * rng.standard_normal(P.nt)
    Z, _, _ = oracle.group_norms(P, a, b)
    assert np.count_nonzero(Z > P.mu * P.gamma) > 10
    S = oracle.ScreenState(P, a + 10.0, b)
    S.extract(a, b)
    assert not S.inN.any()
    # at the point itself as snapshot, the same blocks are extracted
    S0 = oracle.ScreenState(P, a, b)
    S0.extract(a, b)
    assert S0.inN.any()


def test_first_refresh_extracts_against_the_zero_snapshot():
    """Algorithm 1 builds N from the bounds of the previous snapshot before
    refreshing it.  The first refresh (after r iterations) therefore uses the
    zero snapshot, where f = -C <= 0 gives k~ = o~ and a lower bound <= 0:
    its N is empty, and no block is evaluated because of N before the second
    refresh, although extracting against the refreshed snapshot itself would
    have filled N.  Later refreshes do use N."""
    inst = synth.paper_synthetic(10, g=10)
    C, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    P = oracle.Problem(C, inst["labels"], 10, *oracle.rho_form(1.0, 0.8))
    r10 = oracle.solve(P, max_iter=10, r=10, use_screen=True)
    S = oracle.ScreenState(P, r10["alpha"], r10["beta"])
    S.extract(r10["alpha"], r10["beta"])
    assert S.inN.any()
    r1 = oracle.solve(P, max_iter=19, r=10, use_screen=True)
    assert r1["iters"] == 19 and r1["s_r"] == 1 and r1["s_i"] == 0
    r3 = oracle.solve(P, max_iter=100, r=10, use_screen=True)
    assert r3["s_r"] == 10 and r3["s_i"] > 0


def test_screened_solve_follows_the_dense_trajectory():
    """Theorem 2: Algorithm 1 reaches the same objective as the original
    method; here every iterate agrees, and gradients were skipped."""
    inst = synth.paper_synthetic(8, g=10)
    C, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    g, mu = oracle.rho_form(0.1, 0.8)
    P = oracle.Problem(C, inst["labels"], 8, g, mu)
    rd = oracle.solve(P, max_iter=300, use_screen=False)
    rs = oracle.solve(P, max_iter=300, use_screen=True)
    n = min(rd["trace"].size, rs["trace"].size)
    np.testing.assert_allclose(rs["trace"][:n], rd["trace"][:n], rtol=1e-12)
    assert rs["s_u"] + rs["s_i"] < rs["evals"] * P.L * P.nt


def test_rho_form_mapping():
    """Sec. 5.2 parameterises the regulariser by (gamma, rho); it equals Eq. 3
    with gamma' = gamma (1 - rho), mu' = rho / (1 - rho)."""
    rng = np.random.default_rng(41)
    labels = rng.integers(0, 3, 10)
    for gamma, rho in [(1e3, 0.8), (0.1, 0.2), (1.0, 0.6)]:
        t = np.abs(rng.standard_normal(10))
        grp = sum(np.linalg.norm(t[labels == l]) for l in range(3))
        psi_rho = gamma * (0.5 * (1 - rho) * t @ t + rho * grp)
        g2, m2 = oracle.rho_form(gamma, rho)
        assert abs(Psi(t, labels, 3, g2, m2) - psi_rho) < 1e-12 * psi_rho
    with pytest.raises(ValueError):
        oracle.rho_form(1.0, 1.0)


# --------------------------------------------------------------- Table 1

def _table1():
    rows = {}
    with open(os.path.join(HERE, "golden", "table1_max_objective.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                L, o, s = line.split()
                rows[int(L)] = (float(o), float(s))
    return rows


def test_table1_scale_on_the_paper_synthetic_set():
    """Table 1 lists the largest converged objective over the (gamma, rho)
    grid.  At gamma = 1e3, rho = 0.8 with g = 10, Cauchy-Schwarz gives
    D* >= gamma rho / sqrt(g) = 252.98 (group term of any feasible plan is at
    least 1/sqrt(g)); with the cost normalised by its maximum the transport
    term adds about 0.01-0.08.  The oracle must land there and reproduce the
    printed 2.530e2 for 20 classes to four significant digits."""
    rows = _table1()
    g10, mu = oracle.rho_form(1e3, 0.8)
    lb = 1e3 * 0.8 / math.sqrt(10)
    for L in (10, 20, 40):
        inst = synth.paper_synthetic(L)
        C, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
        P = oracle.Problem(C, inst["labels"], L, g10, mu)
        r = oracle.solve(P, max_iter=2000, gtol=1e-9)
        assert lb <= r["obj"] < lb + 0.2
        if L == 20:
            assert float(f"{r['obj']:.3e}") == rows[20][0] == rows[20][1]
    # every printed row is origin == ours (Theorem 2)
    assert all(o == s for o, s in rows.values())


# --------------------------------------------------------------- cost

def test_cost_matches_scipy_cdist():
    rng = np.random.default_rng(50)
    xs, xt = rng.standard_normal((13, 5)), rng.standard_normal((9, 5))
    np.testing.assert_allclose(oracle.cost_sqeuclid(xs, xt), cdist(xs, xt, "sqeuclidean"),
                               rtol=1e-13, atol=1e-13)


def test_parallel_definition_equals_the_serial_one():
    """orc_dual_grad_par is the same definition with the columns shared among
    threads: every value equal bit for bit, whatever the thread count (an
    empty label, uneven groups), and the solve that uses it follows the same
    trajectory."""
    P = rand_problem(47, 300, 211, 5, gamma=0.2, mu=0.3, sizes=[100, 0, 150, 7, 43])
    rng = np.random.default_rng(47)
    a = 0.4 + 0.3 * rng.standard_normal(P.ns)
    b = 0.3 * rng.standard_normal(P.nt)
    ref = oracle.dual_grad(P, a, b)
    for nt in (1, 2, 3, 8):
        got = oracle.dual_grad_par(P, a, b, nthreads=nt)
        for x, y in zip(ref, got):
            assert np.array_equal(x, y)
    r1 = oracle.solve(P, max_iter=60)
    r2 = oracle.solve(P, max_iter=60, nthreads=4)
    assert np.array_equal(r1["trace"], r2["trace"]) and np.array_equal(r1["alpha"], r2["alpha"])


# --------------------------------------------------------------- barycentric mapping (Sec. 2.1)

def test_mapping_with_a_single_source_is_that_source():
    """n_src = 1: every plan column is b_j (the only feasible plan, reached at
    the optimum), so every target is mapped onto the one source point."""
    rng = np.random.default_rng(48)
    C = rng.uniform(0.1, 1.0, (1, 7))
    P = oracle.Problem(C, np.zeros(1, np.int32), 1, 0.4, 0.3)
    r = oracle.solve(P, max_iter=500, gtol=1e-13)
    X = rng.standard_normal((1, 3))
    Y = oracle.transport(P, r["alpha"], r["beta"], X)
    np.testing.assert_allclose(Y, np.repeat(X, 7, axis=0), rtol=1e-9, atol=1e-12)


def test_mapping_is_affine_and_a_barycentre_at_the_optimum():
    """y(X + v) - y(X) = v (sum_i T_ij) / b_j exactly (linear in X); at the
    optimum the column sums equal b (marginal satisfaction), so a shift of
    every source moves every target image by the same vector, and each y_j
    lies in the box spanned by the sources."""
    P = rand_problem(49, 30, 20, 3, gamma=0.3, mu=0.2)
    rng = np.random.default_rng(49)
    r = oracle.solve(P, max_iter=3000, gtol=1e-12)
    X = rng.standard_normal((P.ns, 4))
    v = rng.standard_normal(4)
    Y = oracle.transport(P, r["alpha"], r["beta"], X)
    Y2 = oracle.transport(P, r["alpha"], r["beta"], X + v)
    T = oracle.plan(P, r["alpha"], r["beta"])
    np.testing.assert_allclose(Y2 - Y, np.outer(T.sum(0) / P.b, v), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(T.sum(0), P.b, atol=1e-9)
    np.testing.assert_allclose(Y2 - Y, np.tile(v, (P.nt, 1)), atol=1e-6)
    assert np.all(Y >= X.min(0) - 1e-6) and np.all(Y <= X.max(0) + 1e-6)


# --------------------------------------------------------------- sanitizers

def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """Every oracle entry point on small problems (an empty label, a single
    source row, a single target) in a standalone C test program built with
    -fsanitize=address,undefined: no memory error, leak or undefined
    arithmetic, and the program's own invariants hold."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = os.path.join(HERE, os.pardir, "oracle")
    exe = str(tmp_path / "orc_sanitized")
    subprocess.check_call([gcc, "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe,
                           os.path.join(src, "sanitize_driver.c"), os.path.join(src, "otgs_oracle.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok") == 4, r.stdout
