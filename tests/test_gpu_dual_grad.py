"""Parity of the HIP dual-gradient path with the FP64 oracle, through the C ABI.

Bar: 1e-6 absolute on gradients and 1e-5 relative on the objective at points
of a real L-BFGS trajectory (computed by the oracle); at arbitrary points
the gradient error is also bounded relative to the plan mass of the row or
column (float32 sums of O(1) entries cannot meet 1e-6 there).  Screened and
dense evaluations must agree bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from tests import cases

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _otgs():
    import paper_2303_07597_amd.otgs as O
    return O


def _dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def make_handle(C32, P, **extra):
    O = _otgs()
    prob = dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu,
                cost=_dev(C32), cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN)
    prob.update(extra)
    return O.Handle([prob])


def gpu_grad(h, a32, b32, mode=0):
    al, be = _dev(a32), _dev(b32)
    ga = torch.empty_like(al)
    gb = torch.empty_like(be)
    obj = torch.empty(h.count, dtype=torch.float64, device="cuda")
    h.dual_grad(al, be, ga, gb, obj, mode=mode)
    torch.cuda.synchronize()
    return ga.cpu().numpy(), gb.cpu().numpy(), obj.cpu().numpy()


def check_parity(P, a32, b32, ga, gb, D, traj=True):
    oa, ob, oD, T = oracle.dual_grad(P, a32.astype(np.float64), b32.astype(np.float64), want_plan=True)
    assert abs(D - oD) <= 1e-5 * max(1.0, abs(oD)), (D, oD)
    if traj:
        np.testing.assert_allclose(ga, oa, rtol=0, atol=1e-6)
        np.testing.assert_allclose(gb, ob, rtol=0, atol=1e-6)
    else:
        ra = 1e-6 + 4e-6 * (np.abs(T).sum(1) + np.abs(P.a))
        rb = 1e-6 + 4e-6 * (np.abs(T).sum(0) + np.abs(P.b))
        assert np.all(np.abs(ga - oa) <= ra), np.max(np.abs(ga - oa) / ra)
        assert np.all(np.abs(gb - ob) <= rb), np.max(np.abs(gb - ob) / rb)


def trajectory_points(P, iters):
    pts = []
    for k in iters:
        r = oracle.solve(P, max_iter=k) if k > 0 else dict(alpha=np.zeros(P.ns), beta=np.zeros(P.nt))
        pts.append((r["alpha"].astype(np.float32), r["beta"].astype(np.float32)))
    return pts


def test_dense_matches_oracle_on_trajectory_small():
    inst = synth.gaussian4_2d()
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    for a32, b32 in trajectory_points(P, [0, 1, 3, 10, 40, 200]):
        ga, gb, D = gpu_grad(h, a32, b32)
        check_parity(P, a32, b32, ga, gb, D[0])


@pytest.mark.parametrize("seed,sizes,nt", [
    (1, [1, 17, 0, 600, 64, 3], 129),      # empty label, singleton, a 600-row group, ragged columns
    (2, [16, 16, 32, 31, 33], 64),         # sizes on and around the 16-row class edges
    (3, [513, 1100, 7], 200),              # a group in the 1024-2048 row buckets
    (6, [2100, 4500, 30, 1800], 70),       # split groups (3 and 5 chunks), a 1800-row whole group
    (4, [5], 1),                           # one group, one column
    (5, [2, 1], 70),
])
def test_dense_matches_oracle_ragged(seed, sizes, nt):
    inst = cases.ragged(seed, sum(sizes), nt, sizes)
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    for k in range(3):
        a32, b32 = cases.dual_point(P, seed * 10 + k)
        ga, gb, D = gpu_grad(h, a32, b32)
        check_parity(P, a32, b32, ga, gb, D[0], traj=False)
    for a32, b32 in trajectory_points(P, [2, 25]):
        ga, gb, D = gpu_grad(h, a32, b32)
        check_parity(P, a32, b32, ga, gb, D[0])


def test_mu_zero_and_large_gamma():
    for gamma, mu in [(0.25, 0.0), (50.0, 2.0)]:
        inst = cases.ragged(7, 90, 77, [30, 40, 20], gamma=gamma, mu=mu)
        C32, P = cases.with_cost(inst)
        h = make_handle(C32, P)
        a32, b32 = cases.dual_point(P, 7, spread=0.5)
        ga, gb, D = gpu_grad(h, a32, b32)
        check_parity(P, a32, b32, ga, gb, D[0], traj=False)


def test_batch_is_bitwise_equal_to_single_instances():
    O = _otgs()
    insts = [cases.ragged(20 + i, n, m, s) for i, (n, m, s) in
             enumerate([(40, 70, [10, 30]), (600, 33, [580, 20]), (9, 130, [3, 3, 3])])]
    probs, singles, pts = [], [], []
    for i, inst in enumerate(insts):
        C32, P = cases.with_cost(inst)
        pr = dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                  cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN)
        probs.append(pr)
        singles.append((O.Handle([pr]), P))
        pts.append(cases.dual_point(P, 30 + i))
    hb = O.Handle(probs)
    ga_b, gb_b, D_b = gpu_grad(hb, np.concatenate([p[0] for p in pts]), np.concatenate([p[1] for p in pts]))
    oa = ob = 0
    for i, ((h, P), (a32, b32)) in enumerate(zip(singles, pts)):
        ga, gb, D = gpu_grad(h, a32, b32)
        np.testing.assert_array_equal(ga, ga_b[oa:oa + P.ns])
        np.testing.assert_array_equal(gb, gb_b[ob:ob + P.nt])
        assert D[0] == D_b[i]
        oa += P.ns
        ob += P.nt


# (2600, 2): 1300-row whole groups; (4400, 2): split groups (3 chunks)
@pytest.mark.parametrize("n_src,n_groups", [(1200, 6), (2600, 2), (4400, 2)])
def test_screened_is_bitwise_equal_to_dense(n_src, n_groups):
    """Theorem 2 on the device: after a snapshot, screened evaluations at
    nearby points reproduce the dense ones exactly, and skip tiles.  The
    snapshot evaluation itself (first call on a fresh handle) matches the
    oracle."""
    O = _otgs()
    inst = synth.blobs(seed=11, n_src=n_src, n_tgt=900, d=8, n_groups=n_groups, gamma=0.1, mu=0.5)
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    r = oracle.solve(P, max_iter=60)
    base_a, base_b = r["alpha"].astype(np.float32), r["beta"].astype(np.float32)
    snap = gpu_grad(h, base_a, base_b, mode=O.OT_GS_SNAPSHOT)
    check_parity(P, base_a, base_b, *snap[:2], snap[2][0])
    h.stats(reset=True)
    rng = np.random.default_rng(0)
    for k in range(6):
        eps = [0.0, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2][k]
        a32 = (base_a + eps * rng.standard_normal(P.ns)).astype(np.float32)
        b32 = (base_b + eps * rng.standard_normal(P.nt)).astype(np.float32)
        d = gpu_grad(h, a32, b32, mode=O.OT_GS_DENSE)
        s = gpu_grad(h, a32, b32, mode=O.OT_GS_SCREENED)
        for x, y in zip(d, s):
            np.testing.assert_array_equal(x, y)
        check_parity(P, a32, b32, *s[:2], s[2][0], traj=False)
    st = h.stats()
    assert st["tiles_computed"] < st["tiles_total"]
    assert st["pairs_checked"] > 0


def test_modes_after_an_evaluation_elsewhere():
    """Each mode recomputes every partial it uses: after an evaluation at
    another point, SNAPSHOT, SCREENED and DENSE at a new point agree with the
    oracle there (split groups included)."""
    O = _otgs()
    inst = cases.ragged(41, 3700, 150, [2300, 1100, 300])
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    pts = trajectory_points(P, [5, 15, 16])
    gpu_grad(h, *pts[0], mode=O.OT_GS_DENSE)
    for mode, (a32, b32) in ((O.OT_GS_SNAPSHOT, pts[1]), (O.OT_GS_SCREENED, pts[2]), (O.OT_GS_DENSE, pts[1])):
        ga, gb, D = gpu_grad(h, a32, b32, mode=mode)
        check_parity(P, a32, b32, ga, gb, D[0])


def test_plan_matches_oracle():
    inst = cases.ragged(40, 150, 90, [50, 0, 70, 30])
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    r = oracle.solve(P, max_iter=30)
    a32, b32 = r["alpha"].astype(np.float32), r["beta"].astype(np.float32)
    T = torch.empty((P.ns, P.nt), dtype=torch.float32, device="cuda")
    h.plan(_dev(a32), _dev(b32), T)
    Tref = oracle.plan(P, a32.astype(np.float64), b32.astype(np.float64))
    # entries carry the float32 rounding of f = alpha + beta - c (|alpha|,
    # |beta| ~ 1), i.e. an absolute error of a few 1e-8 / gamma; far below
    # the 1e-6 gradient bar (grad = marginal - row or column sums of T)
    np.testing.assert_allclose(T.cpu().numpy(), Tref, rtol=2e-5, atol=1e-7)
    assert np.array_equal(T.cpu().numpy() > 0, Tref > 0)


def csr_blocks(row_ptr, col, val, ns, nt):
    """Dense per-instance blocks from the CSR plan (rows stacked, local
    columns), checking its structure on the way."""
    rp, c, v = row_ptr.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == c.size == v.size
    out, r0 = [], 0
    for n, m in zip(ns, nt):
        T = np.zeros((n, m), np.float32)
        for i in range(n):
            cols = c[rp[r0 + i]:rp[r0 + i + 1]]
            assert np.all((cols >= 0) & (cols < m)) and np.unique(cols).size == cols.size
            T[i, cols] = v[rp[r0 + i]:rp[r0 + i + 1]]
        assert np.all(v[rp[r0]:rp[r0 + n]] > 0)
        out.append(T)
        r0 += n
    return out


@pytest.mark.parametrize("seed,sizes,nt", [(40, [50, 0, 70, 30], 90), (42, [2300, 300, 5], 130)])
def test_plan_csr_equals_dense_plan(seed, sizes, nt):
    """The sparse plan holds exactly the nonzero entries of the dense plan,
    bit for bit (an empty label, a split group of 2300 rows, a ragged column
    tail), and matches the oracle's plan."""
    inst = cases.ragged(seed, sum(sizes), nt, sizes)
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    r = oracle.solve(P, max_iter=30)
    a32, b32 = r["alpha"].astype(np.float32), r["beta"].astype(np.float32)
    T = torch.empty((P.ns, P.nt), dtype=torch.float32, device="cuda")
    h.plan(_dev(a32), _dev(b32), T)
    rp, col, val = h.plan_csr(_dev(a32), _dev(b32))
    torch.cuda.synchronize()
    Td = T.cpu().numpy()
    (Ts,) = csr_blocks(rp, col, val, [P.ns], [P.nt])
    np.testing.assert_array_equal(Ts, Td)
    assert col.numel() == int(np.count_nonzero(Td))
    Tref = oracle.plan(P, a32.astype(np.float64), b32.astype(np.float64))
    np.testing.assert_allclose(Ts, Tref, rtol=2e-5, atol=1e-7)
    # a fill at another point than the count is refused (nothing written
    # outside the caller's arrays)
    import ctypes as ct
    O = _otgs()
    nnz = ct.c_longlong()
    rp2 = torch.empty(P.ns + 1, dtype=torch.int64, device="cuda")
    al, be = _dev(a32), _dev(b32)
    assert O.lib().ot_gs_plan_csr(h.h, al.data_ptr(), be.data_ptr(), rp2.data_ptr(), None, None,
                                  ct.byref(nnz), None) == 0
    c2 = torch.full((max(nnz.value, 1) + 64,), -7, dtype=torch.int32, device="cuda")
    v2 = torch.full((max(nnz.value, 1) + 64,), -7.0, dtype=torch.float32, device="cuda")
    al2 = _dev((a32 + 0.05).astype(np.float32))
    rc = O.lib().ot_gs_plan_csr(h.h, al2.data_ptr(), be.data_ptr(), rp2.data_ptr(), c2.data_ptr(),
                                v2.data_ptr(), None, None)
    assert rc == O.OT_GS_EINVAL
    assert torch.all(c2[nnz.value:] == -7) and torch.all(v2[nnz.value:] == -7.0)


def test_plan_csr_batched():
    O = _otgs()
    insts = [cases.ragged(70 + i, n, m, s) for i, (n, m, s) in
             enumerate([(40, 70, [10, 30]), (600, 33, [580, 20]), (9, 130, [3, 3, 3])])]
    probs, Ps, pts = [], [], []
    for i, inst in enumerate(insts):
        C32, P = cases.with_cost(inst)
        probs.append(dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                          cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN))
        Ps.append(P)
        pts.append(cases.dual_point(P, 80 + i))
    h = O.Handle(probs)
    al = _dev(np.concatenate([p[0] for p in pts]))
    be = _dev(np.concatenate([p[1] for p in pts]))
    T = torch.empty(sum(P.ns * P.nt for P in Ps), dtype=torch.float32, device="cuda")
    h.plan(al, be, T)
    rp, col, val = h.plan_csr(al, be)
    torch.cuda.synchronize()
    blocks = csr_blocks(rp, col, val, [P.ns for P in Ps], [P.nt for P in Ps])
    Tn, off = T.cpu().numpy(), 0
    for P, B in zip(Ps, blocks):
        np.testing.assert_array_equal(B, Tn[off:off + P.ns * P.nt].reshape(P.ns, P.nt))
        off += P.ns * P.nt


def test_argument_errors():
    O = _otgs()
    inst = cases.ragged(50, 20, 10, [10, 10])
    C32, P = cases.with_cost(inst)
    bad = P.labels.copy()
    bad[3] = 7
    with pytest.raises(O.OTGSError) as e:
        O.Handle([dict(labels=_dev(bad), n_groups=2, gamma=0.1, mu=0.1, cost=_dev(C32), cost_scale=1.0)])
    assert e.value.code == O.OT_GS_EINVAL
    Cn = C32.copy()
    Cn[2, 2] = np.nan
    with pytest.raises(O.OTGSError) as e:
        O.Handle([dict(labels=_dev(P.labels), n_groups=2, gamma=0.1, mu=0.1, cost=_dev(Cn), cost_scale=1.0)])
    assert e.value.code == O.OT_GS_ENUMERIC
    with pytest.raises(O.OTGSError) as e:
        O.Handle([dict(labels=_dev(P.labels), n_groups=2, gamma=0.0, mu=0.1, cost=_dev(C32), cost_scale=1.0)])
    assert e.value.code == O.OT_GS_EINVAL


def test_prepared_call_equals_dual_grad():
    O = _otgs()
    inst = synth.gaussian4_2d()
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    a32, b32 = cases.dual_point(P, 3)
    ga, gb, D = gpu_grad(h, a32, b32)
    al, be = _dev(a32), _dev(b32)
    ga2, gb2 = torch.empty_like(al), torch.empty_like(be)
    obj = torch.empty(1, dtype=torch.float64, device="cuda")
    call = h.prepare_dual_grad(al, be, ga2, gb2, obj, mode=O.OT_GS_DENSE)
    for _ in range(3):
        call()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ga, ga2.cpu().numpy())
    np.testing.assert_array_equal(gb, gb2.cpu().numpy())
    assert D[0] == obj.item()
