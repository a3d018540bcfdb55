"""The C ABI's checks and inspection calls on the device.

- the snapshot and the set N the device builds (Algorithm 1: N from the
  lower bound of Eq. 7 against the previous snapshot, Eq. 8), read back with
  ot_gs_screen_state and compared with the oracle's group norms (Defs. 1-2)
  and its extraction, pair by pair away from the threshold;
- OT_GS_CHECK / ot_gs_check: NaN or Inf duals reported as OT_GS_ENUMERIC;
- OT_GS_VERIFY and the solve's verify option: screened evaluations repeated
  densely must agree bit for bit (Lemma 2);
- marginals validated at create (finite, nonnegative, equal mass).
"""
import numpy as np
import pytest

import oracle
import synth
from tests import cases
from tests.test_gpu_dual_grad import _dev, gpu_grad, make_handle, trajectory_points

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def _instance():
    inst = synth.blobs(seed=11, n_src=1200, n_tgt=900, d=8, n_groups=6, gamma=0.1, mu=0.5)
    C32, P = cases.with_cost(inst)
    return C32, P


def norm_tol(P, a32, b32, K):
    """Float32 error of a group norm computed by the device: each f carries
    at most e = 2u(|alpha| + |beta| + c) of rounding (so the norm moves by
    at most sqrt(g) e), and the sum of g squares then the square root add
    (g + 2) u relative."""
    g = P.group_sizes().astype(np.float64)[:, None]
    e = 2 * U32 * (np.abs(a32).max() + np.abs(b32).max() + P.C.max())
    return 1e-7 + np.sqrt(g) * e + (g + 2) * U32 * K


@pytest.mark.parametrize("which", ["blobs", "small groups"])
def test_snapshot_norms_and_set_N_match_the_oracle(which):
    """Blobs (groups of 200 rows, few blocks single-signed, N small) and
    groups of one or two rows (most active blocks single-signed, so Eq. 7 is
    nearly tight at a nearby point and N holds most of them)."""
    O = _O()
    if which == "blobs":
        C32, P = _instance()
        it = 60
    else:
        C32, P = cases.with_cost(cases.ragged(67, 80, 200, [1] * 40 + [2] * 20, gamma=0.2, mu=0.2))
        it = 80
    h = make_handle(C32, P)
    ((a0, b0),) = trajectory_points(P, [it])
    # the second point lies close to the first, so that Eq. 7 can put
    # blocks in N (a full L-BFGS step apart it puts none)
    rng = np.random.default_rng(65)
    a1 = (a0 + 1e-5 * rng.standard_normal(P.ns)).astype(np.float32)
    b1 = (b0 + 1e-5 * rng.standard_normal(P.nt)).astype(np.float32)
    # first snapshot at the 60-iteration point
    gpu_grad(h, a0, b0, mode=O.OT_GS_SNAPSHOT)
    as_, bs_, z, o, n = (x.cpu().numpy() for x in h.screen_state([P.L]))
    np.testing.assert_array_equal(as_, a0)
    np.testing.assert_array_equal(bs_, b0)
    Z, Od, K = oracle.group_norms(P, a0.astype(np.float64), b0.astype(np.float64))
    tol = norm_tol(P, a0, b0, K)
    z, o = z.reshape(P.L, P.nt), o.reshape(P.L, P.nt)
    assert np.all(np.abs(z - Z) <= tol), float(np.max(np.abs(z - Z) / tol))
    assert np.all(np.abs(o - Od) <= tol), float(np.max(np.abs(o - Od) / tol))
    # the first extraction used the zero snapshot (f = -C <= 0): N is empty
    assert not n.any()
    # a refresh at the nearby point: N from Eq. 7 against the 60-iteration snapshot
    gpu_grad(h, a1, b1, mode=O.OT_GS_SNAPSHOT)
    as2, _, z2, _, n2 = (x.cpu().numpy() for x in h.screen_state([P.L]))
    np.testing.assert_array_equal(as2, a1)
    N = n2.reshape(P.L, P.nt).astype(bool)
    S = oracle.ScreenState(P, a0.astype(np.float64), b0.astype(np.float64))
    S.extract(a1.astype(np.float64), b1.astype(np.float64))
    Zl = oracle.lower_bound(P, a1.astype(np.float64), b1.astype(np.float64), S.alpha_s, S.beta_s, S.Ks, S.Os)
    thr = P.mu * P.gamma
    # pairs whose lower bound is clear of the threshold by more than the
    # float32 error of the snapshot norms (Eq. 7 is 1-Lipschitz in k~, o~)
    clear = np.abs(Zl - thr) > 4 * tol
    assert clear.mean() > 0.9
    np.testing.assert_array_equal(N[clear], S.inN.astype(bool)[clear])
    if which != "blobs":
        Z1, _, _ = oracle.group_norms(P, a1.astype(np.float64), b1.astype(np.float64))
        assert N.sum() > 0.5 * (Z1 > thr).sum() > 0
    # Lemma 5 on the device: every block in N is active at the point
    Z1, _, _ = oracle.group_norms(P, a1.astype(np.float64), b1.astype(np.float64))
    assert np.all(Z1[N] > thr)
    # an evaluation in SCREENED mode leaves the snapshot and N as they were
    gpu_grad(h, a1, b1, mode=O.OT_GS_SCREENED)
    _, _, z3, _, n3 = (x.cpu().numpy() for x in h.screen_state([P.L]))
    np.testing.assert_array_equal(z3, z2)
    np.testing.assert_array_equal(n3, n2)


def test_screen_state_layout_with_empty_labels_and_batches():
    """Caller layout: per instance [n_groups x n_tgt], label-major, caller's
    target order; empty labels read zero."""
    O = _O()
    insts = [cases.ragged(60, 50, 40, [20, 0, 30]), cases.ragged(61, 33, 70, [0, 33])]
    probs, Ps = [], []
    for inst in insts:
        C32, P = cases.with_cost(inst)
        probs.append(dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                          cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN))
        Ps.append(P)
    h = O.Handle(probs)
    pts = [cases.dual_point(P, 62 + i) for i, P in enumerate(Ps)]
    al = np.concatenate([p[0] for p in pts])
    be = np.concatenate([p[1] for p in pts])
    gpu_grad(h, al, be, mode=O.OT_GS_SNAPSHOT)
    as_, bs_, z, o, _ = (x.cpu().numpy() for x in h.screen_state([P.L for P in Ps]))
    np.testing.assert_array_equal(as_, al)
    np.testing.assert_array_equal(bs_, be)
    off = 0
    for P, (a32, b32) in zip(Ps, pts):
        Z, Od, K = oracle.group_norms(P, a32.astype(np.float64), b32.astype(np.float64))
        zz = z[off:off + P.L * P.nt].reshape(P.L, P.nt)
        empty = P.group_sizes() == 0
        assert np.all(zz[empty] == 0)
        assert np.all(np.abs(zz - Z) <= norm_tol(P, a32, b32, K))
        off += P.L * P.nt


def test_checked_calls_report_nonfinite_duals():
    O = _O()
    C32, P = cases.with_cost(cases.ragged(63, 80, 50, [30, 50]))
    h = make_handle(C32, P)
    a32, b32 = cases.dual_point(P, 63)
    bad = a32.copy()
    bad[7] = np.nan
    al, be = _dev(bad), _dev(b32)
    ga, gb = torch.empty_like(al), torch.empty_like(be)
    obj = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(O.OTGSError) as e:
        h.dual_grad(al, be, ga, gb, obj, mode=O.OT_GS_DENSE | O.OT_GS_CHECK)
    assert e.value.code == O.OT_GS_ENUMERIC
    # asynchronous call: accepted, reported by the next check, then cleared
    b2 = b32.copy()
    b2[3] = np.inf
    h.dual_grad(_dev(a32), _dev(b2), ga, gb, obj, mode=O.OT_GS_DENSE)
    with pytest.raises(O.OTGSError) as e:
        h.check()
    assert e.value.code == O.OT_GS_ENUMERIC
    h.check()
    # finite inputs: a checked call succeeds and equals the unchecked one
    d1 = gpu_grad(h, a32, b32, mode=O.OT_GS_SCREENED | O.OT_GS_CHECK)
    d2 = gpu_grad(h, a32, b32, mode=O.OT_GS_SCREENED)
    for x, y in zip(d1, d2):
        np.testing.assert_array_equal(x, y)
    # a solve from a start point with a NaN
    with pytest.raises(O.OTGSError) as e:
        h.solve(_dev(bad), _dev(b32), init_user=1, max_iter=5)
    assert e.value.code == O.OT_GS_ENUMERIC
    h.solve(_dev(a32), _dev(b32), init_user=1, max_iter=5)


def test_verified_evaluations_and_solve():
    O = _O()
    C32, P = _instance()
    h = make_handle(C32, P)
    (a0, b0), (a1, b1) = trajectory_points(P, [40, 45])
    gpu_grad(h, a0, b0, mode=O.OT_GS_SNAPSHOT | O.OT_GS_VERIFY)
    h.stats(reset=True)
    v = gpu_grad(h, a1, b1, mode=O.OT_GS_SCREENED | O.OT_GS_VERIFY)
    st = h.stats(reset=True)
    s = gpu_grad(h, a1, b1, mode=O.OT_GS_SCREENED)
    for x, y in zip(v, s):
        np.testing.assert_array_equal(x, y)
    # the dense repetition is not counted
    assert st["evals"] == 1 and st["tiles_computed"] < st["tiles_total"]
    K = 150
    runs = []
    for ver in (0, 1):
        tr = torch.full((K + 1,), float("nan"), dtype=torch.float64, device="cuda")
        a, b, info, rc = h.solve(max_iter=K, use_screen=1, verify=ver, obj_trace=tr)
        torch.cuda.synchronize()
        runs.append((a.cpu().numpy(), tr.cpu().numpy(), info[0]))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])


def test_marginals_are_validated_at_create():
    O = _O()
    C32, P = cases.with_cost(cases.ragged(64, 40, 30, [15, 25]))
    a = np.full(P.ns, 1.0 / P.ns, np.float32)
    b = np.full(P.nt, 1.0 / P.nt, np.float32)
    b_heavy = b * np.float32(1.001)
    for aa, bb, code in [(a, b_heavy, O.OT_GS_EINVAL), (-a, b, O.OT_GS_EINVAL)]:
        with pytest.raises(O.OTGSError) as e:
            make_handle(C32, P, a=_dev(aa), b=_dev(bb))
        assert e.value.code == code
    an = a.copy()
    an[0] = np.nan
    with pytest.raises(O.OTGSError) as e:
        make_handle(C32, P, a=_dev(an), b=_dev(b))
    assert e.value.code == O.OT_GS_ENUMERIC
    make_handle(C32, P, a=_dev(a), b=_dev(b))
