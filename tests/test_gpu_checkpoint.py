"""Solver checkpoint and resume (ot_gs_solver_state_size / _save / _load and
ot_gs_solve with resume): a solve stopped at an iteration limit and resumed
- on the same handle, or from a saved state in a new handle built from the
same problems - gives the same objective trace, point and info, bit for bit,
as one uninterrupted solve; also across a re-centring, whose working cost
the restored state rebuilds from its reference.  Per-iteration statistics
and gradient-norm traces are checked against the handle's counters and the
solve's own gradient norm.  The state's size, the shape check and the
errors of the calls are exercised too."""
import numpy as np
import pytest

import synth
from tests import cases
from tests.test_gpu_dual_grad import _dev
from tests.test_gpu_solve import handle_for

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def traced(h, K, **kw):
    tr = torch.full((h.count * (K + 1),), float("nan"), dtype=torch.float64, device="cuda")
    a, b, info, rc = h.solve(obj_trace=tr, max_iter=K, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), info, tr.cpu().numpy().reshape(h.count, K + 1)


def _instance(n_src=900, n_groups=6):
    inst = synth.blobs(seed=21, n_src=n_src, n_tgt=700, d=8, n_groups=n_groups, gamma=0.1, mu=0.3)
    return cases.with_cost(inst)


@pytest.mark.parametrize("use_screen", [0, 1])
@pytest.mark.parametrize("via_bytes", [False, True])
def test_resume_equals_uninterrupted(use_screen, via_bytes):
    C32, P = _instance()
    K, M = 160, 70
    a_ref, b_ref, info_ref, tr_ref = traced(handle_for(C32, P), K, use_screen=use_screen)
    h = handle_for(C32, P)
    _, _, info_m, tr_m = traced(h, M, use_screen=use_screen)
    assert info_m[0]["iters"] == M
    if via_bytes:
        state = h.solver_state()
        h.close()
        h = handle_for(C32, P)
        h.load_solver_state(state)
    a, b, info, tr = traced(h, K, use_screen=use_screen, resume=1)
    np.testing.assert_array_equal(tr_m[0][:M + 1], tr_ref[0][:M + 1])
    # iterations M+1..K are written by the resumed call
    np.testing.assert_array_equal(tr[0][M + 1:], tr_ref[0][M + 1:])
    np.testing.assert_array_equal(a, a_ref)
    np.testing.assert_array_equal(b, b_ref)
    assert info[0] == info_ref[0]


def test_resume_in_a_batch_keeps_finished_instances():
    O = _O()
    insts = [synth.blobs(seed=50 + i, n_src=300 + 100 * i, n_tgt=250, d=8, n_groups=4, gamma=0.2, mu=0.3)
             for i in range(3)]
    Cs = [cases.with_cost(x) for x in insts]
    probs = [dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32), cost_scale=1.0,
                  cost_mode=O.OT_GS_COST_GIVEN) for C32, P in Cs]
    K, M = 120, 45
    a_ref, b_ref, info_ref, tr_ref = traced(O.Handle(probs), K, use_screen=1, gtol=1e-5)
    h = O.Handle(probs)
    traced(h, M, use_screen=1, gtol=1e-5)
    state = h.solver_state()
    h2 = O.Handle(probs)
    h2.load_solver_state(state)
    a, b, info, tr = traced(h2, K, use_screen=1, gtol=1e-5, resume=1)
    np.testing.assert_array_equal(a, a_ref)
    np.testing.assert_array_equal(b, b_ref)
    for k in range(3):
        assert info[k] == info_ref[k]
        np.testing.assert_array_equal(tr[k][M + 1:], tr_ref[k][M + 1:])


def test_resume_across_a_recentring():
    """The held-out instance whose solve needs re-centrings (4009 x 457):
    stopped late (after the first re-centring), saved, restored into a new
    handle and resumed, it ends where the uninterrupted solve does."""
    O = _O()
    inst = synth.instance_from_generator((6, 69), n_hi=4096)

    def handle():
        return O.Handle([dict(labels=_dev(inst["labels"]), n_groups=inst["n_groups"], gamma=inst["gamma"],
                              mu=inst["mu"], x_src=_dev(inst["xs"]), x_tgt=_dev(inst["xt"]),
                              cost_mode=O.OT_GS_COST_MATERIALIZE, cost_scale=0.0)])
    K = 8000
    a_ref, b_ref, info_ref, tr_ref = traced(handle(), K, use_screen=1)
    n = info_ref[0]["iters"]
    M = int(0.9 * n)
    h = handle()
    traced(h, M, use_screen=1)
    state = h.solver_state()
    h2 = handle()
    h2.load_solver_state(state)
    a, b, info, tr = traced(h2, K, use_screen=1, resume=1)
    np.testing.assert_array_equal(tr[0][M + 1:n + 1], tr_ref[0][M + 1:n + 1])
    np.testing.assert_array_equal(a, a_ref)
    np.testing.assert_array_equal(b, b_ref)
    assert info[0] == info_ref[0]


def test_state_errors():
    O = _O()
    C32, P = _instance()
    h = handle_for(C32, P)
    with pytest.raises(O.OTGSError) as e:
        h.solver_state()
    assert e.value.code == O.OT_GS_EINVAL
    with pytest.raises(O.OTGSError) as e:
        h.solve(max_iter=10, resume=1)
    assert e.value.code == O.OT_GS_EINVAL
    traced(h, 20, use_screen=1)
    state = h.solver_state()
    # another instance shape
    C2, P2 = _instance(n_src=901)
    h2 = handle_for(C2, P2)
    with pytest.raises(O.OTGSError) as e:
        h2.load_solver_state(state)
    assert e.value.code == O.OT_GS_EINVAL
    # truncated
    h3 = handle_for(C32, P)
    with pytest.raises(O.OTGSError) as e:
        h3.load_solver_state(state[:len(state) // 2])
    assert e.value.code == O.OT_GS_EINVAL
    # another history size
    h3.load_solver_state(state)
    with pytest.raises(O.OTGSError) as e:
        h3.solve(max_iter=30, resume=1, hist=5)
    assert e.value.code == O.OT_GS_EINVAL
    # an accelerated-ascent solve replaces the state
    h.solve(max_iter=5, solver=O.OT_GS_SOLVER_AGD)
    with pytest.raises(O.OTGSError) as e:
        h.solver_state()
    assert e.value.code == O.OT_GS_EINVAL


def test_statistics_and_gradient_traces():
    O = _O()
    C32, P = _instance()
    h = handle_for(C32, P)
    K = 80
    st = torch.zeros(((K + 1) * 8,), dtype=torch.int64, device="cuda")
    gn = torch.full((K + 1,), float("nan"), dtype=torch.float64, device="cuda")
    h.stats(reset=True)
    a, b, info, rc = h.solve(max_iter=K, use_screen=1, stats_trace=st, gnorm_trace=gn)
    torch.cuda.synchronize()
    total = h.stats()
    S = st.cpu().numpy().reshape(K + 1, 8)
    g = gn.cpu().numpy()
    it = info[0]["iters"]
    # counters never decrease, the last row is the handle's total (no
    # evaluation after the last accepted one in a solve that hit max_iter)
    assert np.all(np.diff(S[:it + 1], axis=0) >= 0)
    names = ["evals", "pairs_total", "pairs_in_N", "pairs_checked", "pairs_unskipped", "refreshes", "tiles_total",
             "tiles_computed"]
    if info[0]["status"] == O.OT_GS_NOT_CONVERGED:
        for c, nm in enumerate(names):
            assert S[it, c] == total[nm], nm
    assert S[it, 0] == info[0]["evals"]
    # the gradient norm at the last accepted point is the one the solve reports
    assert g[it] == info[0]["gnorm_inf"]
    assert np.all(np.isfinite(g[:it + 1]))
    # each iteration computed at most the tiles it covered
    d = np.diff(S[:it + 1], axis=0)
    assert np.all(d[:, 7] <= d[:, 6])


def test_resume_with_the_cost_on_the_fly():
    from tests.test_gpu_onthefly import int_instance, otf_handle
    inst = int_instance(42, [300, 40, 7, 200], 250, 20, gamma=0.2, mu=0.3)
    scale = 2.0 ** -9
    K, M = 150, 60
    a_ref, b_ref, info_ref, tr_ref = traced(otf_handle(inst, scale), K, use_screen=1)
    h = otf_handle(inst, scale)
    traced(h, M, use_screen=1)
    state = h.solver_state()
    h2 = otf_handle(inst, scale)
    h2.load_solver_state(state)
    a, b, info, tr = traced(h2, K, use_screen=1, resume=1)
    np.testing.assert_array_equal(tr[0][M + 1:], tr_ref[0][M + 1:])
    np.testing.assert_array_equal(a, a_ref)
    np.testing.assert_array_equal(b, b_ref)
    assert info[0] == info_ref[0]
