"""Edge cases of the HIP path, through the C ABI.

Empty and out-of-range inputs are rejected when the handle is created,
before any device work.  The degenerate shapes of the method match the FP64
oracle: one source row, one target column, every group a single row, the
widest label range (16384 labels, most of them unused), a point where every
(group, target) block is zero (T = 0, so grad = marginals and D = a.alpha +
b.beta) and one where every block is active."""
import numpy as np
import pytest

import oracle
from tests import cases
from tests.test_gpu_dual_grad import _dev, _otgs, check_parity, gpu_grad, make_handle, trajectory_points

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

MAX_LABELS = 16384   # label range limit of ot_gs_create


def _create(labels, C, **kw):
    O = _otgs()
    p = dict(labels=_dev(labels), n_groups=2, gamma=0.1, mu=0.1, cost=_dev(C), cost_scale=1.0,
             cost_mode=O.OT_GS_COST_GIVEN)
    p.update(kw)
    return O.Handle([p])


def test_empty_and_out_of_range_inputs_are_rejected():
    O = _otgs()
    C = np.ones((4, 3), np.float32)
    lab = np.array([0, 1, 0, 1], np.int32)
    cases_ = [
        (np.zeros(0, np.int32), np.ones((0, 3), np.float32), {}),      # no source row
        (lab, np.ones((4, 0), np.float32), {}),                         # no target column
        (lab, C, dict(n_groups=0)),
        (lab, C, dict(n_groups=MAX_LABELS + 1)),
        (lab, C, dict(mu=-1e-3)),
        (lab, C, dict(gamma=float("inf"))),
        (lab, C, dict(gamma=-1.0)),
    ]
    for labels, cost, kw in cases_:
        with pytest.raises(O.OTGSError) as e:
            _create(labels, cost, **kw)
        assert e.value.code == O.OT_GS_EINVAL, kw
    # a negative label and a label past n_groups
    for bad in (-1, 2):
        lb = lab.copy()
        lb[1] = bad
        with pytest.raises(O.OTGSError) as e:
            _create(lb, C)
        assert e.value.code == O.OT_GS_EINVAL
    h = _create(lab, C)
    a, b = np.zeros(4, np.float32), np.zeros(3, np.float32)
    with pytest.raises(O.OTGSError) as e:
        gpu_grad(h, a, b, mode=7)
    assert e.value.code == O.OT_GS_EINVAL


def _scattered_labels(seed, ns, L_used, L):
    rng = np.random.default_rng(seed)
    used = np.sort(rng.choice(L, L_used, replace=False))
    return used[rng.integers(0, L_used, ns)].astype(np.int32)


@pytest.mark.parametrize("name", ["one_source_row", "one_target_column", "singleton_groups",
                                  "widest_label_range"])
def test_degenerate_shapes_match_oracle(name):
    if name == "one_source_row":
        inst = cases.ragged(81, 1, 50, [1])
    elif name == "one_target_column":
        inst = cases.ragged(82, 10, 1, [7, 3])
    elif name == "singleton_groups":
        inst = cases.ragged(83, 300, 70, [1] * 300)
    else:
        inst = cases.ragged(84, 500, 90, [500])
        inst["labels"] = _scattered_labels(85, 500, 40, MAX_LABELS)
        inst["n_groups"] = MAX_LABELS
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    for a32, b32 in trajectory_points(P, [0, 3, 20]):
        ga, gb, D = gpu_grad(h, a32, b32)
        check_parity(P, a32, b32, ga, gb, D[0])
    a32, b32 = cases.dual_point(P, 86)
    ga, gb, D = gpu_grad(h, a32, b32)
    check_parity(P, a32, b32, ga, gb, D[0], traj=False)


def test_every_block_zero_and_every_block_active():
    O = _otgs()
    inst = cases.ragged(87, 700, 150, [300, 0, 250, 150])
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    # f = alpha + beta - c < 0 everywhere: every block is zero, T = 0
    a32 = np.full(P.ns, -1.0, np.float32)
    b32 = np.full(P.nt, -1.0, np.float32)
    ga, gb, D = gpu_grad(h, a32, b32)
    np.testing.assert_array_equal(ga, np.full(P.ns, 1.0 / P.ns, np.float32))
    np.testing.assert_array_equal(gb, np.full(P.nt, 1.0 / P.nt, np.float32))
    assert abs(D[0] - (-2.0)) <= 1e-12
    T = torch.empty((P.ns, P.nt), dtype=torch.float32, device="cuda")
    h.plan(_dev(a32), _dev(b32), T)
    assert not torch.any(T != 0).item()
    # f > 0 everywhere and far above the threshold: every block is active
    a32 = np.full(P.ns, 1.5, np.float32)
    b32 = np.full(P.nt, 0.5, np.float32)
    Z, _, _ = oracle.group_norms(P, a32.astype(np.float64), b32.astype(np.float64))
    sizes = P.group_sizes()
    assert np.all(Z[sizes > 0] > P.mu * P.gamma)
    ga, gb, D = gpu_grad(h, a32, b32)
    check_parity(P, a32, b32, ga, gb, D[0], traj=False)
    # screened at both points equals dense
    for a_, b_ in ((np.full(P.ns, -1.0, np.float32), np.full(P.nt, -1.0, np.float32)), (a32, b32)):
        gpu_grad(h, a_, b_, mode=O.OT_GS_SNAPSHOT)
        d = gpu_grad(h, a_, b_, mode=O.OT_GS_DENSE)
        s = gpu_grad(h, a_, b_, mode=O.OT_GS_SCREENED)
        for x, y in zip(d, s):
            np.testing.assert_array_equal(x, y)
