"""Barycentric mapping y_j = (1/b_j) sum_i T_ij x_i (the paper's n T^T X_S,
Sec. 2.1) on the device against the oracle's (the oracle's plan times the
features): ragged groups with an empty label and a split group, several
feature widths, a batch of instances with non-uniform b."""
import numpy as np
import pytest

import oracle
from tests import cases
from tests.test_gpu_dual_grad import _dev, make_handle, trajectory_points

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


U32 = 2.0 ** -24


def check(P, a32, b32, X, Y):
    a64, b64 = a32.astype(np.float64), b32.astype(np.float64)
    ref = oracle.transport(P, a64, b64, X.astype(np.float64))
    T = oracle.plan(P, a64, b64)
    # float32 entries of T: f = alpha + beta - c carries 2u(|alpha| + |beta|
    # + c), and a block's map f -> t is (1/gamma)-Lipschitz, so an entry of
    # an active (or nearly active) block moves by at most (1 + sqrt(g)) e /
    # gamma; then the float32 products and sums add a few u of sum T |x|
    Z, _, _ = oracle.group_norms(P, a64, b64)
    g = P.group_sizes().astype(np.float64)
    e = 2 * U32 * (np.abs(a64)[:, None] + np.abs(b64)[None, :] + P.C)
    near = Z[P.labels] > (P.mu * P.gamma - np.sqrt(g)[P.labels][:, None] * e.max())
    dT = near * e * (1 + np.sqrt(g[P.labels]))[:, None] / P.gamma
    xm = np.abs(X).max(1)
    tol = 1e-6 + ((dT.T @ xm) + 8 * U32 * (np.abs(T).T @ xm)) / P.b
    tol = tol[:, None]
    assert np.all(np.abs(Y - ref) <= tol), float(np.max(np.abs(Y - ref) / tol))


@pytest.mark.parametrize("seed,sizes,nt,d", [(100, [40, 0, 300, 17], 211, 5), (101, [2300, 90], 97, 70),
                                             (102, [64] * 6, 64, 256)])
def test_transport_matches_oracle(seed, sizes, nt, d):
    inst = cases.ragged(seed, sum(sizes), nt, sizes)
    C32, P = cases.with_cost(inst)
    h = make_handle(C32, P)
    X = np.random.default_rng(seed).standard_normal((P.ns, d)).astype(np.float32)
    for a32, b32 in trajectory_points(P, [5, 60]):
        Y = h.transport(_dev(a32), _dev(b32), _dev(X))
        torch.cuda.synchronize()
        check(P, a32, b32, X, Y.cpu().numpy())


def test_transport_batched_nonuniform_b():
    O = _O()
    insts = [cases.ragged(103, 120, 70, [50, 70]), cases.ragged(104, 90, 150, [30, 0, 60])]
    probs, Ps, pts, Xs = [], [], [], []
    rng = np.random.default_rng(103)
    for inst in insts:
        C32, P0 = cases.with_cost(inst)
        b = rng.uniform(0.3, 1.7, P0.nt)
        b32 = (b / b.sum()).astype(np.float32)
        P = oracle.Problem(C32.astype(np.float64), inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"],
                           b=b32.astype(np.float64))
        probs.append(dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                          cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN, b=_dev(b32)))
        Ps.append(P)
        pts.append(trajectory_points(P, [30])[0])
        Xs.append(rng.standard_normal((P.ns, 9)).astype(np.float32))
    h = O.Handle(probs)
    Y = h.transport(_dev(np.concatenate([p[0] for p in pts])), _dev(np.concatenate([p[1] for p in pts])),
                    _dev(np.concatenate(Xs))).cpu().numpy()
    off = 0
    for P, (a32, b32), X in zip(Ps, pts, Xs):
        check(P, a32, b32, X, Y[off:off + P.nt])
        off += P.nt
