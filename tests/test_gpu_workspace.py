"""Handles in a caller workspace (ot_gs_workspace_size, ot_gs_create_ws):
every call gives the same bits as on a handle that allocates for itself,
for a materialised batch and an on-the-fly instance; a workspace of half
the size is refused."""
import numpy as np
import pytest

import oracle
from tests import cases
from tests.test_gpu_dual_grad import _dev

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def outputs(h, al, be, x_src):
    O = _O()
    ga, gb = torch.empty_like(al), torch.empty_like(be)
    obj = torch.empty(h.count, dtype=torch.float64, device="cuda")
    res = []
    for mode in (O.OT_GS_SNAPSHOT, O.OT_GS_SCREENED, O.OT_GS_DENSE):
        h.dual_grad(al, be, ga, gb, obj, mode=mode)
        res += [ga.clone(), gb.clone(), obj.clone()]
    a, b, info, _ = h.solve(max_iter=150, use_screen=1)
    res += [a, b, torch.tensor([x["obj"] for x in info])]
    res += list(h.plan_csr(al, be))
    if x_src is not None:
        res.append(h.transport(al, be, x_src))
    torch.cuda.synchronize()
    return [r.cpu() for r in res]


@pytest.mark.parametrize("kind", ["materialized batch", "on the fly"])
def test_workspace_handle_equals_allocating_handle(kind):
    O = _O()
    probs, x_src = [], None
    if kind == "materialized batch":
        for i, (n, m, s) in enumerate([(300, 200, [100, 0, 200]), (2300, 90, [2250, 50])]):
            inst = cases.ragged(110 + i, n, m, s)
            probs.append(dict(labels=_dev(inst["labels"]), n_groups=inst["n_groups"], gamma=inst["gamma"],
                              mu=inst["mu"], x_src=_dev(inst["xs"]), x_tgt=_dev(inst["xt"]),
                              cost_mode=O.OT_GS_COST_MATERIALIZE, cost_scale=0.0))
        x_src = torch.cat([p["x_src"] for p in probs])
    else:
        r = np.random.default_rng(112)
        labels = r.integers(0, 3, 1500).astype(np.int32)
        probs.append(dict(labels=_dev(labels), n_groups=3, gamma=0.3, mu=0.2,
                          x_src=_dev(r.integers(-3, 4, (1500, 24)).astype(np.float32)),
                          x_tgt=_dev(r.integers(-3, 4, (700, 24)).astype(np.float32)),
                          cost_mode=O.OT_GS_COST_ONTHEFLY, cost_scale=2.0 ** -9))
    nb = O.workspace_size(probs, max_hist=10)
    assert nb > 0
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    hw = O.Handle(probs, workspace=ws, max_hist=10)
    ha = O.Handle(probs)
    ns, nt = sum(ha.n_src), sum(ha.n_tgt)
    rng = np.random.default_rng(113)
    al = _dev((0.3 + 0.2 * rng.standard_normal(ns)).astype(np.float32))
    be = _dev((0.1 * rng.standard_normal(nt)).astype(np.float32))
    for x, y in zip(outputs(ha, al, be, x_src), outputs(hw, al, be, x_src)):
        assert torch.equal(x, y)
    # a longer history than reserved is refused; a short workspace too
    with pytest.raises(O.OTGSError) as e:
        hw.solve(max_iter=5, hist=11)
    assert e.value.code == O.OT_GS_EINVAL
    hw.close()
    small = torch.empty(nb // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(O.OTGSError) as e:
        O.Handle(probs, workspace=small, max_hist=10)
    assert e.value.code == O.OT_GS_ENOMEM
