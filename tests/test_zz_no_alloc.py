"""ot_gs_plan_csr_static (no device allocations, scratch in a fixed device
array) against ot_gs_plan_csr, through the C ABI: identical row pointers,
column indices and values, on two calls in a row (the second on a smaller
input, so it reuses the array the first one left behind); sizes beyond the
array are refused before any work."""
import ctypes as ct

import numpy as np
import pytest

import oracle
from tests import cases

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def static_csr(h, al, be, n_rows):
    O = _O()
    L = O.lib()
    L.ot_gs_plan_csr_static.argtypes = [ct.c_void_p] * 6 + [ct.POINTER(ct.c_longlong), ct.c_void_p]
    nnz = ct.c_longlong(-1)
    rp = torch.full((n_rows + 1,), -5, dtype=torch.int64, device="cuda")
    s = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.ot_gs_plan_csr_static(h.h, al.data_ptr(), be.data_ptr(), rp.data_ptr(), None, None, ct.byref(nnz), s)
    assert rc == 0, L.ot_gs_last_error()
    col = torch.full((max(nnz.value, 1),), -7, dtype=torch.int32, device="cuda")
    val = torch.full((max(nnz.value, 1),), -7.0, dtype=torch.float32, device="cuda")
    rc = L.ot_gs_plan_csr_static(h.h, al.data_ptr(), be.data_ptr(), rp.data_ptr(), col.data_ptr(),
                                 val.data_ptr(), None, s)
    assert rc == 0, L.ot_gs_last_error()
    torch.cuda.synchronize()
    return rp, col[:nnz.value], val[:nnz.value]


@pytest.mark.parametrize("order", [0, 1])
def test_static_plan_csr_equals_plan_csr(order):
    O = _O()
    specs = [(80, [2300, 300, 5], 130), (81, [50, 0, 70, 30], 90)]
    if order:
        specs = specs[::-1]
    for seed, sizes, nt in specs:
        inst = cases.ragged(seed, sum(sizes), nt, sizes)
        C32, P = cases.with_cost(inst)
        h = O.Handle([dict(labels=_dev(P.labels), n_groups=P.L, gamma=P.gamma, mu=P.mu, cost=_dev(C32),
                           cost_scale=1.0, cost_mode=O.OT_GS_COST_GIVEN)])
        r = oracle.solve(P, max_iter=30)
        al, be = _dev(r["alpha"].astype(np.float32)), _dev(r["beta"].astype(np.float32))
        rp1, c1, v1 = h.plan_csr(al, be)
        rp2, c2, v2 = static_csr(h, al, be, P.ns)
        torch.cuda.synchronize()
        assert c1.numel() > 0
        assert torch.equal(rp1, rp2) and torch.equal(c1, c2) and torch.equal(v1, v2)
        h.close()


def test_static_plan_csr_refuses_oversized_handles():
    """50000 rows x 128 column blocks need 76.8 MB of scratch for a fill."""
    O = _O()
    r = np.random.default_rng(82)
    ns, nt, d = 50000, 4096, 16
    labels = r.integers(0, 4, ns).astype(np.int32)
    xs = r.integers(-2, 3, (ns, d)).astype(np.float32)
    xt = r.integers(-2, 3, (nt, d)).astype(np.float32)
    h = O.Handle([dict(labels=_dev(labels), n_groups=4, gamma=0.5, mu=0.1, x_src=_dev(xs), x_tgt=_dev(xt),
                       cost_mode=O.OT_GS_COST_ONTHEFLY, cost_scale=2.0 ** -8)])
    L = O.lib()
    L.ot_gs_plan_csr_static.argtypes = [ct.c_void_p] * 6 + [ct.POINTER(ct.c_longlong), ct.c_void_p]
    al = torch.zeros(ns, dtype=torch.float32, device="cuda")
    be = torch.zeros(nt, dtype=torch.float32, device="cuda")
    rp = torch.zeros(ns + 1, dtype=torch.int64, device="cuda")
    col = torch.zeros(16, dtype=torch.int32, device="cuda")
    val = torch.zeros(16, dtype=torch.float32, device="cuda")
    rc = L.ot_gs_plan_csr_static(h.h, al.data_ptr(), be.data_ptr(), rp.data_ptr(), col.data_ptr(), val.data_ptr(),
                                 None, None)
    assert rc == O.OT_GS_EINVAL
    assert b"scratch" in L.ot_gs_last_error()
