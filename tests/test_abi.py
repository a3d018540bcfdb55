"""The C ABI library loads and exports every entry point that include/otgs.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "otgs.h")
LIB = os.path.join(ROOT, "paper_2303_07597_amd", "libotgs.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_gs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    syms = declared_symbols()
    for name in ("ot_gs_create", "ot_gs_destroy", "ot_gs_dual_grad", "ot_gs_solve", "ot_gs_plan",
                 "ot_gs_plan_csr"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libotgs.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libotgs.so not built")
def test_host_only_entry_points():
    import paper_2303_07597_amd.otgs as O
    assert "gfx950" in O.ot_gs_version()
    g, m = O.ot_gs_rho_to_mu(1e3, 0.8)
    assert abs(g - 200.0) < 1e-9 and abs(m - 4.0) < 1e-12
    with pytest.raises(O.OTGSError):
        O.ot_gs_rho_to_mu(1.0, 1.0)
    o = O.ot_gs_options()
    O.lib().ot_gs_default_options(ctypes.byref(o))
    assert (o.max_iter, o.hist, o.refresh, o.use_screen, o.max_ls) == (200, 10, 10, 1, 40)
    # the struct's last field (its layout agrees up to its end)
    assert o.recenter_tol == 1e-9
