"""The C-ABI library loads and exports every entry point its header declares (no GPU
calls).  Also checks the host-side argument validation paths that run before any launch."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int32_t|size_t|const char\*)\s+(rt_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["rt_sample_resonance", "rt_trace_forward", "rt_trace_backward", "rt_bin_flux", "rt_flux_grad"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_2309_08655_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("librt.so not built")
    L = C.CDLL(rt.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_workspace_sizes_and_version():
    import paper_2309_08655_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("librt.so not built")
    L = rt.lib()
    assert L.rt_workspace_size(rt.OP_TRACE_FORWARD, 1000) >= 76 * 1000
    assert L.rt_workspace_size(rt.OP_BIN, 1000) >= 4 * 1000
    assert L.rt_workspace_size(rt.OP_FLUX_GRAD, 1000) == L.rt_flux_grad_workspace_size(1000, 64, 64, 2001) > 0
    assert L.rt_flux_grad_workspace_size(1000, 65, 64, 64) == 0
    # the checkpoint pool: 96 bytes a slot, between 1 and 2^31 - 1 slots
    base = L.rt_flux_grad_workspace_size(1000, 8, 64, 1000)
    assert L.rt_flux_grad_workspace_size(1000, 8, 64, 1000 + 4096) - base == 96 * 4096
    assert L.rt_flux_grad_workspace_size(1000, 8, 64, 0) == 0
    assert L.rt_flux_grad_workspace_size(1000, 8, 64, 2**31) == 0
    assert b"gfx950" in L.rt_version()


def test_validation_before_launch():
    """Invalid stars are rejected on the host (no device is touched)."""
    import paper_2309_08655_amd as rt
    import workloads as W
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("librt.so not built")
    L = rt.lib()
    bad = dict(W.CFG1["star"])
    bad["m_a_eV"] = -1.0
    s = rt.make_star(bad)
    rc = L.rt_sample_resonance(C.byref(s), 0, 0, 0, 10, None, None, None)
    assert rc == -1
    assert b"positive" in L.rt_last_error()
    bad = dict(W.CFG1["star"])
    bad["M_Msun"] = 4.0  # r_s > R
    s = rt.make_star(bad)
    assert L.rt_sample_resonance(C.byref(s), 0, 0, 0, 10, None, None, None) == -1
