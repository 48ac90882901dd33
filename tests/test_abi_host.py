"""Host-side checks of the C ABI that need no GPU: the library loads, every
symbol declared in include/icp.h is exported, struct layouts agree, and
argument validation fails cleanly before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2007_07627_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "icp.h")).read()
    return sorted(set(re.findall(r"\b(icp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTED)


def test_params_default_matches_paper():
    p = B.icp_params_default(B.ICP_P2P_WELSCH)
    assert p.anderson_m == 5 and p.eps == 1e-5 and p.iter_first == 1000 and p.iter_cap == 1000
    q = B.icp_params_default(B.ICP_P2PL_WELSCH)
    assert (q.iter_first, q.iter_inc, q.iter_cap, q.max_line_search) == (6, 1, 10, 10)
    assert list(q.T0) == list(np.eye(4).reshape(16))
    assert B.lib().icp_params_default(7, C.byref(B.icp_params())) == B.ICP_ERR_INVALID_ARG


def test_params_classical_match_appendix_e():
    """The comparison methods (App. E): no mixing, no line search, one stage
    of at most 1000 iterations, ||dT||_F^2 < 1e-5."""
    for mode in (B.ICP_P2P_L2, B.ICP_P2PL_L2):
        p = B.icp_params_classical(mode)
        assert p.mode == mode and p.anderson_m == 0 and p.max_line_search == 0
        assert (p.iter_first, p.iter_inc, p.iter_cap) == (1000, 0, 1000)
        assert abs(p.eps * p.eps - 1e-5) <= 1e-20
    q = B.icp_params_default(B.ICP_P2PL_L2)
    assert q.anderson_m == 0 and q.max_line_search == 0 and q.iter_first == 1000
    for mode in (B.ICP_P2P_WELSCH, B.ICP_P2PL_WELSCH, 9):
        assert B.lib().icp_params_classical(mode, C.byref(B.icp_params())) == B.ICP_ERR_INVALID_ARG


def test_struct_sizes():
    assert C.sizeof(B.icp_params) == 192
    assert C.sizeof(B.icp_result) == 200
    assert C.sizeof(B.icp_profile_stats) == 32


def test_status_strings():
    for s in range(9):
        assert B.icp_status_str(s)


def test_null_context_and_bad_device_fail_cleanly():
    L = B.lib()
    assert L.icp_destroy(None) == B.ICP_ERR_INVALID_ARG
    h = C.c_void_p()
    assert L.icp_create(-1, 0, C.byref(h)) == B.ICP_ERR_DEVICE
    assert L.icp_poll(None, 1, None) == B.ICP_ERR_INVALID_ARG
