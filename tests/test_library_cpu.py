"""Host-side checks of the HIP library (no GPU needed): the shared library
loads, exports every symbol include/rbmc.h declares, and its decomposition
planner reproduces the oracle's breadth-first overlap growth bit for bit."""
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd import binding as B
from paper_2309_05435_amd.inputs import obs_mask

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "rbmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rbmc_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    declared = header_symbols()
    assert set(declared) == set(B.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("mx,my,T,P,tx,ty,n_l", [
    (16, 16, 10, 4, 1, 1, 1), (12, 10, 9, 3, 2, 2, 1), (13, 13, 8, 2, 3, 2, 2),
    (9, 9, 7, 7, 1, 1, 0), (20, 17, 5, 1, 3, 4, 2), (7, 7, 1, 1, 1, 1, 1)])
def test_planner_matches_oracle_bfs(mx, my, T, P, tx, ty, n_l):
    n = mx * my * T
    mask = obs_mask(n, 0.3, 3)
    h = 1.0 / (max(mx, my) - 1)
    desc, _m = B.make_desc(mx, my, T, h, (2.0, 0.0, 0.9, 0.0), mask)
    dc = B.rbmc_decomp_desc(P, tx, ty, n_l)
    lab = np.zeros(n, np.int32)
    B.rbmc_plan_query(desc, dc, 0, label_out=lab)
    np.testing.assert_array_equal(lab, O.grid_cores(mx, my, T, P, tx, ty))
    M = O.OracleModel(mx, my, T, h, 2.0, 0.0, 0.9, 0.0, mask)
    for p in range(P * tx * ty):
        st = np.zeros(n, np.uint8)
        B.rbmc_plan_query(desc, dc, p, state_out=st)
        np.testing.assert_array_equal(st, M.subdomain_state(lab, p, n_l))


@pytest.mark.parametrize("bad", [
    dict(mx=1), dict(T=0), dict(P=11), dict(tx=0), dict(n_l=-1), dict(h=0.0)])
def test_planner_rejects_bad_arguments(bad):
    cfg = dict(mx=8, my=8, T=10, P=2, tx=1, ty=1, n_l=1, h=1 / 7)
    cfg.update(bad)
    n = max(cfg["mx"], 1) * cfg["my"] * max(cfg["T"], 1)
    desc, _m = B.make_desc(cfg["mx"], cfg["my"], cfg["T"], cfg["h"], (2.0, 0.0, 0.9, 0.0),
                           np.zeros(n, np.uint8))
    dc = B.rbmc_decomp_desc(cfg["P"], cfg["tx"], cfg["ty"], cfg["n_l"])
    lab = np.zeros(n, np.int32)
    if "h" in bad:
        pytest.skip("h is validated at model creation (needs a device)")
    with pytest.raises(B.RbmcError) as e:
        B.rbmc_plan_query(desc, dc, 0, label_out=lab)
    assert e.value.status == B.RBMC_E_ARG


def test_planner_rejects_models_beyond_32_bit_node_indices():
    """A sample's node indices are 32-bit in the kernels: mx my T >= 2^31 is
    refused before anything is read or allocated (2^31 - 1 nodes would pass
    this check)."""
    mask = np.zeros(1, np.uint8)  # never read: the size check comes first
    for mx, my, T in ((8192, 8192, 32), (65536, 65536, 1)):
        desc, _m = B.make_desc(mx, my, T, 1.0, (2.0, 0.0, 0.9, 0.0), mask)
        with pytest.raises(B.RbmcError) as e:
            B.rbmc_plan_query(desc, B.rbmc_decomp_desc(1, 1, 1, 0), 0)
        assert e.value.status == B.RBMC_E_ARG
        assert "2^31" in str(e.value)


def test_posterior_mean_rejects_a_null_model_before_any_device_call():
    """rbmc_posterior_mean checks its arguments before it touches a device."""
    import ctypes as C
    rep = B.rbmc_report()
    st = B.lib().rbmc_posterior_mean(None, C.byref(B.make_opts(1)), None, 0, None, None, None,
                                     None, None, None, C.byref(rep))
    assert st == B.RBMC_E_ARG
    assert b"NULL" in B.lib().rbmc_last_error()


def test_grad_log_posterior_rejects_a_null_model_before_any_device_call():
    import ctypes as C
    rep = B.rbmc_report()
    g = (C.c_double * 4)()
    st = B.lib().rbmc_grad_log_posterior(None, C.byref(B.make_opts(0)), None, None,
                                         C.c_uint64(0), g, None, None, C.byref(rep))
    assert st == B.RBMC_E_ARG
    assert b"NULL" in B.lib().rbmc_last_error()
