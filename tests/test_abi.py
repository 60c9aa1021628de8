"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/nmc.h, builds energy grids on the host and rejects bad
arguments before touching the device; likewise the measurement library of the
FMA probe (include/nmc_probe.h), which the solver library does not export."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2601_00976_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="nmc.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nmc_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = N.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(N.EXPORTED)
    assert not hasattr(L, "nmc_probe_fma_f64")


def test_probe_library_exports_and_checks():
    from paper_2601_00976_amd import probe as PR
    L = PR.lib()
    assert declared_functions("nmc_probe.h") == ["nmc_probe_fma_f64"]
    for waves, iters, out in ((0, 8, 1), (1, 0, 1), (1, 8, None), (1 << 21, 8, 1)):
        assert L.nmc_probe_fma_f64(waves, iters, out, None) == N.NMC_E_INVALID_ARG


def _grid(**kw):
    d = N.GridDesc(kw.get("n_elem", 16), kw.get("npe", 2), kw.get("lo", 1.0), kw.get("hi", 300.0),
                   kw.get("spacing", N.SPACING_LOG), kw.get("zoom", 0.0))
    h = C.c_void_p()
    rc = N.lib().nmc_grid_create(C.byref(d), C.byref(h))
    return rc, h


def _query(h):
    nq = C.c_int()
    N.check(N.lib().nmc_grid_query(h, C.byref(nq), None, None, None))
    out = [np.zeros(nq.value) for _ in range(3)]
    N.check(N.lib().nmc_grid_query(h, None, *[o.ctypes.data_as(C.c_void_p) for o in out]))
    return out


def test_grid_host_values():
    rc, h = _grid()
    assert rc == N.NMC_OK
    eps, w2, w3 = _query(h)
    assert len(eps) == 32
    assert w2.sum() == pytest.approx((300.0**3 - 1) / 3, rel=1e-14)
    assert w3.sum() == pytest.approx((300.0**4 - 1) / 4, rel=1e-14)
    edges = 300.0 ** (np.arange(17) / 16)
    c, d = 0.5 * (edges[:-1] + edges[1:]), np.diff(edges)
    assert np.allclose(eps[0::2], c - d / (2 * np.sqrt(3)), rtol=1e-15)
    N.lib().nmc_grid_destroy(h)


def test_zoom_grid_matches_table():
    for line in open(os.path.join(ROOT, "tests", "golden", "energy_grids_table.txt")):
        if line.startswith("#"):
            continue
        name, n, zoom, d1, dn = line.split()
        rc, h = _grid(n_elem=int(n), spacing=N.SPACING_ZOOM, zoom=float(zoom), hi=300.0)
        assert rc == N.NMC_OK, name
        eps, w2, _ = _query(h)
        assert w2.sum() == pytest.approx(300.0**3 / 3, rel=1e-13), name
        N.lib().nmc_grid_destroy(h)


@pytest.mark.parametrize("kw,code", [(dict(npe=3), N.NMC_E_UNSUPPORTED), (dict(n_elem=0), N.NMC_E_INVALID_ARG),
                                     (dict(n_elem=33), N.NMC_E_INVALID_ARG), (dict(lo=-1.0), N.NMC_E_INVALID_ARG),
                                     (dict(spacing=7), N.NMC_E_INVALID_ARG),
                                     (dict(spacing=N.SPACING_ZOOM, zoom=-2.0), N.NMC_E_INVALID_ARG)])
def test_grid_validation(kw, code):
    rc, h = _grid(**kw)
    assert rc == code and not h.value
    assert len(N.lib().nmc_last_error()) > 0


def test_solve_rejects_null_arguments_before_launch():
    L = N.lib()
    prm = N.SolverParams()
    L.nmc_solver_params_default(C.byref(prm))
    bi, bo = N.BatchIn(), N.BatchOut()
    rc = L.nmc_solve_batch(None, C.byref(prm), 10, 1e-3, C.byref(bi), C.byref(bo), None, 0, None, None)
    assert rc == N.NMC_E_INVALID_ARG
    assert L.nmc_workspace_bytes(None, 10) == 0
    assert L.nmc_error_string(N.NMC_E_UNSUPPORTED) == b"unsupported configuration"
    rc = L.nmc_init_state(None, 1, None, None, None, None, None, None, 1.0, 0.1, 0.1, None, None, None, None)
    assert rc == N.NMC_E_INVALID_ARG


def test_default_descriptors():
    d = N.ModelDesc()
    N.lib().nmc_model_desc_default(C.byref(d))
    assert d.n_species == 3 and d.flags == N.ALL_PHYSICS and d.rho11_min == 1e-4
    p = N.SolverParams()
    N.lib().nmc_solver_params_default(C.byref(p))
    assert (p.tol_inner, p.m_inner, p.m_outer, p.max_inner, p.max_outer) == (1e-10, 3, 3, 100, 50)


def test_projection_descriptor_defaults_and_bounds():
    """The projected equilibrium is off by default with the documented bounds;
    out-of-range bounds are rejected before any device call."""
    d = N.ModelDesc()
    N.lib().nmc_model_desc_default(C.byref(d))
    assert d.fd_projection == 0 and d.deq_min == 1e-150 and d.deq_max == 1.0 - 1e-12
    rc, g = _grid()
    assert rc == N.NMC_OK
    for field, val in (("deq_min", 0.0), ("deq_min", 1e-200), ("deq_min", 0.1), ("deq_max", 1.0),
                       ("deq_max", 0.5), ("fd_projection", 2)):
        dd = N.ModelDesc()
        N.lib().nmc_model_desc_default(C.byref(dd))
        dd.fd_projection = 1
        setattr(dd, field, val)
        h = C.c_void_p()
        assert N.lib().nmc_model_create(g, C.byref(dd), C.byref(h)) == N.NMC_E_INVALID_ARG, (field, val)
        assert not h.value
    N.lib().nmc_grid_destroy(g)


def test_projection_gauss_rule_constants():
    """The 8-point Gauss-Legendre rule written into the projection's device
    code is the rule numpy computes (nodes and weights to rounding)."""
    src = open(os.path.join(ROOT, "paper_2601_00976_amd", "csrc", "nmc_fdproj.h")).read()
    num = r"(-?\d\.\d+)"
    gx = [float(v) for v in re.findall(num, re.search(r"kGx\[8\] = \{(.*?)\};", src, re.S).group(1))]
    gw = [float(v) for v in re.findall(num, re.search(r"kGw\[8\] = \{(.*?)\};", src, re.S).group(1))]
    x, w = np.polynomial.legendre.leggauss(8)
    assert len(gx) == 8 and len(gw) == 8
    assert np.max(np.abs(np.array(gx) - x)) <= 2e-16
    assert np.max(np.abs(np.array(gw) - w)) <= 5e-16
