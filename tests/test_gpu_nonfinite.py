"""Failure injection: a point whose old state holds a NaN ends with status
NONFINITE, and the points that share its work-group (the other half of its
wavefront in the two-points-per-wavefront kernel, and the points the same
work-group solves after it) are solved exactly as the oracle solves them.

Launches are non-persistent with several points per work-group, so that a
work-group solves valid points on top of the LDS state the NaN point left.
Both sides build their inputs from the same draws and receive the same NaN
entries."""
import numpy as np
import pytest

import oracle as O
from paper_2601_00976_amd import native as N
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

ALL3 = (O.NU_E, O.NU_E_BAR, O.NU_X)
# (point, species slot, node, array): D* of point 3 (second half of pair 1),
# I* of point 8 (first half of pair 4)
NANS = ((3, 1, 5, "D"), (8, 2, 17, "I"))


def _inputs(n_elem, flags, P=24):
    nq = 2 * n_elem
    d = W.radial_profile(P=1 << 16, nq=nq).take(np.linspace(0, 30000, P).astype(np.int64))
    return d, np.concatenate([np.ones(nq), [PT.A_NES, PT.A_PAIR]])


@pytest.mark.parametrize("n_elem,flags,store,chunk", [
    (16, O.ALL_PHYSICS, N.KERNELS_PAIRED, 3),
    (16, O.EMAB | O.ISO, N.KERNELS_PAIRED, 3),
    (16, O.ALL_PHYSICS, N.KERNELS_WAVE, 4),
    (16, O.ALL_PHYSICS, N.KERNELS_REGEN, 4),
    (16, O.ALL_PHYSICS, N.KERNELS_REGISTERS, 4),
    (16, O.EMAB | O.ISO, N.KERNELS_WAVE, 4),
    (32, O.ALL_PHYSICS, N.KERNELS_ON_CHIP, 4),
])
def test_nan_point_is_nonfinite_and_neighbours_match(n_elem, flags, store, chunk):
    import torch
    print(f"[case] NaN injection: {2 * n_elem} nodes, flags {flags}, kernel store {store}, chunk {chunk}",
          flush=True)
    d, theta = _inputs(n_elem, flags)
    m = PT.oracle_model(ALL3, flags, n_elem)
    D0, I0, e0 = m.init_state(d.T, d.rho11, d.ye, d.uD, d.uI)
    for p, s, q, arr in NANS:
        (D0 if arr == "D" else I0)[p, s, q] = np.nan
    ref = O.solve_batch(m, O.Params(), theta, W.DTAU_KM, D0, I0, d.rho11, d.ye, e0)

    gm = S.Model(S.Grid(n_elem), species=ALL3, flags=flags)
    t = S.to_device(d)
    gD0, gI0, ge0 = S.init_state(gm, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    for p, s, q, arr in NANS:
        (gD0 if arr == "D" else gI0)[p, s, q] = float("nan")
    launch = S.LaunchConfig(chunk=chunk, persistent=False, kernel_store=store)
    # a first solve with NaN points leaves their LDS state behind; the second
    # call is the one compared
    for _ in range(2):
        out = S.solve(gm, S.Params(), W.DTAU_KM, gD0, gI0, t["rho11"], t["ye"], ge0,
                      torch.as_tensor(theta, device="cuda"), launch=launch)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    bad = np.zeros(d.P, dtype=bool)
    bad[[p for p, _, _, _ in NANS]] = True
    assert np.all(ref["status"][bad] == O.NONFINITE)
    assert np.array_equal(ref["status"], got["status"]), (ref["status"], got["status"])
    assert np.array_equal(ref["n_outer"][bad], got["n_outer"][bad])
    assert np.array_equal(ref["n_inner"][bad], got["n_inner"][bad])
    ok = ~bad
    assert np.all(got["status"][ok] == O.OK)
    eD, eI, eY, eE = PT.parity_errors({k: v[ok] for k, v in ref.items()}, {k: v[ok] for k, v in got.items()}, m.w2)
    RY, RE = PT.reservoir_ratios(m.c.kcoup, d.rho11[ok], ref["D"][ok], ref["ye"][ok], ref["e"][ok], m.w2, m.w3)
    eY, eE = eY / np.maximum(RY, 1.0), eE / np.maximum(RE, 1.0)
    print(f"neighbours: D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} e {eE.max():.2e}", flush=True)
    assert max(eD.max(), eI.max(), eY.max(), eE.max()) <= 1e-9


def test_nan_point_o_v():
    import torch
    print("[case] NaN injection: O(v) solve, chunk 4", flush=True)
    dv = W.radial_profile_v(P=1 << 16).take(np.linspace(0, 30000, 16).astype(np.int64))
    theta = np.concatenate([np.ones(32), [PT.A_NES, PT.A_PAIR]])
    prm = dict(tol_inner=1e-12, tol_outer=1e-10)
    m = O.Model()
    D0, _, e0 = m.init_state(dv.T, dv.rho11, dv.ye, dv.uD, dv.uI)
    I0 = 0.1 * D0[:, :, None, :] * dv.uI3
    ef0 = e0 + 0.5 * O.MU_C2 * np.sum(dv.v * dv.v, axis=1)
    D0[5, 0, 3] = np.nan
    I0[6, 1, 2, 9] = np.nan
    ref = O.solve_batch_v(m, O.Params(**prm), theta, W.DTAU_KM, D0, I0, dv.rho11, dv.ye, ef0, dv.v)
    gm = S.Model(S.Grid())
    tv = S.to_device(dv)
    gD, gI, gef = S.init_state_v(gm, tv)
    gD[5, 0, 3] = float("nan")
    gI[6, 1, 2, 9] = float("nan")
    launch = S.LaunchConfig(chunk=4, persistent=False)
    for _ in range(2):
        out = S.solve_v(gm, S.Params(**prm), W.DTAU_KM, gD, gI, tv["rho11"], tv["ye"], gef, tv["v"],
                        torch.as_tensor(theta, device="cuda"), launch=launch)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    assert ref["status"][5] == O.NONFINITE and ref["status"][6] == O.NONFINITE
    assert np.array_equal(ref["status"], got["status"]), (ref["status"], got["status"])
    ok = np.ones(16, dtype=bool)
    ok[[5, 6]] = False
    sub = lambda r: {k: v[ok] for k, v in r.items()}
    eD, eI, eY, eE, eV = PT.parity_errors_v(sub(ref), sub(got), m.w2, m.w3, m.c.kcoup, dv.rho11[ok])
    print(f"neighbours: D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} ef {eE.max():.2e} v {eV.max():.2e}",
          flush=True)
    assert max(eD.max(), eI.max(), eY.max(), eE.max(), eV.max()) <= 1e-9
