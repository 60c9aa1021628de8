"""GPU parity of the O(v) solve with the linear-order (Phi_1) NES and pair
corrections (Eqs. zerothMomentCollisionTerm_NES/_Pair,
firstMomentCollisionTerm_NES/_Pair with Eqs. linearCorrectionsNES/Pair)
against the oracle: the moving profile with pass-through (both kernels: two
points per wavefront, the default, and one point per wavefront), fast flow,
species subsets."""
import numpy as np
import pytest

import oracle as O
from paper_2601_00976_amd import native as N
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

TOL = 1e-9
PRM = dict(tol_inner=1e-12, tol_outer=1e-10)
R_NES, R_PAIR = 0.3, -0.25


def _theta():
    return np.concatenate([np.ones(32), [PT.A_NES, PT.A_PAIR]])


def _run(d, species=(0, 1, 2), flags=O.ALL_PHYSICS, r=(R_NES, R_PAIR), launch=None):
    import torch
    om = O.Model(species=tuple(species), flags=flags, overrides=dict(phi1_nes=r[0], phi1_pair=r[1]))
    D0, _, e0 = om.init_state(d.T, d.rho11, d.ye, d.uD, d.uI)
    I0 = 0.1 * D0[:, :, None, :] * d.uI3
    ef0 = e0 + 0.5 * O.MU_C2 * np.sum(d.v * d.v, axis=1)
    ref = O.solve_batch_v(om, O.Params(**PRM), _theta(), W.DTAU_KM, D0, I0, d.rho11, d.ye, ef0, d.v)
    gm = S.Model(S.Grid(), species=tuple(species), flags=flags, phi1_nes=r[0], phi1_pair=r[1])
    t = S.to_device(d)
    gD, gI, gef = S.init_state_v(gm, t)
    out = S.solve_v(gm, S.Params(**PRM), W.DTAU_KM, gD, gI, t["rho11"], t["ye"], gef, t["v"],
                    torch.as_tensor(_theta(), device="cuda"), launch=launch)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    return om, ref, got


def _compare(om, ref, got, rho11, species=(0, 1, 2)):
    assert np.array_equal(ref["status"], got["status"]), (np.bincount(ref["status"]), np.bincount(got["status"]))
    ok = ref["status"] == 0
    eD, eI, eY, eE, eV = PT.parity_errors_v({k: v[ok] for k, v in ref.items()}, {k: v[ok] for k, v in got.items()},
                                            om.w2, om.w3, om.c.kcoup, rho11[ok], species=species)
    print(f"max errors D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} ef {eE.max():.2e} v {eV.max():.2e}; "
          f"median inner {np.median(got['n_inner'][got['n_outer'] > 0])}", flush=True)
    assert max(eD.max(), eI.max(), eY.max(), eE.max(), eV.max()) <= TOL


@pytest.mark.parametrize("store", [0, 5], ids=["two_points_per_wave", "one_point_per_wave"])
def test_phi1_moving_profile_parity(store):
    print(f"[case] Phi_1 terms, O(v) moving profile sample with pass-through, P=400, kernel_store {store}",
          flush=True)
    d = W.radial_profile_v(P=1 << 16).take(np.linspace(0, 45000, 400).astype(np.int64))
    om, ref, got = _run(d, launch=S.LaunchConfig(chunk=1, kernel_store=store))
    _compare(om, ref, got, d.rho11)
    # the corrections act: the isotropic solve of the same inputs differs
    _, iso, _ = _run(d.take(np.arange(0, 400, 8)), r=(0.0, 0.0))
    live = d.rho11[::8] >= 1e-4
    assert np.max(np.abs(iso["I"][live] - ref["I"][::8][live])) > 1e-8


def test_phi1_fast_flow_and_launches():
    print("[case] Phi_1 terms, |v| in [0.2, 0.4), P=200, non-persistent chunk 3", flush=True)
    d = W.radial_profile_v(P=1 << 16).take(np.linspace(0, 45000, 200).astype(np.int64))
    rng = np.random.default_rng(43)
    n = d.v / np.linalg.norm(d.v, axis=1, keepdims=True)
    d.v = np.ascontiguousarray(n * rng.uniform(0.2, 0.4, (200, 1)))
    om, ref, got = _run(d, launch=S.LaunchConfig(chunk=3, persistent=False))
    either = (ref["status"] == O.MAX_OUTER) | (got["status"] == O.MAX_OUTER)
    assert np.array_equal(ref["status"][~either], got["status"][~either])
    ok = (ref["status"] == 0) & (got["status"] == 0)
    assert ok.mean() > 0.97
    _compare(om, {k: v[ok] for k, v in ref.items()}, {k: v[ok] for k, v in got.items()}, d.rho11[ok])


@pytest.mark.parametrize("species,flags,r", [
    ((O.NU_E, O.NU_E_BAR), O.ALL_PHYSICS, (R_NES, R_PAIR)),
    ((O.NU_X,), O.NES | O.PAIR | O.ISO, (-0.2, 0.3)),
    ((O.NU_E, O.NU_E_BAR, O.NU_X), O.EMAB | O.ISO | O.NES, (1.0 / 3.0, 0.0)),
])
def test_phi1_species_and_physics(species, flags, r):
    print(f"[case] Phi_1 terms, species {species} flags {flags} ratios {r}", flush=True)
    d = W.radial_profile_v(P=1 << 16, ns=len(species)).take(np.linspace(0, 45000, 160).astype(np.int64))
    om, ref, got = _run(d, species=species, flags=flags, r=r)
    _compare(om, ref, got, d.rho11, species=species)


def test_phi1_ratio_range_is_checked():
    for bad in (0.34, -0.5, float("nan")):
        with pytest.raises(N.NmcError) as ei:
            S.Model(S.Grid(), phi1_nes=bad)
        assert ei.value.code == N.NMC_E_INVALID_ARG
