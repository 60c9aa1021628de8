"""GPU parity of the O(v) solve (nonzero fluid velocity) against the oracle:
the moving radial profile with its low-density pass-through, the moving
equilibrium fixed point, ragged and in-place launches, and argument checks."""
import numpy as np
import pytest

import oracle as O
from paper_2601_00976_amd import native as N
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

TOL = 1e-9
# The fixed-point form with lambda < 1 converges linearly in the inner loop;
# its residual error, amplified by the neutrino/matter reservoir ratio at the
# low-density edge of the profile, would exceed an outer tolerance equal to
# the inner one there, so the O(v) workloads solve the inner loop 100 times
# tighter.
ORA_PRM = dict(tol_inner=1e-12, tol_outer=1e-10)


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _theta():
    return np.concatenate([np.ones(32), [PT.A_NES, PT.A_PAIR]])


def _profile(P, lo=0, hi=1 << 16):
    full = W.radial_profile_v(P=1 << 16)
    return full.take(np.linspace(lo, hi - 1, P).astype(np.int64))


@pytest.mark.parametrize("store", [N.KERNELS_ON_CHIP, N.KERNELS_WAVE])
def test_moving_profile_parity(store):
    """The default two-points-per-wavefront kernel and the one-point kernel
    (kernel_store WAVE), each against the oracle."""
    _say(f"O(v) radial profile sample with pass-through, P=600, kernel_store {store}")
    d = _profile(600)
    m, ref = PT.run_oracle_v(d, W.DTAU_KM, O.Params(**ORA_PRM), _theta())
    _, got = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta(), launch=S.LaunchConfig(kernel_store=store))
    assert np.max(np.abs(got["D0"] - ref["D0"])) <= 1e-15
    assert np.max(np.abs(got["I0"] - ref["I0"])) <= 1e-15
    assert np.max(np.abs(got["ef0"] - ref["ef0"]) / ref["ef0"]) <= 1e-15
    print("status", np.bincount(ref["status"], minlength=5), np.bincount(got["status"], minlength=5), flush=True)
    ok = (ref["status"] == 0) & (got["status"] == 0)
    # a point whose outer iteration stalls at its noise floor may end with
    # MAX_OUTER on one side only; every other status agrees
    either = (ref["status"] == O.MAX_OUTER) | (got["status"] == O.MAX_OUTER)
    assert np.array_equal(ref["status"][~either], got["status"][~either])
    assert ok.mean() > 0.99
    eD, eI, eY, eE, eV = PT.parity_errors_v({k: v[ok] for k, v in ref.items()},
                                            {k: v[ok] for k, v in got.items()}, m.w2, m.w3, m.c.kcoup,
                                            d.rho11[ok])
    print(f"max errors D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} ef {eE.max():.2e} v {eV.max():.2e}",
          flush=True)
    assert eD.max() <= TOL and eI.max() <= TOL
    assert eY.max() <= TOL and eE.max() <= TOL and eV.max() <= TOL
    skip = d.rho11 < 1e-4
    assert skip.any() and (~skip).any()
    assert np.all(got["n_outer"][skip] == 0)
    assert np.array_equal(got["D"][skip], got["D0"][skip]) and np.array_equal(got["I"][skip], got["I0"][skip])
    assert np.array_equal(got["v"][skip], d.v[skip])
    # the velocity moved where neutrinos exchanged momentum
    assert np.max(np.abs(got["v"][~skip] - d.v[~skip])) > 1e-6


def test_moving_equilibrium_fixed_point():
    _say("O(v) moving equilibrium: D* = D_eq, I* = 0")
    d = _profile(256, 0, 30000)
    d.uD = np.zeros_like(d.uD)  # D* = D_eq exactly (a = 1, b uD = 0)
    d.uI3 = np.zeros_like(d.uI3)
    _, got = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta())
    assert np.all(got["status"] == 0)
    m = O.Model()
    dn = np.sqrt(np.sum(m.w2 * got["D0"] ** 2, axis=-1))
    assert np.max(np.sqrt(np.sum(m.w2 * (got["D"] - got["D0"]) ** 2, axis=-1)) / dn) < 1e-11
    # D* is the equilibrium to rounding only, so the flux settles at rounding level
    assert np.max(np.abs(got["I"]), axis=(1, 2, 3)).max() <= 1e-14 * got["D0"].max()
    assert np.allclose(got["ye"], d.ye, rtol=1e-12, atol=0)
    assert np.allclose(got["ef"], got["ef0"], rtol=1e-12, atol=0)
    assert np.allclose(got["v"], d.v, rtol=1e-12, atol=0)


@pytest.mark.parametrize("launch", [S.LaunchConfig(persistent=False, chunk=1),
                                    S.LaunchConfig(persistent=True, chunk=3, blocks_per_cu=1),
                                    S.LaunchConfig(persistent=False, chunk=7),
                                    S.LaunchConfig(persistent=True, chunk=2, kernel_store=N.KERNELS_PAIRED)])
def test_ragged_launches_bitwise(launch):
    _say(f"O(v) ragged launch {launch}")
    d = _profile(517, 1000, 20000)
    _, a = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta())
    _, b = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta(), launch=launch)
    for k in ("D", "I", "ye", "ef", "v", "T", "n_outer", "n_inner", "status"):
        assert np.array_equal(a[k], b[k]), k


def test_in_place_step():
    _say("O(v) in-place step")
    d = _profile(300, 0, 40000)
    _, a = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta())
    _, b = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta(), inplace=True)
    for k in ("D", "I", "ye", "ef", "v", "T", "n_outer", "n_inner", "status"):
        assert np.array_equal(a[k], b[k]), k


def test_argument_checks():
    _say("O(v) argument checks")
    import torch
    m64 = S.Model(S.Grid(n_elem=32))
    P = 4
    f = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")
    with pytest.raises(N.NmcError) as e:
        S.solve_v(m64, S.Params(), 1e-3, f(P, 3, 64), f(P, 3, 3, 64), f(P) + 1, f(P) + 0.3, f(P) + 10, f(P, 3),
                  f(66))
    assert e.value.code == N.NMC_E_UNSUPPORTED
    m = S.Model(S.Grid())
    with pytest.raises(N.NmcError) as e:
        S.solve_v(m, S.Params(), 1e-3, f(P, 3, 32), f(P, 3, 3, 32), f(P) + 1, f(P) + 0.3, f(P) + 10, f(P, 3),
                  f(34), launch=S.LaunchConfig(kernel_store=N.KERNELS_REGEN))
    assert e.value.code == N.NMC_E_UNSUPPORTED
    with pytest.raises(N.NmcError) as e:
        S.solve_v(m, S.Params(), 0.0, f(P, 3, 32), f(P, 3, 3, 32), f(P) + 1, f(P) + 0.3, f(P) + 10, f(P, 3), f(34))
    assert e.value.code == N.NMC_E_INVALID_ARG
    # an empty batch enqueues nothing
    S.solve_v(m, S.Params(), 1e-3, f(0, 3, 32), f(0, 3, 3, 32), f(0), f(0), f(0), f(0, 3), f(34))


def test_single_point_and_all_skipped():
    _say("O(v) one point; a batch entirely below the coupling density")
    d = _profile(1, 20000, 20001)
    m, ref = PT.run_oracle_v(d, W.DTAU_KM, O.Params(**ORA_PRM), _theta())
    _, got = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta())
    assert got["status"][0] == ref["status"][0] == 0 and got["n_outer"][0] > 0
    eD, eI, eY, eE, eV = PT.parity_errors_v(ref, got, m.w2, m.w3, m.c.kcoup, d.rho11)
    assert max(eD.max(), eI.max(), eY.max(), eE.max(), eV.max()) <= TOL
    low = _profile(50, 62000, 65535)
    assert np.all(low.rho11 < 1e-4)
    _, got = PT.run_gpu_v(low, W.DTAU_KM, S.Params(**ORA_PRM), _theta())
    assert np.all(got["n_outer"] == 0) and np.all(got["status"] == 0)
    assert np.array_equal(got["D"], got["D0"]) and np.array_equal(got["I"], got["I0"])
    assert np.array_equal(got["v"], low.v) and np.array_equal(got["ef"], got["ef0"])


def _oracle_status_spread(om, idx, D, I, rho11, ye, ef, v, draws=512):
    """Statuses the oracle itself returns at points idx when every entry of
    the old moments D* moves by a seeded random -1, 0 or +1 ulp (``draws``
    runs per point)."""
    rng = np.random.default_rng(17)
    rep = np.repeat(idx, draws)
    Dp = D[rep] * (1.0 + rng.integers(-1, 2, D[rep].shape) * 2.0 ** -52)
    r = O.solve_batch_v(om, O.Params(**ORA_PRM), _theta(), W.DTAU_KM, Dp, I[rep], rho11[rep], ye[rep], ef[rep],
                        v[rep])
    return [set(int(x) for x in r["status"][i * draws:(i + 1) * draws]) for i in range(len(idx))]


def test_full_size_chain_every_point():
    """The 2^16-point moving profile at the launch shape bench.py times, three
    chained in-place steps on the GPU and in the oracle, every point of every
    step compared.

    Statuses: equal at every point, except where the oracle's own status is
    decided by rounding.  At the low-density edge of the profile the outer
    iteration of a few points hovers at its noise floor (the neutrino/matter
    reservoir ratio amplifies the inner loop's residual), and whether it meets
    the outer tolerance within max_outer there flips with 1-ulp changes of
    the old moments.  A status mismatch is accepted only where the GPU's
    status is one the oracle returns under such a perturbation of its own
    input (512 seeded draws: a status taken in 2.5% of them is then seen with
    probability 1 - 4e-6), and on at most 0.1% of the points.  Points
    that are not OK on either side are not converged states: their moments
    are not compared, and from then on their chained inputs differ.
    Moments and matter of every other point: after step k, k * 1e-9 (as for
    the static chain), per species, except for a species more than 12 orders
    of magnitude below the point's largest (nu_e at ~0.3 MeV, ~1e-22 of
    anti-nu_e at the low-density edge): there the outer iteration of the two
    sides stops at different counts within its tolerance, the temperature
    differs at that level, and that species' exponential tail answers with a
    factor (eps - mu) / T of 50-100, so it is compared in the point's
    all-species W-norm, the reading used for the low-temperature case."""
    _say("O(v) full size 2^16, 3 chained steps, every point")
    import torch
    full = W.radial_profile_v(P=1 << 16)
    m = S.Model(S.Grid())
    t = S.to_device(full)
    D, I, ef = S.init_state_v(m, t)
    ye, v = t["ye"].clone(), t["v"].clone()
    theta = torch.as_tensor(_theta(), dtype=torch.float64, device="cuda")
    prm = S.Params(**ORA_PRM)
    out = S.alloc_outputs_v(m, 1 << 16)
    out.update(D=D, I=I, ye=ye, ef=ef, v=v)
    om = O.Model()
    D0, _, e0 = om.init_state(full.T, full.rho11, full.ye, full.uD, full.uI)
    Io = 0.1 * D0[:, :, None, :] * full.uI3
    efo = e0 + 0.5 * O.MU_C2 * np.sum(full.v * full.v, axis=1)
    Do, yeo, vo = D0, full.ye.copy(), full.v.copy()
    live = np.ones(1 << 16, dtype=bool)  # converged on both sides in every step so far
    for k in range(1, 4):
        S.solve_v(m, prm, W.DTAU_KM, D, I, t["rho11"], ye, ef, v, theta, out=out, launch=S.LaunchConfig(chunk=1))
        torch.cuda.synchronize()
        got = {n: x.cpu().numpy() for n, x in out.items()}
        r = O.solve_batch_v(om, O.Params(**ORA_PRM), _theta(), W.DTAU_KM, Do, Io, full.rho11, yeo, efo, vo)
        mism = np.where(live & (r["status"] != got["status"]))[0]
        print(f"step {k}: oracle status {np.bincount(r['status'], minlength=5)}, "
              f"GPU {np.bincount(got['status'], minlength=5)}, {len(mism)} mismatches", flush=True)
        if len(mism):
            seen = _oracle_status_spread(om, mism, Do, Io, full.rho11, yeo, efo, vo)
            for i, p in enumerate(mism):
                print(f"  point {p} (rho11 {full.rho11[p]:.2e}): oracle {r['status'][p]}, GPU {got['status'][p]}, "
                      f"oracle under 1-ulp changes of D* {sorted(seen[i])}", flush=True)
            assert all(int(got["status"][p]) in seen[i] for i, p in enumerate(mism)), f"step {k}: status mismatch"
            assert len(mism) <= 1e-3 * len(live)
        Do, Io, yeo, efo, vo = r["D"], r["I"], r["ye"], r["ef"], r["v"]
        live &= (r["status"] == 0) & (got["status"] == 0)
        assert live.mean() > 0.999
        eD, eI, eY, eE, eV = PT.parity_errors_v({n: x[live] for n, x in r.items()},
                                                {n: x[live] for n, x in got.items()},
                                                om.w2, om.w3, om.c.kcoup, full.rho11[live])
        print(f"step {k}: max errors D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} ef {eE.max():.2e} "
              f"v {eV.max():.2e} over {int(live.sum())} points", flush=True)
        # a species more than 12 orders of magnitude below the point's largest
        # is compared in the point's all-species W-norm (see the docstring)
        dn = PT.wnorm(r["D"][live], om.w2)
        tiny = dn < 1e-12 * dn.max(axis=1, keepdims=True)
        scale = np.where(tiny, np.sqrt(np.sum(dn * dn, axis=1, keepdims=True)), 1.0)
        eDs, eIs = np.where(tiny, eD * dn / scale, eD), np.where(tiny, eI * dn / scale, eI)
        li = np.where(live)[0]
        for w in np.where(np.max(np.maximum(eD, eI), axis=1) > k * TOL)[0]:
            p = li[w]
            print(f"  point {p}: rho11 {full.rho11[p]:.3e} T {r['T'][p]:.3f} errors D {eD[w]} I {eI[w]} "
                  f"||D_s|| {dn[w]} n_outer {r['n_outer'][p]}/{got['n_outer'][p]}", flush=True)
        print(f"step {k}: with tiny species in the point norm: D {eDs.max():.2e} I {eIs.max():.2e} "
              f"({int(tiny.sum())} tiny species)", flush=True)
        assert max(eDs.max(), eIs.max(), eY.max(), eE.max(), eV.max()) <= k * TOL, f"step {k}"


@pytest.mark.parametrize("species,flags,fixed", [
    ((O.NU_E, O.NU_E_BAR, O.NU_X), O.EMAB | O.ISO, False),
    ((O.NU_E, O.NU_E_BAR), O.ALL_PHYSICS, False),
    ((O.NU_X,), O.NES | O.PAIR | O.ISO, False),
    ((O.NU_E, O.NU_E_BAR, O.NU_X), O.ALL_PHYSICS, True),
])
def test_species_physics_and_fixed_matter(species, flags, fixed):
    _say(f"O(v) species {species} flags {flags} fixed_matter {fixed}")
    d = W.radial_profile_v(P=1 << 16, ns=len(species)).take(np.linspace(0, 45000, 200).astype(np.int64))
    m, ref = PT.run_oracle_v(d, W.DTAU_KM, O.Params(fixed_matter=fixed, **ORA_PRM), _theta(), species=species,
                             flags=flags)
    _, got = PT.run_gpu_v(d, W.DTAU_KM, S.Params(fixed_matter=fixed, **ORA_PRM), _theta(), species=species,
                          flags=flags)
    assert np.array_equal(ref["status"], got["status"])
    ok = ref["status"] == 0
    assert ok.mean() > 0.99
    eD, eI, eY, eE, eV = PT.parity_errors_v({k: v[ok] for k, v in ref.items()}, {k: v[ok] for k, v in got.items()},
                                            m.w2, m.w3, m.c.kcoup, d.rho11[ok], species=species)
    print(f"max errors D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} ef {eE.max():.2e} v {eV.max():.2e}",
          flush=True)
    assert max(eD.max(), eI.max(), eY.max(), eE.max(), eV.max()) <= TOL
    if fixed:
        assert np.array_equal(got["ye"], d.ye) and np.array_equal(got["v"], d.v)
        assert np.array_equal(got["ef"], got["ef0"])


def test_fast_flow_parity():
    """Speeds 0.2-0.4 c, up to the bound below which the fixed-point map of
    the moment equations is a contraction."""
    _say("O(v) fast flow, |v| in [0.2, 0.4), P=256")
    d = _profile(256, 0, 45000)
    rng = np.random.default_rng(41)
    n = d.v / np.linalg.norm(d.v, axis=1, keepdims=True)
    d.v = np.ascontiguousarray(n * rng.uniform(0.2, 0.4, (256, 1)))
    m, ref = PT.run_oracle_v(d, W.DTAU_KM, O.Params(**ORA_PRM), _theta())
    _, got = PT.run_gpu_v(d, W.DTAU_KM, S.Params(**ORA_PRM), _theta())
    either = (ref["status"] == O.MAX_OUTER) | (got["status"] == O.MAX_OUTER)
    assert np.array_equal(ref["status"][~either], got["status"][~either])
    ok = (ref["status"] == 0) & (got["status"] == 0)
    assert ok.mean() > 0.97
    eD, eI, eY, eE, eV = PT.parity_errors_v({k: v[ok] for k, v in ref.items()}, {k: v[ok] for k, v in got.items()},
                                            m.w2, m.w3, m.c.kcoup, d.rho11[ok])
    print(f"status {np.bincount(ref['status'], minlength=5)}; max errors D {eD.max():.2e} I {eI.max():.2e} "
          f"Ye {eY.max():.2e} ef {eE.max():.2e} v {eV.max():.2e}; median inner {np.median(got['n_inner'])}",
          flush=True)
    assert max(eD.max(), eI.max(), eY.max(), eE.max(), eV.max()) <= TOL
