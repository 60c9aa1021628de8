"""Parity at the benchmark's full sizes and launch shapes: the whole radial
profile (2^16 points at 32 nodes, 2^18 at 64 nodes) is solved on the GPU for
three chained in-place steps at the launch shape bench.py times (autotune
cache), and every point of every step is compared with the oracle's own
chain of the same three steps.

Bar: the statuses agree at every point of every step; after step k the
moments agree to k * 1e-9 in the per-species W-norm, and Ye and e to
k * 1e-9 times the neutrino/matter reservoir ratio (at least 1).  Each step
solves to the relative tolerance 1e-10 and agrees with the oracle's step to
1e-9 from the same input; the chained input differences are carried through
the next step's implicit map, whose response to the old state is damped
(1 / (1 + dtau chi) per node), so the differences add at most linearly over
the steps.  The measured per-step maxima are printed."""
import numpy as np
import pytest

import oracle as O
from paper_2601_00976_amd import autotune as AT
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

STEPS = 3


@pytest.mark.parametrize("n_elem,P,wid", [(16, 1 << 16, 3), (32, 1 << 18, 4)])
def test_full_size_chain_every_point(n_elem, P, wid):
    import torch
    nq = 2 * n_elem
    print(f"[case] full size {P} points, {nq} nodes, {STEPS} chained steps at the bench launch, every point",
          flush=True)
    full = W.radial_profile(P=P, nq=nq, wid=wid)
    m = S.Model(S.Grid(n_elem))
    t = S.to_device(full)
    D, I, e = S.init_state(m, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    ye = t["ye"].clone()
    theta = m.default_theta()
    launch = AT.best_launch(m, P)
    out = S.alloc_outputs(m, P)
    out.update(D=D, I=I, ye=ye, e=e)
    om = O.Model(n_elem=n_elem)
    th = theta.cpu().numpy()
    Do, Io, eo = om.init_state(full.T, full.rho11, full.ye, full.uD, full.uI)
    yeo = full.ye.copy()
    for k in range(1, STEPS + 1):
        S.solve(m, S.Params(), W.DTAU_KM, D, I, t["rho11"], ye, e, theta, out=out, launch=launch)
        torch.cuda.synchronize()
        got = {n: x.cpu().numpy() for n, x in out.items()}
        r = O.solve_batch(om, O.Params(), th, W.DTAU_KM, Do, Io, full.rho11, yeo, eo)
        Do, Io, yeo, eo = r["D"], r["I"], r["ye"], r["e"]
        assert np.array_equal(r["status"], got["status"]), f"step {k}: status mismatch"
        assert np.all(r["status"] == O.OK)
        assert np.array_equal(r["n_outer"] == 0, got["n_outer"] == 0)
        eD, eI, eY, eE = PT.parity_errors(r, got, om.w2)
        RY, RE = PT.reservoir_ratios(om.c.kcoup, full.rho11, r["D"], r["ye"], r["e"], om.w2, om.w3)
        eY, eE = eY / np.maximum(RY, 1.0), eE / np.maximum(RE, 1.0)
        print(f"step {k}: max errors D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} e {eE.max():.2e}; "
              f"solved {int(np.sum(got['n_outer'] > 0))}", flush=True)
        assert max(eD.max(), eI.max(), eY.max(), eE.max()) <= k * 1e-9, f"step {k}"


def test_full_size_every_point_solved():
    """The 2^16-point profile with the low-density pass-through switched off,
    so that every point is solved, down to T ~ 0.065 MeV at its outer edge (the
    NES factors there span more powers of two than the symmetric contraction
    can carry, and the kernel takes its orientation form).  One step, every
    point.

    Far out, the neutrino reservoir dwarfs the matter's: the ratio R of
    neutrino to matter lepton number or energy (from the oracle's result)
    exceeds 1e5 on the outer 17% of the profile and reaches 1e7.  The matter
    update multiplies the rounding of the moments by R, so beyond
    R = 1e5 ~ tol_outer / (10 eps_mach) the outer test at 1e-10 is decided
    by rounding: there the oracle and the GPU (same algorithm, different
    summation order and FMAs) end with different statuses (MAX_OUTER, EOS
    domain, OK) at ~150 points and different converged states; such points
    are counted, not compared (the paper switches the coupling off there).
    Where R <= 1e5 the statuses agree exactly, converged points agree to 1e-9
    (species more than 12 orders of magnitude below their point's largest in
    the point's all-species norm), and EOS-domain exits, the last iterate of a
    diverging iteration, to 1e-5."""
    import torch
    print("[case] full size 65536 points, 32 nodes, every point solved (rho11_min = 0), one step", flush=True)
    full = W.radial_profile(P=1 << 16)
    m = S.Model(S.Grid(16), rho11_min=0.0)
    t = S.to_device(full)
    D, I, e = S.init_state(m, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    theta = m.default_theta()
    out = S.solve(m, S.Params(), W.DTAU_KM, D, I, t["rho11"], t["ye"], e, theta, launch=AT.best_launch(m, 1 << 16))
    torch.cuda.synchronize()
    got = {n: x.cpu().numpy() for n, x in out.items()}
    om = O.Model(overrides=dict(rho11_min=0.0))
    th = theta.cpu().numpy()
    Do, Io, eo = om.init_state(full.T, full.rho11, full.ye, full.uD, full.uI)
    r = O.solve_batch(om, O.Params(), th, W.DTAU_KM, Do, Io, full.rho11, full.ye, eo)
    assert np.all(got["n_outer"] > 0)
    RY, RE = PT.reservoir_ratios(om.c.kcoup, full.rho11, r["D"], r["ye"], r["e"], om.w2, om.w3)
    well = np.maximum(RY, RE) <= 1e5
    far = ~well
    print(f"R <= 1e5 at {int(well.sum())} points (T >= {full.T[well].min():.3f} MeV); oracle status "
          f"{np.bincount(r['status'][well], minlength=5)}, GPU {np.bincount(got['status'][well], minlength=5)}; "
          f"beyond: oracle {np.bincount(r['status'][far], minlength=5)}, GPU "
          f"{np.bincount(got['status'][far], minlength=5)}, {int(np.sum(r['status'][far] != got['status'][far]))} "
          f"status differences", flush=True)
    assert well.mean() > 0.8
    assert np.array_equal(r["status"][well], got["status"][well])
    ok = well & (r["status"] == O.OK)
    eos = well & (r["status"] == O.EOS_DOMAIN)
    eD, eI, eY, eE = PT.parity_errors({n: x[ok] for n, x in r.items()}, {n: x[ok] for n, x in got.items()}, om.w2)
    dn = PT.wnorm(r["D"][ok], om.w2)
    tiny = dn < 1e-12 * dn.max(axis=1, keepdims=True)
    scale = np.where(tiny, np.sqrt(np.sum(dn * dn, axis=1, keepdims=True)), 1.0)
    eD, eI = np.where(tiny, eD * dn / scale, eD), np.where(tiny, eI * dn / scale, eI)
    eY, eE = eY / np.maximum(RY[ok], 1.0), eE / np.maximum(RE[ok], 1.0)
    print(f"converged {int(ok.sum())}: D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} e {eE.max():.2e}",
          flush=True)
    assert max(eD.max(), eI.max(), eY.max(), eE.max()) <= 1e-9
    if eos.any():
        xD, xI, _, _ = PT.parity_errors({n: x[eos] for n, x in r.items()}, {n: x[eos] for n, x in got.items()},
                                        om.w2)
        print(f"EOS-domain exits {int(eos.sum())}: D {xD.max():.2e} I {xI.max():.2e}", flush=True)
        assert xD.max() <= 1e-5 and xI.max() <= 1e-5
