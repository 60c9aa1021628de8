"""The paper's relaxation problem (Sec. 6.1) with the O(v) solve and the
synthetic opacities: neutrinos start far from equilibrium in a moving fluid,
and chained backward-Euler steps relax them.  Checked: GPU against the
oracle step by step, conservation of the total lepton number, energy and
momentum over the chain, and the approach to the comoving equilibrium
(Fermi-Dirac number moments of the electron flavours, vanishing flux)."""
import numpy as np
import pytest

import oracle as O
from paper_2601_00976_amd import solver as S
from tests import parity as PT

pytestmark = pytest.mark.gpu

MC2 = O.MU_C2
PRM = dict(tol_inner=1e-12, tol_outer=1e-10, max_outer=100)
STEPS, DTAU = 12, 0.5  # km


def _initial(P):
    """Initial moments of f0 = 0.99 exp(-((e - 2T)/10 MeV)^2 / 2) H(mu) for every
    species: D = (1/2) int f0 dmu, I^1 = (1/2) int f0 mu dmu along the first
    axis; matter rho = 1e12 g/cm^3, T = 7.6 MeV, Ye = 0.135, v = (0.1, 0, 0) at
    the first point, the other points with other speeds and directions."""
    m = O.Model()
    eps = m.eps
    rng = np.random.default_rng(2535)
    T = np.full(P, 7.6)
    T[1:] = rng.uniform(5.0, 10.0, P - 1)
    rho = np.full(P, 10.0)
    ye = np.full(P, 0.135)
    n = rng.standard_normal((P, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n[0] = (1.0, 0.0, 0.0)
    speed = np.concatenate([[0.1], rng.uniform(0.0, 0.2, P - 1)])
    v = speed[:, None] * n
    G = 0.99 * np.exp(-0.5 * ((eps[None, :] - 2.0 * T[:, None]) / 10.0) ** 2)
    D = np.repeat((0.5 * G)[:, None, :], 3, axis=1)
    I = np.zeros((P, 3, 3, m.nq))
    I[:, :, :, :] = (0.25 * G)[:, None, None, :] * n[:, None, :, None]
    e = 1.5 * T * (1.0 + ye) + 3.0 * ye ** (4.0 / 3.0) * np.cbrt(rho)
    ef = e + 0.5 * MC2 * speed ** 2
    return m, D, I, rho, ye, ef, v


def _totals(m, D, I, ye, ef, v, rho):
    """Matter plus neutrino lepton number, energy and momentum per baryon
    (Eulerian neutrino integrals at the given velocity)."""
    g = np.array([1.0, -1.0, 0.0])
    d = np.array([1.0, 1.0, 4.0])
    K = m.c.kcoup / rho
    vI = np.einsum("pj,psjq->psq", v, I)
    N = np.einsum("s,q,psq->p", g, m.w2, D + vI)
    E = np.einsum("s,q,psq->p", d, m.w3, D + 2 * vI)
    P_, ns, nq = D.shape
    F = np.zeros((P_, 3))
    for p in range(P_):
        for s in range(ns):
            for q in range(nq):
                F[p] += d[s] * m.w3[q] * (I[p, s, :, q] + v[p] * D[p, s, q] + O.eddington(D[p, s, q], I[p, s, :, q]) @ v[p])
    return ye + K * N, ef + K * E, v + (K / MC2)[:, None] * F


def test_relaxation_chain():
    print("[case] O(v) relaxation problem, 32 points, 12 steps of 0.5 km", flush=True)
    import torch
    P = 32
    m, D, I, rho, ye, ef, v = _initial(P)
    th = np.concatenate([np.ones(32), [PT.A_NES, PT.A_PAIR]])
    gm = S.Model(S.Grid())
    f = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    gD, gI, grho, gye, gef, gv, gth = f(D), f(I), f(rho), f(ye), f(ef), f(v), f(th)
    out = S.alloc_outputs_v(gm, P)
    out.update(D=gD, I=gI, ye=gye, ef=gef, v=gv)
    L0 = _totals(m, D, I, ye, ef, v, rho)
    oD, oI, oye, oef, ov = D, I, ye, ef, v
    for k in range(STEPS):
        r = O.solve_batch_v(m, O.Params(**PRM), th, DTAU, oD, oI, rho, oye, oef, ov)
        oD, oI, oye, oef, ov = r["D"], r["I"], r["ye"], r["ef"], r["v"]
        S.solve_v(gm, S.Params(**PRM), DTAU, gD, gI, grho, gye, gef, gv, gth, out=out)
        torch.cuda.synchronize()
        got = {key: x.cpu().numpy() for key, x in out.items()}
        assert np.all(r["status"] == 0) and np.all(got["status"] == 0), k
        eD, eI, eY, eE, eV = PT.parity_errors_v(r, got, m.w2, m.w3, m.c.kcoup, rho)
        worst = max(eD.max(), eI.max(), eY.max(), eE.max(), eV.max())
        print(f"step {k}: n_inner max {got['n_inner'].max()}, worst parity {worst:.2e}", flush=True)
        assert worst <= 1e-9 * (k + 1), k
    # conservation over the chain (the output matter state is the matter
    # right-hand side at the final moments: exact up to the solver tolerance)
    L1 = _totals(m, got["D"], got["I"], got["ye"], got["ef"], got["v"], rho)
    assert np.max(np.abs(L1[0] - L0[0]) / np.abs(L0[0])) <= 1e-8
    assert np.max(np.abs(L1[1] - L0[1]) / np.abs(L0[1])) <= 1e-8
    vs = np.maximum(np.linalg.norm(L0[2], axis=1), 1e-3)
    assert np.max(np.abs(L1[2] - L0[2]) / vs[:, None]) <= 1e-8
    # relaxed: Fermi-Dirac number moments at the final matter state, no flux
    e_int = got["ef"] - 0.5 * MC2 * np.sum(got["v"] ** 2, axis=1)
    T = (e_int - 3.0 * got["ye"] ** (4.0 / 3.0) * np.cbrt(rho)) / (1.5 * (1.0 + got["ye"]))
    assert np.allclose(T, got["T"], rtol=1e-12)
    mu = 20.0 * (got["ye"] - 0.3) * np.cbrt(rho) + 5.0 * np.log(T / 5.0)
    sgn = np.array([1.0, -1.0, 0.0])
    x = (m.eps[None, None, :] - sgn[None, :, None] * mu[:, None, None]) / T[:, None, None]
    deq = 1.0 / (np.exp(x) + 1.0)
    rel = PT.wnorm(got["D"] - deq, m.w2) / PT.wnorm(deq, m.w2)
    flux = np.sqrt(np.sum(m.w2 * got["I"] ** 2, axis=(-2, -1))) / PT.wnorm(got["D"], m.w2)
    print(f"after {STEPS} steps: max |D - D_eq| / |D_eq| {rel.max():.2e}, max |I| / |D| {flux.max():.2e}", flush=True)
    # the electron flavours equilibrate through emission and absorption; the
    # heavy-lepton stand-in has no absorption, and NES conserves its number,
    # so only the slower pair processes bring it to its equilibrium
    D0rel = PT.wnorm(D - deq, m.w2) / PT.wnorm(deq, m.w2)
    assert np.all(rel[:, :2] < 1e-3 * D0rel[:, :2])
    assert flux.max() < 1e-3
