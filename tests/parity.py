"""Shared helpers of the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W

A_NES = S.DEFAULT_A_NES
A_PAIR = S.DEFAULT_A_PAIR


def oracle_model(ns_species, flags, n_elem=16, **ov):
    return O.Model(n_elem=n_elem, species=tuple(ns_species), flags=flags, overrides=ov)


def run_oracle(draws: W.Draws, species, flags, dtau, params: O.Params, theta, n_elem=16, **ov):
    m = oracle_model(species, flags, n_elem, **ov)
    D0, I0, e0 = m.init_state(draws.T, draws.rho11, draws.ye, draws.uD, draws.uI, draws.a, draws.b, draws.c,
                              mu=draws.mu)
    fixedT = params.fixed_matter and draws.mu is not None
    r = O.solve_batch(m, params, theta, dtau, D0, I0, draws.rho11, draws.ye, e0, chi0=draws.chi0,
                      T_fixed=draws.T if fixedT else None, mu_fixed=draws.mu if fixedT else None)
    r["D0"], r["I0"], r["e0"] = D0, I0, e0
    return m, r


def run_gpu(draws: W.Draws, species, flags, dtau, params: S.Params, theta_np, n_elem=16, launch=None, **ov):
    import torch
    g = S.Grid(n_elem=n_elem)
    m = S.Model(g, species=tuple(species), flags=flags, **ov)
    t = S.to_device(draws)
    D0, I0, e0 = S.init_state(m, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"], draws.a, draws.b, draws.c,
                              mu=t["mu"])
    theta = torch.as_tensor(theta_np, dtype=torch.float64, device="cuda")
    fixedT = params.fixed_matter and draws.mu is not None
    out = S.solve(m, params, dtau, D0, I0, t["rho11"], t["ye"], e0, theta, chi0=t["chi0"],
                  T_fixed=t["T"] if fixedT else None, mu_fixed=t["mu"] if fixedT else None, launch=launch)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["D0"], res["I0"], res["e0"] = D0.cpu().numpy(), I0.cpu().numpy(), e0.cpu().numpy()
    return m, res


def wnorm(x, w2):
    return np.sqrt(np.sum(w2 * x * x, axis=-1))


def parity_errors(ref, got, w2):
    """Per point and species W-weighted relative errors of D and I (reference
    ||D||), and relative errors of Ye and e."""
    dref = wnorm(ref["D"], w2)
    scale = np.where(dref > 0, dref, 1.0)
    eD = wnorm(got["D"] - ref["D"], w2) / scale
    eI = wnorm(got["I"] - ref["I"], w2) / scale
    eY = np.abs(got["ye"] - ref["ye"]) / np.abs(ref["ye"])
    eE = np.abs(got["e"] - ref["e"]) / np.abs(ref["e"])
    return eD, eI, eY, eE


def reservoir_ratios(kcoup, rho11, D, ye, e, w2, w3, species=(0, 1, 2)):
    """Neutrino-to-matter ratios of lepton number and energy per point.  The
    output matter state is recomputed from the final moments, so a relative
    error tol in the moments becomes tol * ratio in Ye and e."""
    g = np.array([[1.0, 1.0, 0.0][s] for s in species])[None, :, None]
    mult = np.array([[1.0, 1.0, 4.0][s] for s in species])[None, :, None]
    K = kcoup / rho11
    RY = K * np.sum(g * w2 * D, axis=(1, 2)) / np.abs(ye)
    RE = K * np.sum(mult * w3 * D, axis=(1, 2)) / np.abs(e)
    return RY, RE


# ---- O(v) solve (nonzero fluid velocity) ------------------------------------

def run_oracle_v(draws: W.Draws, dtau, params: O.Params, theta, c=0.1, species=(0, 1, 2), flags=O.ALL_PHYSICS):
    m = O.Model(species=tuple(species), flags=flags)
    D0, _, e0 = m.init_state(draws.T, draws.rho11, draws.ye, draws.uD, draws.uI)
    I0 = c * D0[:, :, None, :] * draws.uI3
    ef0 = e0 + 0.5 * O.MU_C2 * np.sum(draws.v * draws.v, axis=1)
    r = O.solve_batch_v(m, params, theta, dtau, D0, I0, draws.rho11, draws.ye, ef0, draws.v)
    r["D0"], r["I0"], r["ef0"] = D0, I0, ef0
    return m, r


def run_gpu_v(draws: W.Draws, dtau, params: S.Params, theta_np, launch=None, inplace=False, species=(0, 1, 2),
              flags=O.ALL_PHYSICS):
    import torch
    m = S.Model(S.Grid(), species=tuple(species), flags=flags)
    t = S.to_device(draws)
    D0, I0, ef0 = S.init_state_v(m, t)
    theta = torch.as_tensor(theta_np, dtype=torch.float64, device="cuda")
    keep = dict(D0=D0.cpu().numpy(), I0=I0.cpu().numpy(), ef0=ef0.cpu().numpy())
    out = None
    if inplace:
        P = D0.shape[0]
        i32 = dict(dtype=torch.int32, device="cuda")
        out = dict(D=D0, I=I0, ye=t["ye"], ef=ef0, v=t["v"], T=torch.empty_like(ef0),
                   n_outer=torch.empty(P, **i32), n_inner=torch.empty(P, **i32), status=torch.empty(P, **i32))
    out = S.solve_v(m, params, dtau, D0, I0, t["rho11"], t["ye"], ef0, t["v"], theta, out=out, launch=launch)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res.update(keep)
    return m, res


def parity_errors_v(ref, got, w2, w3, kcoup, rho11, species=None):
    """Per point and species W-weighted relative errors of D and of the flux
    vector (reference ||D||); Ye and ef relative errors divided by the
    neutrino/matter reservoir ratio (at least 1); velocity errors relative to
    the larger of |v| and the neutrino momentum scale K / (m_u c^2) sum W3 D."""
    dref = wnorm(ref["D"], w2)
    scale = np.where(dref > 0, dref, 1.0)
    eD = wnorm(got["D"] - ref["D"], w2) / scale
    dI = got["I"] - ref["I"]
    eI = np.sqrt(np.sum(w2 * dI * dI, axis=(-2, -1))) / scale
    sp = species if species is not None else (0, 1, 2)
    mult = np.array([[1.0, 1.0, 4.0][s] for s in sp])[None, :, None]
    g = np.array([[1.0, 1.0, 0.0][s] for s in sp])[None, :, None]
    K = kcoup / rho11
    RY = np.maximum(K * np.sum(g * w2 * ref["D"], axis=(1, 2)) / np.abs(ref["ye"]), 1.0)
    RE = np.maximum(K * np.sum(mult * w3 * ref["D"], axis=(1, 2)) / np.abs(ref["ef"]), 1.0)
    eY = np.abs(got["ye"] - ref["ye"]) / np.abs(ref["ye"]) / RY
    eE = np.abs(got["ef"] - ref["ef"]) / np.abs(ref["ef"]) / RE
    vs = np.maximum(np.linalg.norm(ref["v"], axis=1), K / O.MU_C2 * np.sum(mult * w3 * ref["D"], axis=(1, 2)))
    eV = np.max(np.abs(got["v"] - ref["v"]), axis=1) / vs
    return eD, eI, eY, eE, eV
