"""Pins of the oracle's O(v) solve (nonzero fluid velocity) against what the
paper and the mathematics fix, independently of the oracle's own code:

* the Minerbo closure (Eqs. eddingtonFactorMinerbo, eddingtonTensor) against
  its limits, the trace and eigen-structure of the Eddington tensor, and the
  exact Maxwell-Boltzmann maximum-entropy closure it approximates;
* the solve at dtau = 0 (the old state is the exact solution), at equilibrium
  with motion (isotropic Fermi-Dirac moments are a fixed point for any v), and
  at v = 0 without flux (it reduces to the zero-velocity solve);
* the definition of the result: the unrearranged implicit equations
  (Eqs. implicitNumberNodal, implicitNumberFluxNodal, implicitFluidNodal with
  eulerianMomentumLG, eulerianEnergyLG, eulerianNumberLG) hold at the solution,
  and dense Newton on them from the old state reaches the same root.
"""
from __future__ import annotations

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle as O

THETA_A = 1e-7
MC2 = O.MU_C2


def test_minerbo_limits_and_max_entropy():
    assert O.minerbo_psi(0.0) == pytest.approx(1.0 / 3.0, abs=1e-16)
    assert O.minerbo_psi(1.0) == pytest.approx(1.0, abs=1e-15)
    hs = np.linspace(0.0, 1.0, 201)
    ps = np.array([O.minerbo_psi(h) for h in hs])
    assert np.all(np.diff(ps) > 0)
    # Maxwell-Boltzmann maximum entropy: f ~ exp(Z mu), h = coth Z - 1/Z,
    # psi = 1 - 2 h / Z; the polynomial fits it to about half a percent
    lang = lambda z: 1.0 / np.tanh(z) - 1.0 / z
    for h in np.linspace(0.02, 0.98, 49):
        Z = brentq(lambda z: lang(z) - h, 1e-8, 1e4)
        assert abs((1.0 - 2.0 * h / Z) - O.minerbo_psi(h)) < 6e-3
    # flux factor: zero without flux, limited to 1
    assert O.flux_factor(1.0, 0.0) == 0.0
    assert O.flux_factor(0.5, 0.25) == 0.5
    assert O.flux_factor(0.5, 0.75) == 1.0
    assert O.flux_factor(0.0, 0.1) == 1.0


def test_eddington_tensor_structure():
    rng = np.random.default_rng(11)
    for _ in range(50):
        D = rng.uniform(0.01, 1.0)
        I3 = rng.uniform(-1, 1, 3)
        I3 *= rng.uniform(0.0, 1.0) * D / np.linalg.norm(I3)
        K = O.eddington(D, I3)
        h = np.linalg.norm(I3) / D
        n = I3 / np.linalg.norm(I3)
        psi = O.minerbo_psi(h)
        assert np.allclose(K, K.T, rtol=0, atol=1e-16)
        assert np.trace(K) == pytest.approx(D, rel=1e-14)           # trace condition
        assert np.allclose(K @ n, psi * D * n, rtol=1e-13, atol=0)  # psi = n.k.n along the flux
        e = np.cross(n, rng.standard_normal(3))
        e /= np.linalg.norm(e)
        assert np.allclose(K @ e, 0.5 * (1 - psi) * D * e, rtol=1e-12, atol=1e-16)
    # isotropic and free-streaming limits
    assert np.allclose(O.eddington(0.7, np.zeros(3)), 0.7 / 3.0 * np.eye(3), rtol=1e-15, atol=0)
    n = np.array([0.6, 0.0, 0.8])
    assert np.allclose(O.eddington(0.7, 0.7 * n), 0.7 * np.outer(n, n), rtol=0, atol=1e-15)


def _state(P, nq_elem=16, seed=3, v_scale=0.1, eq=False, zero_flux=False):
    m = O.Model(n_elem=nq_elem)
    rng = np.random.default_rng([77, seed])
    rho = 10.0 ** rng.uniform(-1.0, 1.0, P)
    T = rng.uniform(5.0, 30.0, P)
    ye = rng.uniform(0.15, 0.45, P)
    uD = rng.uniform(-1, 1, (P, m.ns, m.nq))
    D0, _, e0 = m.init_state(T, rho, ye, uD, uD, a=1.0, b=0.0 if eq else 0.1, c=0.0)
    I0 = 0.0 if (eq or zero_flux) else 0.1 * D0[:, :, None, :] * rng.uniform(-1, 1, (P, m.ns, 3, m.nq))
    I0 = np.zeros((P, m.ns, 3, m.nq)) + I0
    v = v_scale * rng.uniform(-1, 1, (P, 3)) / np.sqrt(3.0)
    ef0 = e0 + 0.5 * MC2 * np.sum(v * v, axis=1)
    return m, rho, ye, D0, I0, e0, ef0, v


def test_dtau_zero_returns_old_state():
    m, rho, ye, D0, I0, e0, ef0, v = _state(64)
    th = m.default_theta(THETA_A, THETA_A)
    r = O.solve_batch_v(m, O.Params(), th, 0.0, D0, I0, rho, ye, ef0, v)
    assert np.all(r["status"] == O.OK) and np.all(r["n_outer"] == 1)
    assert np.allclose(r["D"], D0, rtol=1e-14, atol=1e-300)
    assert np.allclose(r["I"], I0, rtol=1e-13, atol=1e-15 * np.max(np.abs(D0)))
    assert np.allclose(r["ye"], ye, rtol=1e-14, atol=0)
    assert np.allclose(r["ef"], ef0, rtol=1e-14, atol=0)
    assert np.allclose(r["v"], v, rtol=1e-12, atol=1e-16)


def test_moving_equilibrium_is_fixed_point():
    m, rho, ye, D0, I0, e0, ef0, v = _state(64, eq=True)
    th = m.default_theta(THETA_A, THETA_A)
    r = O.solve_batch_v(m, O.Params(), th, 1e-3, D0, I0, rho, ye, ef0, v)
    assert np.all(r["status"] == O.OK)
    dn = np.sqrt(np.sum(m.w2 * D0 * D0, axis=-1))
    assert np.max(np.sqrt(np.sum(m.w2 * (r["D"] - D0) ** 2, axis=-1)) / dn) < 1e-12
    assert np.array_equal(r["I"], I0)
    assert np.allclose(r["ye"], ye, rtol=1e-12, atol=0)
    assert np.allclose(r["ef"], ef0, rtol=1e-12, atol=0)
    assert np.allclose(r["v"], v, rtol=1e-12, atol=0)


def test_zero_velocity_without_flux_reduces_to_static_solve():
    m, rho, ye, D0, I0, e0, ef0, v = _state(48, zero_flux=True, v_scale=0.0)
    th = m.default_theta(THETA_A, THETA_A)
    prm = O.Params(tol_inner=1e-13, tol_outer=1e-13, max_outer=200)
    r = O.solve_batch_v(m, prm, th, 1e-3, D0, I0, rho, ye, e0, v)
    s = O.solve_batch(m, prm, th, 1e-3, D0, np.zeros_like(D0), rho, ye, e0)
    # the matter update sums the Eulerian integrals before differencing them,
    # the static solve sums the differences: equal up to rounding order, which
    # can move an iteration count and so the result within the tolerance
    assert np.array_equal(r["status"], s["status"])
    dn = np.sqrt(np.sum(m.w2 * s["D"] ** 2, axis=-1))
    eD = np.sqrt(np.sum(m.w2 * (r["D"] - s["D"]) ** 2, axis=-1)) / dn
    assert np.max(eD) < 1e-11 and np.median(eD) < 1e-13
    assert np.allclose(r["ye"], s["ye"], rtol=1e-10, atol=0) and np.allclose(r["ef"], s["e"], rtol=1e-10, atol=0)
    assert not np.any(r["I"]) and not np.any(r["v"])


# ---- definition of the result -------------------------------------------

def _closure(D, I3):
    """Eddington tensor times D from the paper's formulas (test-side copy of
    the definition: Eqs. eddingtonFactorMinerbo, eddingtonTensor)."""
    a = np.linalg.norm(I3)
    h = 0.0 if a == 0 else (1.0 if D <= 0 else min(a / D, 1.0))
    psi = 1 / 3 + 2 / 15 * (3 - h + 3 * h * h) * h * h
    n = I3 / a if a > 0 else np.zeros(3)
    return D * (0.5 * (1 - psi) * np.eye(3) + 0.5 * (3 * psi - 1) * np.outer(n, n))


def _eulerian(m, D, I, v):
    g = np.array([1.0, -1.0, 0.0])
    d = np.array([1.0, 1.0, 4.0])
    N = E = 0.0
    F = np.zeros(3)
    for s in range(m.ns):
        for q in range(m.nq):
            I3 = I[s, :, q]
            K = _closure(D[s, q], I3)
            N += g[s] * m.w2[q] * (D[s, q] + v @ I3)
            E += d[s] * m.w3[q] * (D[s, q] + 2 * v @ I3)
            F += d[s] * m.w3[q] * (I3 + v * D[s, q] + K @ v)
    return N, E, F


def _residual(m, th, dtau, rho, Ds, Is, ys, efs, vs, x):
    ns, nq = m.ns, m.nq
    D = x[: ns * nq].reshape(ns, nq)
    I = x[ns * nq: 4 * ns * nq].reshape(ns, 3, nq)
    ye, ef, v = x[-5], x[-4], x[-3:]
    T = m.eos_temperature(ef - 0.5 * MC2 * (v @ v), ye, rho)
    mu = m.eos_mu(ye, T, rho)
    eta, chi, kap = m.rates(th, rho, 10.0 * rho, T, mu, D)
    RD = np.zeros((ns, nq))
    RI = np.zeros((ns, 3, nq))
    for s in range(ns):
        for q in range(nq):
            Ns = Ds[s, q] + vs @ Is[s, :, q]
            Gs = Is[s, :, q] + _closure(Ds[s, q], Is[s, :, q]) @ vs
            RD[s, q] = D[s, q] + v @ I[s, :, q] - Ns - dtau * (eta[s, q] - chi[s, q] * D[s, q])
            RI[s, :, q] = I[s, :, q] + _closure(D[s, q], I[s, :, q]) @ v - Gs + dtau * kap[s, q] * I[s, :, q]
    K = m.c.kcoup / rho
    N1, E1, F1 = _eulerian(m, D, I, v)
    N0, E0, F0 = _eulerian(m, Ds, Is, vs)
    Ry = ye - ys + K * (N1 - N0)
    Re = ef - efs + K * (E1 - E0)
    Rv = v - vs + K / MC2 * (F1 - F0)
    return np.concatenate([RD.ravel(), RI.ravel(), [Ry, Re], Rv])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_definition_residual_and_newton(seed):
    m = O.Model(n_elem=2, eps_lo=2.0, eps_hi=60.0)  # 4 energy nodes, 3 species: 53 unknowns
    rng = np.random.default_rng([78, seed])
    rho = np.array([rng.uniform(0.3, 3.0)])
    T = np.array([rng.uniform(6.0, 15.0)])
    ye = np.array([rng.uniform(0.2, 0.4)])
    uD = rng.uniform(-1, 1, (1, m.ns, m.nq))
    D0, _, e0 = m.init_state(T, rho, ye, uD, uD, a=1.0, b=0.3, c=0.0)
    I0 = 0.3 * D0[:, :, None, :] * rng.uniform(-1, 1, (1, m.ns, 3, m.nq))
    v = np.array([[0.12, -0.05, 0.03]]) * rng.uniform(0.5, 1.5)
    ef0 = e0 + 0.5 * MC2 * np.sum(v * v, axis=1)
    th = m.default_theta(1e-6, 1e-6)
    dtau = 0.05
    r = O.solve_batch_v(m, O.Params(tol_inner=1e-14, tol_outer=1e-14, max_inner=400, max_outer=400), th, dtau,
                        D0, I0, rho, ye, ef0, v)
    assert r["status"][0] == O.OK
    args = (m, th, dtau, rho[0], D0[0], I0[0], ye[0], ef0[0], v[0])
    x_ora = np.concatenate([r["D"][0].ravel(), r["I"][0].ravel(), [r["ye"][0], r["ef"][0]], r["v"][0]])
    scale = np.concatenate([np.full(m.ns * m.nq * 4, np.max(D0)), [ye[0], ef0[0]], np.full(3, 0.1)])
    R = _residual(*args, x_ora)
    assert np.max(np.abs(R) / scale) < 1e-10
    # the solve moved the state well beyond that residual
    x0 = np.concatenate([D0[0].ravel(), I0[0].ravel(), [ye[0], ef0[0]], v[0]])
    assert np.max(np.abs(x_ora - x0) / scale) > 1e-4
    # dense Newton (finite-difference Jacobian) on the unrearranged equations
    x = x0.copy()
    for _ in range(30):
        R = _residual(*args, x)
        if np.max(np.abs(R) / scale) < 1e-14:
            break
        J = np.zeros((len(x), len(x)))
        for j in range(len(x)):
            hj = 1e-7 * max(abs(x[j]), scale[j] * 1e-3)
            xp, xm = x.copy(), x.copy()
            xp[j] += hj
            xm[j] -= hj
            J[:, j] = (_residual(*args, xp) - _residual(*args, xm)) / (2 * hj)
        x = x - np.linalg.solve(J, R)
    assert np.max(np.abs(_residual(*args, x)) / scale) < 1e-13
    assert np.max(np.abs(x - x_ora) / scale) < 1e-10
