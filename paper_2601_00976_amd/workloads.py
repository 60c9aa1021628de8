"""Seeded synthetic input draws for the coupling-solve workloads.

This module holds random draws only (no physics): point densities,
temperatures, electron fractions, chemical potentials, opacity scales and the
uniform noise arrays from which an initial neutrino state is built.  Turning a
draw into a state (equation of state, Fermi-Dirac equilibrium) is done by the
consumer.  The draws stand in for the paper's tabulated microphysics and
supernova profiles, which are not available: the shapes follow the paper's
production setup (32 energy nodes, Sec. 7.1) reduced to three species.

Every generator is deterministic in (workload id, seed) through
``numpy.random.default_rng([wid, seed])``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

DTAU_KM = 1.0e-3  # implicit step length c*dt in km


@dataclass
class Draws:
    """Raw draws for P points; arrays are float64 and C-contiguous."""

    T: np.ndarray             # (P,) MeV
    rho11: np.ndarray         # (P,) density in 1e11 g/cm^3
    ye: np.ndarray            # (P,) electron fraction
    uD: np.ndarray            # (P, ns, nq) noise for the number moments
    uI: np.ndarray            # (P, ns, nq) noise in [-1, 1) for the flux moments
    mu: np.ndarray | None = None    # (P,) prescribed nu_e chemical potential (fixed matter)
    chi0: np.ndarray | None = None  # (P,) prescribed absorption scale, 1/km
    r_km: np.ndarray | None = None  # (P,) radius for profile workloads
    a: float = 1.0            # D* = clip(D_eq (a + b uD))
    b: float = 0.1
    c: float = 0.1            # I* = c D* uI
    v: np.ndarray | None = None    # (P, 3) fluid velocity [c] (O(v) workloads)
    uI3: np.ndarray | None = None  # (P, ns, 3, nq) noise in [-1, 1) for three flux components

    @property
    def P(self):
        return len(self.T)

    def take(self, idx):
        idx = np.asarray(idx)
        sel = lambda x: None if x is None else np.ascontiguousarray(x[idx])
        return Draws(sel(self.T), sel(self.rho11), sel(self.ye), sel(self.uD), sel(self.uI),
                     sel(self.mu), sel(self.chi0), sel(self.r_km), self.a, self.b, self.c,
                     sel(self.v), sel(self.uI3))


def emab_iso_fixed(P: int = 1000, ns: int = 2, nq: int = 32, seed: int = 0) -> Draws:
    """Emission/absorption + isoenergetic scattering at fixed matter.

    chi0 ~ LogUniform(1e-3, 1e2) /km, T ~ U(2, 20) MeV, mu ~ U(-10, 20) MeV,
    D* = U(0, 1) D_eq, I* = 0.1 D* U(-1, 1)."""
    rng = np.random.default_rng([1, seed])
    chi0 = 10.0 ** rng.uniform(-3.0, 2.0, P)
    T = rng.uniform(2.0, 20.0, P)
    mu = rng.uniform(-10.0, 20.0, P)
    uD = rng.uniform(0.0, 1.0, (P, ns, nq))
    uI = rng.uniform(-1.0, 1.0, (P, ns, nq))
    rho11 = np.ones(P)
    ye = np.full(P, 0.3)
    return Draws(T, rho11, ye, uD, uI, mu=mu, chi0=chi0, a=0.0, b=1.0, c=0.1)


def uniform_box(P: int = 4096, ns: int = 3, nq: int = 32, seed: int = 0) -> Draws:
    """Full coupled solve on a box of matter states.

    rho11 ~ LogUniform(1e-3, 10), T ~ U(2, 40) MeV, Ye ~ U(0.1, 0.5),
    D* = clip(D_eq (1 + 0.1 U(-1, 1))), I* = 0.1 D* U(-1, 1)."""
    rng = np.random.default_rng([2, seed])
    rho11 = 10.0 ** rng.uniform(-3.0, 1.0, P)
    T = rng.uniform(2.0, 40.0, P)
    ye = rng.uniform(0.1, 0.5, P)
    uD = rng.uniform(-1.0, 1.0, (P, ns, nq))
    uI = rng.uniform(-1.0, 1.0, (P, ns, nq))
    return Draws(T, rho11, ye, uD, uI)


def radial_profile(P: int = 1 << 16, ns: int = 3, nq: int = 32, seed: int = 0, wid: int = 3) -> Draws:
    """Supernova-like radial profile: r_i = 300 i / (P-1) km,
    rho11 = 10 exp(-r/20) exp(0.05 Z1), T = 30 exp(-r/50) exp(0.05 Z2) MeV,
    Ye ~ U(0.1, 0.5), near-equilibrium neutrinos as in ``uniform_box``."""
    rng = np.random.default_rng([wid, seed])
    r = 300.0 * np.arange(P, dtype=np.float64) / max(P - 1, 1)
    z1 = rng.standard_normal(P)
    z2 = rng.standard_normal(P)
    rho11 = 10.0 * np.exp(-r / 20.0) * np.exp(0.05 * z1)
    T = 30.0 * np.exp(-r / 50.0) * np.exp(0.05 * z2)
    ye = rng.uniform(0.1, 0.5, P)
    uD = rng.uniform(-1.0, 1.0, (P, ns, nq))
    uI = rng.uniform(-1.0, 1.0, (P, ns, nq))
    return Draws(T, rho11, ye, uD, uI, r_km=r)


def radial_profile_v(P: int = 1 << 16, ns: int = 3, nq: int = 32, seed: int = 0, wid: int = 6) -> Draws:
    """The radial profile of ``radial_profile`` with fluid motion, for the
    O(v) solve: every point sits at its radius in a random direction n (uniform
    on the sphere) and moves with v = v_r(r) n + 0.005 Z3 (c units),
    v_r = -0.1 (1 - exp(-r/50)) (infall that vanishes at the centre); the
    three flux components get independent noise (I*_j = 0.1 D* uI3_j)."""
    d = radial_profile(P, ns, nq, seed, wid)
    rng = np.random.default_rng([wid, seed, 1])
    n = rng.standard_normal((P, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    vr = -0.1 * (1.0 - np.exp(-d.r_km / 50.0))
    d.v = np.ascontiguousarray(vr[:, None] * n + 0.005 * rng.standard_normal((P, 3)))
    d.uI3 = rng.uniform(-1.0, 1.0, (P, ns, 3, nq))
    return d


def fd_sample(P_total: int, n: int, seed: int = 0) -> np.ndarray:
    """Indices of n points drawn without replacement, for finite-difference checks."""
    rng = np.random.default_rng([5, seed])
    return np.sort(rng.choice(P_total, size=n, replace=False))
