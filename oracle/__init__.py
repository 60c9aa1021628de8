"""Test infrastructure, not product code.

ctypes front end of the plain FP64 CPU oracle (``nmc_oracle.c``) of the
implicit neutrino-matter coupling solve (paper Sec. 3.5).  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_nmc.so")
SRC = os.path.join(HERE, "nmc_oracle.c")
TALLY_PATH = os.path.join(HERE, "liboracle_tally.so")
TALLY_SRC = os.path.join(HERE, "flop_tally.cpp")

MAX_NQ = 64
MAX_NS = 3
NU_E, NU_E_BAR, NU_X = 0, 1, 2
EMAB, ISO, NES, PAIR = 1, 2, 4, 8
ALL_PHYSICS = EMAB | ISO | NES | PAIR
OK, MAX_OUTER, MAX_INNER, NONFINITE, EOS_DOMAIN = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP over points)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c99", "-Wall",
               "-shared", "-fPIC", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Model(C.Structure):
    _fields_ = [
        ("nq", C.c_int), ("ns", C.c_int), ("species", C.c_int * MAX_NS),
        ("eps", C.c_double * MAX_NQ), ("w2", C.c_double * MAX_NQ), ("w3", C.c_double * MAX_NQ),
        ("flags", C.c_uint),
        ("chi_ref", C.c_double), ("eps_ref", C.c_double), ("chi_power", C.c_double),
        ("sigma_ratio", C.c_double),
        ("eos_a", C.c_double), ("eos_b", C.c_double), ("mu_a", C.c_double), ("mu_ye0", C.c_double),
        ("mu_b", C.c_double), ("mu_t0", C.c_double),
        ("kcoup", C.c_double), ("rho11_min", C.c_double),
        ("phi1_nes", C.c_double), ("phi1_pair", C.c_double),
        ("fd_projection", C.c_int), ("deq_min", C.c_double), ("deq_max", C.c_double),
        ("edges", C.c_double * (MAX_NQ // 2 + 1)),
    ]


class _Params(C.Structure):
    _fields_ = [
        ("tol_inner", C.c_double), ("tol_outer", C.c_double),
        ("m_inner", C.c_int), ("m_outer", C.c_int), ("max_inner", C.c_int), ("max_outer", C.c_int),
        ("fixed_matter", C.c_int),
    ]


def build_tally(force: bool = True) -> str:
    """Compile the counting build of the oracle (flop_tally.cpp: the same
    source with every double replaced by an operation-counting wrapper)."""
    if force or not os.path.exists(TALLY_PATH):
        tmp = TALLY_PATH + ".tmp"
        cmd = ["g++", "-O2", "-ffp-contract=off", "-fopenmp", "-fpermissive", "-std=c++17", "-w",
               "-shared", "-fPIC", TALLY_SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, TALLY_PATH)
    return TALLY_PATH


_lib = None
_tally = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _load(LIB_PATH)
    return _lib


def tally_lib():
    """The counting build (same C ABI, plus ora_tally_read / ora_tally_reset)."""
    global _tally
    if _tally is None:
        if not os.path.exists(TALLY_PATH):
            build_tally()
        L = _load(TALLY_PATH)
        L.ora_tally_read.argtypes = [np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")]
        L.ora_tally_reset.argtypes = []
        _tally = L
    return _tally


def _load(path):
    if True:
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        L.ora_grid_loguniform.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp, dp]
        L.ora_grid_zoom.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp, dp]
        L.ora_model_defaults.argtypes = [C.POINTER(_Model)]
        for f in ("ora_fermi_dirac", "ora_fermi_dirac_complement"):
            getattr(L, f).argtypes = [C.c_double] * 3
            getattr(L, f).restype = C.c_double
        for f in ("ora_eos_energy", "ora_eos_temperature", "ora_eos_mu"):
            getattr(L, f).argtypes = [C.POINTER(_Model), C.c_double, C.c_double, C.c_double]
            getattr(L, f).restype = C.c_double
        L.ora_kernels.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.ora_rates.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                dp, dp, dp, dp]
        L.ora_anderson.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.ora_anderson.restype = C.c_int
        L.ora_solve_batch.argtypes = [C.POINTER(_Model), C.POINTER(_Params), dp, C.c_long, C.c_double,
                                      dp, dp, dp, dp, dp, vp, vp, vp,
                                      dp, dp, dp, dp, dp, ip, ip, ip, C.c_int]
        L.ora_residual.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, C.c_double,
                                   dp, dp, C.c_double, C.c_double, dp, dp, C.c_double, C.c_double, dp]
        L.ora_jacobian.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, C.c_double,
                                   dp, C.c_double, C.c_double, dp]
        L.ora_newton.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, C.c_double,
                                 dp, dp, C.c_double, C.c_double, dp, dp,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_int]
        L.ora_newton.restype = C.c_int
        L.ora_adjoint_batch.argtypes = [C.POINTER(_Model), dp, C.c_long, C.c_double, dp, vp,
                                        dp, dp, dp, dp, dp, vp, C.c_int]
        L.ora_adjoint_batch.restype = C.c_int
        L.ora_init_state.argtypes = [C.POINTER(_Model), C.c_long, dp, vp, dp, dp, dp, dp,
                                     C.c_double, C.c_double, C.c_double, dp, dp, vp]
        L.ora_minerbo_psi.argtypes = [C.c_double]
        L.ora_minerbo_psi.restype = C.c_double
        L.ora_flux_factor.argtypes = [C.c_double, C.c_double]
        L.ora_flux_factor.restype = C.c_double
        L.ora_eddington.argtypes = [C.c_double, dp, dp]
        L.ora_primitive_batch.argtypes = [C.POINTER(_Model), C.c_long, dp, dp, dp, C.c_int, C.c_double, C.c_int,
                                          dp, dp, ip, C.c_int]
        L.ora_pdars_step_v.argtypes = [C.POINTER(_Model), C.POINTER(_Params), dp, C.c_long, C.c_double,
                                       dp, dp, dp, dp, dp, dp, vp, C.c_int, C.c_double, C.c_int,
                                       dp, dp, dp, dp, dp, dp, ip, ip, ip, C.c_int]
        L.ora_gauss_legendre.argtypes = [C.c_int, dp, dp]
        L.ora_gauss_legendre.restype = C.c_int
        L.ora_fd_projection.argtypes = [C.POINTER(_Model), C.c_double, C.c_double, dp, dp, dp]
        L.ora_kernels_odds.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, dp, dp, dp, dp, dp]
        L.ora_phi1_terms.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.ora_solve_batch_v.argtypes = [C.POINTER(_Model), C.POINTER(_Params), dp, C.c_long, C.c_double,
                                        dp, dp, dp, dp, dp, dp, vp,
                                        dp, dp, dp, dp, dp, dp, ip, ip, ip, C.c_int]
    return L


def _vp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# grids

def grid_loguniform(n_elem: int, eps_lo: float = 1.0, eps_hi: float = 300.0, with_edges: bool = False):
    nq = 2 * n_elem
    edges, eps, w2, w3 = np.zeros(n_elem + 1), np.zeros(nq), np.zeros(nq), np.zeros(nq)
    if lib().ora_grid_loguniform(n_elem, eps_lo, eps_hi, edges, eps, w2, w3) != 0:
        raise ValueError("bad grid")
    return (edges, eps, w2, w3) if with_edges else (eps, w2, w3)


def grid_zoom(n_elem: int, zoom: float, width: float = 300.0):
    nq = 2 * n_elem
    edges, eps, w2, w3 = np.zeros(n_elem + 1), np.zeros(nq), np.zeros(nq), np.zeros(nq)
    if lib().ora_grid_zoom(n_elem, zoom, width, edges, eps, w2, w3) != 0:
        raise ValueError("bad grid")
    return edges, eps, w2, w3


# ---------------------------------------------------------------------------
# model

@dataclass
class Model:
    n_elem: int = 16
    eps_lo: float = 1.0
    eps_hi: float = 300.0
    species: tuple = (NU_E, NU_E_BAR, NU_X)
    flags: int = ALL_PHYSICS
    overrides: dict = field(default_factory=dict)
    zoom: float | None = None  # geometric grid of Table energyGrids on [0, eps_hi]

    def __post_init__(self):
        m = _Model()
        lib().ora_model_defaults(C.byref(m))
        if self.zoom:
            edges, eps, w2, w3 = grid_zoom(self.n_elem, self.zoom, self.eps_hi)
        else:
            edges, eps, w2, w3 = grid_loguniform(self.n_elem, self.eps_lo, self.eps_hi, with_edges=True)
        self.set_grid(edges, eps, w2, w3, m)

    def set_grid(self, edges, eps, w2, w3, m=None):
        m = m if m is not None else self.c
        m.nq = len(eps)
        m.ns = len(self.species)
        for i, s in enumerate(self.species):
            m.species[i] = s
        for i in range(len(eps)):
            m.eps[i], m.w2[i], m.w3[i] = eps[i], w2[i], w3[i]
        for i in range(len(edges)):
            m.edges[i] = edges[i]
        m.flags = self.flags
        for k, v in self.overrides.items():
            setattr(m, k, v)
        self.c = m

    @property
    def nq(self):
        return self.c.nq

    @property
    def ns(self):
        return self.c.ns

    @property
    def eps(self):
        return np.array(self.c.eps[: self.nq])

    @property
    def w2(self):
        return np.array(self.c.w2[: self.nq])

    @property
    def w3(self):
        return np.array(self.c.w3[: self.nq])

    @property
    def edges(self):
        return np.array(self.c.edges[: self.nq // 2 + 1])

    def ref(self):
        return C.byref(self.c)

    def default_theta(self, a_nes: float, a_pair: float):
        return np.concatenate([np.ones(self.nq), [a_nes, a_pair]])

    # thermodynamics
    def fd(self, eps, mu, T):
        return lib().ora_fermi_dirac(eps, mu, T)

    def fd_complement(self, eps, mu, T):
        return lib().ora_fermi_dirac_complement(eps, mu, T)

    def eos_energy(self, T, ye, rho11):
        return lib().ora_eos_energy(self.ref(), T, ye, rho11)

    def eos_temperature(self, e, ye, rho11):
        return lib().ora_eos_temperature(self.ref(), e, ye, rho11)

    def eos_mu(self, ye, T, rho11):
        return lib().ora_eos_mu(self.ref(), ye, T, rho11)

    def kernels(self, theta, rho11, T):
        nq = self.nq
        out = [np.zeros(nq * nq) for _ in range(4)]
        lib().ora_kernels(self.ref(), _f64(theta), rho11, T, *out)
        return [o.reshape(nq, nq) for o in out]  # phi_in, phi_out, phi_pro, phi_ann

    def rates(self, theta, rho11, chi0, T, mu, D):
        nn = self.ns * self.nq
        eta, chi, kap = np.zeros(nn), np.zeros(nn), np.zeros(nn)
        lib().ora_rates(self.ref(), _f64(theta), rho11, chi0, T, mu, _f64(D).ravel(), eta, chi, kap)
        shp = (self.ns, self.nq)
        return eta.reshape(shp), chi.reshape(shp), kap.reshape(shp)

    def residual(self, theta, dtau, rho11, chi0, Dstar, Istar, ye_star, e_star, D, I, ye, e):
        nn = self.ns * self.nq
        R = np.zeros(2 * nn + 2)
        lib().ora_residual(self.ref(), _f64(theta), dtau, rho11, chi0, _f64(Dstar).ravel(),
                           _f64(Istar).ravel(), ye_star, e_star, _f64(D).ravel(), _f64(I).ravel(),
                           ye, e, R)
        return R

    def jacobian(self, theta, dtau, rho11, chi0, D, ye, e):
        n = self.ns * self.nq + 2
        J = np.zeros(n * n)
        lib().ora_jacobian(self.ref(), _f64(theta), dtau, rho11, chi0, _f64(D).ravel(), ye, e, J)
        return J.reshape(n, n)

    def newton(self, theta, dtau, rho11, chi0, Dstar, Istar, ye_star, e_star, D0=None, I0=None,
               ye0=None, e0=None, tol=1e-14, max_it=100):
        D = _f64(Dstar if D0 is None else D0).ravel().copy()
        I = _f64(Istar if I0 is None else I0).ravel().copy()
        ye = C.c_double(ye_star if ye0 is None else ye0)
        e = C.c_double(e_star if e0 is None else e0)
        it = lib().ora_newton(self.ref(), _f64(theta), dtau, rho11, chi0, _f64(Dstar).ravel(),
                              _f64(Istar).ravel(), ye_star, e_star, D, I, C.byref(ye), C.byref(e),
                              tol, max_it)
        shp = (self.ns, self.nq)
        return D.reshape(shp), I.reshape(shp), ye.value, e.value, it

    def init_state(self, T, rho11, ye, uD, uI, a=1.0, b=0.1, c=0.1, mu=None):
        T, rho11, ye = _f64(T), _f64(rho11), _f64(ye)
        P = len(T)
        nn = self.ns * self.nq
        D0, I0, e0 = np.zeros(P * nn), np.zeros(P * nn), np.zeros(P)
        mu_arr = None if mu is None else _f64(mu)
        lib().ora_init_state(self.ref(), P, T, _vp(mu_arr), rho11, ye, _f64(uD).ravel(), _f64(uI).ravel(),
                             a, b, c, D0, I0, _vp(e0))
        shp = (P, self.ns, self.nq)
        return D0.reshape(shp), I0.reshape(shp), e0


@dataclass
class Params:
    tol_inner: float = 1e-10
    tol_outer: float = 1e-10
    m_inner: int = 3
    m_outer: int = 3
    max_inner: int = 100
    max_outer: int = 50
    fixed_matter: bool = False

    def c(self):
        return _Params(self.tol_inner, self.tol_outer, self.m_inner, self.m_outer, self.max_inner,
                       self.max_outer, int(self.fixed_matter))


def anderson(Qh, Fh):
    """One Anderson step over a history (oldest first); returns (x_new, columns used)."""
    Qh, Fh = _f64(Qh), _f64(Fh)
    mem, n = Qh.shape
    out = np.zeros(n)
    ncol = lib().ora_anderson(n, mem, Qh.ravel(), Fh.ravel(), out)
    return out, ncol


def solve_batch(model: Model, params: Params, theta, dtau, D0, I0, rho11, ye0, e0, chi0=None,
                T_fixed=None, mu_fixed=None, nthreads: int = 0, library=None):
    """Batched forward solve (Algorithm neutrinoMatterCoupling), one point per item.
    ``library``: the loaded oracle build to run (default lib(); tally_lib()
    for the operation count, with nthreads = 1)."""
    D0 = _f64(D0)
    P = D0.shape[0]
    nn = model.ns * model.nq
    D, I = np.zeros(P * nn), np.zeros(P * nn)
    ye, e, T = np.zeros(P), np.zeros(P), np.zeros(P)
    no, ni, st = np.zeros(P, np.int32), np.zeros(P, np.int32), np.zeros(P, np.int32)
    chi0 = None if chi0 is None else _f64(chi0)
    T_fixed = None if T_fixed is None else _f64(T_fixed)
    mu_fixed = None if mu_fixed is None else _f64(mu_fixed)
    pc = params.c()
    rc = (library or lib()).ora_solve_batch(model.ref(), C.byref(pc), _f64(theta), P, dtau, D0.ravel(),
                               _f64(I0).ravel(), _f64(rho11), _f64(ye0), _f64(e0), _vp(chi0),
                               _vp(T_fixed), _vp(mu_fixed), D, I, ye, e, T, no, ni, st, nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    shp = (P, model.ns, model.nq)
    return dict(D=D.reshape(shp), I=I.reshape(shp), ye=ye, e=e, T=T, n_outer=no, n_inner=ni, status=st)


def flop_tally(model: Model, params: Params, theta, dtau, D0, I0, rho11, ye0, e0):
    """Runs the forward solve through the counting build on one thread and
    returns (result, counts) with counts = {add, mul, div, sqrt, trans}:
    the additions/subtractions, products, quotients, square roots and
    transcendental calls the oracle performed."""
    L = tally_lib()
    L.ora_tally_reset()
    r = solve_batch(model, params, theta, dtau, D0, I0, rho11, ye0, e0, nthreads=1, library=L)
    c = np.zeros(5, dtype=np.uint64)
    L.ora_tally_read(c)
    return r, dict(zip(("add", "mul", "div", "sqrt", "trans"), (int(x) for x in c)))


def adjoint_batch(model: Model, theta, dtau, rho11, D, ye, e, gbar, chi0=None, per_point=False,
                  nthreads: int = 0):
    P = len(rho11)
    nt = model.nq + 2
    g = np.zeros(nt)
    gpp = np.zeros(P * nt) if per_point else None
    chi0 = None if chi0 is None else _f64(chi0)
    rc = lib().ora_adjoint_batch(model.ref(), _f64(theta), P, dtau, _f64(rho11), _vp(chi0),
                                 _f64(D).ravel(), _f64(ye), _f64(e), _f64(gbar).ravel(), g, _vp(gpp),
                                 nthreads)
    if rc != 0:
        raise RuntimeError("singular Jacobian in the oracle adjoint")
    return (g, gpp.reshape(P, nt)) if per_point else g



# ---------------------------------------------------------------------------
# O(v) coupling (nonzero fluid velocity)

MU_C2 = 931.49410242  # atomic mass unit rest energy [MeV]


def minerbo_psi(h: float) -> float:
    return lib().ora_minerbo_psi(h)


def flux_factor(D: float, Imag: float) -> float:
    return lib().ora_flux_factor(D, Imag)


def eddington(D: float, I3) -> np.ndarray:
    K = np.zeros(9)
    lib().ora_eddington(D, _f64(I3), K)
    return K.reshape(3, 3)


def phi1_terms(model: Model, theta, rho11, T, D, I):
    """Linear-order corrections of the NES and pair collision terms at one
    point: (C1D (ns, nq), C1I (ns, 3, nq)) for moments D (ns, nq), I (ns, 3, nq)."""
    ns, nq = model.ns, model.nq
    C1D, C1I = np.zeros(ns * nq), np.zeros(3 * ns * nq)
    lib().ora_phi1_terms(model.ref(), _f64(theta), rho11, T, _f64(D).ravel(), _f64(I).ravel(), C1D, C1I)
    return C1D.reshape(ns, nq), C1I.reshape(ns, 3, nq)


def solve_batch_v(model: Model, params: Params, theta, dtau, D0, I0, rho11, ye0, ef0, v0, chi0=None,
                  nthreads: int = 0):
    """Batched O(v) forward solve.  D0 (P, ns, nq), I0 (P, ns, 3, nq), v0 (P, 3);
    ef0 is the specific fluid energy (internal plus kinetic) [MeV/baryon]."""
    D0 = _f64(D0)
    P = D0.shape[0]
    nn = model.ns * model.nq
    D, I = np.zeros(P * nn), np.zeros(P * 3 * nn)
    ye, ef, v, T = np.zeros(P), np.zeros(P), np.zeros(P * 3), np.zeros(P)
    no, ni, st = np.zeros(P, np.int32), np.zeros(P, np.int32), np.zeros(P, np.int32)
    chi0 = None if chi0 is None else _f64(chi0)
    pc = params.c()
    rc = lib().ora_solve_batch_v(model.ref(), C.byref(pc), _f64(theta), P, dtau, D0.ravel(),
                                 _f64(I0).ravel(), _f64(rho11), _f64(ye0), _f64(ef0), _f64(v0).ravel(),
                                 _vp(chi0), D, I, ye, ef, v, T, no, ni, st, nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return dict(D=D.reshape(P, model.ns, model.nq), I=I.reshape(P, model.ns, 3, model.nq), ye=ye, ef=ef,
                v=v.reshape(P, 3), T=T, n_outer=no, n_inner=ni, status=st)


def primitive_batch(model: Model, N, G, v, mem=3, tol=1e-8, max_it=100, nthreads: int = 0):
    """Primitive-moment recovery (Sec. 3.4): conserved N (P, ns, nq), G (P, ns, 3, nq)
    at velocity v (P, 3) -> (D, I, iters); iters = -1 at the cap, -2 non-finite."""
    N = _f64(N)
    P = N.shape[0]
    nn = model.ns * model.nq
    D, I, it = np.zeros(P * nn), np.zeros(P * 3 * nn), np.zeros(P * nn, np.int32)
    rc = lib().ora_primitive_batch(model.ref(), P, N.ravel(), _f64(G).ravel(), _f64(v).ravel(), mem, tol, max_it,
                                   D, I, it, nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return D.reshape(P, model.ns, model.nq), I.reshape(P, model.ns, 3, model.nq), it.reshape(P, model.ns, model.nq)


def pdars_step_v(model: Model, params: Params, theta, dt, D0, I0, rho11, ye0, ef0, v0, chi0=None, c2p_mem=3,
                 c2p_tol=1e-8, c2p_max=100, nthreads: int = 0):
    """One PD-ARS IMEX step (Eq. butcherPDARS) of the coupling alone, O(v) form."""
    D0 = _f64(D0)
    P = D0.shape[0]
    nn = model.ns * model.nq
    D, I = np.zeros(P * nn), np.zeros(P * 3 * nn)
    ye, ef, v, T = np.zeros(P), np.zeros(P), np.zeros(P * 3), np.zeros(P)
    no, ni, st = np.zeros(P, np.int32), np.zeros(P, np.int32), np.zeros(P, np.int32)
    chi0 = None if chi0 is None else _f64(chi0)
    pc = params.c()
    rc = lib().ora_pdars_step_v(model.ref(), C.byref(pc), _f64(theta), P, dt, D0.ravel(), _f64(I0).ravel(),
                                _f64(rho11), _f64(ye0), _f64(ef0), _f64(v0).ravel(), _vp(chi0), c2p_mem, c2p_tol,
                                c2p_max, D, I, ye, ef, v, T, no, ni, st, nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return dict(D=D.reshape(P, model.ns, model.nq), I=I.reshape(P, model.ns, 3, model.nq), ye=ye, ef=ef,
                v=v.reshape(P, 3), T=T, n_outer=no, n_inner=ni, status=st)


def gauss_legendre(n: int):
    """Gauss-Legendre rule with n points on (-1, 1)."""
    x, w = np.zeros(n), np.zeros(n)
    if lib().ora_gauss_legendre(n, x, w) != 0:
        raise ValueError("bad rule size")
    return x, w


def fd_projection(model: Model, T, mu):
    """Nodal values of the weighted L2 projection of f(eps; mu, T) per energy
    element before the bound-enforcing limiter, after it, and the limited
    complement 1 - D."""
    dt, dl, cl = np.zeros(model.nq), np.zeros(model.nq), np.zeros(model.nq)
    lib().ora_fd_projection(model.ref(), T, mu, dt, dl, cl)
    return dt, dl, cl


def kernels_odds(model: Model, theta, rho11, T, odds):
    """Kernels with detailed balance for equilibrium odds (ns, nq):
    phi_in, phi_out, phi_pro (ns, nq, nq), phi_ann (nq, nq)."""
    ns, nq = model.ns, model.nq
    pin, pout, ppro = np.zeros(ns * nq * nq), np.zeros(ns * nq * nq), np.zeros(ns * nq * nq)
    pann = np.zeros(nq * nq)
    lib().ora_kernels_odds(model.ref(), _f64(theta), rho11, T, _f64(odds).ravel(), pin, pout, ppro, pann)
    return (pin.reshape(ns, nq, nq), pout.reshape(ns, nq, nq), ppro.reshape(ns, nq, nq), pann.reshape(nq, nq))
