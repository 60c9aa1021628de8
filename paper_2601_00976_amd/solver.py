"""Python front end of the MI355X coupling solver (``libnmc.so``).

Thin wrappers: shape and dtype checks plus argument marshalling.  Every step
of the solve runs in the HIP kernels behind the C ABI of ``include/nmc.h``;
torch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import native as N

DEFAULT_A_NES = 1.0e-10   # NES kernel amplitude per rho11 [1/(km MeV^5)]
DEFAULT_A_PAIR = 1.0e-10  # pair kernel amplitude per rho11 [1/(km MeV^5)]


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _req(t: torch.Tensor, name: str, shape, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Grid:
    """Energy grid (2 Legendre-Gauss nodes per element)."""

    def __init__(self, n_elem: int = 16, eps_lo: float = 1.0, eps_hi: float = 300.0, zoom: float | None = None):
        d = N.GridDesc(n_elem, 2, eps_lo, eps_hi, N.SPACING_ZOOM if zoom else N.SPACING_LOG, zoom or 0.0)
        h = C.c_void_p()
        N.check(N.lib().nmc_grid_create(C.byref(d), C.byref(h)))
        self._h = h
        nq = C.c_int()
        N.check(N.lib().nmc_grid_query(h, C.byref(nq), None, None, None))
        self.nq = nq.value
        import numpy as np
        eps, w2, w3 = (np.zeros(self.nq) for _ in range(3))
        N.check(N.lib().nmc_grid_query(h, None, eps.ctypes.data_as(C.c_void_p), w2.ctypes.data_as(C.c_void_p),
                                       w3.ctypes.data_as(C.c_void_p)))
        self.eps, self.w2, self.w3 = eps, w2, w3

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and N is not None and N._lib is not None:
            N.lib().nmc_grid_destroy(h)
            self._h = None


class Model:
    """Species set, physics flags and synthetic microphysics constants on a grid."""

    def __init__(self, grid: Grid, species=(N.NU_E, N.NU_E_BAR, N.NU_X), flags: int = N.ALL_PHYSICS, **overrides):
        d = N.ModelDesc()
        N.lib().nmc_model_desc_default(C.byref(d))
        d.n_species = len(species)
        for i, s in enumerate(species):
            d.species[i] = s
        d.flags = flags
        for k, v in overrides.items():
            setattr(d, k, v)
        h = C.c_void_p()
        N.check(N.lib().nmc_model_create(grid._h, C.byref(d), C.byref(h)))
        self._h = h
        self.grid = grid
        self.ns = len(species)
        self.nq = grid.nq
        self.flags = flags
        self.desc = d

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and N is not None and N._lib is not None:
            N.lib().nmc_model_destroy(h)
            self._h = None

    def workspace_bytes(self, P: int) -> int:
        return int(N.lib().nmc_workspace_bytes(self._h, P))

    def kernel_store_bytes(self, P: int) -> int:
        """Extra workspace bytes of a solve with the kernels precomputed in HBM."""
        return int(N.lib().nmc_kernel_store_bytes(self._h, P))

    def default_theta(self, a_nes: float = DEFAULT_A_NES, a_pair: float = DEFAULT_A_PAIR, device="cuda"):
        th = torch.ones(self.nq + 2, dtype=torch.float64, device=device)
        th[self.nq] = a_nes
        th[self.nq + 1] = a_pair
        return th


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
        return N.SolverParams(self.tol_inner, self.tol_outer, self.m_inner, self.m_outer, self.max_inner,
                              self.max_outer, int(self.fixed_matter))


@dataclass
class LaunchConfig:
    blocks_per_cu: int = 0
    chunk: int = 4
    persistent: bool = True
    kernel_store: int = 0  # N.KERNELS_ON_CHIP or N.KERNELS_HBM (64-node roofline study)

    def c(self):
        return N.Launch(self.blocks_per_cu, self.chunk, int(self.persistent), int(self.kernel_store))


class Workspace:
    """Device workspace for solve calls (allocated once, reused)."""

    def __init__(self, model: Model, P: int, device="cuda", kernel_store: bool = False):
        nb = max(model.workspace_bytes(P) + (model.kernel_store_bytes(P) if kernel_store else 0), 256)
        self.buf = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        self.ptr = self.buf.data_ptr() + off
        self.nbytes = nb


def alloc_outputs(model: Model, P: int, device="cuda"):
    f64 = dict(dtype=torch.float64, device=device)
    i32 = dict(dtype=torch.int32, device=device)
    return dict(D=torch.empty(P, model.ns, model.nq, **f64), I=torch.empty(P, model.ns, model.nq, **f64),
                ye=torch.empty(P, **f64), e=torch.empty(P, **f64), T=torch.empty(P, **f64),
                n_outer=torch.empty(P, **i32), n_inner=torch.empty(P, **i32), status=torch.empty(P, **i32))


def _batch_in(model, P, D0, I0, rho11, ye0, e0, theta, chi0, T_fixed, mu_fixed):
    ns, nq = model.ns, model.nq
    _req(D0, "D0", (P, ns, nq))
    _req(I0, "I0", (P, ns, nq))
    for n, t in (("rho11", rho11), ("ye0", ye0), ("e0", e0)):
        _req(t, n, (P,))
    _req(theta, "theta", (nq + 2,))
    for n, t in (("chi0", chi0), ("T_fixed", T_fixed), ("mu_fixed", mu_fixed)):
        if t is not None:
            _req(t, n, (P,))
    return N.BatchIn(*[None if t is None else t.data_ptr()
                       for t in (D0, I0, rho11, ye0, e0, chi0, T_fixed, mu_fixed, theta)])


def _batch_out(model, P, out):
    ns, nq = model.ns, model.nq
    _req(out["D"], "D", (P, ns, nq))
    _req(out["I"], "I", (P, ns, nq))
    for n in ("ye", "e", "T"):
        _req(out[n], n, (P,))
    for n in ("n_outer", "n_inner", "status"):
        _req(out[n], n, (P,), torch.int32)
    return N.BatchOut(*[out[n].data_ptr() for n in ("D", "I", "ye", "e", "T", "n_outer", "n_inner", "status")])


def solve(model: Model, params: Params, dtau: float, D0, I0, rho11, ye0, e0, theta, chi0=None, T_fixed=None,
          mu_fixed=None, out=None, workspace: Workspace | None = None, launch: LaunchConfig | None = None,
          stream=None):
    """Enqueue one batched implicit solve on the current (or given) stream.

    Returns the output dict (tensors on the GPU; not synchronized)."""
    P = D0.shape[0]
    if out is None:
        out = alloc_outputs(model, P, D0.device)
    bi = _batch_in(model, P, D0, I0, rho11, ye0, e0, theta, chi0, T_fixed, mu_fixed)
    bo = _batch_out(model, P, out)
    launch = launch or LaunchConfig()
    if workspace is None:
        workspace = Workspace(model, P, D0.device)
    pc, lc = params.c(), launch.c()
    N.check(N.lib().nmc_solve_batch(model._h, C.byref(pc), P, float(dtau), C.byref(bi), C.byref(bo),
                                    C.c_void_p(workspace.ptr), workspace.nbytes, C.byref(lc),
                                    _stream_handle(stream)))
    return out


def solve_noalloc(model: Model, params: Params, dtau: float, D0, I0, rho11, ye0, e0, theta, out, chi0=None,
                  T_fixed=None, mu_fixed=None, launch: LaunchConfig | None = None, stream=None):
    """``solve`` through nmc_solve_batch_noalloc: no workspace, the outputs
    ``out`` given by the caller (see ``alloc_outputs``); the library's static
    per-device scratch holds the work-queue counters, so calls that overlap on
    one device race.  Returns ``out`` (not synchronized)."""
    P = D0.shape[0]
    bi = _batch_in(model, P, D0, I0, rho11, ye0, e0, theta, chi0, T_fixed, mu_fixed)
    bo = _batch_out(model, P, out)
    pc, lc = params.c(), (launch or LaunchConfig()).c()
    N.check(N.lib().nmc_solve_batch_noalloc(model._h, C.byref(pc), P, float(dtau), C.byref(bi), C.byref(bo),
                                            C.byref(lc), _stream_handle(stream)))
    return out


def alloc_outputs_v(model: Model, P: int, device="cuda"):
    f64 = dict(dtype=torch.float64, device=device)
    i32 = dict(dtype=torch.int32, device=device)
    return dict(D=torch.empty(P, model.ns, model.nq, **f64), I=torch.empty(P, model.ns, 3, model.nq, **f64),
                ye=torch.empty(P, **f64), ef=torch.empty(P, **f64), v=torch.empty(P, 3, **f64),
                T=torch.empty(P, **f64), n_outer=torch.empty(P, **i32), n_inner=torch.empty(P, **i32),
                status=torch.empty(P, **i32))


def solve_v(model: Model, params: Params, dtau: float, D0, I0, rho11, ye0, ef0, v0, theta, chi0=None, out=None,
            workspace: Workspace | None = None, launch: LaunchConfig | None = None, stream=None):
    """Enqueue one batched O(v) solve (nonzero fluid velocity): D0 (P, ns, nq),
    I0 (P, ns, 3, nq), v0 (P, 3), ef0 the specific fluid energy (internal plus
    kinetic) per baryon.  Returns the output dict (not synchronized)."""
    P = D0.shape[0]
    ns, nq = model.ns, model.nq
    _req(D0, "D0", (P, ns, nq))
    _req(I0, "I0", (P, ns, 3, nq))
    for n, t in (("rho11", rho11), ("ye0", ye0), ("ef0", ef0)):
        _req(t, n, (P,))
    _req(v0, "v0", (P, 3))
    _req(theta, "theta", (nq + 2,))
    if chi0 is not None:
        _req(chi0, "chi0", (P,))
    if out is None:
        out = alloc_outputs_v(model, P, D0.device)
    _req(out["D"], "D", (P, ns, nq))
    _req(out["I"], "I", (P, ns, 3, nq))
    for n in ("ye", "ef", "T"):
        _req(out[n], n, (P,))
    _req(out["v"], "v", (P, 3))
    for n in ("n_outer", "n_inner", "status"):
        _req(out[n], n, (P,), torch.int32)
    bi = N.BatchVIn(*[None if t is None else t.data_ptr() for t in (D0, I0, rho11, ye0, ef0, v0, chi0, theta)])
    bo = N.BatchVOut(*[out[n].data_ptr() for n in ("D", "I", "ye", "ef", "v", "T", "n_outer", "n_inner", "status")])
    launch = launch or LaunchConfig(chunk=1)
    if workspace is None:
        workspace = Workspace(model, P, D0.device)
    pc, lc = params.c(), launch.c()
    N.check(N.lib().nmc_solve_batch_v(model._h, C.byref(pc), P, float(dtau), C.byref(bi), C.byref(bo),
                                      C.c_void_p(workspace.ptr), workspace.nbytes, C.byref(lc),
                                      _stream_handle(stream)))
    return out


@dataclass
class C2pParams:
    """Primitive-moment recovery: Anderson memory, relative tolerance, cap."""
    mem: int = 3
    tol: float = 1e-8
    max_it: int = 100

    def c(self):
        return N.C2pParams(self.mem, self.tol, self.max_it)


def primitive_recovery(model: Model, Nc, G, v, params: C2pParams | None = None, stream=None, out=None):
    """Primitive moments (D (P, ns, nq), I (P, ns, 3, nq)) of conserved ones
    Nc (P, ns, nq), G (P, ns, 3, nq) at velocity v (P, 3), with the iteration
    counts (P, ns, nq) int32 (-1 at the cap, -2 non-finite).  ``out`` = (D, I,
    it) to write into (allocated if None; D and I must not alias Nc and G).
    Not synchronized."""
    P = Nc.shape[0]
    ns, nq = model.ns, model.nq
    _req(Nc, "N", (P, ns, nq))
    _req(G, "G", (P, ns, 3, nq))
    _req(v, "v", (P, 3))
    if out is None:
        D = torch.empty_like(Nc)
        I = torch.empty_like(G)
        it = torch.empty(P, ns, nq, dtype=torch.int32, device=Nc.device)
    else:
        D, I, it = out
        _req(D, "D", (P, ns, nq))
        _req(I, "I", (P, ns, 3, nq))
        _req(it, "iters", (P, ns, nq), torch.int32)
    pc = (params or C2pParams()).c()
    N.check(N.lib().nmc_primitive_recovery(model._h, C.byref(pc), P, Nc.data_ptr(), G.data_ptr(), v.data_ptr(),
                                           D.data_ptr(), I.data_ptr(), it.data_ptr(), _stream_handle(stream)))
    return D, I, it


class PdarsWorkspace:
    """Device workspace of ``pdars_step_v`` (allocated once, reused)."""

    def __init__(self, model: Model, P: int, device="cuda"):
        nb = max(int(N.lib().nmc_pdars_workspace_bytes(model._h, P)), 256)
        self.buf = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        self.ptr = self.buf.data_ptr() + (-self.buf.data_ptr()) % 256
        self.nbytes = nb


def pdars_step_v(model: Model, params: Params, dt: float, D0, I0, rho11, ye0, ef0, v0, theta, chi0=None, out=None,
                 c2p: C2pParams | None = None, workspace: PdarsWorkspace | None = None,
                 launch: LaunchConfig | None = None, stream=None):
    """One PD-ARS IMEX step of the coupling (O(v) form): two solves (dt,
    dt/2) with the stage combination in conserved moments and primitive
    recovery between them.  Arguments as for ``solve_v``; returns the output
    dict (not synchronized)."""
    P = D0.shape[0]
    ns, nq = model.ns, model.nq
    _req(D0, "D0", (P, ns, nq))
    _req(I0, "I0", (P, ns, 3, nq))
    for n, t in (("rho11", rho11), ("ye0", ye0), ("ef0", ef0)):
        _req(t, n, (P,))
    _req(v0, "v0", (P, 3))
    _req(theta, "theta", (nq + 2,))
    if chi0 is not None:
        _req(chi0, "chi0", (P,))
    if out is None:
        out = alloc_outputs_v(model, P, D0.device)
    bi = N.BatchVIn(*[None if t is None else t.data_ptr() for t in (D0, I0, rho11, ye0, ef0, v0, chi0, theta)])
    bo = N.BatchVOut(*[out[n].data_ptr() for n in ("D", "I", "ye", "ef", "v", "T", "n_outer", "n_inner", "status")])
    if workspace is None:
        workspace = PdarsWorkspace(model, P, D0.device)
    pc, cc, lc = params.c(), (c2p or C2pParams()).c(), (launch or LaunchConfig(chunk=1)).c()
    N.check(N.lib().nmc_pdars_step_v(model._h, C.byref(pc), C.byref(cc), P, float(dt), C.byref(bi), C.byref(bo),
                                     C.c_void_p(workspace.ptr), workspace.nbytes, C.byref(lc),
                                     _stream_handle(stream)))
    return out


def adjoint(model: Model, dtau: float, rho11, theta, fwd, gbar, chi0=None, grad_theta=None, per_point=False,
            workspace: Workspace | None = None, stream=None, params: Params | None = None):
    """Enqueue the implicit-function-theorem adjoint of a converged forward
    solve (``fwd`` = its output dict, solved with ``params``, default
    ``Params()``) for the per-point loss
    L_p = gbar[p, 0] (e*_p - e_p) + gbar[p, 1] (Ye_p - Ye*_p).

    Adds dL/dtheta into ``grad_theta`` (allocated zero if None) and returns it,
    with the (P, nq + 2) per-point terms when ``per_point``.  A forward solve
    with fixed matter is rejected (NmcError, NMC_E_UNSUPPORTED)."""
    P = rho11.shape[0]
    nq = model.nq
    _req(rho11, "rho11", (P,))
    _req(theta, "theta", (nq + 2,))
    _req(gbar, "gbar", (P, 2))
    if chi0 is not None:
        _req(chi0, "chi0", (P,))
    bo = _batch_out(model, P, fwd)
    bi = N.BatchIn(None, None, rho11.data_ptr(), None, None, None if chi0 is None else chi0.data_ptr(), None, None,
                   theta.data_ptr())
    if grad_theta is None:
        grad_theta = torch.zeros(nq + 2, dtype=torch.float64, device=rho11.device)
    _req(grad_theta, "grad_theta", (nq + 2,))
    gpp = torch.empty(P, nq + 2, dtype=torch.float64, device=rho11.device) if per_point else None
    if workspace is None:
        workspace = Workspace(model, P, rho11.device)
    pc = (params or Params()).c()
    N.check(N.lib().nmc_solve_batch_adjoint(model._h, C.byref(pc), P, float(dtau), C.byref(bi), C.byref(bo),
                                            gbar.data_ptr(),
                                            grad_theta.data_ptr(), None if gpp is None else gpp.data_ptr(),
                                            C.c_void_p(workspace.ptr), workspace.nbytes, _stream_handle(stream)))
    return (grad_theta, gpp) if per_point else grad_theta


class NMCSolve(torch.autograd.Function):
    """Differentiable batched solve with respect to theta = (s_1..s_nq, a_nes, a_pair).

    forward(theta, model, params, dtau, D0, I0, rho11, ye0, e0) returns
    (D, I, Ye, e, L_E, L_Y) with L_E = e* - e and L_Y = Ye - Ye* per point.
    backward folds the cotangents of Ye, e, L_E and L_Y into the per-point
    loss weights of the adjoint; cotangents on D or I are not supported."""

    @staticmethod
    def forward(ctx, theta, model, params, dtau, D0, I0, rho11, ye0, e0):
        if params.fixed_matter:
            raise NotImplementedError("NMCSolve: the adjoint differentiates the coupled system; "
                                      "fixed_matter is not supported")
        out = solve(model, params, dtau, D0, I0, rho11, ye0, e0, theta)
        ctx.model, ctx.dtau, ctx.params = model, dtau, params
        ctx.out = out
        ctx.save_for_backward(theta, rho11)
        return out["D"], out["I"], out["ye"], out["e"], e0 - out["e"], out["ye"] - ye0

    @staticmethod
    def backward(ctx, gD, gI, gYe, ge, gLE, gLY):
        for g, n in ((gD, "D"), (gI, "I")):
            if g is not None and bool(torch.any(g != 0)):
                raise NotImplementedError(f"NMCSolve.backward: cotangents on {n} are not supported")
        theta, rho11 = ctx.saved_tensors
        P = rho11.shape[0]
        z = torch.zeros(P, dtype=torch.float64, device=rho11.device)
        gE = (gLE if gLE is not None else z) - (ge if ge is not None else z)
        gY = (gLY if gLY is not None else z) + (gYe if gYe is not None else z)
        gbar = torch.stack([gE, gY], dim=1).contiguous()
        g = adjoint(ctx.model, ctx.dtau, rho11, theta, ctx.out, gbar, params=ctx.params)
        return g, None, None, None, None, None, None, None, None


def init_state(model: Model, T, rho11, ye, uD, uI, a=1.0, b=0.1, c=0.1, mu=None, stream=None):
    """Initial state on the GPU from raw draws (EOS energy, perturbed equilibrium)."""
    P = T.shape[0]
    ns, nq = model.ns, model.nq
    for n, t in (("T", T), ("rho11", rho11), ("ye", ye)):
        _req(t, n, (P,))
    _req(uD, "uD", (P, ns, nq))
    _req(uI, "uI", (P, ns, nq))
    if mu is not None:
        _req(mu, "mu", (P,))
    D0 = torch.empty(P, ns, nq, dtype=torch.float64, device=T.device)
    I0 = torch.empty_like(D0)
    e0 = torch.empty(P, dtype=torch.float64, device=T.device)
    N.check(N.lib().nmc_init_state(model._h, P, T.data_ptr(), None if mu is None else mu.data_ptr(),
                                   rho11.data_ptr(), ye.data_ptr(), uD.data_ptr(), uI.data_ptr(), float(a),
                                   float(b), float(c), D0.data_ptr(), I0.data_ptr(), e0.data_ptr(),
                                   _stream_handle(stream)))
    return D0, I0, e0


def to_device(draws, device="cuda"):
    """Move a workloads.Draws bundle to the GPU as float64 tensors."""
    f = lambda x: None if x is None else torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()
    return dict(T=f(draws.T), rho11=f(draws.rho11), ye=f(draws.ye), uD=f(draws.uD), uI=f(draws.uI),
                mu=f(draws.mu), chi0=f(draws.chi0), v=f(draws.v), uI3=f(draws.uI3))


MU_C2 = 931.49410242  # atomic mass unit rest energy [MeV]


def init_state_v(model: Model, t: dict, c: float = 0.1):
    """Old state of an O(v) workload from device draws ``t`` (see
    ``to_device``): D* and e* from ``init_state``, I*_j = c D* uI3_j and the
    specific fluid energy ef* = e* + m_u c^2 |v|^2 / 2."""
    D0, _, e0 = init_state(model, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    I0 = (c * D0[:, :, None, :] * t["uI3"]).contiguous()
    ef0 = e0 + 0.5 * MU_C2 * (t["v"] * t["v"]).sum(dim=1)
    return D0, I0, ef0
