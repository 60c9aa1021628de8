"""The persistent work queue under adversarial cost orderings, and parity at
a tight solver tolerance.

Queue: the profile's points reordered so that all stiff (dense) points come
first, or last, and solved in place by a persistent grid of one work-group
per CU in chunks of 1 and 4 points, give per point bit-identical results to
the out-of-place solve in profile order.  An in-place solve would show a
point visited twice (its second solve starts from the first one's output)
or not at all (its state unchanged), so this also checks that the queue
hands out every point exactly once.

Tolerance: with the inner and outer tolerances at 1e-13 instead of 1e-10,
the GPU and the oracle, which run the same iteration with different
rounding, still agree to 1e-11 (a hundred times the tolerance).  A point's
outer test compares matter updates whose rounding the matter update scales
by the neutrino/matter reservoir ratio R, so it is decided by rounding once
R eps_mach approaches the tolerance; statuses are compared where
R <= 1e-13 / (100 eps_mach), and converged states wherever both sides
converged."""
import numpy as np
import pytest

import oracle as O
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

ALL3 = (O.NU_E, O.NU_E_BAR, O.NU_X)
KEYS = ("D", "I", "ye", "e", "T", "n_outer", "n_inner", "status")


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _theta():
    return np.concatenate([np.ones(32), [PT.A_NES, PT.A_PAIR]])


def _solve(d, launch=None, inplace=False):
    import torch
    m = S.Model(S.Grid(16))
    t = S.to_device(d)
    D0, I0, e0 = S.init_state(m, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"], d.a, d.b, d.c)
    theta = torch.as_tensor(_theta(), dtype=torch.float64, device="cuda")
    ye0 = t["ye"].clone()
    out = S.alloc_outputs(m, d.P)
    for k in ("D", "I", "ye", "e", "T"):
        out[k].fill_(float("nan"))
    for k in ("n_outer", "n_inner", "status"):
        out[k].fill_(-7)
    if inplace:
        out.update(D=D0, I=I0, ye=ye0, e=e0)
    S.solve(m, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], ye0, e0, theta, out=out, launch=launch)
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy() for k in KEYS}


@pytest.mark.parametrize("chunk", [1, 4])
def test_adversarial_orderings_in_place(chunk):
    full = W.radial_profile(P=1 << 16)
    d = full.take(np.arange(0, 1 << 16, 16))
    _say(f"queue orderings, {d.P} profile points, in place, persistent 1 work-group per CU, chunk {chunk}")
    ref = _solve(d)
    for k in ("n_outer", "n_inner", "status"):
        assert np.all(ref[k] >= 0), k
    assert np.all(np.isfinite(ref["D"])) and np.all(np.isfinite(ref["T"]))
    launch = S.LaunchConfig(persistent=True, chunk=chunk, blocks_per_cu=1)
    for name, perm in (("stiff first", np.argsort(-d.rho11, kind="stable")),
                       ("stiff last", np.argsort(d.rho11, kind="stable"))):
        got = _solve(d.take(perm), launch=launch, inplace=True)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm))
        for k in KEYS:
            assert np.array_equal(got[k][inv], ref[k], equal_nan=False), f"{name}: {k}"
        print(f"{name}: bit-identical to the profile-order solve", flush=True)


def test_tight_tolerance_parity():
    tol = 1e-13
    full = W.radial_profile(P=1 << 16)
    d = full.take(np.linspace(0, 45000, 600).astype(np.int64))
    _say(f"profile sample, {d.P} points, tol_inner = tol_outer = {tol}")
    theta = _theta()
    m, ref = PT.run_oracle(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, O.Params(tol_inner=tol, tol_outer=tol, max_outer=200,
                                                                        max_inner=400), theta)
    _, got = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(tol_inner=tol, tol_outer=tol, max_outer=200,
                                                                     max_inner=400), theta)
    RY, RE = PT.reservoir_ratios(m.c.kcoup, d.rho11, ref["D"], ref["ye"], ref["e"], m.w2, m.w3)
    R = np.maximum(np.maximum(RY, RE), 1.0)
    solved = ref["n_outer"] > 0
    safe = solved & (R <= tol / (100 * np.finfo(float).eps))
    print(f"solved {int(solved.sum())}, R within the rounding bound at {int(safe.sum())}; oracle status "
          f"{np.bincount(ref['status'][solved], minlength=5)}, GPU {np.bincount(got['status'][solved], minlength=5)}",
          flush=True)
    assert np.array_equal(ref["status"][safe], got["status"][safe])
    ok = solved & (ref["status"] == O.OK) & (got["status"] == O.OK)
    assert ok.sum() >= 0.9 * solved.sum()
    eD, eI, eY, eE = PT.parity_errors({k: v[ok] for k, v in ref.items()}, {k: v[ok] for k, v in got.items()}, m.w2)
    eY, eE = eY / np.maximum(RY[ok], 1.0), eE / np.maximum(RE[ok], 1.0)
    print(f"converged {int(ok.sum())}: max errors D {eD.max():.2e} I {eI.max():.2e} Ye {eY.max():.2e} "
          f"e {eE.max():.2e}", flush=True)
    assert max(eD.max(), eI.max(), eY.max(), eE.max()) <= 100 * tol
