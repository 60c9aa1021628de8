"""The no-allocation forward solve (nmc_solve_batch_noalloc) against the
workspace-taking one (nmc_solve_batch): same inputs, same launch, results
bitwise equal (both run the same kernels; the solve's reductions have a fixed
order).  Two calls in a row, the second with a smaller input, so that the
second starts from the static scratch the first left behind."""
import numpy as np
import pytest

from paper_2601_00976_amd import native as N
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(m, d):
    t = S.to_device(d)
    D0, I0, e0 = S.init_state(m, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    return t, D0, I0, e0


@pytest.mark.parametrize("launch", [S.LaunchConfig(chunk=4), S.LaunchConfig(chunk=1, blocks_per_cu=2),
                                    S.LaunchConfig(chunk=3, persistent=False)])
def test_noalloc_matches_workspace_solve(launch):
    import torch
    print(f"[case] no-allocation solve vs workspace solve, launch {launch}", flush=True)
    m = S.Model(S.Grid(16))
    theta = m.default_theta()
    full = W.radial_profile(P=1 << 16)
    for P in (4099, 1031):  # the second call is smaller
        d = full.take(np.linspace(0, (1 << 16) - 1, P).astype(np.int64))
        t, D0, I0, e0 = _case(m, d)
        ref = S.solve(m, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, launch=launch)
        out = S.alloc_outputs(m, P)
        for v in out.values():
            v.fill_(-7)
        got = S.solve_noalloc(m, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, out, launch=launch)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], got[k]), f"P={P}: {k} differs"
        assert int((got["status"] != 0).sum()) == 0
        assert int((got["n_outer"] > 0).sum()) > 0


def test_noalloc_64_nodes_and_limits():
    import torch
    print("[case] no-allocation solve, 64 nodes, and the scratch limit of the HBM kernel store", flush=True)
    m = S.Model(S.Grid(32))
    theta = m.default_theta()
    full = W.radial_profile(P=1 << 18, nq=64, wid=4)
    for P, store in ((777, N.KERNELS_ON_CHIP), (40, N.KERNELS_HBM), (9, N.KERNELS_HBM)):
        d = full.take(np.linspace(0, 200000, P).astype(np.int64))
        t, D0, I0, e0 = _case(m, d)
        launch = S.LaunchConfig(chunk=2, kernel_store=store)
        ws = S.Workspace(m, P, kernel_store=store == N.KERNELS_HBM)
        ref = S.solve(m, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, launch=launch, workspace=ws)
        out = S.alloc_outputs(m, P)
        got = S.solve_noalloc(m, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, out, launch=launch)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], got[k]), f"P={P}: {k} differs"
    # beyond the static scratch: a clear error, nothing launched
    d = full.take(np.arange(64))
    t, D0, I0, e0 = _case(m, d)
    out = S.alloc_outputs(m, 64)
    with pytest.raises(N.NmcError) as ei:
        S.solve_noalloc(m, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, out,
                        launch=S.LaunchConfig(kernel_store=N.KERNELS_HBM))
    assert ei.value.code == N.NMC_E_WORKSPACE
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
