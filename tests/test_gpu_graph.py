"""Captured-graph replays of the chained solve equal the eager result
bitwise, replay after replay, with eager work and synchronisations between
the replays (the persistent kernel's work-queue counter is reset by a kernel
node inside the graph, not by a memset)."""
import numpy as np
import pytest

from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_elem", [16, 32])
def test_graph_replays_match_eager(n_elem):
    import torch
    print(f"[case] graph replay of 3 chained steps, {2 * n_elem} nodes, P=2048", flush=True)
    nq = 2 * n_elem
    d = W.radial_profile(P=1 << 16, nq=nq).take(np.arange(0, 1 << 16, 32))
    P = len(d.rho11)
    m = S.Model(S.Grid(n_elem))
    t = S.to_device(d)
    D0, I0, e0 = S.init_state(m, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    theta = m.default_theta()
    ws = S.Workspace(m, P)
    work = dict(D=D0.clone(), I=I0.clone(), ye=t["ye"].clone(), e=e0.clone())
    outs = [S.alloc_outputs(m, P) for _ in range(3)]
    for o in outs:
        o["D"], o["I"], o["ye"], o["e"] = work["D"], work["I"], work["ye"], work["e"]

    def chain():
        work["D"].copy_(D0)
        work["I"].copy_(I0)
        work["ye"].copy_(t["ye"])
        work["e"].copy_(e0)
        for o in outs:
            S.solve(m, S.Params(), W.DTAU_KM, work["D"], work["I"], t["rho11"], work["ye"], work["e"], theta,
                    out=o, workspace=ws)

    chain()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in work.items()}
    ref_cnt = [o["n_inner"].clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        chain()
    for rep in range(4):
        # unrelated eager work between replays
        work["D"].fill_(0.5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(work[k], ref[k]), f"replay {rep}: {k}"
        for o, c in zip(outs, ref_cnt):
            assert torch.equal(o["n_inner"], c), f"replay {rep}: n_inner"
