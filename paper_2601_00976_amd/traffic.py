"""HBM traffic of the solve kernels from rocprofv3 counters.

Two steps, each run on a machine with the GPU:

  cd /tmp && export TMPDIR=/tmp
  rocprofv3 --pmc FETCH_SIZE -d <dir>/fetch -o run -- python3 <repo>/paper_2601_00976_amd/traffic.py run
  rocprofv3 --pmc WRITE_SIZE -d <dir>/write -o run -- python3 <repo>/paper_2601_00976_amd/traffic.py run
  python3 <repo>/paper_2601_00976_amd/traffic.py summarize <dir>/fetch/run_results.db <dir>/write/run_results.db

`run` launches a plain device-to-device copy of a known size (the
calibration: it must read and write exactly that many bytes), the forward
solve (default and one-point-per-wave kernels, and the default with the
projected equilibrium) and the adjoint on the first step of the 2^16-point
radial profile, the O(v) solve (two points and one point per wavefront) on
the first step of the 2^16-point moving profile (and with the Phi_1
corrections), the primitive recovery of that profile's moments, and the
64-node solves
(kernels on chip and in HBM) on the first step of the 2^18-point profile,
each at the launch shape of the autotune cache.
`summarize` scales each kernel's per-dispatch counter by copy bytes / copy
counter and writes profiles/traffic_<kernel>.txt with the source hash of the
kernels, so that stale measurements are recognised.
"""
from __future__ import annotations

import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 28  # 256 MiB calibration copy
KERNELS = {
    "fwd_pair_kernel<3, true, false>": ("fwd_pair_kernel_nq32_ns3", "radial profile, 2^16 points, 32 nodes, step 1"),
    "fwd_pair_kernel<3, true, true>": ("fwd_pair_kernel_nq32_ns3_proj", "radial profile, 2^16 points, 32 nodes, "
                                       "step 1, projected equilibrium"),
    "fwd_kernel<3, 32, true, 2>": ("fwd_kernel_nq32_ns3", "radial profile, 2^16 points, 32 nodes, step 1, "
                                   "one point per wavefront"),
    "adj_kernel<3>": ("adj_kernel_nq32_ns3", "radial profile, 2^16 points, 32 nodes, step 1"),
    "fwd_v_kernel<3, true, false>": ("fwd_v_kernel_nq32_ns3", "moving radial profile (O(v) solve), 2^16 points, "
                                     "32 nodes, step 1, one point per wavefront"),
    "fwd_vpair_kernel<3, true, false>": ("fwd_vpair_kernel_nq32_ns3", "moving radial profile (O(v) solve), 2^16 "
                                  "points, 32 nodes, step 1, two points per wavefront"),
    "fwd_vpair_kernel<3, true, true>": ("fwd_vpair_kernel_nq32_ns3_phi1", "moving radial profile (O(v) solve "
                                        "with the Phi_1 corrections), 2^16 points, 32 nodes, step 1, two points "
                                        "per wavefront"),
    "c2p_kernel": ("c2p_kernel_nq32_ns3", "primitive recovery of every node of the moving radial profile, "
                   "2^16 points x 3 species x 32 nodes"),
    "fwd64_kernel<3, true, false>": ("fwd64_kernel_nq64_ns3", "radial profile, 2^18 points, 64 nodes, step 1"),
    "fwd64_kernel<3, true, true>": ("fwd64_kernel_nq64_ns3_hbm",
                                    "radial profile, 2^18 points, 64 nodes, step 1, kernels in HBM"),
}


def run():
    sys.path.insert(0, ROOT)
    import torch

    from paper_2601_00976_amd import solver as S
    from paper_2601_00976_amd import workloads as W

    dev = torch.device("cuda:0")
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    model = S.Model(S.Grid(16))
    t = S.to_device(W.radial_profile(P=1 << 16), dev)
    D0, I0, e0 = S.init_state(model, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    theta = model.default_theta()
    ws = S.Workspace(model, 1 << 16, dev)
    out = S.alloc_outputs(model, 1 << 16, dev)
    from paper_2601_00976_amd import autotune as AT

    # the launch shape bench.py times (autotune cache); the one-point-per-wave
    # kernel once as well
    for store in (0, 0, 0, 5):
        L = AT.best_launch(model, 1 << 16)
        L.kernel_store = store
        S.solve(model, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, out=out, workspace=ws,
                launch=L)
    gbar = torch.ones(1 << 16, 2, dtype=torch.float64, device=dev)
    S.adjoint(model, W.DTAU_KM, t["rho11"], theta, out, gbar, workspace=ws)
    torch.cuda.synchronize()
    # the projected equilibrium, at the same launch shape
    mp = S.Model(S.Grid(16), fd_projection=1)
    S.solve(mp, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, out=out, workspace=ws,
            launch=AT.best_launch(model, 1 << 16))
    torch.cuda.synchronize()
    # the O(v) solve on the moving profile, at the launch shape bench.py uses
    tv = S.to_device(W.radial_profile_v(P=1 << 16, wid=6), dev)
    Dv, Iv, efv = S.init_state_v(model, tv)
    outv = S.alloc_outputs_v(model, 1 << 16, dev)
    for store in (0, 5):  # two points per wavefront (default), then one
        S.solve_v(model, S.Params(tol_inner=1e-12, tol_outer=1e-10), W.DTAU_KM, Dv, Iv, tv["rho11"], tv["ye"], efv,
                  tv["v"], theta, out=outv, workspace=ws, launch=S.LaunchConfig(chunk=1, kernel_store=store))
    # the same with the Phi_1 corrections (two points per wavefront), and the
    # primitive recovery of the profile's moments at its velocity
    m1 = S.Model(S.Grid(16), phi1_nes=0.3, phi1_pair=-0.25)
    S.solve_v(m1, S.Params(tol_inner=1e-12, tol_outer=1e-10), W.DTAU_KM, Dv, Iv, tv["rho11"], tv["ye"], efv,
              tv["v"], theta, out=outv, workspace=ws, launch=S.LaunchConfig(chunk=1))
    S.primitive_recovery(model, Dv, Iv, tv["v"])
    torch.cuda.synchronize()
    del ws, out, gbar, D0, I0, e0, t, tv, Dv, Iv, efv, outv
    # 64 nodes, 2^18 points: kernels on chip, then precomputed in HBM
    P64 = 1 << 18
    m64 = S.Model(S.Grid(32))
    t = S.to_device(W.radial_profile(P=P64, nq=64, wid=4), dev)
    D0, I0, e0 = S.init_state(m64, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    th64 = m64.default_theta()
    out = S.alloc_outputs(m64, P64, dev)
    ws = S.Workspace(m64, P64, dev, kernel_store=True)
    for store in (0, 1):
        L = AT.best_launch(m64, P64)
        L.kernel_store = store
        S.solve(m64, S.Params(), W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, th64, out=out, workspace=ws,
                launch=L)
    torch.cuda.synchronize()
    print("traffic run done", flush=True)


def _per_dispatch(db, counter):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, value from counters_collection where counter_name = ?",
                     (counter,)).fetchall()
    acc = {}
    for name, v in rows:
        acc.setdefault(name, []).append(float(v))
    return acc


def _match(acc, key):
    for name, vals in acc.items():
        if key in name:
            return sum(vals) / len(vals), len(vals)
    return None, 0


def _copy_reading(acc):
    """Counter of the calibration copy: the largest copy dispatch (the
    workload's own small host-to-device copies also use the copy kernel)."""
    vals = [v for name, vs in acc.items() if "copyBuffer" in name or "copy" in name for v in vs]
    return max(vals) if vals else None


def summarize(fetch_db, write_db):
    sys.path.insert(0, ROOT)
    from paper_2601_00976_amd.autotune import kernel_source_hash

    f, w = _per_dispatch(fetch_db, "FETCH_SIZE"), _per_dispatch(write_db, "WRITE_SIZE")
    cf, cw = _copy_reading(f), _copy_reading(w)
    kib = COPY_BYTES / 1024.0
    sf, sw = kib / cf, kib / cw
    h = kernel_source_hash()
    for key, (tag, what) in KERNELS.items():
        vf, nf = _match(f, key)
        vw, nw = _match(w, key)
        if vf is None or vw is None:
            continue
        total = (vf * sf + vw * sw) * 1024.0
        path = os.path.join(ROOT, "profiles", f"traffic_{tag}.txt")
        with open(path, "w") as o:
            o.write(f"# HBM traffic of {key} ({what})\n")
            o.write("# commands (GPU host, from the repository root; source_hash = code-only hash of csrc/, "
                    "see autotune.kernel_source_hash):\n")
            o.write("#   cd /tmp && export TMPDIR=/tmp\n")
            o.write("#   rocprofv3 --pmc FETCH_SIZE -d <dir>/fetch -o run -- python3 <repo>/paper_2601_00976_amd/traffic.py run\n")
            o.write("#   rocprofv3 --pmc WRITE_SIZE -d <dir>/write -o run -- python3 <repo>/paper_2601_00976_amd/traffic.py run\n")
            o.write("#   python3 <repo>/paper_2601_00976_amd/traffic.py summarize <fetch db> <write db>\n")
            o.write(f"calibration_copy_bytes: {COPY_BYTES}\n")
            o.write(f"copy_fetch_kib: {cf:.1f}  (scale {sf:.4f})\n")
            o.write(f"copy_write_kib: {cw:.1f}  (scale {sw:.4f})\n")
            o.write(f"fetch_kib_per_dispatch: {vf:.1f}  (dispatches {nf})\n")
            o.write(f"write_kib_per_dispatch: {vw:.1f}  (dispatches {nw})\n")
            o.write(f"source_hash: {h}\n")
            o.write(f"fetch_bytes_per_launch: {vf * sf * 1024.0:.6e}\n")
            o.write(f"write_bytes_per_launch: {vw * sw * 1024.0:.6e}\n")
            o.write(f"hbm_bytes_per_launch: {total:.6e}\n")
        print(open(path).read())


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "run":
        run()
    elif len(sys.argv) == 4 and sys.argv[1] == "summarize":
        summarize(sys.argv[2], sys.argv[3])
    else:
        print(__doc__)
        sys.exit(2)
