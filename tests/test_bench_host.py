"""Host-side checks of bench.py (no GPU): the one-GPU guard and the
accounting conventions of the roofline line."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flop_and_byte_conventions():
    # per inner iteration: four energy-coupling mat-vecs per species (8 Ns Nq^2)
    # and the pointwise and Anderson work (40 Ns Nq); per outer iteration the
    # kernel build and matter update (4 Nq^2 + 30 Ns Nq)
    assert bench.flops_per_point(1, 0, 32, 3) == 24576 + 3840
    assert bench.flops_per_point(1, 0, 64, 3) == 98304 + 7680
    assert bench.flops_per_point(0, 1, 32, 3) == 4 * 1024 + 30 * 96
    # D*, I* and three scalars in; D, I, three scalars and three counters out
    assert bench.bytes_per_point(32, 3) == 2 * 96 * 8 + 24 + 2 * 96 * 8 + 24 + 12
    # O(v): D and three flux components each way, six scalars each way
    assert bench.bytes_per_point_v(32, 3) == 2 * 4 * 96 * 8 + 48 + 48 + 12
    # Phi_1: four contractions per species against each of three flux
    # components (24 Ns Nq^2) and 70 Ns Nq pointwise, per inner iteration
    assert (bench.flops_per_point_v_phi1(1, 0, 32, 3) - bench.flops_per_point_v(1, 0, 32, 3)
            == 24 * 3 * 1024 + 70 * 96)
    assert bench.flops_per_point_v_phi1(0, 1, 32, 3) == bench.flops_per_point_v(0, 1, 32, 3)
    # recovery: 158 per iteration and 30 per node; 68 bytes per node plus the
    # velocity shared by the point's 96 nodes
    assert bench.flops_per_node_c2p(5) == 5 * 158 + 30
    assert bench.bytes_per_node_c2p(3, 32) == 68 + 24 / 96


def test_iteration_summary_histograms():
    import numpy as np
    n_in = np.array([[3, 0, 7], [3, 5, 0]], dtype=float)
    n_out = np.array([[1, 0, 2], [1, 2, 0]], dtype=float)  # zeros: points passed through
    s = bench.iteration_summary(n_in, n_out)
    assert s["inner_hist"] == [0, 0, 0, 2, 0, 1, 0, 1]
    assert s["outer_hist"] == [0, 2, 2]
    assert (s["inner_min"], s["inner_max"], s["outer_max"]) == (3, 7, 2)
    assert sum(s["inner_hist"]) == 4
