"""The FP64 FMA throughput probe behind the roofline denominator: its lanes
hold the values of the recurrence x <- x a + b it claims to run (so the
FLOP count it reports is the work done), and the measured rate is of the
order of the published FP64 vector peak."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_probe_values_and_rate():
    import torch

    from paper_2601_00976_amd import probe as PR

    print("probe: 4 waves x 64 lanes, 64 rounds; then the default rate probe", flush=True)
    waves, iters = 4, 64
    out = torch.empty(waves * 64, dtype=torch.float64, device="cuda")
    PR.fma_f64(waves, iters, out)
    torch.cuda.synchronize()
    lane = np.arange(waves * 64) % 64
    a, b = 0.9999999, 1e-7
    ref = np.zeros(waves * 64)
    for k in range(16):
        x = 1.0 + 1e-3 * k + 1e-9 * lane
        for _ in range(iters):
            x = x * a + b
        ref += x
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-13, atol=0)
    tf = PR.fma_tflops("cuda")
    assert 20.0 < tf < 100.0, tf
