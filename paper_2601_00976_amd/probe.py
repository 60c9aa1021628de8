"""The FP64 FMA throughput probe (``libnmc_probe.so``, declared in
``include/nmc_probe.h``): a measurement of the device's FP64 FMA rate that the
benchmark reports beside the published peak.  Not part of the solver."""
from __future__ import annotations

import ctypes as C
import os

import torch

from . import native as N

_lib = None


def lib():
    """Load libnmc_probe.so (built in-tree by ``paper_2601_00976_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(N.PROBE_LIB_PATH):
            raise RuntimeError(f"{N.PROBE_LIB_PATH} is missing: build it with `python -m paper_2601_00976_amd.build`")
        L = C.CDLL(N.PROBE_LIB_PATH)
        L.nmc_probe_fma_f64.argtypes = [C.c_int64, C.c_int, C.c_void_p, C.c_void_p]
        L.nmc_probe_fma_f64.restype = C.c_int
        _lib = L
    return _lib


def fma_f64(waves: int, iters: int, out: torch.Tensor, stream=None) -> None:
    """Enqueue the probe: `waves` one-wavefront work-groups, each lane
    running 16 FMA chains for `iters` rounds (rounded up to 8), writing
    waves * 64 sums to `out`."""
    rc = lib().nmc_probe_fma_f64(waves, iters, out.data_ptr(), None if stream is None else stream.cuda_stream)
    if rc != 0:
        raise N.NmcError(rc, "probe_fma_f64 rejected its arguments or failed to launch")


def fma_tflops(device="cuda", waves=None, iters=4096, reps=3):
    """Measured FP64 FMA throughput of the device (TFLOP/s, best of `reps`):
    8 one-wavefront work-groups per SIMD, timed with HIP events on the
    current stream."""
    props = torch.cuda.get_device_properties(device)
    if waves is None:
        waves = props.multi_processor_count * 4 * 8
    iters = (iters + 7) // 8 * 8
    out = torch.empty(waves * 64, dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(device)
    best = 0.0
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fma_f64(waves, iters, out, stream)
        b.record(stream)
        b.synchronize()
        flops = waves * 64.0 * 32.0 * iters
        best = max(best, flops / (a.elapsed_time(b) * 1e-3) / 1e12)
    return best
