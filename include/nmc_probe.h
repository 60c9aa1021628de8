/*
 * Measurement library (libnmc_probe.so), not part of the solver's C ABI:
 * the FP64 FMA throughput probe whose measured rate the benchmark reports
 * beside the published FP64 peak of the roofline.
 */
#ifndef NMC_PROBE_H
#define NMC_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NMC_PROBE_OK 0
#define NMC_PROBE_E_INVALID_ARG (-1)
#define NMC_PROBE_E_HIP (-3)

/* Launches `waves` work-groups of one wavefront each on `stream` (a
 * hipStream_t, NULL for the default stream); every lane runs R rounds of 16
 * independent FMA chains (x <- x a + b), R = `iters` rounded up to a multiple
 * of 8 (8 rounds per loop trip), i.e. 32 R FLOP per lane and
 * waves * 64 * 32 * R FLOP in total, and writes its 16 chain values' sum to
 * out[lane] (out: device array of waves * 64 doubles, caller-owned), so that
 * no FMA is dead.  The caller times the launch on `stream`.
 * Returns NMC_PROBE_E_INVALID_ARG (before any launch) for waves < 1,
 * waves > 2^20, iters < 1, iters > 2^24 or a null out; NMC_PROBE_E_HIP if the
 * launch fails. */
int nmc_probe_fma_f64(int64_t waves, int iters, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NMC_PROBE_H */
