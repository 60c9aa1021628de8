"""GPU parity of the two-points-per-wave 32-node solve (kernel_store = PAIRED)
against the CPU oracle, including the cases particular to it: batches of odd
size (the last wave has one point), neighbouring points with different
iteration counts and statuses (one half of a wave finishes first), and
low-density pass-through next to a solved point."""
import numpy as np
import pytest

import oracle as O
from paper_2601_00976_amd import native as N
from paper_2601_00976_amd import solver as S
from paper_2601_00976_amd import workloads as W
from tests import parity as PT
from tests.test_gpu_parity import ALL3, _box_sample, _compare, _say, _theta

pytestmark = pytest.mark.gpu

PAIRED = S.LaunchConfig(kernel_store=N.KERNELS_PAIRED)


def test_paired_profile_box_and_species():
    _say("paired: profile P=513 (odd), box P=255 (odd), species subsets")
    theta = _theta(32)
    d = W.radial_profile(P=1 << 16).take(np.arange(0, 1 << 16, 128)[:513])
    m, ref = PT.run_oracle(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, O.Params(), theta)
    _, got = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=PAIRED)
    _compare(ref, got, m.w2, model=m, rho11=d.rho11)
    assert np.array_equal(ref["n_outer"], got["n_outer"])
    d = _box_sample(255, seed=3)
    m, ref = PT.run_oracle(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, O.Params(), theta)
    _, got = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=PAIRED)
    _compare(ref, got, m.w2, model=m, rho11=d.rho11)
    for sp in ((O.NU_E, O.NU_E_BAR), (O.NU_X,)):
        dd = W.radial_profile(P=1 << 16, ns=len(sp)).take(np.arange(0, 1 << 16, 512))
        m, ref = PT.run_oracle(dd, sp, O.ALL_PHYSICS, W.DTAU_KM, O.Params(), theta)
        _, got = PT.run_gpu(dd, sp, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=PAIRED)
        _compare(ref, got, m.w2, model=m, rho11=dd.rho11, species=sp)


def test_paired_mixed_neighbours():
    """Interleave transparent (skipped), stiff and ordinary points, so that the
    two halves of most waves differ in iteration counts and paths."""
    _say("paired: alternating skipped / stiff / ordinary neighbours, P=301")
    full = W.radial_profile(P=1 << 16)
    idx = np.stack([np.arange(0, 100) * 200, 60000 + np.arange(0, 100) * 50, np.arange(0, 100) * 7 + 1000], 1)
    idx = np.concatenate([idx.ravel(), [65535]])
    d = full.take(idx)
    theta = _theta(32)
    m, ref = PT.run_oracle(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, O.Params(), theta)
    _, got = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=PAIRED)
    _compare(ref, got, m.w2, model=m, rho11=d.rho11)
    assert np.array_equal(ref["n_outer"], got["n_outer"])
    skip = ref["n_outer"] == 0
    assert skip.any() and (~skip).any()
    assert np.array_equal(got["D"][skip], got["D0"][skip])


def test_paired_caps_statuses_and_eos_exits():
    _say("paired: iteration caps (exact statuses and counts), EOS-domain exits")
    d = W.radial_profile(P=1 << 16).take(np.arange(0, 1 << 15, 64))
    theta = _theta(32)
    for kw in (dict(max_inner=2), dict(max_outer=1)):
        m, ref = PT.run_oracle(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, O.Params(**kw), theta)
        _, got = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(**kw), theta, launch=PAIRED)
        assert np.array_equal(ref["status"], got["status"]), kw
        assert np.any(got["status"] != O.OK), kw
        assert np.array_equal(ref["n_inner"], got["n_inner"]) and np.array_equal(ref["n_outer"], got["n_outer"])
        _compare(ref, got, m.w2, model=m, rho11=d.rho11)
    d = W.uniform_box(P=1023, seed=7)
    m, ref = PT.run_oracle(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, O.Params(), theta)
    _, got = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=PAIRED)
    bad = ref["status"] == O.EOS_DOMAIN
    assert bad.any()
    assert np.array_equal(ref["status"], got["status"])
    eD, eI, _, _ = PT.parity_errors({k: v[bad] for k, v in ref.items()}, {k: v[bad] for k, v in got.items()}, m.w2)
    assert eD.max() <= 1e-5 and eI.max() <= 1e-5
    ok = ~bad
    _compare({k: v[ok] for k, v in ref.items()}, {k: v[ok] for k, v in got.items()}, m.w2, model=m,
             rho11=d.rho11[ok])


def test_paired_fixed_matter_and_single():
    _say("paired: emission/absorption closed form (fixed matter), P=1")
    d = W.emab_iso_fixed(P=999)
    sp = (O.NU_E, O.NU_E_BAR)
    fl = O.EMAB | O.ISO
    theta = _theta(32, 0.0, 0.0)
    m, ref = PT.run_oracle(d, sp, fl, W.DTAU_KM, O.Params(fixed_matter=True), theta)
    _, got = PT.run_gpu(d, sp, fl, W.DTAU_KM, S.Params(fixed_matter=True), theta, launch=PAIRED)
    _compare(ref, got, m.w2)
    assert np.all(got["n_inner"] == 2) and np.all(got["n_outer"] == 1)
    d = W.uniform_box(P=1, seed=11)
    theta = _theta(32)
    mo, ref = PT.run_oracle(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, O.Params(), theta)
    _, got = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=PAIRED)
    _compare(ref, got, mo.w2, model=mo, rho11=d.rho11)


@pytest.mark.parametrize("launch", [S.LaunchConfig(kernel_store=N.KERNELS_PAIRED, persistent=False, chunk=1),
                                    S.LaunchConfig(kernel_store=N.KERNELS_PAIRED, persistent=True, chunk=3,
                                                   blocks_per_cu=1),
                                    S.LaunchConfig(kernel_store=N.KERNELS_PAIRED, persistent=True, chunk=1,
                                                   blocks_per_cu=2)])
def test_paired_ragged_launches_bitwise(launch):
    _say(f"paired ragged launch {launch}")
    d = W.radial_profile(P=1 << 16).take(np.arange(20000, 20000 + 1037))
    theta = _theta(32)
    _, a = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=PAIRED)
    _, b = PT.run_gpu(d, ALL3, O.ALL_PHYSICS, W.DTAU_KM, S.Params(), theta, launch=launch)
    for k in ("D", "I", "ye", "e", "T", "n_outer", "n_inner", "status"):
        assert np.array_equal(a[k], b[k]), k
