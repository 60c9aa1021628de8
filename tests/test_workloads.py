"""Host-side checks of the seeded workload draws (no GPU)."""
import numpy as np

from paper_2601_00976_amd import workloads as W


def test_moving_profile_draws():
    a = W.radial_profile_v(P=4096)
    b = W.radial_profile_v(P=4096)
    for k in ("T", "rho11", "ye", "uD", "uI", "v", "uI3"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert a.v.shape == (4096, 3) and a.uI3.shape == (4096, 3, 3, 32)
    speed = np.linalg.norm(a.v, axis=1)
    # the fixed-point map of the moment equations is a contraction below
    # sqrt(2) - 1 (remark on the step-size parameter)
    assert speed.max() < np.sqrt(2.0) - 1.0
    # infall: the velocity points inward (against the radial direction) away
    # from the centre, where it vanishes up to the noise
    r = a.r_km
    assert np.median(speed[r > 150]) > 0.08 and np.median(speed[r < 5]) < 0.02
    # the static profile's draws are those of its own workload id
    s = W.radial_profile(P=4096)
    assert not np.array_equal(s.T, a.T)
    assert np.all(np.abs(a.uI3) <= 1.0)


def test_take_keeps_velocity_fields():
    a = W.radial_profile_v(P=512)
    idx = np.array([3, 100, 511])
    t = a.take(idx)
    assert np.array_equal(t.v, a.v[idx]) and np.array_equal(t.uI3, a.uI3[idx])
    assert t.P == 3
