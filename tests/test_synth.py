"""The seeded input generators match the workload recipe (no GPU): the
Gaussian random field has the squared-exponential covariance it is built
from (variance and correlation at several lags, estimated over many seeds),
the contrast rescaling makes k span exactly [c^-1/2, c^1/2], the contrast is
drawn inside its range, and seeds reproduce their systems."""
import numpy as np
import pytest

import synth


def _samples(n, h, count, ell=0.1):
    return np.stack([synth.grf(synth.rng(5000 + s), n, h, ell) for s in range(count)])


def test_grf_variance_and_correlation():
    n, h, ell = 32, 1.0 / 33, 0.1
    z = _samples(n, h, 400, ell)
    assert abs(np.mean(z)) < 0.05
    assert abs(np.mean(z * z) - 1.0) < 0.05
    for lag in (1, 3, 6):
        d = lag * h
        want = np.exp(-d * d / (2 * ell * ell))
        got_x = np.mean(z[:, lag:, :] * z[:, :-lag, :])
        got_y = np.mean(z[:, :, lag:] * z[:, :, :-lag])
        assert abs(got_x - want) < 0.05 and abs(got_y - want) < 0.05, (lag, want, got_x, got_y)
    # a diagonal lag: the covariance is a product of the two directions
    d2 = 2 * (3 * h) ** 2
    got_d = np.mean(z[:, 3:, 3:] * z[:, :-3, :-3])
    assert abs(got_d - np.exp(-d2 / (2 * ell * ell))) < 0.05


@pytest.mark.parametrize("N", [16, 33, 64])
def test_contrast_rescaling_spans_the_range(N):
    for seed in range(5):
        k, f, u0, c = synth.system(100 + seed, N, (10.0, 1000.0))
        assert 10.0 <= c <= 1000.0
        assert k.shape == (N + 2, N + 2) and f.shape == (N, N) and u0.shape == (N, N)
        assert np.isclose(k.max() / k.min(), c, rtol=1e-12)
        assert np.isclose(k.max() * k.min(), 1.0, rtol=1e-12)
        assert np.all(k > 0)


def test_seeds_reproduce_systems_and_batches_stack_them():
    a = synth.system(7, 24, (10.0, 1000.0))
    b = synth.system(7, 24, (10.0, 1000.0))
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    k, f, u0, cs = synth.batch(3, 4, 24, (10.0, 1000.0))
    assert k.shape == (4, 26, 26) and f.shape == (4, 24, 24) and u0.shape == (4, 24, 24)
    one = synth.system(3000 + 2, 24, (10.0, 1000.0))
    assert np.array_equal(k[2], one[0]) and np.array_equal(f[2], one[1])
