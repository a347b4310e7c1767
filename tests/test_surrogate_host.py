"""Host logic of the surrogate's calibration (no GPU)."""
import math

import numpy as np
import pytest

from paper_2306_07552_amd import surrogate


def _normal_cdf(x):
    return 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_skip_threshold_skips_no_held_out_positive(seed):
    rng = np.random.default_rng(seed)
    z = rng.normal(3.0, 2.0, 20000)
    p = 1.0 / (1.0 + np.exp(-z))
    skip, tau = surrogate.skip_threshold(p, safety=0.25)
    assert tau == pytest.approx(p.min())
    assert skip <= 0.25 * tau
    assert (p <= skip).sum() == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_skip_threshold_extrapolates_the_tail(seed):
    """Positive logits ~ N(3, 2): with n held-out positives the smallest sits
    near the 1/n quantile; the threshold must leave a true tail mass well
    below 1/n, so that a deployment with many more positives than the
    held-out set skips none of them."""
    rng = np.random.default_rng(seed)
    n = 30000
    z = rng.normal(3.0, 2.0, n)
    p = 1.0 / (1.0 + np.exp(-z))
    skip, _ = surrogate.skip_threshold(p, safety=0.25)
    z_skip = math.log(skip) - math.log1p(-skip)
    mass = _normal_cdf((z_skip - 3.0) / 2.0)
    assert mass < 0.05 / n


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_skip_threshold_heavy_tail(seed):
    """Positive logits with an exponential lower tail (Laplace(3, 1.5)): a
    fixed factor below the smallest probability leaves a tail mass of order
    1/n; the tail extrapolation leaves at most a quarter of it."""
    rng = np.random.default_rng(seed)
    n = 30000
    z = rng.laplace(3.0, 1.5, n)
    p = 1.0 / (1.0 + np.exp(-z))
    skip, tau = surrogate.skip_threshold(p, safety=0.25)
    tail = lambda x: 0.5 * math.exp((x - 3.0) / 1.5)   # P(z < x) below the median
    z_skip = math.log(skip) - math.log1p(-skip)
    z_fixed = math.log(0.25 * tau) - math.log1p(-0.25 * tau)
    assert tail(z_skip) < 0.25 * tail(z_fixed)
    assert tail(z_skip) < 0.2 / n


def test_skip_threshold_without_positives():
    skip, tau = surrogate.skip_threshold(np.zeros(0), safety=0.25)
    assert tau == 1.0 and skip == 0.25
