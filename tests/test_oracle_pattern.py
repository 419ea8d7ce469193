"""Pins for the oracle's point-pair pattern (Section 3, after Eq. 2: pairs
drawn from an isotropic Gaussian inside the S x S window; Section 4.1:
n = 4096, S = 26, spread 4).

The generator is splitmix64 -> Box-Muller -> floor(sigma*z + 0.5), redrawn
outside the window.  It is pinned to the published splitmix64 outputs, to the
normal distribution, and to the exact probability mass of the rounded,
truncated normal.
"""
import numpy as np
import pytest
from scipy import stats


def test_splitmix64_published_vectors(orc):
    # Published reference outputs of splitmix64 started from state 0.
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
              0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    assert orc.splitmix64(0, 5) == expect


def test_box_muller_is_standard_normal(orc):
    z = orc.normal_draws(12345, 20000)
    assert abs(z.mean()) < 0.03
    assert abs(z.std() - 1.0) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # consecutive draws are independent
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 0.03


def _window(S):
    return -(S // 2), (S - 1) // 2


def _pmf(S, sigma):
    lo, hi = _window(S)
    k = np.arange(lo, hi + 1)
    p = stats.norm.cdf((k + 0.5) / sigma) - stats.norm.cdf((k - 0.5) / sigma)
    return k, p / p.sum()


@pytest.mark.parametrize("S,sigma", [(15, 4 * 15 / 26), (26, 4.0), (31, 4 * 31 / 26), (3, 1.0)])
def test_pattern_bounds_and_distinct(orc, S, sigma):
    pat = orc.make_pattern(7, 4096, S, sigma).astype(int)
    lo, hi = _window(S)
    assert pat.min() >= lo and pat.max() <= hi
    assert not np.any((pat[:, 0] == pat[:, 2]) & (pat[:, 1] == pat[:, 3]))


def test_pattern_deterministic_and_seeded(orc):
    a = orc.make_pattern(99, 1024, 31, 4.77)
    b = orc.make_pattern(99, 1024, 31, 4.77)
    c = orc.make_pattern(100, 1024, 31, 4.77)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    # draws are consumed in pair order, so a longer pattern starts with the
    # shorter one drawn from the same seed
    d = orc.make_pattern(99, 64, 31, 4.77)
    assert np.array_equal(a[:64], d)


@pytest.mark.parametrize("S,sigma", [(26, 4.0), (31, 4 * 31 / 26), (15, 4 * 15 / 26)])
def test_pattern_matches_rounded_truncated_normal(orc, S, sigma):
    pat = orc.make_pattern(2020, 4096, S, sigma).astype(int)
    k, pmf = _pmf(S, sigma)
    exact_mean = (k * pmf).sum()
    exact_std = np.sqrt(((k - exact_mean) ** 2 * pmf).sum())
    p = pat[:, :2].ravel()          # p coordinates: exactly the pmf above
    q = pat[:, 2:].ravel()          # q is conditioned on q != p (tiny effect)
    for s in (p, q):
        assert abs(s.mean() - exact_mean) < 4 * exact_std / np.sqrt(s.size)
        assert abs(s.std() / exact_std - 1.0) < 0.05
    counts = np.array([(p == kk).sum() for kk in k], float)
    expected = pmf * p.size
    keep = expected >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(expected[keep], expected[~keep].sum())
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    # isotropy: x and y spreads agree
    assert abs(pat[:, 0].std() / pat[:, 1].std() - 1) < 0.08


def test_pattern_rejects_bad_args(orc):
    with pytest.raises(ValueError):
        orc.make_pattern(1, 64, 1, 1.0)
    with pytest.raises(ValueError):
        orc.make_pattern(1, 64, 15, 0.0)
