"""Pins of the oracle's statistical tests (Sec. III: Eqs. 4-11) against what
the mathematics and the paper fix, and of the library's host-side formulas
(which work from integer counts) against the oracle.

* Eq. 4 equals the population variance of the 256 counts (numpy.var); a
  uniform histogram gives 0 and a one-level histogram of N pixels gives
  255 N^2 / 256^2.
* Eq. 5 equals scipy's chi-square statistic against equal expected counts;
  a one-level histogram gives 255 N; the critical value 293.25 is scipy's
  95% quantile of chi-square with 255 degrees of freedom.
* Eq. 10 equals scipy's entropy in base 2; 256 equiprobable levels give
  8 bits, two give 1, one gives 0.
* Eq. 11 on uniformly random bytes: the mean over many frames meets the
  paper's ideal 7.902469317 for k = 30, T_B = 1936 and lies in its
  interval; single frames spread as the plug-in entropy's variance says.
* Eqs. 6-9 equal numpy.corrcoef on the same pairs; a ramp correlates +1,
  a checkerboard -1 horizontally and vertically and +1 diagonally;
  independent random bytes give |r| of order 1/sqrt(N).
* Pair moments match a pure-Python loop over a tiny frame."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import stats as O


def rand_frame(rng, h, w):
    return rng.integers(0, 256, (h, w, 3), dtype=np.uint8)


# ---------------------------------------------------------------- histograms

def test_histogram_matches_bincount_and_brute_force():
    rng = np.random.default_rng(1)
    f = rand_frame(rng, 37, 41)
    H = O.frame_histograms(f)
    for c in range(3):
        assert np.array_equal(H[c], np.bincount(f[..., c].ravel(), minlength=256))
    tiny = rand_frame(rng, 3, 4)
    for c in range(3):
        brute = [0] * 256
        for r in range(3):
            for x in range(4):
                brute[int(tiny[r, x, c])] += 1
        assert list(O.frame_histograms(tiny)[c]) == brute


# ---------------------------------------------------------------- Eq. 4

def test_variance_is_population_variance_of_counts():
    rng = np.random.default_rng(2)
    for _ in range(5):
        z = rng.integers(0, 5000, 256)
        assert O.histogram_variance(z) == pytest.approx(np.var(z.astype(np.float64)), rel=1e-12)


def test_variance_special_cases():
    assert O.histogram_variance(np.full(256, 17)) == 0.0
    z = np.zeros(256, dtype=np.int64)
    z[200] = 1000
    assert O.histogram_variance(z) == pytest.approx(255 * 1000 ** 2 / 256 ** 2, rel=1e-14)


# ---------------------------------------------------------------- Eq. 5

def test_chi_square_matches_scipy():
    rng = np.random.default_rng(3)
    z = np.bincount(rng.integers(0, 256, 512 * 512), minlength=256)
    assert O.chi_square(z) == pytest.approx(scipy.stats.chisquare(z).statistic, rel=1e-12)


def test_chi_square_special_cases_and_critical_value():
    assert O.chi_square(np.full(256, 9)) == 0.0
    z = np.zeros(256, dtype=np.int64)
    z[0] = 4096
    assert O.chi_square(z) == pytest.approx(255 * 4096, rel=1e-14)
    # the paper's critical value at alpha = 0.05 with 255 degrees of freedom
    assert round(scipy.stats.chi2.ppf(0.95, 255), 2) == 293.25


# ---------------------------------------------------------------- Eq. 10

def test_entropy_matches_scipy_and_special_cases():
    rng = np.random.default_rng(4)
    z = rng.integers(0, 300, 256)
    z[rng.integers(0, 256, 20)] = 0
    assert O.entropy(z) == pytest.approx(scipy.stats.entropy(z, base=2), rel=1e-12)
    assert O.entropy(np.full(256, 3)) == pytest.approx(8.0, rel=1e-15)
    two = np.zeros(256, dtype=np.int64)
    two[[5, 77]] = 11
    assert O.entropy(two) == pytest.approx(1.0, rel=1e-15)
    one = np.zeros(256, dtype=np.int64)
    one[9] = 100
    assert O.entropy(one) == 0.0


# ---------------------------------------------------------------- Eq. 11

def origins_grid(rng, h, w, k=30, side=44):
    cells = rng.choice((h // side) * (w // side), size=k, replace=False)
    gc = w // side
    return np.stack([(cells // gc) * side, (cells % gc) * side], axis=1)


def test_local_entropy_is_mean_of_block_entropies():
    rng = np.random.default_rng(5)
    f = rand_frame(rng, 300, 400)
    org = origins_grid(rng, 300, 400)
    for c in range(3):
        ents = [scipy.stats.entropy(np.bincount(f[r:r + 44, x:x + 44, c].ravel(), minlength=256), base=2)
                for r, x in org]
        assert O.local_entropy(f, c, org, 44, 44) == pytest.approx(np.mean(ents), rel=1e-12)
    assert O.local_entropy(np.zeros((300, 400, 3), np.uint8), 0, org, 44, 44) == 0.0


def test_local_entropy_of_random_bytes_meets_the_papers_ideal():
    """k = 30 blocks of T_B = 1936 random bytes: the mean over frames meets
    the paper's ideal value (Sec. III-C) and lies inside its interval; the
    spread of single frames matches the second-order variance of the
    plug-in entropy of a uniform source, (K - 1) / (2 T_B^2 ln^2 2) per
    block with K = 256 levels, divided by k."""
    rng = np.random.default_rng(6)
    vals = []
    for _ in range(40):
        f = rand_frame(rng, 264, 352)   # 6 x 8 cells of 44 x 44
        org = origins_grid(rng, 264, 352)
        vals += [O.local_entropy(f, c, org, 44, 44) for c in range(3)]
    vals = np.array(vals)
    sd = math.sqrt(255 / (2 * 1936 ** 2 * math.log(2) ** 2) / 30)    # about 1.54e-3
    assert abs(vals.mean() - 7.902469317) < 4 * sd / math.sqrt(len(vals))
    assert 7.901515798 < vals.mean() < 7.903422936
    assert 0.75 * sd < vals.std() < 1.25 * sd


# ---------------------------------------------------------------- Eqs. 6-9

def test_correlation_matches_corrcoef():
    rng = np.random.default_rng(7)
    f = rand_frame(rng, 60, 70)
    f[..., 1] = np.minimum(255, f[..., 0].astype(np.int32) // 2 + 40).astype(np.uint8)
    pos = np.stack([rng.integers(0, 59, 3000), rng.integers(0, 69, 3000)], axis=1)
    for d in range(3):
        for c in range(3):
            x, y = O.pairs(f, c, d, pos)
            assert O.correlation(f, c, d, pos) == pytest.approx(np.corrcoef(x, y)[0, 1], rel=1e-10, abs=1e-12)


def test_correlation_special_cases():
    h, w = 20, 30
    ramp = np.zeros((h, w, 3), np.uint8)
    ramp[...] = (np.arange(w, dtype=np.uint8) * 7 + 3)[None, :, None]
    ramp = ramp + (np.arange(h, dtype=np.uint8) * 2)[:, None, None]
    for d in range(3):
        assert O.correlation(ramp, 0, d) == pytest.approx(1.0, abs=1e-12)
    chk = ((np.arange(h)[:, None] + np.arange(w)[None, :]) % 2 * 255).astype(np.uint8)
    chk = np.repeat(chk[..., None], 3, axis=2)
    assert O.correlation(chk, 1, 0) == pytest.approx(-1.0, abs=1e-12)
    assert O.correlation(chk, 1, 1) == pytest.approx(-1.0, abs=1e-12)
    assert O.correlation(chk, 1, 2) == pytest.approx(1.0, abs=1e-12)
    rng = np.random.default_rng(8)
    f = rand_frame(rng, 300, 400)
    for d in range(3):
        assert abs(O.correlation(f, 2, d)) < 5 / math.sqrt(299 * 399)


def test_pair_moments_brute_force():
    rng = np.random.default_rng(9)
    f = rand_frame(rng, 5, 6)
    want = np.zeros((3, 3, 5), dtype=np.int64)
    for d, (dr, dc) in enumerate([(0, 1), (1, 0), (1, 1)]):
        for c in range(3):
            for r in range(4):
                for x in range(5):
                    a, b = int(f[r, x, c]), int(f[r + dr, x + dc, c])
                    want[d, c] += [a, b, a * a, b * b, a * b]
    assert np.array_equal(O.pair_moments(f), want)
    pos = np.array([[0, 0], [3, 4], [3, 4], [2, 1]])
    want = np.zeros((3, 3, 5), dtype=np.int64)
    for d, (dr, dc) in enumerate([(0, 1), (1, 0), (1, 1)]):
        for c in range(3):
            for r, x in pos:
                a, b = int(f[r, x, c]), int(f[r + dr, x + dc, c])
                want[d, c] += [a, b, a * a, b * b, a * b]
    assert np.array_equal(O.pair_moments(f, pos), want)


# ------------------------------------------- library host formulas vs oracle

def test_library_formulas_from_counts_match_the_oracle():
    from paper_2505_07158_amd import stats as S
    rng = np.random.default_rng(10)
    f = rand_frame(rng, 200, 330)
    f[..., 2] = (f[..., 2] // 16) * 16   # 16 levels only
    H = O.frame_histograms(f)
    for c in range(3):
        assert S.histogram_variance(H[c]) == pytest.approx(O.histogram_variance(H[c]), rel=1e-12)
        assert S.chi_square(H[c]) == pytest.approx(O.chi_square(H[c]), rel=1e-12)
        assert S.entropy(H[c]) == pytest.approx(O.entropy(H[c]), rel=1e-12)
    pos = S.sample_pair_positions(rng, 200, 330, 5000).astype(np.int64)
    M = O.pair_moments(f, pos)
    for d in range(3):
        for c in range(3):
            assert S.correlation(M[d, c], len(pos)) == pytest.approx(O.correlation(f, c, d, pos), rel=1e-10)
    assert math.isnan(S.correlation([5, 5, 5, 5, 5], 5))   # constant x: undefined


def test_library_samplers():
    from paper_2505_07158_amd import stats as S
    rng = np.random.default_rng(11)
    pos = S.sample_pair_positions(rng, 7, 9, 20000)
    assert pos[:, 0].max() == 5 and pos[:, 1].max() == 7 and pos.min() == 0
    org = S.sample_block_origins(rng, 1080, 1920)
    assert org.shape == (30, 2) and len({tuple(o) for o in org}) == 30
    assert (org % 44 == 0).all() and (org[:, 0] + 44 <= 1080).all() and (org[:, 1] + 44 <= 1920).all()
    with pytest.raises(ValueError):
        S.sample_block_origins(rng, 100, 100)
    with pytest.raises(ValueError):
        S.sample_pair_positions(rng, 1, 100)
    assert S.CHI2_CRITICAL == 293.25 and S.LSE_INTERVAL == (7.901515798, 7.903422936)
