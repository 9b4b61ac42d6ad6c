"""Pins of the oracle's sampler (Alg. 1 "uniformly sample Q"; Sec. III-A):
Philox4x32-10 against the published Random123 known-answer vectors, the
24-bit unit mapping against its lattice, and the distribution against a
Kolmogorov-Smirnov test."""
import os

import numpy as np
import pytest
from scipy import stats

import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(orc, ctr, key, out):
    assert list(orc.philox4x32_10(ctr, key)) == out


def test_words_counter_layout(orc):
    # counter = (n, m, stage, stream << 16 | block), key = (seed lo, seed hi)
    seed = 0x0123456789ABCDEF
    w = orc.sample_words(seed, 7, 0, 5, 3, 1)
    ref = orc.philox4x32_10([5, 3, 7, (0 << 16) | 1], [seed & 0xFFFFFFFF, seed >> 32])
    assert list(w) == list(ref)


def test_samples_in_box_on_24bit_lattice(orc):
    lo, hi = wl.box_limits("point2d", 2)
    Q = orc.sample_layers(3, 500, 2, lo, hi, seed=11, stage=0)
    assert Q.dtype == np.float32
    assert np.all(Q >= lo) and np.all(Q < hi)
    # on the unit box the sample is the unit itself: (w >> 8) * 2^-24, an
    # integer multiple of 2^-24 whose top byte-shifted word is the Philox word
    z, one = np.zeros(2, np.float32), np.ones(2, np.float32)
    U = orc.sample_layers(2, 40, 2, z, one, seed=11, stage=3)
    k = U.astype(np.float64) * 2**24
    assert np.array_equal(k, np.round(k)) and k.min() >= 0 and k.max() < 2**24
    w = orc.sample_words(11, 3, 0, 7, 1, 0)
    assert int(k[1, 7, 0]) == int(w[0]) >> 8 and int(k[1, 7, 1]) == int(w[1]) >> 8


def test_samples_uniform_ks(orc):
    lo, hi = wl.box_limits("arm", 7)
    Q = orc.sample_layers(2, 4000, 7, lo, hi, seed=3, stage=5).reshape(-1, 7).astype(np.float64)
    for j in range(7):
        p = stats.kstest(Q[:, j], stats.uniform(loc=lo[j], scale=hi[j] - lo[j]).cdf).pvalue
        assert p > 1e-4, (j, p)
    # coordinates are uncorrelated
    c = np.corrcoef(Q.T)
    assert np.max(np.abs(c - np.eye(7))) < 0.05


def test_samples_deterministic_and_stage_dependent(orc):
    lo, hi = wl.box_limits("point2d", 2)
    a = orc.sample_layers(2, 64, 2, lo, hi, seed=1, stage=0)
    b = orc.sample_layers(2, 64, 2, lo, hi, seed=1, stage=0)
    c = orc.sample_layers(2, 64, 2, lo, hi, seed=1, stage=1)
    d = orc.sample_layers(2, 64, 2, lo, hi, seed=2, stage=0)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert not np.array_equal(a, d)


def test_layer_coverage_of_a_corridor():
    """Sec. III (Layered Sampling Model): a layer of N independent draws misses
    a set A with probability (1 - pi(A))^N for the uniform sampler, within the
    paper's bound (1 - pi(A)/2)^N for the fair-coin mixture.  A = the corridor
    |x| <= 0.5 of the 2D box [-10, 10]^2, pi(A) = 0.05, N = 40."""
    import oracle
    from scipy import stats
    lo, hi = np.array([-10.0, -10.0]), np.array([10.0, 10.0])
    N, trials = 40, 3000
    miss = 0
    for t in range(trials):
        Q = oracle.sample_layers(1, N, 2, lo, hi, 1000 + t, 7)[0]
        miss += int(not np.any(np.abs(Q[:, 0]) <= 0.5))
    p_exact = (1 - 0.05) ** N
    assert stats.binomtest(miss, trials, p_exact).pvalue > 1e-3
    assert miss / trials <= (1 - 0.05 / 2) ** N
