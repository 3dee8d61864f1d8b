"""The seeded input generator's Zipf keys (input generation only): P(k)
proportional to k**-0.5 on 1..N, rows independent of where a chunk starts."""
import math

import numpy as np

from paper_2606_24647_amd import datagen as dg


def test_zipf_thresholds_are_the_distribution_function():
    N = 9
    t = dg.zipf_thresholds(N)
    w = [1 / math.sqrt(k) for k in range(1, N + 1)]
    cdf = np.cumsum(w) / sum(w)
    assert t.dtype == np.uint64 and len(t) == N - 1
    assert np.all(np.diff(t.astype(np.float64)) > 0)
    assert np.allclose(t.astype(np.float64) / 2.0 ** 63, cdf[:-1], rtol=0, atol=1e-15)


def test_zipf_frequencies_match_k_to_the_minus_half():
    N, n = 6, 600_000
    k = dg.zipf(11, 0, 0, n, N)
    freq = np.bincount(k, minlength=N + 1)[1:] / n
    p = np.array([k ** -0.5 for k in range(1, N + 1)])
    p /= p.sum()
    sigma = np.sqrt(p * (1 - p) / n)
    assert np.all(np.abs(freq - p) < 5 * sigma), (freq, p)


def test_zipf_bounds_degenerate_and_chunking():
    assert set(dg.zipf(3, 0, 0, 1000, 1).tolist()) == {1}
    N = 15_000_000
    k = dg.zipf(3, 0, 0, 200_000, N)
    assert k.min() >= 1 and k.max() <= N
    # The top key's share is 1 / H(N, 1/2) = 1.29e-4 (Euler-Maclaurin: 2 sqrt(N) + zeta(1/2)).
    top = 1 / (2 * math.sqrt(N) - 1.4603545)
    assert abs(top - 1.2913e-4) < 1e-7
    assert abs((k == 1).mean() - top) < 6 * math.sqrt(top / 200_000)
    assert np.array_equal(dg.zipf(5, 2, 100, 50, 1000), dg.zipf(5, 2, 0, 150, 1000)[100:])
