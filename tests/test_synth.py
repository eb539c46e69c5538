"""CPU checks of the seeded input generators that are not part of the method."""
import numpy as np

from synth import workload
from synth.generators import robin_candidates


def test_robin_candidates_ranges_and_determinism():
    h = 1.0 / 32
    p, q = robin_candidates(128, h, seed=0)
    assert p.shape == q.shape == (128,)
    assert np.all(p >= h ** -1.5) and np.all(p <= 10.0 / h)
    assert np.all(q >= 0.0) and np.all(q <= h)
    # log-uniform in p: log p spreads over the whole log range
    lp = (np.log(p) - np.log(h ** -1.5)) / (np.log(10.0 / h) - np.log(h ** -1.5))
    assert lp.min() < 0.05 and lp.max() > 0.95 and abs(lp.mean() - 0.5) < 0.1
    p2, q2 = robin_candidates(128, h, seed=0)
    assert np.array_equal(p, p2) and np.array_equal(q, q2)
    p3, _ = robin_candidates(128, h, seed=1)
    assert not np.array_equal(p, p3)


def test_candidate_copy_workload_matches_the_large_one_per_subdomain():
    small, large = workload("c5copy"), workload("c5")
    # both have 16^3-element subdomains, so p h and q / h carry over
    assert [small.ne[a] // (len(small.cuts[a]) + 1) for a in range(3)] == [16, 16, 16]
    assert [large.ne[a] // (len(large.cuts[a]) + 1) for a in range(3)] == [16, 16, 16]
