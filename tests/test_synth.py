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


def test_crater_field_vertical_axis_is_a_relabelling():
    from synth.generators import crater_density
    a = crater_density((6, 4, 5), (1.0, 0.3, 0.8), seed=2, up=1)   # y vertical
    b = crater_density((6, 5, 4), (1.0, 0.8, 0.3), seed=2, up=2)   # z vertical, y and z swapped
    assert np.allclose(a.reshape(5, 4, 6).transpose(1, 0, 2), b.reshape(4, 5, 6))


def test_slab_workloads_have_the_paper_shape():
    for parts in (32, 64, 128):
        wl = workload(f"slab{parts}")
        assert wl.nparts == (parts, 1, 1) and wl.tol == 1e-6 and wl.up == 2
        widths = np.diff([0, *wl.cuts[0], wl.ne[0]])
        assert widths.sum() == 320 and widths.max() - widths.min() <= 1
        assert abs(wl.lengths[2] / wl.lengths[0] - 15.0 / 250.0) < 1e-12 and wl.lengths[1] == wl.lengths[0]
        assert wl.n_nodes == 641 * 641 * 39
        assert wl.extra["kmin"] < wl.extra["kmax"]
