"""CMA-ES search of the transmission coefficients (Sec. 4) in the native
library (host code, no GPU), against the oracle's closed form, brute-force
grid minimax, its own cost evaluation and the paper's Table 1."""
import os

import numpy as np
import pytest

from oracle import fourier
from paper_2112_03851_amd import sos

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_cmaes.txt")
KMIN, KMAX = 0.0174, 1.0


def table1():
    rows = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            name, *v = line.split()
            rows[name] = [float(x) for x in v]
    return rows


def test_zeroth_order_symmetric_matches_closed_form():
    pq, rho, it = sos.optimize_robin(0, KMIN, KMAX)
    p, r = fourier.oo0_symmetric_optimum(KMIN, KMAX)
    assert abs(pq[0] - p) <= 1e-6 * p and pq[0] == pq[2] and pq[1] == pq[3] == 0.0
    assert abs(rho - r) <= 1e-9
    assert it < 7200


@pytest.mark.parametrize("kind", [1, 2])
def test_two_parameter_optimum_at_least_as_good_as_grid_minimax(kind):
    pq, rho, _ = sos.optimize_robin(kind, KMIN, KMAX)
    grid, _ = fourier.grid_minimax(kind, KMIN, KMAX)
    assert rho <= grid * (1 + 1e-3)


@pytest.mark.parametrize("kind,name", [(0, "oo0_symmetric"), (1, "oo0_unsymmetric"),
                                       (2, "oo2_symmetric"), (3, "oo2_unsymmetric")])
def test_optimum_no_worse_than_table1_and_cost_consistent(kind, name):
    pq, rho, it = sos.optimize_robin(kind, KMIN, KMAX, seed=7)
    ref = table1()[name][4]
    assert rho <= ref
    # the oracle's evaluation of the returned coefficients on a finer sampling
    dense = fourier.rho_max(*pq, KMIN, KMAX, n=200001)
    assert rho <= dense <= rho * (1 + 1e-4)
    assert all(v >= 0 for v in pq)


def test_deterministic_for_a_seed_and_rejects_bad_arguments():
    a = sos.optimize_robin(3, KMIN, KMAX, seed=3)
    b = sos.optimize_robin(3, KMIN, KMAX, seed=3)
    assert a == b
    for args in [(4, KMIN, KMAX), (0, 0.0, KMAX), (0, 1.0, 0.5)]:
        with pytest.raises(sos.SosError):
            sos.optimize_robin(*args)
    with pytest.raises(sos.SosError):
        sos.optimize_robin(0, KMIN, KMAX, popsize=2)
