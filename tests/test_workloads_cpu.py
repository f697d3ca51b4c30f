"""Input generators of the paper's test problems (host only)."""
import os
import sys

import numpy as np
import pytest

import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads"))
import breaktime_sweep as S  # noqa: E402


@pytest.mark.parametrize("n", [5.0, 10.0, 20.0, 40.0, 80.0, 120.0])
def test_poisson_truncation_matches_scipy(n):
    """Sec. IV.A truncation: the smallest N_max with Poisson weight >= 0.999."""
    from scipy.stats import poisson

    assert S.poisson_nmax(n) == int(poisson.ppf(0.999, n))


def test_exact_interactions_conserve_exactly():
    M = 5
    for V in (W.V_contact_exact(M), W.V_longrange_exact(M)):
        i, j, k, l = np.nonzero(V)
        assert np.all(i + j == k + l)
    # every transfer term of the long-range form is 1/q^2 with q = k - i != 0
    V = W.V_longrange_exact(M)
    for i, j, k, l in zip(*np.nonzero(V)):
        assert k != i and V[i, j, k, l] == 1.0 / (k - i) ** 2
    # ... and it is not the periodic one: 0 + 4 -> 1 + 3 is allowed with q = 1, 4 + 4 -> 3 + 0 (mod 5) is not
    assert W.V_longrange_exact(M)[0, 4, 1, 3] == 1.0
    assert W.V_longrange_exact(M)[4, 4, 3, 0] == 0.0 and W.V_longrange(M)[4, 4, 3, 0] != 0.0


def test_paper_problem_states():
    w = W.paper_problem("number", "longrange", 3)
    assert list(w.init_params) == [0, 6, 6, 3, 0]
    assert w.meta["P_exact"] == 6 + 12 + 9
    assert w.sectors == [(15, 27 % 5)]
    wc = W.paper_problem("coherent", "contact-", 2)
    z = wc.init_params[0]
    np.testing.assert_allclose(np.abs(z) ** 2, [0, 4, 4, 2, 0], atol=1e-12)
    assert wc.Lambda == pytest.approx(-0.05) and np.allclose(wc.omega, np.arange(5) / 2)
    # the same phases for every r and init
    zf = W.paper_problem("fieldnumber", "longrange", 7).init_params[0]
    np.testing.assert_allclose(np.angle(zf[1:4]), np.angle(z[1:4]), atol=1e-12)
    with pytest.raises(ValueError):
        W.paper_problem("number", "other", 1)


def test_periodic_psi_has_no_short_repeats():
    x = W.periodic_psi(3_000_000, 4)
    assert x.dtype == np.complex128
    # indices differing by p1 share the real part but not the imaginary one
    assert x[5].real == x[5 + 1_000_003].real and x[5].imag != x[5 + 1_000_003].imag
