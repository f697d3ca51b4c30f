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


# ----------------------------------------- the sweep runner's analysis (f1) --
def test_refine_minimum_on_synthetic_series():
    """The V_min refinement: exact for samples of a parabola, the plain sample at
    the ends, around non-finite neighbours and where the parabola does not open
    upward; NaN for an all-NaN series."""
    t = np.linspace(0.0, 1.0, 21)
    for t0, v0 in ((0.437, 0.61), (0.5, 0.2), (0.52, -1.0)):
        v = 3.0 * (t - t0) ** 2 + v0
        tm, vm = S.refine_minimum(t, v)
        assert abs(tm - t0) <= 1e-12 and abs(vm - v0) <= 1e-12
    # minimum at the first / last sample: no refinement
    assert S.refine_minimum(t, t) == (0.0, 0.0)
    assert S.refine_minimum(t, -t) == (1.0, -1.0)
    # a NaN next to the minimum: the sample itself
    v = (t - 0.437) ** 2
    v[9] = np.nan
    k = int(np.nanargmin(v))
    assert S.refine_minimum(t, v) == (t[k], v[k])
    # flat around the minimum (no upward parabola): the sample itself
    v = np.ones_like(t)
    assert S.refine_minimum(t, v) == (0.0, 1.0)
    tm, vm = S.refine_minimum(t, np.full_like(t, np.nan))
    assert np.isnan(tm) and np.isnan(vm)


def test_squeezing_onset_prediction_closed_forms():
    """t_sqz = 0.05 n_tot / |<H_int>| (Sec. II.E) against closed forms: the
    single-mode Kerr field, <H_int> = (Lambda/2)|z|^4, so t_sqz = 0.1 / (Lambda
    |z|^2); and the paper's long-range coherent problem, where n_tot |chi| =
    |<H_int>| / n_tot = |0.13 + 0.08 sqrt(2) cos(theta1 + theta3 - 2 theta2)| for
    every r (pin P10), so t_sqz = 0.05 / that."""
    import math

    for Lam, z in ((0.01, 7.0 * np.exp(0.3j)), (0.2, 1.5)):
        t, n, e = S.squeezing_onset_prediction(np.ones((1, 1, 1, 1)), Lam, [z])
        assert abs(t - 0.1 / (Lam * abs(z) ** 2)) <= 1e-12 * t
        assert abs(n - abs(z) ** 2) <= 1e-12 and abs(e - 0.5 * Lam * abs(z) ** 4) <= 1e-9
    for r in (1, 2, 8):
        w = W.paper_problem("coherent", "longrange", r)
        z = w.init_params[0]
        th = np.angle(z[1:4])
        nchi = abs(0.13 + 0.08 * math.sqrt(2) * math.cos(th[0] + th[2] - 2 * th[1]))
        t, n, _ = S.squeezing_onset_prediction(w.V, w.Lambda, z)
        assert abs(n - 5 * r) <= 1e-12
        assert abs(t - 0.05 / nchi) <= 1e-12 * t
    t, _, _ = S.squeezing_onset_prediction(np.zeros((2,) * 4), 0.3, [1.0, 2.0])
    assert t == float("inf")


def test_classical_distance_at_t0(oracle_lib):
    """Sec. IV.B distance sum_k |<n_k> - |alpha_k|^2| / n_tot at t = 0, from the
    oracle's moments of the paper's coherent state (r = 1): zero up to the
    truncation when every sector up to a far Poisson tail is kept, and the
    dropped weight's order (< 5e-3) with the 0.999 truncation the runner uses."""
    from oracle import Oracle, derived, states

    w = W.paper_problem("coherent", "longrange", 1)
    z = w.init_params[0]
    n_tot = float(np.sum(np.abs(z) ** 2))
    for nmax, bound in ((30, 1e-12), (S.poisson_nmax(n_tot), 5e-3)):
        o = Oracle(w.M, w.M, w.omega, w.Lambda, w.V, W.all_sectors(w.M, nmax))
        d = derived.observe(o, states.coherent_state(o, z))
        dev = S.classical_distance(np.real(np.diag(d["M"]))[None, :], (np.abs(z) ** 2)[None, :], n_tot)
        assert dev.shape == (1,) and 0.0 <= dev[0] <= bound
    # two records, one mode off by 1 in the second: distance 1 / n_tot there
    nm = np.array([[1.0, 2.0], [1.0, 3.0]])
    np.testing.assert_allclose(S.classical_distance(nm, [[1.0, 2.0], [1.0, 2.0]], 4.0), [0.0, 0.25])
