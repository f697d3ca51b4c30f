"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/fockhip.h with the binding's signature, and the host-only
entry points (argument validation, fh_derive) behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fockhip.h")
LIB = os.path.join(ROOT, "paper_2111_00050_amd", "libfockhip.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfockhip.so not built")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fh_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared in fockhip.h but not exported"


def test_binding_covers_the_header():
    import paper_2111_00050_amd as fh

    assert set(header_functions()) == set(fh.SIGNATURES)


def test_host_validation_paths():
    import paper_2111_00050_amd as fh

    lib = fh._lib
    h = ctypes.c_void_p()
    M = 3
    om = np.zeros(M)
    V = np.zeros((M,) * 4)
    # M out of range / pmod != M are rejected before any device work
    assert lib.fh_model_create(11, 11, fh._np_ptr(np.zeros(11)), 1.0, fh._np_ptr(np.zeros((11,) * 4)),
                               ctypes.byref(h)) == fh.FH_EUNSUPPORTED
    assert lib.fh_model_create(M, M + 1, fh._np_ptr(om), 1.0, fh._np_ptr(V), ctypes.byref(h)) == fh.FH_EUNSUPPORTED
    # a non-conserving interaction entry: 0 + 0 != 0 + 1 (mod 3)
    Vb = V.copy()
    Vb[0, 0, 0, 1] = 1.0
    assert lib.fh_model_create(M, M, fh._np_ptr(om), 1.0, fh._np_ptr(Vb), ctypes.byref(h)) == fh.FH_EINVAL
    assert b"conserve" in lib.fh_last_error()
    Vn = V.copy()
    Vn[0, 0, 0, 0] = np.nan
    assert lib.fh_model_create(M, M, fh._np_ptr(om), 1.0, fh._np_ptr(Vn), ctypes.byref(h)) == fh.FH_EINVAL
    # duplicate sectors, bad P, no sectors
    N = np.array([4, 4], np.int32)
    P = np.array([1, 1], np.int32)
    assert lib.fh_basis_create(M, M, 2, fh._np_ptr(N), fh._np_ptr(P), ctypes.byref(h)) == fh.FH_EINVAL
    P2 = np.array([0, 3], np.int32)
    assert lib.fh_basis_create(M, M, 2, fh._np_ptr(N), fh._np_ptr(P2), ctypes.byref(h)) == fh.FH_EINVAL
    assert lib.fh_basis_create(M, M, 0, fh._np_ptr(N), fh._np_ptr(P), ctypes.byref(h)) == fh.FH_EINVAL
    # a sector of 2^28 states or more (M=10, N=42: 304,232,500) is refused before any device work
    big_N, big_P = np.array([42], np.int32), np.array([0], np.int32)
    assert lib.fh_basis_create(10, 10, 1, fh._np_ptr(big_N), fh._np_ptr(big_P), ctypes.byref(h)) == fh.FH_EOVERFLOW
    assert b"2^28" in lib.fh_last_error()
    assert lib.fh_adjoint_work_states(0, 10) == -1
    assert lib.fh_adjoint_work_states(3000, 100) == 30 + 100 + 10
    assert lib.fh_adjoint_work_states_kept(3000, 100) == 30 + 400 + 10
    assert lib.fh_adjoint_work_states_kept(7, 100) == 1 + 28 + 10
    assert lib.fh_adjoint_work_states_kept(5, 0) == -1


def test_derive_host_only_against_oracle():
    """fh_derive (own Jacobi eigensolver) against the oracle's numpy path on
    moments of random states: Hermitian M, random <a>, symmetric A."""
    import paper_2111_00050_amd as fh
    from oracle import derived

    rng = np.random.default_rng(3)
    for M in (1, 2, 5, 10):
        X = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
        Mij = X.conj().T @ X + M * np.eye(M)
        a = 0.3 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
        A = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
        A = A + A.T
        n2 = 1.7
        g = fh.derive(M, n2, a * n2, Mij * n2, A * n2)
        o = derived.derive(n2, a * n2, Mij * n2, A * n2)
        for k in ("n_tot", "Q", "lambda_p", "po_deficit", "vminus"):
            assert abs(g[k] - o[k]) <= 1e-12 * max(1.0, abs(o[k])), (M, k)
        np.testing.assert_allclose(g["vminus_mode"], o["vminus_mode"], rtol=1e-12, atol=1e-12)
        # eigenvector up to a phase
        ph = np.vdot(o["xi"], g["xi"])
        assert abs(abs(ph) - 1) < 1e-10


def test_chebyshev_coefficients_host_only():
    """Series coefficients of exp(-i x T): c_0 = J_0(x), c_k = 2 (-i)^k J_k(x)
    (scipy's Bessel functions as the reference) and the oracle's term count."""
    import paper_2111_00050_amd as fh
    from scipy.special import jv

    from oracle import evolve

    for x, tol in ((0.05, 1e-14), (3.7, 1e-14), (41.0, 1e-12)):
        c = fh.chebyshev_coefficients(x, tol)
        assert len(c) == evolve.chebyshev_terms(x, tol)
        k = np.arange(len(c))
        want = np.where(k == 0, 1.0, 2.0) * (-1j) ** k * jv(k, x)
        np.testing.assert_allclose(c, want, rtol=0, atol=1e-14)
    with pytest.raises(ValueError):
        fh.chebyshev_coefficients(-1.0)
    with pytest.raises(ValueError):
        fh.chebyshev_coefficients(5000.0)


def test_first_crossing_host_only():
    """Breaktime extraction: exact on piecewise-linear data, within the linear
    interpolation bound h^2 max|y''| / 8 on a smooth curve, NaN when the level
    is never reached, errors on bad arguments."""
    import paper_2111_00050_amd as fh

    t = np.linspace(0.0, 2.0, 21)
    assert abs(fh.first_crossing(t, 3.0 * t - 1.0, 2.0) - 1.0) <= 1e-15
    assert abs(fh.first_crossing(t, 1.0 - 0.25 * t, 0.8, -1) - 0.8) <= 1e-15
    h = t[1] - t[0]
    got = fh.first_crossing(t, t ** 2, 0.15)
    # the chord of a convex curve lies above it: the crossing comes early
    assert 0.0 < np.sqrt(0.15) - got <= h * h * 2.0 / 8.0 / (2.0 * (np.sqrt(0.15) - h))
    assert np.isnan(fh.first_crossing(t, t ** 2, 9.0))
    assert fh.first_crossing(t, t + 1.0, 0.5) == 0.0          # already past at the first sample
    y = t ** 2
    y[3] = np.nan
    assert abs(fh.first_crossing(t, y, y[2] + 1e-3) - t[4]) <= 1e-15  # bracket broken by NaN
    assert np.isnan(fh.first_crossing(np.zeros(0), np.zeros(0), 1.0))
    with pytest.raises(fh.FockError):
        fh.first_crossing(t[::-1].copy(), y, 0.5)
    with pytest.raises(fh.FockError):
        fh.first_crossing(t, y, 0.5, direction=0)
    s = {"t": t, "Q": 0.1 * t, "po_deficit": 0.05 * t, "vminus": 1.0 - 0.1 * t}
    bt = fh.breaktimes(s)
    assert abs(bt["t_Q"] - 1.5) < 1e-14 and abs(bt["t_PO"] - 2.0) < 1e-14 and abs(bt["t_sqz"] - 2.0) < 1e-14


def test_derive_principal_mode_on_a_site_kerr_state():
    """fh_derive's V_- of the principal mode on the pinned state of S3: a
    contact interaction with one occupied site mode b_1 (M = 4), evolved
    exactly.  fh_derive takes the oracle's unnormalised moments and must
    return the single-mode Kerr V_- (xi, not conj(xi)), the normalised
    moments and the mode occupations n_k = <a_k^+ a_k>/<psi|psi>."""
    import math

    import paper_2111_00050_amd as fh
    import workloads as W
    from oracle import Oracle, derived, states

    from test_oracle_pins import _expm_by_sector, _kerr_moments, _single_mode_vminus

    M, Lam, x, Nmax = 4, 0.3, 1, 17
    F = np.exp(2j * np.pi * np.outer(np.arange(M), np.arange(M)) / M) / math.sqrt(M)
    beta = np.zeros(M, np.complex128)
    beta[x] = np.exp(0.7j)
    o = Oracle(M, M, np.zeros(M), Lam, W.V_contact(M), W.all_sectors(M, Nmax))
    psi0 = states.coherent_state(o, F.conj().T @ beta)
    for t in (0.25, 1.2):
        psi = 1.7 * _expm_by_sector(o, psi0, t)  # unnormalised on purpose
        n2, a, Mij, A = o.moments(psi)
        g = fh.derive(M, n2, a, Mij, A)
        want = _single_mode_vminus(*_kerr_moments(beta[x], Lam * M, t))
        assert abs(g["vminus"] - want) <= 1e-10
        od = derived.derive(n2, a, Mij, A)
        np.testing.assert_allclose(g["a"], od["a"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(g["M"], od["M"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(g["A"], od["A"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(g["n_modes"], np.real(np.diag(Mij)) / n2, rtol=0, atol=1e-14)
        assert abs(np.sum(g["n_modes"]) - g["n_tot"]) <= 1e-13
    # a zero norm gives NaN everywhere and FH_ESTATE (mapped to NaN, no raise)
    z = np.zeros(M, np.complex128)
    g = fh.derive(M, 0.0, z, np.zeros((M, M), np.complex128), np.zeros((M, M), np.complex128))
    assert np.isnan(g["n_tot"]) and np.all(np.isnan(g["n_modes"])) and np.all(np.isnan(g["M"]))
