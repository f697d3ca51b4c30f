"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's own formula: each compares it with
something computed a different way (brute force, a closed form, a textbook
identity, a dense-matrix propagator, a printed number of the paper).

  P1  basis == brute-force filter of {0..N}^M sorted lexicographically
  P2  sector sizes == closed form from Ramanujan sums (multisets of Z_M)
  P3  Hermiticity of H for symmetric V; scatter form == gather form
  P4  Lambda = 0: H is diagonal with E(n) = sum w n; RK4 multiplies by R(-iE dt)^s
  P5  contact interaction, w = 0: spectrum (Lambda M/2) sum_x n_x(n_x - 1) and
      site-wise Kerr dynamics of a coherent state
  P6  single-mode Kerr closed forms for <a>, <a^2>, Q
  P7  dense RK4 propagator and dense expm
  P8  momentum conservation (block structure), norm/energy within the RK4 bound
  P9  coherent state at t = 0 (Q = 0, lambda_p = n_tot, V_- = 1, normal order)
  P10 the paper's long-range coherent test problem, n_tot |chi| (Sec. IV.E)
  P11 field-number and number eigenstates (Sec. II.B, Sec. IV.C/D remarks)
  C1-C4 classical field equations: free phases, single-mode and site-wise
      Kerr rotations, invariants of the flow
  T1-T2 the paper's second-order step (Eq. Q_int): free factor 1 + z + c2 z^2,
      dense propagator, second order only with c2 = 1/2
  X1-X2 Chebyshev propagator: equal to exp(-i H t) (dense expm) and to the
      free phases exp(-i E t), at steps where RK4 is unstable
  E1-E2 the paper's exact interactions (Eq. Lambda) and their embedding in
      periodic sectors
  S1-S2 single-mode squeezing: the large-n approximation and the early slope
  S3  V_- of the principal mode (Eq. generalVminus, Eq. a_op) for M > 1 where
      the state is one Kerr-evolved site mode (catches xi <-> conj(xi))
  S4  per-mode V_- against Kerr closed forms (M = 1; one Kerr mode of M = 4)
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import Oracle, count_sector
from oracle import dense, derived, evolve, states


# --------------------------------------------------------------------- P1 --
@pytest.mark.parametrize("M,N,pmod", [(1, 5, 1), (2, 6, 2), (3, 5, 3), (4, 6, 4), (5, 4, 5), (4, 5, 7), (3, 6, 13)])
def test_p1_basis_bruteforce(oracle_lib, M, N, pmod):
    brute = [n for n in itertools.product(range(N + 1), repeat=M) if sum(n) == N]
    for P in range(pmod):
        want = sorted(n for n in brute if sum(j * x for j, x in enumerate(n)) % pmod == P)
        o = Oracle(M, pmod, np.zeros(M), 0.0, np.zeros((M,) * 4), [(N, P)])
        got = [tuple(int(v) for v in r) for r in o.occupations(0)]
        assert got == want
        if want:
            idx = o.rank(0, np.array(want, dtype=np.uint8))
            assert list(idx) == list(range(len(want)))


# --------------------------------------------------------------------- P2 --
def _ramanujan(d, P):
    return sum(math.cos(2 * math.pi * a * P / d) for a in range(1, d + 1) if math.gcd(a, d) == 1)


def closed_form_dim(M, N, P):
    """Multisets of size N from Z_M with element sum == P (mod M):
    (1/M) sum_{d | gcd(M, N)} c_d(P) C(N/d + M/d - 1, M/d - 1), c_d = Ramanujan sum."""
    tot = 0.0
    for d in range(1, M + 1):
        if M % d == 0 and N % d == 0:
            tot += _ramanujan(d, P) * math.comb(N // d + M // d - 1, M // d - 1)
    return int(round(tot / M))


@pytest.mark.parametrize("M,N", [(5, 8), (6, 12), (8, 12), (4, 9), (10, 6), (6, 30)])
def test_p2_sector_sizes_closed_form(oracle_lib, M, N):
    dims = [count_sector(M, M, N, P) for P in range(M)]
    assert dims == [closed_form_dim(M, N, P) for P in range(M)]
    assert sum(dims) == math.comb(N + M - 1, M - 1)


def test_p2_workload_sizes(oracle_lib):
    # tiny number state sector (M=5, N=8, P=2) and its whole N=8 space
    assert count_sector(5, 5, 8, 2) == 99
    assert sum(count_sector(5, 5, 8, P) for P in range(5)) == 495
    # one large sector: M=8, N=48, P=0, by enumeration and by closed form
    assert closed_form_dim(8, 48, 0) == 25_366_335
    assert count_sector(8, 8, 48, 0) == 25_366_335
    # batched coherent: M=6, N <= 90, all P
    assert sum(closed_form_dim(6, N, P) for N in range(91) for P in range(6)) == math.comb(96, 6)
    # field-number draws: M=10, N=30, all P
    assert sum(closed_form_dim(10, 30, P) for P in range(10)) == math.comb(39, 9)


# --------------------------------------------------------------------- P3 --
def _small_model(M=4, N=(3, 4, 5), seed=7, sym=True):
    V = W.V_random_symmetric(M, seed) if sym else W.V_random(M, seed)
    omega = np.random.default_rng(seed + 1).uniform(-1, 1, M)
    secs = [(n, p) for n in N for p in range(M)]
    return Oracle(M, M, omega, 0.7, V, secs)


def test_p3_hermitian(oracle_lib):
    o = _small_model()
    x = W.random_psi(o.total, 1)
    y = W.random_psi(o.total, 2)
    lhs = np.vdot(x, o.apply_h(y))
    rhs = np.vdot(o.apply_h(x), y)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_p3_scatter_equals_gather(oracle_lib):
    for sym in (True, False):
        o = _small_model(sym=sym)
        x = W.random_psi(o.total, 3)
        full = o.apply_h(x)
        rows = np.arange(o.total)
        np.testing.assert_allclose(o.apply_h_rows(x, rows), full, rtol=0, atol=1e-12 * np.abs(full).max())


def test_p3_threaded_gather_equals_scatter(oracle_lib):
    """The oracle's threaded gather apply (row blocks in parallel) equals its
    scatter form on a multi-sector basis of an M = 8 long-range model."""
    M = 8
    secs = [(10, 0), (9, 3), (8, 5)]
    o1 = Oracle(M, M, W.omega_quadratic(M), 0.02, W.V_longrange(M), secs)
    o4 = Oracle(M, M, W.omega_quadratic(M), 0.02, W.V_longrange(M), secs, threads=4)
    assert o1.total >= 4096
    x = W.random_psi(o1.total, 8)
    full = o1.apply_h(x)
    np.testing.assert_allclose(o4.apply_h(x), full, rtol=0, atol=1e-12 * np.abs(full).max())


def test_p3_nonsymmetric_v_transpose(oracle_lib):
    """H(V[k,l,i,j]) is the transpose of H(V): <x, H y> = <H' x, y> for real x-conjugation."""
    o = _small_model(sym=False)
    oT = o.transposed()
    x = W.random_psi(o.total, 4)
    y = W.random_psi(o.total, 5)
    assert abs(np.vdot(x, o.apply_h(y)) - np.vdot(oT.apply_h(x), y)) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * 10


# --------------------------------------------------------------------- P4 --
def test_p4_free_evolution(oracle_lib):
    M = 5
    omega = W.omega_quadratic(M)
    o = Oracle(M, M, omega, 0.0, W.V_contact(M), [(6, p) for p in range(M)])
    psi0 = W.random_psi(o.total, 11)
    E = o.all_occupations().astype(float) @ omega
    np.testing.assert_allclose(o.apply_h(psi0), E * psi0, rtol=1e-15, atol=0)
    dt, s = 0.01, 50
    z = -1j * E * dt
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    psi, _ = evolve.rk4(o, psi0, dt, s)
    np.testing.assert_allclose(psi, R ** s * psi0, rtol=1e-13, atol=0)


# --------------------------------------------------------------------- P5 --
def test_p5_contact_spectrum(oracle_lib):
    M, N, Lam = 4, 5, 0.3
    o = Oracle(M, M, np.zeros(M), Lam, W.V_contact(M), [(N, p) for p in range(M)])
    H = dense.dense_h(o)
    ev = np.sort(np.linalg.eigvalsh(H))
    pos = [x for x in itertools.product(range(N + 1), repeat=M) if sum(x) == N]
    want = np.sort([0.5 * Lam * M * sum(n * (n - 1) for n in x) for x in pos])
    np.testing.assert_allclose(ev, want, rtol=0, atol=1e-12)


def test_p5_contact_coherent_sitewise_kerr(oracle_lib):
    M, Lam, Nmax = 3, 0.4, 14
    alpha = W.coherent_amplitudes(21, M, 1.0)
    o = Oracle(M, M, np.zeros(M), Lam, W.V_contact(M), W.all_sectors(M, Nmax))
    psi0 = states.coherent_state(o, alpha)
    H = dense.dense_h(o)
    F = np.exp(2j * np.pi * np.outer(np.arange(M), np.arange(M)) / M) / math.sqrt(M)  # b = F a
    beta = F @ alpha
    for t in (0.3, 1.1):
        psi = dense.expm_evolve(H, psi0, t)
        obs = derived.observe(o, psi)
        b_t = beta * np.exp(np.abs(beta) ** 2 * (np.exp(-1j * Lam * M * t) - 1))
        a_t = F.conj().T @ b_t
        np.testing.assert_allclose(obs["a"], a_t, rtol=0, atol=1e-9)


# --------------------------------------------------------------------- P6 --
def test_p6_single_mode_kerr(oracle_lib):
    Lam, alpha, Nmax, dt, nsteps = 0.1, 1.3 + 0.9j, 40, 1e-3, 2000
    o = Oracle(1, 1, np.zeros(1), Lam, np.ones((1, 1, 1, 1)), [(n, 0) for n in range(Nmax + 1)])
    psi0 = states.coherent_state(o, [alpha])
    a2 = abs(alpha) ** 2

    def check(step, t, psi):
        obs = derived.observe(o, psi)
        a_want = alpha * np.exp(a2 * (np.exp(-1j * Lam * t) - 1))
        aa_want = alpha ** 2 * np.exp(-1j * Lam * t) * np.exp(a2 * (np.exp(-2j * Lam * t) - 1))
        Q_want = 1 - np.exp(-2 * a2 * (1 - np.cos(Lam * t)))
        assert abs(obs["a"][0] - a_want) < 1e-10
        assert abs(obs["A"][0, 0] - aa_want) < 1e-10
        assert abs(obs["n_tot"] - a2) < 1e-10
        assert abs(obs["Q"] - Q_want) < 1e-10
        return obs

    _, outs = evolve.rk4(o, psi0, dt, nsteps, every=500, observe=check)
    assert len(outs) == 5


# --------------------------------------------------------------------- P7 --
def test_p7_dense_rk4_and_expm(oracle_lib):
    w = W.tiny_number()
    o = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    psi0 = states.number_state(o, w.init_params)
    H = dense.dense_h(o)
    nsteps = 200
    psi, _ = evolve.rk4(o, psi0, w.dt, nsteps)
    np.testing.assert_allclose(psi, dense.rk4_dense_evolve(H, psi0, w.dt, nsteps), rtol=0, atol=1e-12)
    Emax = np.abs(np.linalg.eigvalsh(H)).max()
    T = nsteps * w.dt
    bound = 4 * T * (Emax * w.dt) ** 4 * Emax / 120 + 1e-13
    assert np.linalg.norm(psi - dense.expm_evolve(H, psi0, T)) <= bound


# --------------------------------------------------------------------- P8 --
def test_p8_momentum_blocks_and_conservation(oracle_lib):
    M, N = 5, 6
    for V in (W.V_contact(M), W.V_longrange(M)):
        o = Oracle(M, M, W.omega_quadratic(M), 0.2, V, [(N, p) for p in range(M)])
        H = dense.dense_h(o)
        for a in range(M):
            for b in range(M):
                if a != b:
                    blk = H[o.offsets[a]:o.offsets[a] + o.dims[a], o.offsets[b]:o.offsets[b] + o.dims[b]]
                    assert np.all(blk == 0)
        assert np.allclose(H, H.conj().T, atol=1e-14)
    # norm and energy drift under RK4 bounded by |R(ix)|^2 = 1 - x^6/72 + x^8/576
    psi0 = W.random_psi(o.total, 9)
    psi0 /= np.linalg.norm(psi0)
    dt, nsteps = 2e-3, 300
    psi, _ = evolve.rk4(o, psi0, dt, nsteps)
    xmax = np.abs(np.linalg.eigvalsh(H)).max() * dt
    assert 0 <= 1 - np.linalg.norm(psi) ** 2 <= nsteps * xmax ** 6 / 72 + 1e-13
    E0 = np.vdot(psi0, o.apply_h(psi0)).real
    E1 = np.vdot(psi, o.apply_h(psi)).real
    assert abs(E1 - E0) <= nsteps * xmax ** 6 / 72 * np.abs(np.linalg.eigvalsh(H)).max() + 1e-12


# --------------------------------------------------------------------- P9 --
def test_p9_coherent_initial_moments(oracle_lib):
    M, Lam = 4, 0.3
    alpha = W.coherent_amplitudes(5, M, 2.0)
    V = W.V_longrange(M)
    o = Oracle(M, M, np.zeros(M), Lam, V, W.all_sectors(M, 22))
    psi0 = states.coherent_state(o, alpha)
    obs = derived.observe(o, psi0)
    tail = 1 - obs["norm2"]
    assert 0 <= tail < 1e-9
    assert abs(obs["Q"]) < 1e-8
    assert abs(obs["n_tot"] - np.sum(np.abs(alpha) ** 2)) < 1e-7
    assert abs(obs["lambda_p"] - obs["n_tot"]) < 1e-8
    assert abs(obs["vminus"] - 1) < 1e-7
    np.testing.assert_allclose(obs["M"], np.outer(alpha.conj(), alpha), atol=1e-7)
    # normal-ordered interaction energy
    Eint = np.vdot(psi0, o.apply_h(psi0)).real / obs["norm2"]
    want = 0.5 * Lam * np.einsum("ijkl,i,j,k,l->", V, alpha.conj(), alpha.conj(), alpha, alpha).real
    assert abs(Eint - want) < 1e-7 * max(1, abs(want))


# -------------------------------------------------------------------- P10 --
def test_p10_long_range_interaction_energy(oracle_lib):
    """Sec. IV.E: n_tot |chi| of the long-range coherent test problem equals
    |0.13 + 0.08 sqrt(2) cos(theta1 + theta3 - 2 theta2)| (independent of r), whose
    maximum 0.243 covers the printed value 0.242."""
    M = 5
    V = W.V_longrange(M)
    rng = np.random.default_rng(12)
    for r in (1.0, 3.0):
        C = -0.1 / r
        for _ in range(4):
            th = rng.uniform(0, 2 * np.pi, 3)
            z = np.array([0, math.sqrt(2 * r) * np.exp(1j * th[0]), math.sqrt(2 * r) * np.exp(1j * th[1]),
                          math.sqrt(r) * np.exp(1j * th[2]), 0])
            ntot = 5 * r
            want = abs(0.13 + 0.08 * math.sqrt(2) * math.cos(th[0] + th[2] - 2 * th[1]))
            # periodic minimal-image and exact (p_j = j) transfers agree on modes 1..3
            for VV in (V, W.V_longrange_exact(M)):
                e = 0.5 * C * np.einsum("ijkl,i,j,k,l->", VV, z.conj(), z.conj(), z, z)
                assert abs(abs(e) / ntot - want) < 1e-12
    assert 0.13 + 0.08 * math.sqrt(2) >= 0.242
    # the default phases of the workload generator reproduce the printed value
    w = W.paper_problem("coherent", "longrange", 2)
    z = w.init_params[0]
    e = 0.5 * w.Lambda * np.einsum("ijkl,i,j,k,l->", w.V, z.conj(), z.conj(), z, z)
    assert round(abs(e) / 10.0, 3) == 0.242
    # the oracle's H reproduces the normal-ordered energy on the truncated state (r = 1)
    r, C = 1.0, -0.1
    th = np.array([0.3, 1.7, 0.2])
    z = np.array([0, math.sqrt(2 * r) * np.exp(1j * th[0]), math.sqrt(2 * r) * np.exp(1j * th[1]),
                  math.sqrt(r) * np.exp(1j * th[2]), 0])
    o = Oracle(M, M, np.zeros(M), C, V, W.all_sectors(M, 26))
    psi = states.coherent_state(o, z)
    e_or = np.vdot(psi, o.apply_h(psi)).real / np.vdot(psi, psi).real
    want = 5 * r * (0.13 + 0.08 * math.sqrt(2) * math.cos(th[0] + th[2] - 2 * th[1])) * np.sign(C)
    assert abs(e_or - want) < 1e-8


# -------------------------------------------------------------------- P11 --
def test_p11_fieldnumber_and_number_states(oracle_lib):
    M, N = 4, 6
    o = Oracle(M, M, W.omega_quadratic(M), 0.2, W.V_contact(M), [(N, p) for p in range(M)])
    z = W.coherent_amplitudes(8, M, 3.0)
    psi0 = states.fieldnumber_state(o, z)
    obs = derived.observe(o, psi0)
    u = z / np.linalg.norm(z)
    np.testing.assert_allclose(obs["M"], N * np.outer(u.conj(), u), atol=1e-12)
    assert abs(obs["lambda_p"] - N) < 1e-12
    psi, outs = evolve.rk4(o, psi0, 1e-2, 40, every=20, observe=lambda s, t, p: derived.observe(o, p))
    for ob in outs:
        assert np.all(ob["a"] == 0) and ob["Q"] == 1.0
    # number eigenstate: M stays diagonal, <a> = 0, Q = 1
    n1 = [1, 2, 0, 3]
    o1 = Oracle(M, M, W.omega_quadratic(M), 0.2, W.V_longrange(M), [(N, W.momentum(n1, M))])
    psi1 = states.number_state(o1, n1)
    _, outs = evolve.rk4(o1, psi1, 1e-2, 40, every=20, observe=lambda s, t, p: derived.observe(o1, p))
    for ob in outs:
        assert np.all(ob["a"] == 0) and ob["Q"] == 1.0
        assert np.all(ob["M"][~np.eye(M, dtype=bool)] == 0)


# -------------------------------------------------------------------- P12 --
def _forward_J(M, omega, Lam, V, sectors, alpha, dt, nsteps, objective):
    o = Oracle(M, M, omega, Lam, V, sectors)
    psi0 = states.coherent_state(o, alpha)
    psi, _ = evolve.rk4(o, psi0, dt, nsteps)
    return objective(o)(psi)[0]


def test_p12_adjoint_kerr_closed_form(oracle_lib):
    """M = 1: dQ/dLambda = 2|a|^2 t sin(Lt) e^{-2|a|^2(1-cos Lt)},
    dQ/dRe a = 2 Re a g, dQ/dIm a = 2 Im a g, g = 2(1 - cos Lt) e^{-2|a|^2(1-cos Lt)}."""
    Lam, alpha, Nmax, dt, nsteps = 0.5, 0.8 - 0.6j, 30, 2e-3, 500
    o = Oracle(1, 1, np.zeros(1), Lam, np.ones((1, 1, 1, 1)), [(n, 0) for n in range(Nmax + 1)])
    psi0 = states.coherent_state(o, [alpha])
    res = evolve.adjoint(o, psi0, dt, nsteps, evolve.objective_Q(o))
    t = dt * nsteps
    a2 = abs(alpha) ** 2
    e = np.exp(-2 * a2 * (1 - np.cos(Lam * t)))
    assert abs(res["J"] - (1 - e)) < 1e-9
    assert abs(res["dLambda"] - 2 * a2 * t * np.sin(Lam * t) * e) < 1e-8
    g = 2 * (1 - np.cos(Lam * t)) * e
    dre, dim = evolve.coherent_alpha_gradient(o, [alpha], psi0, res["g0"])
    assert abs(dre[0] - 2 * alpha.real * g) < 1e-8
    assert abs(dim[0] - 2 * alpha.imag * g) < 1e-8


def test_p12_adjoint_vs_central_differences(oracle_lib):
    M, Lam, dt, nsteps, Nmax = 3, 0.35, 5e-3, 40, 9
    omega = W.omega_quadratic(M)
    V = W.V_longrange(M)
    V[V == 0] = 0.0
    V = V + W.V_contact(M) * 0.3
    sectors = W.all_sectors(M, Nmax)
    alpha = W.coherent_amplitudes(31, M, 1.5)
    for objective in (evolve.objective_Q, evolve.objective_PO, lambda o: evolve.objective_mode_occupation(o, 1)):
        o = Oracle(M, M, omega, Lam, V, sectors)
        psi0 = states.coherent_state(o, alpha)
        res = evolve.adjoint(o, psi0, dt, nsteps, objective(o))
        h = 1e-6
        fd = (_forward_J(M, omega, Lam + h, V, sectors, alpha, dt, nsteps, objective)
              - _forward_J(M, omega, Lam - h, V, sectors, alpha, dt, nsteps, objective)) / (2 * h)
        assert abs(res["dLambda"] - fd) < 1e-7 * max(1, abs(fd))
        # one symmetric and one single ordered V entry
        for idx in [(0, 1, 1, 0), (2, 2, 1, 0)]:
            Vp, Vm = V.copy(), V.copy()
            Vp[idx] += h
            Vm[idx] -= h
            fd = (_forward_J(M, omega, Lam, Vp, sectors, alpha, dt, nsteps, objective)
                  - _forward_J(M, omega, Lam, Vm, sectors, alpha, dt, nsteps, objective)) / (2 * h)
            assert abs(res["dV"][idx] - fd) < 1e-7 * max(1, abs(fd))
        dre, dim = evolve.coherent_alpha_gradient(o, alpha, psi0, res["g0"])
        for k in range(M):
            for comp, d in ((1.0, dre[k]), (1j, dim[k])):
                ap, am = alpha.copy(), alpha.copy()
                ap[k] += comp * h
                am[k] -= comp * h
                fd = (_forward_J(M, omega, Lam, V, sectors, ap, dt, nsteps, objective)
                      - _forward_J(M, omega, Lam, V, sectors, am, dt, nsteps, objective)) / (2 * h)
                assert abs(d - fd) < 1e-7 * max(1, abs(fd))


def test_p12_adjoint_dense_expm_and_zeros(oracle_lib):
    """Number eigenstate at N = 6: Q is identically 1 so its gradient is exactly
    zero; the gradient of <n_0>(T) agrees with central differences of the exact
    (dense expm) evolution to within the RK4 error."""
    w = W.adjoint_number(N=6)
    o = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    psi0 = states.number_state(o, w.init_params)
    dt, nsteps = 1e-3, 300
    res = evolve.adjoint(o, psi0, dt, nsteps, evolve.objective_Q(o))
    assert res["J"] == 1.0 and res["dLambda"] == 0.0 and np.all(res["dV"] == 0)
    res = evolve.adjoint(o, psi0, dt, nsteps, evolve.objective_mode_occupation(o, 0))
    T = dt * nsteps

    def J_exact(Lam):
        oo = Oracle(w.M, w.pmod, w.omega, Lam, w.V, w.sectors)
        psi = dense.expm_evolve(dense.dense_h(oo), psi0, T)
        return evolve.objective_mode_occupation(oo, 0)(psi)[0]

    h = 1e-5
    fd = (J_exact(w.Lambda + h) - J_exact(w.Lambda - h)) / (2 * h)
    assert abs(res["dLambda"] - fd) < 1e-6 * max(1, abs(fd))


# ----------------------------------------------------- classical field (C) --
# The mean-field equations of Sec. II / Sec. III.A (oracle.classical), pinned
# to closed forms of the classical dynamics.
from oracle import classical  # noqa: E402


def _rk4_factor(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_c1_classical_free_phases():
    """Lambda = 0: each amplitude is multiplied by R(-i w dt) per step."""
    M, dt, n = 6, 0.07, 40
    om = W.omega_quadratic(M)
    a0 = np.stack([W.coherent_amplitudes(s, M, 3.0) for s in (1, 2)])
    aT, _ = classical.rk4(om, 0.0, W.V_longrange(M), a0, dt, n)
    np.testing.assert_allclose(aT, a0 * _rk4_factor(-1j * om * dt) ** n, rtol=1e-13, atol=0)


def test_c2_classical_single_mode_kerr():
    """M = 1: d alpha/dt = -i (w + Lambda v |alpha|^2) alpha, a pure rotation."""
    w, v, Lam, a0, dt, n = 0.5, 0.8, 0.35, 1.1 - 0.7j, 1e-3, 3000
    V = np.full((1, 1, 1, 1), v)
    aT, traj = classical.rk4(np.array([w]), Lam, V, np.array([a0]), dt, n, every=500)
    for s, a in enumerate(traj):
        t = s * 500 * dt
        assert abs(a[0] - a0 * np.exp(-1j * (w + Lam * v * abs(a0) ** 2) * t)) <= 1e-10


def test_c3_classical_contact_sitewise_kerr():
    """Contact V, w = 0: with b = F alpha (F_xk = e^{2 pi i k x / M}/sqrt(M)),
    each b_x rotates at rate Lambda M |b_x|^2 (the classical image of P5)."""
    M, Lam, dt, n = 5, 0.3, 1e-3, 2000
    F = np.exp(2j * np.pi * np.outer(np.arange(M), np.arange(M)) / M) / np.sqrt(M)
    a0 = W.coherent_amplitudes(9, M, 2.0)
    aT, _ = classical.rk4(np.zeros(M), Lam, W.V_contact(M), a0, dt, n)
    b0 = F @ a0
    bT = b0 * np.exp(-1j * Lam * M * np.abs(b0) ** 2 * n * dt)
    np.testing.assert_allclose(F @ aT, bT, rtol=0, atol=1e-10)


def test_c4_classical_invariants():
    """Hermitian V: sum |alpha|^2 and the mean-field energy are invariants of the
    flow (conserved to the RK4 error); a non-Hermitian V breaks the first."""
    M, Lam, dt, n = 5, 0.6, 2e-4, 2000
    om = np.random.default_rng(4).uniform(0, 2, M)
    V = W.V_random_symmetric(M, 7)
    a0 = W.coherent_amplitudes(11, M, 2.0)
    aT, _ = classical.rk4(om, Lam, V, a0, dt, n)
    assert abs(np.sum(np.abs(aT) ** 2) - np.sum(np.abs(a0) ** 2)) <= 1e-11
    assert abs(classical.energy(om, Lam, V, aT) - classical.energy(om, Lam, V, a0)) <= 1e-10
    Vn = W.V_random(M, 7)
    aN, _ = classical.rk4(om, Lam, Vn, a0, dt, n)
    assert abs(np.sum(np.abs(aN) ** 2) - np.sum(np.abs(a0) ** 2)) > 1e-6


# ----------------------------------------------- second-order step (T) ------
@pytest.mark.parametrize("c2", [0.5, 1.0])
def test_t1_taylor2_free_factor(oracle_lib, c2):
    """Lambda = 0: each amplitude is multiplied by 1 + z + c2 z^2, z = -i E dt."""
    M, dt, n = 4, 0.02, 30
    sectors = [(5, p) for p in range(M)]
    o = Oracle(M, M, W.omega_quadratic(M), 0.0, W.V_contact(M), sectors)
    psi0 = W.random_psi(o.total, 3)
    E = o.all_occupations() @ W.omega_quadratic(M)
    psi, _ = evolve.taylor2(o, psi0, dt, n, c2=c2)
    z = -1j * E * dt
    np.testing.assert_allclose(psi, psi0 * (1 + z + c2 * z * z) ** n, rtol=1e-13, atol=0)


def test_t2_taylor2_dense_propagator(oracle_lib):
    """Interacting sector: the step equals the dense matrix (I - i dt H - dt^2 H^2 / 2)
    applied n times; the printed c2 = 1 gives a different, first-order step."""
    w = W.tiny_number()
    o = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    psi0 = states.number_state(o, w.init_params)
    H = dense.dense_h(o)
    n = 100
    Pm = np.eye(H.shape[0]) - 1j * w.dt * H - 0.5 * w.dt ** 2 * (H @ H)
    want = np.linalg.matrix_power(Pm, n) @ psi0
    psi, _ = evolve.taylor2(o, psi0, w.dt, n)
    np.testing.assert_allclose(psi, want, rtol=0, atol=1e-12)
    # second order: error against exp(-i H t) about t (E dt)^2 E / 6; c2 = 1 is first order
    T = n * w.dt
    exact = dense.expm_evolve(H, psi0, T)
    err_half = np.linalg.norm(psi - exact)
    psi1, _ = evolve.taylor2(o, psi0, w.dt, n, c2=1.0)
    assert err_half < 0.1 * np.linalg.norm(psi1 - exact)


# ------------------------------------------------ Chebyshev propagator (X) ---
def test_x1_chebyshev_equals_exponential(oracle_lib):
    """The Chebyshev series reproduces exp(-i H t) psi0 (dense expm) at large
    steps, where RK4 would be unstable (|E| dt > 2.8)."""
    w = W.tiny_number()
    o = Oracle(w.M, w.pmod, w.omega, w.Lambda, w.V, w.sectors)
    psi0 = states.number_state(o, w.init_params)
    H = dense.dense_h(o)
    E = np.linalg.eigvalsh(H)
    emin, emax = E.min() - 0.5, E.max() + 0.5
    dt, n = 0.7, 5
    assert max(abs(emin), abs(emax)) * dt > 2.8
    psi, _ = evolve.chebyshev(o, psi0, dt, n, emin, emax)
    np.testing.assert_allclose(psi, dense.expm_evolve(H, psi0, n * dt), rtol=0, atol=1e-12)


def test_x2_chebyshev_free_phases(oracle_lib):
    """Lambda = 0: each amplitude picks up exp(-i E t) exactly."""
    M, dt, n = 4, 0.9, 4
    sectors = [(6, p) for p in range(M)]
    om = W.omega_quadratic(M)
    o = Oracle(M, M, om, 0.0, W.V_contact(M), sectors)
    psi0 = W.random_psi(o.total, 5)
    E = o.all_occupations() @ om
    psi, _ = evolve.chebyshev(o, psi0, dt, n, -1.0, E.max() + 1.0)
    np.testing.assert_allclose(psi, psi0 * np.exp(-1j * E * n * dt), rtol=0, atol=1e-12)


# ------------------------------------------------------------------ E1-E2 --
def _brute_two_body(occs, quads):
    """<m| sum_q c_q a_a^+ a_b^+ a_c a_d |n> by explicit ladder operators on
    occupation tuples (a^+|n> = sqrt(n+1)|n+1>, a|n> = sqrt(n)|n-1>)."""
    index = {tuple(int(x) for x in o): r for r, o in enumerate(occs)}
    H = np.zeros((len(occs), len(occs)))
    for col, o in enumerate(occs):
        for (a, b, c, d), coef in quads:
            v = [int(x) for x in o]
            amp = coef
            for mode, create in ((d, False), (c, False), (b, True), (a, True)):
                if create:
                    v[mode] += 1
                    amp *= math.sqrt(v[mode])
                else:
                    amp *= math.sqrt(v[mode])
                    v[mode] -= 1
                    if v[mode] < 0:
                        amp = 0.0
                        break
            if amp != 0.0:
                H[index[tuple(v)], col] += amp
    return H


@pytest.mark.parametrize("N", [3, 5])
def test_e1_exact_interactions_are_eq_lambda(oracle_lib, N):
    """Sec. II.A, Eq. (Ham) with Eq. (Lambda) on the grid p_j = j: the
    interaction (1/2) sum Lambda^{ij}_{kl} a_k^+ a_l^+ a_i a_j, each transfer term
    C / (2 (p_k - p_i)^2) kept only where it is finite, built here term by term
    with ladder operators, equals the oracle's H for V_longrange_exact (Lambda = C)
    plus V_contact_exact (Lambda = Lambda_0), in every exact momentum sector."""
    M, C, L0 = 5, -0.3, 0.7
    quads = []
    for i, j, k, l in itertools.product(range(M), repeat=4):
        if i + j != k + l:
            continue
        lam = L0 + sum(C / (2.0 * (k - x) ** 2) for x in (i, j) if x != k)
        quads.append(((k, l, i, j), 0.5 * lam))
    pmod = N * (M - 1) + 1
    for P in range(0, N * (M - 1) + 1, 3):
        oc = Oracle(M, pmod, np.zeros(M), C, W.V_longrange_exact(M), [(N, P)])
        oo = Oracle(M, pmod, np.zeros(M), L0, W.V_contact_exact(M), [(N, P)])
        want = _brute_two_body(oc.occupations(0), quads)
        got = dense.dense_h(oc) + dense.dense_h(oo)
        assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("inter", ["longrange", "contact+"])
def test_e2_periodic_sector_embeds_exact_sectors(oracle_lib, inter):
    """With an exactly conserving V, the periodic sector (N, P mod M) is the union
    of the exact sectors P' = P (mod M), 0 <= P' <= N (M-1), and H does not couple
    them: permuted to exact order, the periodic H is block diagonal with the exact
    sectors' H as blocks (Sec. III.B; exact Sigma j n_j)."""
    w = W.paper_problem("number", inter, 1)
    M, N = w.M, 6
    pmod = N * (M - 1) + 1
    for P in range(M):
        per = Oracle(M, M, w.omega, w.Lambda, w.V, [(N, P)])
        exact_secs = [(N, q) for q in range(P, N * (M - 1) + 1, M)]
        ex = Oracle(M, pmod, w.omega, w.Lambda, w.V, exact_secs)
        row = {tuple(o): r for r, o in enumerate(per.occupations(0))}
        perm = np.array([row[tuple(o)] for o in ex.all_occupations()])
        assert sorted(perm.tolist()) == list(range(per.total))
        Hp = dense.dense_h(per)[np.ix_(perm, perm)]
        He = dense.dense_h(ex)
        assert np.abs(Hp - He).max() <= 1e-13 * np.abs(He).max()


# ------------------------------------------------------------------ S1-S2 --
def _bajer(tau, n):
    s = math.sqrt(1.0 + 4.0 * tau * tau)
    return 1 - 4 * tau * s + 8 * tau ** 2 + 8 * tau ** 3 * (5 + 12 * tau ** 2) / (n * s) - 16 * tau ** 4 / n


def _kerr_vminus(n, taus, Lam=0.01):
    """V_- of a single-mode Kerr coherent state (where the single-field picture
    of Sec. II.E is exact) at the given tau = n_tot |chi| t, by the oracle's RK4."""
    o = Oracle(1, 1, np.zeros(1), Lam, np.ones((1, 1, 1, 1)), [(N, 0) for N in range(W.poisson_cut(n) + 1)])
    z = np.array([math.sqrt(n) * np.exp(0.4j)])
    psi = states.coherent_state(o, z)
    chi = 0.5 * Lam * n        # n_tot |chi| = (1/n) (Lambda/2) |z|^4
    out, t, nsub = [], 0.0, 400
    for tau in taus:
        h = (tau / chi - t) / nsub
        psi, _ = evolve.rk4(o, psi, h, nsub)
        t = tau / chi
        out.append(derived.observe(o, psi)["vminus"])
    return np.array(out)


def test_s1_squeezing_follows_the_large_n_approximation(oracle_lib):
    """Sec. II.E, Eq. (VminusBajer): for n_tot > 20 the approximation is accurate;
    its error is O(1/n_tot^2) (a 2.5x larger n_tot shrinks it about 6x)."""
    taus = [0.01, 0.05, 0.1, 0.3]
    v20 = _kerr_vminus(20.0, taus)
    v50 = _kerr_vminus(50.0, taus)
    e20 = np.abs(v20 - [_bajer(t, 20.0) for t in taus])
    e50 = np.abs(v50 - [_bajer(t, 50.0) for t in taus])
    assert np.all(e50[:3] <= 1e-6) and e50[3] <= 3e-4
    assert 4.0 <= e20[3] / e50[3] <= 9.0


def test_s2_early_time_squeezing_slope(oracle_lib):
    """Sec. II.E: V_- = 1 - 4 tau + O(tau^2) at early times; the onset
    V_- = 0.8 lies near tau = 0.05 (t_sqz = 0.05 / (n_tot |chi|))."""
    taus = [1e-3, 2e-3]
    v = _kerr_vminus(50.0, taus)
    slope = (1.0 - v) / (4.0 * np.array(taus))
    # 1 - slope = O(tau): halving tau halves the gap
    assert abs(1.0 - slope[0]) <= 2e-3
    assert 1.7 <= (1.0 - slope[1]) / (1.0 - slope[0]) <= 2.3
    a, b = _kerr_vminus(50.0, [0.05, 0.06])
    assert a > 0.8 > b


# ------------------------------------------------------------------ S3-S4 --
# Squeezing of a principal mode (Sec. II.E, Eq. generalVminus with the mode of
# Eq. a_op) and of single modes, pinned where the many-mode dynamics reduce to
# one Kerr oscillator whose moments are known in closed form.

def _expm_by_sector(o, psi0, t):
    """exp(-i H t) psi0 with a dense eigendecomposition of each retained sector
    on its own (H never couples sectors, Sec. III.B)."""
    out = np.empty_like(psi0)
    for s, sec in enumerate(o.sectors):
        lo, d = o.offsets[s], o.dims[s]
        if d == 0:
            continue
        one = Oracle(o.M, o.pmod, o.omega, o.Lambda, o.V, [sec])
        out[lo:lo + d] = dense.expm_evolve(dense.dense_h(one), psi0[lo:lo + d], t)
    return out


def _kerr_moments(z, g, t, w=0.0):
    """<b>, <b^2>, <b^+ b> of a coherent state |z> at time t under
    H = w b^+ b + (g/2) b^+ b^+ b b (a rotation times the single-mode Kerr
    evolution of P6)."""
    n = abs(z) ** 2
    m1 = z * np.exp(-1j * w * t) * np.exp(n * (np.exp(-1j * g * t) - 1))
    m2 = z * z * np.exp(-2j * w * t) * np.exp(-1j * g * t) * np.exp(n * (np.exp(-2j * g * t) - 1))
    return m1, m2, n


def _single_mode_vminus(m1, m2, n):
    """Eq. (generalVminus) for one mode with <O> = m1, <O^2> = m2, <O^+ O> = n."""
    return 1.0 + 2.0 * (n - abs(m1) ** 2) - 2.0 * abs(m2 - m1 * m1)


def _principal_vminus(d, conj_xi=False):
    """V_- of O = sum_k c_k a_k with c = xi (or, as a planted mistake, conj(xi))
    from the oracle's normalised moments and principal eigenvector."""
    c = np.conj(d["xi"]) if conj_xi else d["xi"]
    O = complex(np.sum(c * d["a"]))
    OdO = float(np.real(np.conj(c) @ d["M"] @ c))
    O2 = complex(c @ d["A"] @ c)
    return _single_mode_vminus(O, O2, OdO)


@pytest.mark.parametrize("M,r,Nmax", [(3, 1.0, 18), (4, 1.0, 17), (5, 0.6, 11)])
def test_s3_principal_mode_vminus_is_the_site_kerr_oscillator(oracle_lib, M, r, Nmax):
    """Contact interaction, w = 0, and a coherent state with a single occupied
    site mode b_x (x = 1, beta_x = e^{0.7 i}; alpha = F^+ beta has complex
    components).  By P5 the state stays a Kerr-evolved coherent state of b_x
    with rate Lambda M and vacuum in every other b mode, so M_ij has the single
    nonzero eigenvalue |beta_x|^2, the principal mode of Eq. (a_op) is b_x, and
    V_- must equal the single-mode Kerr value at every time.  With conj(xi) the
    operator would be b_{-x}, a vacuum mode (V_- = 1): the pin tells the two
    apart.  |beta_x| = r; the Poisson(r^2) tail beyond Nmax, weighted by n^2
    (it enters <b^2>), stays below 1e-12."""
    Lam, x = 0.3, 1
    F = np.exp(2j * np.pi * np.outer(np.arange(M), np.arange(M)) / M) / math.sqrt(M)  # b = F a
    beta = np.zeros(M, np.complex128)
    beta[x] = r * np.exp(0.7j)
    alpha = F.conj().T @ beta
    assert np.max(np.abs(alpha.imag)) > 0.1
    o = Oracle(M, M, np.zeros(M), Lam, W.V_contact(M), W.all_sectors(M, Nmax))
    psi0 = states.coherent_state(o, alpha)
    for t in (0.25, 1.2, 1.9):
        d = derived.observe(o, _expm_by_sector(o, psi0, t))
        m1, m2, n = _kerr_moments(beta[x], Lam * M, t)
        want = _single_mode_vminus(m1, m2, n)
        assert abs(d["lambda_p"] - n) <= 1e-10
        assert abs(d["vminus"] - want) <= 1e-10, (M, t, d["vminus"], want)
        assert abs(1.0 - want) > 0.05               # the pin is not the vacuum value 1
        assert abs(_principal_vminus(d) - want) <= 1e-10
        assert abs(_principal_vminus(d, conj_xi=True) - want) > 0.05
        assert abs(_principal_vminus(d, conj_xi=True) - 1.0) <= 1e-10


def test_s4_per_mode_vminus_kerr_closed_forms(oracle_lib):
    """Per-mode V_- (Eq. generalVminus with O = a_i) where single modes are
    exact Kerr oscillators: (a) M = 1 against the closed form; (b) M = 4 with
    the interaction V[k,k,k,k] on mode k = 2 only and nonzero frequencies, so
    mode 2 is a rotating Kerr oscillator (rate Lambda V_kkkk) and the other modes
    rotate freely and stay unsqueezed (V_- = 1)."""
    # (a) one mode
    Lam, z, Nmax = 0.2, 1.1 * np.exp(0.4j), 30
    o1 = Oracle(1, 1, np.zeros(1), Lam, np.ones((1, 1, 1, 1)), [(n, 0) for n in range(Nmax + 1)])
    psi0 = states.coherent_state(o1, [z])
    for t in (0.3, 1.2, 4.0):
        d = derived.observe(o1, _expm_by_sector(o1, psi0, t))
        want = _single_mode_vminus(*_kerr_moments(z, Lam, t))
        assert abs(d["vminus_mode"][0] - want) <= 1e-10
        assert abs(1.0 - want) > 0.05
    # (b) one Kerr mode among free ones
    M, k, Vk, Nmax = 4, 2, 1.5, 20
    omega = np.array([0.3, -0.2, 0.5, 0.1])
    V = np.zeros((M,) * 4)
    V[k, k, k, k] = Vk
    alpha = np.array([0.5, 0.4j, 0.9 * np.exp(0.3j), 0.3])
    o = Oracle(M, M, omega, Lam, V, W.all_sectors(M, Nmax))
    psi0 = states.coherent_state(o, alpha)
    for t in (0.5, 2.5):
        d = derived.observe(o, _expm_by_sector(o, psi0, t))
        m1, m2, n = _kerr_moments(alpha[k], Lam * Vk, t, omega[k])
        assert abs(d["a"][k] - m1) <= 1e-10 and abs(d["A"][k, k] - m2) <= 1e-10
        want = _single_mode_vminus(m1, m2, n)
        assert abs(d["vminus_mode"][k] - want) <= 1e-10
        assert abs(1.0 - want) > 0.02
        others = [i for i in range(M) if i != k]
        np.testing.assert_allclose(d["vminus_mode"][others], 1.0, rtol=0, atol=1e-10)
