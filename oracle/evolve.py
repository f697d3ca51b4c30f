"""Time stepping and its discrete adjoint -- TEST INFRASTRUCTURE ONLY.

Forward: the Schroedinger equation d psi/dt = -i H psi (Eq. Schr), restricted
to the retained (N, P) sectors (Sec. III.B), integrated with the classical
fourth-order Runge-Kutta tableau
    k1 = f(y), k2 = f(y + dt/2 k1), k3 = f(y + dt/2 k2), k4 = f(y + dt k3),
    y <- y + dt/6 (k1 + 2 k2 + 2 k3 + k4),   f(y) = -i H y.
(The paper's own second-order step, Eq. Q_int, is not what is integrated here.)

Adjoint: for a real objective J(psi_T) write g = 2 dJ/d conj(psi) so that
dJ = Re <g, d psi>.  A step psi' = R psi with R linear gives g = R^+ g'.
Reversing the stage recursion above with A = -i H (A^+ = +i H^+):
    kb4 = dt/6 g'                ; yb4 = A^+ kb4
    kb3 = dt/3 g' + dt   yb4     ; yb3 = A^+ kb3
    kb2 = dt/3 g' + dt/2 yb3     ; yb2 = A^+ kb2
    kb1 = dt/6 g' + dt/2 yb2     ; yb1 = A^+ kb1
    g   = g' + yb1 + yb2 + yb3 + yb4
and each parameter theta of A collects  sum_stages Re <kb_s, (dA/dtheta) y_s>.
For A = -i H:  dA/dV[i,j,k,l] = -i (Lambda/2) a_i^+ a_j^+ a_k a_l  and
dA/dLambda = -i (1/2) sum V a^+ a^+ a a.
"""
from __future__ import annotations

import numpy as np


def rk4_step(orc, psi, dt):
    f = lambda y: -1j * orc.apply_h(y)
    k1 = f(psi)
    k2 = f(psi + 0.5 * dt * k1)
    k3 = f(psi + 0.5 * dt * k2)
    k4 = f(psi + dt * k3)
    return psi + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk4(orc, psi0, dt, nsteps, every=0, observe=None):
    """Run nsteps steps; when every > 0 call observe(step, t, psi) at
    steps 0, every, 2*every, ... (t = step * dt, not accumulated)."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    out = []
    if every and observe is not None:
        out.append(observe(0, 0.0, psi))
    for s in range(1, nsteps + 1):
        psi = rk4_step(orc, psi, dt)
        if every and observe is not None and s % every == 0:
            out.append(observe(s, s * dt, psi))
    return psi, out


def taylor2(orc, psi0, dt, nsteps, c2=0.5, every=0, observe=None):
    """The paper's second-order step, Eq. (Q_int):
        psi <- psi - i dt H psi - c2 dt^2 H (H psi),
    with c2 = 1/2 for a Taylor step of exp(-i H dt) (the printed equation has
    c2 = 1).  Outputs as in rk4()."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    out = []
    for s in range(nsteps + 1):
        if every > 0 and s % every == 0 and observe is not None:
            out.append(observe(s, s * dt, psi))
        if s == nsteps:
            break
        h1 = orc.apply_h(psi)
        psi = psi - 1j * dt * h1 - c2 * dt * dt * orc.apply_h(h1)
    return psi, out


def chebyshev_terms(x, tol=1e-14):
    """Number of terms K so that the Chebyshev series of exp(-i x T) (|T| <= 1)
    keeps every coefficient 2 |J_k(x)| >= tol for k < K (J_k decays
    super-exponentially once k > x)."""
    from scipy.special import jv

    k = int(x) + 1
    while 2.0 * abs(jv(k, x)) >= tol or k <= x:
        k += 1
    return k + 1


def chebyshev(orc, psi0, dt, nsteps, emin, emax, tol=1e-14, every=0, observe=None):
    """Exact-exponential steps psi <- exp(-i H dt) psi by the Chebyshev series
    (spectrum of H inside [emin, emax]):
        H = a + b T,  a = (emax + emin)/2,  b = (emax - emin)/2,
        exp(-i H dt) = exp(-i a dt) sum_k c_k T_k(T),
        c_0 = J_0(b dt),  c_k = 2 (-i)^k J_k(b dt),
        T_0 psi = psi, T_1 psi = T psi, T_{k+1} psi = 2 T T_k psi - T_{k-1} psi.
    Outputs as in rk4()."""
    from scipy.special import jv

    a, b = 0.5 * (emax + emin), 0.5 * (emax - emin)
    K = chebyshev_terms(b * dt, tol)
    c = np.array([(1.0 if k == 0 else 2.0) * (-1j) ** k * jv(k, b * dt) for k in range(K)])
    phase = np.exp(-1j * a * dt)
    T = lambda v: (orc.apply_h(v) - a * v) / b
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    out = []
    for s in range(nsteps + 1):
        if every > 0 and s % every == 0 and observe is not None:
            out.append(observe(s, s * dt, psi))
        if s == nsteps:
            break
        t_prev, t_cur = psi, T(psi)
        acc = c[0] * t_prev + c[1] * t_cur
        for k in range(2, K):
            t_prev, t_cur = t_cur, 2.0 * T(t_cur) - t_prev
            acc = acc + c[k] * t_cur
        psi = phase * acc
    return psi, out


def _stages(orc, psi, dt):
    f = lambda y: -1j * orc.apply_h(y)
    y1 = psi
    k1 = f(y1)
    y2 = psi + 0.5 * dt * k1
    k2 = f(y2)
    y3 = psi + 0.5 * dt * k2
    k3 = f(y3)
    y4 = psi + dt * k3
    return (y1, y2, y3, y4)


def adjoint(orc, psi0, dt, nsteps, terminal):
    """Discrete adjoint of nsteps RK4 steps.

    terminal(psi_T) -> (J, g_T) with g_T = 2 dJ/d conj(psi_T).
    Returns dict with J, g0 (= 2 dJ/d conj(psi_0)), dV (M^4, real), dLambda.
    The adjoint uses the transposed model so that it is exact also when V is
    not symmetric (H^+ = H with V[k,l,i,j]).
    """
    orcT = orc.transposed()
    Ad = lambda y: 1j * orcT.apply_h(y)  # A^+ = (-i H)^+ = +i H^+
    traj = [np.array(psi0, dtype=np.complex128, copy=True)]
    for _ in range(nsteps):
        traj.append(rk4_step(orc, traj[-1], dt))
    J, g = terminal(traj[-1])
    M = orc.M
    G = np.zeros((M, M, M, M), np.complex128)
    for s in range(nsteps - 1, -1, -1):
        y1, y2, y3, y4 = _stages(orc, traj[s], dt)
        kb4 = (dt / 6.0) * g
        yb4 = Ad(kb4)
        kb3 = (dt / 3.0) * g + dt * yb4
        yb3 = Ad(kb3)
        kb2 = (dt / 3.0) * g + 0.5 * dt * yb3
        yb2 = Ad(kb2)
        kb1 = (dt / 6.0) * g + 0.5 * dt * yb2
        yb1 = Ad(kb1)
        for kb, y in ((kb1, y1), (kb2, y2), (kb3, y3), (kb4, y4)):
            G += orc.quartic_correlators(kb, y)
        g = g + yb1 + yb2 + yb3 + yb4
    # Re <kb, -i c X y> = c Re(-i <kb|X|y>) = c Im <kb|X|y>
    dV = 0.5 * orc.Lambda * np.imag(G)
    dLambda = 0.5 * float(np.sum(orc.V * np.imag(G)))
    return {"J": J, "g0": g, "dV": dV, "dLambda": dLambda, "psiT": traj[-1]}


def coherent_alpha_gradient(orc, alpha, psi0, g0):
    """dJ/dRe(alpha_k), dJ/dIm(alpha_k) for psi0 = coherent(alpha) (Eq. coherentStates).

    psi0(n) = exp(-|alpha|^2/2) prod alpha^n/sqrt(n!):
      d psi0/d Re a_k = (n_k / a_k - Re a_k) psi0,  d psi0/d Im a_k = (i n_k / a_k - Im a_k) psi0,
    with n_k/a_k * psi0 evaluated as n_k a_k^(n_k-1)/sqrt(n_k!) * (rest) so a_k = 0 is fine.
    dJ/dtheta = Re <g0, d psi0/d theta>.
    """
    from .states import _product_amplitudes
    import math

    alpha = np.asarray(alpha, np.complex128)
    occ = orc.all_occupations().astype(np.int64)
    pref = math.exp(-0.5 * float(np.sum(np.abs(alpha) ** 2)))
    M = orc.M
    dre = np.zeros(M)
    dim = np.zeros(M)
    S0 = np.vdot(g0, psi0)
    for k in range(M):
        # n_k alpha_k^(n_k - 1)/sqrt(n_k!) * prod_{m != k} ... times pref
        sub = occ.copy()
        mask = sub[:, k] > 0
        d = np.zeros(len(occ), np.complex128)
        if np.any(mask):
            sub_m = sub[mask].copy()
            nk = sub_m[:, k].astype(np.float64)
            sub_m[:, k] -= 1
            # alpha^(n-1)/sqrt((n-1)!) * n / sqrt(n) = alpha^(n-1)/sqrt((n-1)!) * sqrt(n)
            d[mask] = pref * _product_amplitudes(sub_m, alpha) * np.sqrt(nk)
        Sk = np.vdot(g0, d)
        dre[k] = float(np.real(Sk)) - alpha[k].real * float(np.real(S0))
        dim[k] = float(np.real(1j * Sk)) - alpha[k].imag * float(np.real(S0))
    return dre, dim


# ------------------------------------------------------------- objectives --
# Each returns (J, g) with g = 2 dJ/d conj(psi).  Expectations are normalised
# by nu = <psi|psi>; for <O> = <psi|O|psi>/nu one has
#   d<O>/d conj(psi) = (O psi - <O> psi) / nu.

def objective_Q(orc):
    """J = Q = sum_i <da_i^+ da_i> / n_tot = 1 - sum_i |<a_i>|^2 / n_tot  (Eq. Qparam)."""
    def terminal(psi):
        nu = np.vdot(psi, psi).real
        M = orc.M
        lo = [orc.apply_lower(i, psi) for i in range(M)]
        up = [orc.apply_raise(i, psi) for i in range(M)]
        a = np.array([np.vdot(psi, lo[i]) / nu for i in range(M)])
        Npsi = sum(orc.apply_hop(i, i, psi) for i in range(M))
        n = np.vdot(psi, Npsi).real / nu
        S = float(np.sum(np.abs(a) ** 2))
        dS = sum(np.conj(a[i]) * (lo[i] - a[i] * psi) + a[i] * (up[i] - np.conj(a[i]) * psi)
                 for i in range(M)) / nu
        dn = (Npsi - n * psi) / nu
        J = 1.0 - S / n
        g = 2.0 * (-dS / n + (S / n ** 2) * dn)
        return J, g
    return terminal


def objective_PO(orc):
    """J = 1 - lambda_p / n_tot  (Eq. POcriterion); d lambda_p = xi^+ dM xi."""
    def terminal(psi):
        nu = np.vdot(psi, psi).real
        M = orc.M
        hop = [[orc.apply_hop(i, j, psi) for j in range(M)] for i in range(M)]
        Mm = np.array([[np.vdot(psi, hop[i][j]) / nu for j in range(M)] for i in range(M)])
        w, v = np.linalg.eigh(0.5 * (Mm + Mm.conj().T))
        lam, xi = w[-1], v[:, -1]
        n = np.trace(Mm).real
        OdO = sum(np.conj(xi[i]) * xi[j] * hop[i][j] for i in range(M) for j in range(M))
        Npsi = sum(hop[i][i] for i in range(M))
        dlam = (OdO - lam * psi) / nu
        dn = (Npsi - n * psi) / nu
        J = 1.0 - lam / n
        g = 2.0 * (-dlam / n + (lam / n ** 2) * dn)
        return J, g
    return terminal


def objective_mode_occupation(orc, k):
    """J = <a_k^+ a_k>."""
    def terminal(psi):
        nu = np.vdot(psi, psi).real
        npsi = orc.apply_hop(k, k, psi)
        J = np.vdot(psi, npsi).real / nu
        return J, 2.0 * (npsi - J * psi) / nu
    return terminal
