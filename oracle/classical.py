"""Classical (mean-field) field equations -- TEST INFRASTRUCTURE ONLY.

Sec. II (Eq. clEqnMotion) and Sec. III.A (Eq. classicalFieldEqns): the
Heisenberg equation of a_p with every operator replaced by its mean value.
For H = sum_j w_j a_j^+ a_j + (Lambda/2) sum_{ijkl} V_ijkl a_i^+ a_j^+ a_k a_l
(the same model as the quantum oracle), [H, a_p] gives

    d alpha_p / dt = -i [ w_p alpha_p
                          + (Lambda/2) sum_{jkl} (V_pjkl + V_jpkl) conj(alpha_j) alpha_k alpha_l ].

Integrated with the textbook RK4 tableau, trajectories batched along the
first axis.  The initial conditions of Sec. III.A (sqrt(n_p) for a number
eigenstate, z_p for coherent and field-number states) are plain arrays, built
by the caller.  The contraction is numpy's einsum over the full V.
"""
from __future__ import annotations

import numpy as np


def rhs(omega, Lam, V, a):
    """f(alpha) for alpha of shape [T, M] (or [M])."""
    a = np.asarray(a, dtype=np.complex128)
    Vs = np.asarray(V, dtype=np.float64)
    U = Vs + Vs.transpose(1, 0, 2, 3)
    nl = np.einsum("pjkl,...j,...k,...l->...p", U, np.conj(a), a, a)
    return -1j * (np.asarray(omega) * a + 0.5 * Lam * nl)


def energy(omega, Lam, V, a):
    """H with operators replaced by means: sum w |a|^2 + (Lambda/2) sum V a_i* a_j* a_k a_l."""
    a = np.asarray(a, dtype=np.complex128)
    kin = np.einsum("p,...p->...", np.asarray(omega, dtype=np.float64), np.abs(a) ** 2)
    pot = np.einsum("ijkl,...i,...j,...k,...l->...", np.asarray(V, dtype=np.float64), np.conj(a), np.conj(a), a, a)
    return kin + 0.5 * Lam * pot


def rk4(omega, Lam, V, a0, dt, nsteps, every=0):
    """nsteps RK4 steps from a0 ([T, M] or [M]).  Returns (a_T, outputs) where
    outputs stacks a at steps 0, every, 2 every, ... (empty when every == 0)."""
    a = np.array(a0, dtype=np.complex128, copy=True)
    f = lambda y: rhs(omega, Lam, V, y)
    out = []
    for s in range(nsteps + 1):
        if every > 0 and s % every == 0:
            out.append(a.copy())
        if s == nsteps:
            break
        k1 = f(a)
        k2 = f(a + 0.5 * dt * k1)
        k3 = f(a + 0.5 * dt * k2)
        k4 = f(a + dt * k3)
        a = a + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return a, (np.stack(out) if out else np.zeros((0,) + a.shape, np.complex128))
