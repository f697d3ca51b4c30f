"""Dense-matrix references for small sector sets -- TEST INFRASTRUCTURE ONLY.

The projected Hamiltonian H_lm = <n_l|H|n_m> of Sec. III.B is assembled column
by column from the oracle's H psi on unit vectors.  Then:
  * exact propagation  psi(t) = U exp(-i E t) U^+ psi0   (numpy eigh)
  * the exact one-step RK4 propagator R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 with
    z = -i dt H, so that nsteps of classical RK4 on a linear system equal
    R^nsteps psi0 up to rounding.
"""
from __future__ import annotations

import numpy as np


def dense_h(orc) -> np.ndarray:
    D = orc.total
    H = np.zeros((D, D), np.complex128)
    e = np.zeros(D, np.complex128)
    for c in range(D):
        e[c] = 1.0
        H[:, c] = orc.apply_h(e)
        e[c] = 0.0
    return H


def expm_evolve(H, psi0, t):
    w, U = np.linalg.eigh(H)
    return U @ (np.exp(-1j * w * t) * (U.conj().T @ psi0))


def rk4_propagator(H, dt):
    Z = -1j * dt * H
    I = np.eye(H.shape[0], dtype=np.complex128)
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    Z4 = Z3 @ Z
    return I + Z + Z2 / 2.0 + Z3 / 6.0 + Z4 / 24.0


def rk4_dense_evolve(H, psi0, dt, nsteps):
    R = rk4_propagator(H, dt)
    return np.linalg.matrix_power(R, nsteps) @ psi0
