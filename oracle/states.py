"""Initial states of Sec. II.B, evaluated on the oracle's enumerated basis.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Number eigenstate, Eq. (numEigenstate): one basis vector.
* Coherent state, Eq. (coherentStates): the tensor product over modes of
  exp(-|z|^2/2) z^n / sqrt(n!).  Truncation to the retained sectors keeps the
  amplitudes as they are (no renormalisation): the dropped tail is the
  truncation error of Sec. III.B.
* Field-number state, Eq. (fieldNumState): proportional to prod z^n / sqrt(n!)
  on the states with sum n = N.  The printed normalisation is ambiguous, so the
  oracle normalises it explicitly; this equals (sum_k z_k a_k^+)^N |0> / norm.

Amplitudes are computed from logarithms (lgamma) and the phase sum n*arg(z),
which is a different evaluation order from any recurrence.
"""
from __future__ import annotations

import math

import numpy as np


def number_state(orc, occ) -> np.ndarray:
    occ = np.asarray(occ, dtype=np.int64)
    psi = np.zeros(orc.total, np.complex128)
    N = int(occ.sum())
    P = int((np.arange(orc.M) * occ).sum() % orc.pmod)
    for s, (n, p) in enumerate(orc.sectors):
        if (n, p) == (N, P):
            r = int(orc.rank(s, occ.astype(np.uint8))[0])
            assert r >= 0
            psi[orc.offsets[s] + r] = 1.0
            return psi
    raise ValueError("occupation vector is in no retained sector")


def _product_amplitudes(occ: np.ndarray, z: np.ndarray) -> np.ndarray:
    """prod_k z_k^{n_k} / sqrt(n_k!) for every row of occ, via logs."""
    occ = occ.astype(np.int64)
    out = np.empty(len(occ), np.complex128)
    absz = np.abs(z)
    argz = np.angle(z)
    for r in range(len(occ)):
        logmag = 0.0
        phase = 0.0
        zero = False
        for k, nk in enumerate(occ[r]):
            if nk == 0:
                continue
            if absz[k] == 0.0:
                zero = True
                break
            logmag += nk * math.log(absz[k]) - 0.5 * math.lgamma(nk + 1)
            phase += nk * argz[k]
        out[r] = 0.0 if zero else math.exp(logmag) * complex(math.cos(phase), math.sin(phase))
    return out


def coherent_state(orc, alpha) -> np.ndarray:
    alpha = np.asarray(alpha, dtype=np.complex128)
    occ = orc.all_occupations()
    pref = math.exp(-0.5 * float(np.sum(np.abs(alpha) ** 2)))
    return pref * _product_amplitudes(occ, alpha)


def fieldnumber_state(orc, z) -> np.ndarray:
    z = np.asarray(z, dtype=np.complex128)
    occ = orc.all_occupations()
    psi = _product_amplitudes(occ, z)
    nrm = math.sqrt(float(np.sum(np.abs(psi) ** 2)))
    return psi / nrm
