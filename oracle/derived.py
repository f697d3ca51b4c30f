"""Derived observables from the moments -- TEST INFRASTRUCTURE ONLY.

Expectation values are normalised by the current <psi|psi>.

* n_tot = sum_i <a_i^+ a_i>                          (Sec. II.B)
* Q = sum_i <delta a_i^+ delta a_i> / n_tot          (Eq. Qparam)
      with <delta a^+ delta a> = <a^+ a> - |<a>|^2
* lambda_p, xi = largest eigenpair of M_ij = <a_i^+ a_j>   (Eq. POcriterion)
* principal-mode operator O = sum_k xi_k a_k           (Eq. a_op)
* V_- = 1 + 2 <dO^+ dO> - 2 |<O^2> - <O>^2|            (Eq. generalVminus)
  with <O^+ O> = xi^+ M xi = lambda_p and <O^2> = sum xi_k xi_l <a_k a_l>.
  Here xi is the eigenvector of the matrix M_ij = <a_i^+ a_j>: then
  sum_ij conj(xi_i) xi_j M_ij = lambda_p requires O = sum_k xi_k a_k with the
  eigenvector of M read as <a_i^+ a_j> (i = row).  A near-degenerate top pair
  makes xi ill defined; V_- of the principal mode is NaN then.
* per-mode squeezing uses O = a_i.
* PO deficit = 1 - lambda_p / n_tot.
"""
from __future__ import annotations

import numpy as np


def derive(norm2, a, Mij, Akl, degenerate_rtol=1e-8):
    a = np.asarray(a) / norm2
    Mm = np.asarray(Mij) / norm2
    A = np.asarray(Akl) / norm2
    n_tot = float(np.real(np.trace(Mm)))
    Q = (n_tot - float(np.sum(np.abs(a) ** 2))) / n_tot if n_tot != 0 else float("nan")
    H = 0.5 * (Mm + Mm.conj().T)
    w, v = np.linalg.eigh(H)
    lam = float(w[-1])
    xi = v[:, -1]
    # <O^+ O> for O = sum_k c_k a_k equals sum_ij conj(c_i) c_j M_ij; maximised by
    # the top eigenvector c = xi of M.
    c = xi
    O = complex(np.sum(c * a))
    OdO = float(np.real(np.conj(c) @ Mm @ c))
    O2 = complex(c @ A @ c)
    vminus = 1.0 + 2.0 * (OdO - abs(O) ** 2) - 2.0 * abs(O2 - O * O)
    if len(w) > 1 and (w[-1] - w[-2]) <= degenerate_rtol * abs(w[-1]):
        vminus = float("nan")
    vmode = np.array(
        [1.0 + 2.0 * (np.real(Mm[i, i]) - abs(a[i]) ** 2) - 2.0 * abs(A[i, i] - a[i] ** 2)
         for i in range(len(a))]
    )
    return {
        "norm2": float(norm2),
        "a": a,
        "M": Mm,
        "A": A,
        "n_tot": n_tot,
        "Q": Q,
        "lambda_p": lam,
        "xi": xi,
        "vminus": float(vminus),
        "vminus_mode": vmode,
        "po_deficit": 1.0 - lam / n_tot if n_tot != 0 else float("nan"),
    }


def observe(orc, psi, **kw):
    return derive(*orc.moments(psi), **kw)
