"""torch.autograd binding of the discrete RK4 adjoint.

``QEvolve.apply(alpha_re, alpha_im, Lambda, V, spec)`` evolves the coherent
state of Eq. (coherentStates) with amplitudes alpha = alpha_re + i alpha_im for
spec.nsteps RK4 steps under Eq. (Ham) and returns the objective J at the end
(Q of Eq. Qparam by default).  The forward pass runs the hand-written adjoint
(fh_adjoint_rk4 + fh_coherent_vjp) once and keeps dJ/dalpha, dJ/dLambda and
dJ/dV; backward scales them by the incoming gradient.  Each ordered V entry is
an independent real parameter.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch


@dataclass
class EvolveSpec:
    basis: object           # paper_2111_00050_amd.Basis
    omega: np.ndarray       # [M]
    dt: float
    nsteps: int
    ckpt_every: int = 100
    objective: int = 0      # FH_J_Q, FH_J_PO, FH_J_NMODE
    mode: int = 0


class QEvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha_re, alpha_im, Lam, V, spec: EvolveSpec):
        from . import Model, adjoint_rk4, coherent_vjp, init_coherent

        b = spec.basis
        M = b.M
        alpha = alpha_re.detach().cpu().numpy().astype(np.float64) + 1j * alpha_im.detach().cpu().numpy().astype(
            np.float64)
        model = Model(M, spec.omega, float(Lam.detach().cpu()), V.detach().cpu().numpy().astype(np.float64))
        psi0 = init_coherent(b, alpha)
        res = adjoint_rk4(model, b, psi0, spec.dt, spec.nsteps, min(spec.ckpt_every, spec.nsteps), spec.objective,
                          spec.mode)
        dre, dim = coherent_vjp(b, alpha, res["lambda0"])
        model.close()
        dev, dt = alpha_re.device, torch.float64
        ctx.save_for_backward(
            torch.as_tensor(dre[0], dtype=dt, device=dev),
            torch.as_tensor(dim[0], dtype=dt, device=dev),
            torch.as_tensor(res["dLambda"][0], dtype=dt, device=Lam.device),
            torch.as_tensor(res["dV"][0], dtype=dt, device=V.device),
        )
        return torch.as_tensor(res["J"][0], dtype=dt, device=dev)

    @staticmethod
    def backward(ctx, gJ):
        dre, dim, dl, dv = ctx.saved_tensors
        return gJ * dre, gJ * dim, gJ * dl, gJ * dv, None


def q_of_coherent(alpha_re, alpha_im, Lam, V, spec: EvolveSpec):
    return QEvolve.apply(alpha_re, alpha_im, Lam, V, spec)
