"""Breaktimes of the paper's test problems as the occupation grows (Sec. IV.C-E).

For each average occupation r the chosen problem (Sec. IV.A: number, coherent or
field-number initial state; long-range or contact interactions, exact momentum)
is evolved on the GPU with the Chebyshev propagator in record intervals of
--interval, until Q has reached 0.15, 1 - lambda_p/n_tot has reached 0.1 and V_-
has fallen to 0.8 (or --t-max).  Coherent states keep the sectors N <= N_max with
the smallest N_max whose Poisson weight is >= 0.999 (Sec. IV.A).  One JSON line
per r: sizes, the three breaktimes, the squeezing-onset prediction
t_sqz = 0.05 n_tot / |sum (1/2) Lambda z* z* z z| (Sec. II.E), the deepest
squeezing V_min within the run and its time tau_min = n_tot |chi| t_min
(Sec. IV.E), and the wall time.
With --classical the classical field of the same initial condition (Sec. III.A:
sqrt(n_k) for a number state, z for the others) is evolved beside it and the
distance sum_k |<n_k>(t) - |alpha_k(t)|^2| / n_tot is reported at --t-ref and as
its maximum (the comparison of Sec. IV.B).

    python workloads/breaktime_sweep.py --problem coherent-longrange --r 1 2 4 8
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import workloads as W  # noqa: E402


def poisson_nmax(mean: float, weight: float = 0.999) -> int:
    """Smallest N with P(Poisson(mean) <= N) >= weight."""
    p = math.exp(-mean)
    acc, N = p, 0
    while acc < weight:
        N += 1
        p *= mean / N
        acc += p
    return N


def squeezing_onset_prediction(V, Lam, z):
    """Sec. II.E: the single-field estimate of the squeezing onset,
    t_sqz = 0.05 n_tot / |<H_int>|, with the classical interaction energy
    <H_int> = (Lambda/2) sum V_ijkl z_i* z_j* z_k z_l of the initial field z.
    Returns (t_sqz, n_tot, <H_int>); t_sqz is inf without interaction energy."""
    z = np.asarray(z, dtype=np.complex128)
    n_tot = float(np.sum(np.abs(z) ** 2))
    e_int = 0.5 * Lam * np.einsum("ijkl,i,j,k,l->", V, z.conj(), z.conj(), z, z)
    t_pred = 0.05 * n_tot / abs(e_int) if e_int != 0 else float("inf")
    return t_pred, n_tot, e_int


def refine_minimum(t, v):
    """Deepest sample of v(t) refined by the parabola through it and its two
    neighbours (when both exist, are finite and the parabola opens upward).
    Returns (t_min, v_min), or (nan, nan) if no sample is finite."""
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    if not np.isfinite(v).any():
        return float("nan"), float("nan")
    k = int(np.nanargmin(v))
    t_min, v_min = float(t[k]), float(v[k])
    if 0 < k < len(v) - 1 and np.all(np.isfinite(v[k - 1:k + 2])):
        y0, y1, y2 = v[k - 1], v[k], v[k + 1]
        den = y0 - 2.0 * y1 + y2
        if den > 0:
            off = 0.5 * (y0 - y2) / den
            t_min = float(t[k] + off * (t[k + 1] - t[k]))
            v_min = float(y1 - 0.25 * (y0 - y2) * off)
    return t_min, v_min


def classical_distance(n_modes, n_classical, n_tot):
    """Sec. IV.B comparison: sum_k |<n_k>(t) - |alpha_k(t)|^2| / n_tot per record
    (rows of n_modes and n_classical are records, columns modes)."""
    return np.abs(np.asarray(n_modes) - np.asarray(n_classical)).sum(axis=1) / n_tot


def run(problem: str, r: int, interval: float, t_max: float, seed, margin: float, classical: bool = False,
        t_ref: float = 1.0):
    import torch

    import paper_2111_00050_amd as fh

    init, inter = problem.split("-", 1)
    w = W.paper_problem(init, inter, r, seed=seed)
    if init == "coherent":
        z = w.init_params[0]
        n = float(np.sum(np.abs(z) ** 2))
        sectors = W.all_sectors(w.M, poisson_nmax(n))
    else:
        sectors = w.sectors
    model, b = fh.Model(w.M, w.omega, w.Lambda, w.V), fh.Basis(w.M, sectors)
    if init == "number":
        psi = fh.init_number(b, w.init_params)
        zc = np.sqrt(w.init_params.astype(np.float64))
    elif init == "coherent":
        psi, zc = fh.init_coherent(b, w.init_params[0]), w.init_params[0]
    else:
        psi, zc = fh.init_fieldnumber(b, w.init_params[0]), w.init_params[0]
    t_pred, n_tot, e_int = squeezing_onset_prediction(w.V, w.Lambda, zc)
    rho = margin * fh.spectral_radius(model, b) + 1e-9
    work = torch.empty((4 * b.total,), dtype=torch.complex128, device="cuda")
    t0 = time.time()
    series = {k: [] for k in ("t", "n_tot", "Q", "lambda_p", "po_deficit", "vminus", "n_modes")}
    chunk, t_now = 10, 0.0
    terms_per_step = len(fh.chebyshev_coefficients(rho * interval))
    bt = {"t_Q": float("nan"), "t_PO": float("nan"), "t_sqz": float("nan")}
    while True:
        res = fh.evolve_chebyshev(model, b, psi, interval, chunk, -rho, rho, every=1, work=work)
        s = fh.observable_series(w.M, res, interval)
        first = 0 if not series["t"] else 1  # the chunk's first record repeats the last one
        for k in series:
            vals = s[k][first:] + (t_now if k == "t" else 0.0)
            series[k].extend(list(vals))
        t_now += chunk * interval
        bt = fh.breaktimes({k: np.array(v) for k, v in series.items()})
        done = all(np.isfinite(v) for v in bt.values())
        print(f"  r={r} t={t_now:.3f} Q={series['Q'][-1]:.4f} po={series['po_deficit'][-1]:.4f} "
              f"V-={series['vminus'][-1]:.4f}", file=sys.stderr, flush=True)
        if (done and (not classical or t_now >= t_ref - 1e-12)) or t_now >= t_max - 1e-12:
            break
    torch.cuda.synchronize()
    out = {"problem": problem, "r": r, "n_tot": n_tot, "sectors": len(sectors), "states": b.total,
           "t_end": t_now, **bt, "t_sqz_pred": t_pred, "spectral_radius": rho,
           "h_applies": int(round(t_now / interval)) * terms_per_step, "wall_s": time.time() - t0}
    # deepest squeezing within the run (Sec. IV.E): V_min and tau_min = n_tot |chi| t_min,
    # the minimum refined by the parabola through the three samples around it
    t_min, v_min = refine_minimum(series["t"], series["vminus"])
    if np.isfinite(v_min):
        n_chi = abs(e_int) / n_tot
        out.update(vminus_min=v_min, t_vminus_min=t_min, tau_min=n_chi * t_min, n_chi=n_chi)
    if classical:
        sub = 20
        nrec = len(series["t"])
        _, traj = fh.classical_rk4(model, zc, interval / sub, (nrec - 1) * sub, every=sub)
        ncl = (traj[:, 0, :].abs() ** 2).cpu().numpy()
        dev = classical_distance(series["n_modes"], ncl, n_tot)
        tt = np.array(series["t"])
        out["classical"] = {"t_ref": t_ref, "dev_at_t_ref": float(np.interp(t_ref, tt, dev)),
                            "dev_max": float(dev.max()), "dev_at_0": float(dev[0])}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--problem", default="coherent-longrange",
                    choices=[f"{i}-{p}" for i in ("number", "coherent", "fieldnumber")
                             for p in ("longrange", "contact+", "contact-")])
    ap.add_argument("--r", type=int, nargs="+", default=[1, 2, 4])
    ap.add_argument("--interval", type=float, default=0.02)
    ap.add_argument("--t-max", type=float, default=20.0)
    ap.add_argument("--seed", type=int, default=None, help="phase seed (default: the draw matching n_tot |chi| = 0.242)")
    ap.add_argument("--margin", type=float, default=1.1)
    ap.add_argument("--out", default=None, help="append JSON lines to this file")
    ap.add_argument("--classical", action="store_true", help="compare with the classical field")
    ap.add_argument("--t-ref", type=float, default=1.0, help="time of the classical comparison")
    a = ap.parse_args()
    for r in a.r:
        line = json.dumps(run(a.problem, r, a.interval, a.t_max, a.seed, a.margin, a.classical, a.t_ref))
        print(line, flush=True)
        if a.out:
            with open(a.out, "a") as f:
                f.write(line + "\n")


if __name__ == "__main__":
    main()
