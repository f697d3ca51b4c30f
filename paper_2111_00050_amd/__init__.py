"""fockhip -- MI355X (gfx950) Fock-sector time evolution, Python binding.

Method: Eberhardt, Zamora, Kopp & Abel, arXiv:2111.00050.  The Hamiltonian of
Sec. II.A (Eq. Ham) is applied matrix-free on the number- and momentum-
conserving sectors of Sec. III.B and integrated with classical RK4 on complex
FP64 amplitudes; observables follow Sec. II.C-E.

This module only marshals arguments: every step runs in the hand-written HIP
kernels of ``libfockhip.so`` (C ABI in include/fockhip.h).  PyTorch supplies
device memory and the current stream.  Importing raises if the library has not
been built (``python -m paper_2111_00050_amd.build``); there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfockhip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libfockhip.so not found at {LIB_PATH}; build it with `python paper_2111_00050_amd/build.py`"
    )

_lib = ctypes.CDLL(LIB_PATH)

FH_OK, FH_EINVAL, FH_ENOMEM, FH_EOVERFLOW, FH_EHIP, FH_ESTATE, FH_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FH_PER_SECTOR, FH_GRAPH, FH_TIMING = 1, 2, 4
FH_J_Q, FH_J_PO, FH_J_NMODE = 0, 1, 2

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double


class fh_obs_scalars(ctypes.Structure):
    _fields_ = [(n, _D) for n in ("norm2", "n_tot", "Q", "lambda_p", "po_deficit", "vminus")]


class fh_timing(ctypes.Structure):
    _fields_ = [("stage_ms", _D), ("stage_launches", _I64), ("wall_ms", _D)]


# name -> (restype, argtypes); every exported entry point of include/fockhip.h
SIGNATURES = {
    "fh_last_error": (ctypes.c_char_p, []),
    "fh_version": (_I, []),
    "fh_model_create": (_I, [_I, _I, _P, _D, _P, _P]),
    "fh_model_transpose": (_I, [_P, _P]),
    "fh_model_destroy": (_I, [_P]),
    "fh_basis_create": (_I, [_I, _I, _I, _P, _P, _P]),
    "fh_basis_destroy": (_I, [_P]),
    "fh_basis_info": (_I, [_P, _P, _P, _P, _P]),
    "fh_basis_sizes": (_I, [_P, _P, _P]),
    "fh_basis_rank": (_I, [_P, _I, _I64, _P, _P, _P]),
    "fh_basis_unrank": (_I, [_P, _I, _I64, _P, _P, _P]),
    "fh_basis_occupations": (_I, [_P, _P, _P]),
    "fh_basis_set_launch": (_I, [_P, _I, _I]),
    "fh_basis_set_tile_order": (_I, [_P, _I, _I]),
    "fh_basis_autotune": (_I, [_P, _P, _I, _P, _P, ctypes.c_char_p, _P, _P, _P]),
    "fh_init_number": (_I, [_P, _P, _I, _P, _P]),
    "fh_init_coherent": (_I, [_P, _P, _I, _P, _P]),
    "fh_init_fieldnumber": (_I, [_P, _P, _I, _P, _P]),
    "fh_apply_h": (_I, [_P, _P, _I, _P, _P, _P]),
    "fh_moments": (_I, [_P, _I, _I, _P, _P, _P, _P, _P, _P]),
    "fh_moments_noalloc": (_I, [_P, _I, _I, _P, _P, _P, _P, _P, _P]),
    "fh_derive": (_I, [_I, _D, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "fh_first_crossing": (_I, [_P, _P, _I64, _D, _I, _P]),
    "fh_evolve_rk4": (_I, [_P, _P, _I, _P, _P, _D, _I64, _I64, _P, _I64, _I, _P, _P]),
    "fh_evolve_taylor2": (_I, [_P, _P, _I, _P, _P, _D, _D, _I64, _I64, _P, _I64, _I, _P, _P]),
    "fh_classical_rk4": (_I, [_P, _I, _P, _D, _I64, _I64, _P, _P]),
    "fh_tangent_rk4": (_I, [_P, _P, _I, _P, _P, _P, _D, _I64, _I, _I, _P, _P, _P]),
    "fh_evolve_chebyshev": (_I, [_P, _P, _I, _P, _P, _D, _I64, _D, _D, _D, _I64, _P, _I64, _I, _P, _P]),
    "fh_chebyshev_coefficients": (_I, [_D, _D, _I, _P, _P]),
    "fh_spectral_radius": (_I, [_P, _P, _P, _I, _P, _P]),
    "fh_adjoint_work_states": (_I64, [_I64, _I64]),
    "fh_adjoint_work_states_kept": (_I64, [_I64, _I64]),
    "fh_adjoint_rk4": (_I, [_P, _P, _I, _P, _D, _I64, _I64, _I, _I, _P, _I64, _P, _P, _P, _P, _P]),
    "fh_coherent_vjp": (_I, [_P, _I, _P, _P, _P, _P, _P]),
}
for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class FockError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fockhip status {status}: {msg}")
        self.status = status


def _check(st):
    if st != FH_OK:
        raise FockError(st, _lib.fh_last_error().decode(errors="replace"))


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _torch():
    import torch

    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def moment_doubles(M: int) -> int:
    return 1 + 2 * M + 4 * M * M


# --------------------------------------------------------------- handles ---
class Model:
    """Eq. (Ham): omega[M], Lambda and V[M,M,M,M] (V[i,j,k,l] multiplies a_i^+ a_j^+ a_k a_l)."""

    def __init__(self, M, omega, Lambda, V, pmod=None):
        self.M = int(M)
        self.pmod = self.M if pmod is None else int(pmod)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64).reshape(self.M)
        self.Lambda = float(Lambda)
        self.V = np.ascontiguousarray(V, dtype=np.float64).reshape((self.M,) * 4)
        h = ctypes.c_void_p()
        _check(_lib.fh_model_create(self.M, self.pmod, _np_ptr(self.omega), self.Lambda, _np_ptr(self.V),
                                    ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        # at interpreter shutdown the module globals may already be gone
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fh_model_destroy(self._h)
            self._h = None

    __del__ = close


class Basis:
    """Retained (N, P) sectors (Sec. III.B special Hilbert spaces), in order."""

    def __init__(self, M, sectors, pmod=None):
        self.M = int(M)
        self.pmod = self.M if pmod is None else int(pmod)
        self.sectors = [(int(n), int(p)) for n, p in sectors]
        N = np.array([s[0] for s in self.sectors], dtype=np.int32)
        P = np.array([s[1] for s in self.sectors], dtype=np.int32)
        h = ctypes.c_void_p()
        _check(_lib.fh_basis_create(self.M, self.pmod, len(self.sectors), _np_ptr(N), _np_ptr(P), ctypes.byref(h)))
        self._h = h
        dim = np.zeros(len(self.sectors), np.int64)
        off = np.zeros(len(self.sectors) + 1, np.int64)
        _check(_lib.fh_basis_sizes(self._h, _np_ptr(dim), _np_ptr(off)))
        self.dims = [int(x) for x in dim]
        self.offsets = [int(x) for x in off]
        self.total = int(off[-1])

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fh_basis_destroy(self._h)
            self._h = None

    __del__ = close

    def set_launch(self, blocks_per_cu=0, xcd_order=3):
        _check(_lib.fh_basis_set_launch(self._h, int(blocks_per_cu), int(xcd_order)))

    def set_tile_order(self, order=1, prefix_modes=3):
        """Tiles split at changes of the first prefix_modes occupations, visited
        lexicographically (order 0) or along a Morton curve over the prefix (1)."""
        _check(_lib.fh_basis_set_tile_order(self._h, int(order), int(prefix_modes)))

    def rank(self, sec, occ):
        torch = _torch()
        occ = occ.contiguous()
        count = occ.numel() // self.M
        idx = torch.empty(count, dtype=torch.int64, device=occ.device)
        _check(_lib.fh_basis_rank(self._h, int(sec), count, _dev_ptr(occ, torch.uint8, "occ"),
                                  _dev_ptr(idx, torch.int64, "idx"), _stream()))
        return idx

    def unrank(self, sec, idx):
        torch = _torch()
        idx = idx.contiguous()
        occ = torch.empty((idx.numel(), self.M), dtype=torch.uint8, device=idx.device)
        _check(_lib.fh_basis_unrank(self._h, int(sec), idx.numel(), _dev_ptr(idx, torch.int64, "idx"),
                                    _dev_ptr(occ, torch.uint8, "occ"), _stream()))
        return occ

    def occupations(self, device="cuda"):
        torch = _torch()
        occ = torch.empty((self.total, self.M), dtype=torch.uint8, device=device)
        _check(_lib.fh_basis_occupations(self._h, _dev_ptr(occ, torch.uint8, "occ"), _stream()))
        return occ


# ---------------------------------------------------------------- states ---
def _alloc_state(basis, nrhs, device="cuda"):
    torch = _torch()
    shape = (basis.total,) if nrhs == 1 else (basis.total, nrhs)
    return torch.empty(shape, dtype=torch.complex128, device=device)


def _nrhs_of(basis, psi):
    if psi.dim() == 1:
        if psi.shape[0] != basis.total:
            raise ValueError("state length does not match the basis")
        return 1
    if psi.dim() == 2 and psi.shape[0] == basis.total:
        return int(psi.shape[1])
    raise ValueError("state must have shape [total] or [total, nrhs]")


def init_number(basis, occ, nrhs=1):
    torch = _torch()
    occ = np.ascontiguousarray(occ, dtype=np.uint8).reshape(basis.M)
    psi = _alloc_state(basis, nrhs)
    _check(_lib.fh_init_number(basis.handle, _np_ptr(occ), int(nrhs), _dev_ptr(psi, torch.complex128, "psi"),
                               _stream()))
    return psi


def _amps(basis, z):
    z = np.ascontiguousarray(np.atleast_2d(np.asarray(z, dtype=np.complex128)))
    if z.shape[1] != basis.M:
        raise ValueError("amplitudes must have M columns")
    return z


def init_coherent(basis, alpha):
    """Eq. (coherentStates) truncated to the basis; alpha has shape [M] or [nrhs, M]."""
    torch = _torch()
    a = _amps(basis, alpha)
    psi = _alloc_state(basis, a.shape[0])
    _check(_lib.fh_init_coherent(basis.handle, _np_ptr(a), a.shape[0], _dev_ptr(psi, torch.complex128, "psi"),
                                 _stream()))
    return psi


def init_fieldnumber(basis, z):
    """Eq. (fieldNumState), normalised over the basis; z has shape [M] or [nrhs, M]."""
    torch = _torch()
    a = _amps(basis, z)
    psi = _alloc_state(basis, a.shape[0])
    _check(_lib.fh_init_fieldnumber(basis.handle, _np_ptr(a), a.shape[0],
                                    _dev_ptr(psi, torch.complex128, "psi"), _stream()))
    return psi


# ------------------------------------------------------------- operators ---
def apply_h(model, basis, psi, out=None):
    torch = _torch()
    nrhs = _nrhs_of(basis, psi)
    if out is None:
        out = torch.empty_like(psi)
    _check(_lib.fh_apply_h(model.handle, basis.handle, nrhs, _dev_ptr(psi, torch.complex128, "psi"),
                           _dev_ptr(out, torch.complex128, "out"), _stream()))
    return out


def autotune(model, basis, x, cache_path=None):
    """Pick the fastest launch configuration for H psi on this basis (fh_basis_autotune).
    Returns ({blocks_per_cu, xcd_order, tile_order, prefix_modes}, milliseconds)."""
    torch = _torch()
    nrhs = _nrhs_of(basis, x)
    out = torch.empty_like(x)
    cfg = np.zeros(4, np.intc)
    ms = np.zeros(1)
    _check(_lib.fh_basis_autotune(model.handle, basis.handle, nrhs, _dev_ptr(x, torch.complex128, "x"),
                                  _dev_ptr(out, torch.complex128, "out"),
                                  None if cache_path is None else str(cache_path).encode(), _np_ptr(cfg), _np_ptr(ms),
                                  _stream()))
    keys = ("blocks_per_cu", "xcd_order", "tile_order", "prefix_modes")
    return dict(zip(keys, (int(v) for v in cfg))), float(ms[0])


def moments(basis, psi, rhs=0):
    """Unnormalised (norm2, <a_i>, <a_i^+ a_j>, <a_k a_l>) of one right-hand side."""
    torch = _torch()
    nrhs = _nrhs_of(basis, psi)
    M = basis.M
    n2 = np.zeros(1)
    a = np.zeros(M, np.complex128)
    Mij = np.zeros((M, M), np.complex128)
    Akl = np.zeros((M, M), np.complex128)
    _check(_lib.fh_moments(basis.handle, nrhs, int(rhs), _dev_ptr(psi, torch.complex128, "psi"), _np_ptr(n2),
                           _np_ptr(a), _np_ptr(Mij), _np_ptr(Akl), _stream()))
    return float(n2[0]), a, Mij, Akl


def moments_noalloc(basis, psi, rhs=0):
    """fh_moments_noalloc: the same moments as moments(), with the reduction
    scratch in the library's static device array (no allocation)."""
    torch = _torch()
    nrhs = _nrhs_of(basis, psi)
    M = basis.M
    n2 = np.zeros(1)
    a = np.zeros(M, np.complex128)
    Mij = np.zeros((M, M), np.complex128)
    Akl = np.zeros((M, M), np.complex128)
    _check(_lib.fh_moments_noalloc(basis.handle, nrhs, int(rhs), _dev_ptr(psi, torch.complex128, "psi"), _np_ptr(n2),
                                   _np_ptr(a), _np_ptr(Mij), _np_ptr(Akl), _stream()))
    return float(n2[0]), a, Mij, Akl


def unpack_moments(M, rec):
    rec = np.asarray(rec, dtype=np.float64)
    norm2 = float(rec[0])
    a = rec[1:1 + 2 * M].view(np.complex128).copy()
    Mij = rec[1 + 2 * M:1 + 2 * M + 2 * M * M].view(np.complex128).reshape(M, M).copy()
    Akl = rec[1 + 2 * M + 2 * M * M:1 + 2 * M + 4 * M * M].view(np.complex128).reshape(M, M).copy()
    return norm2, a, Mij, Akl


def derive(M, norm2, a, Mij, Akl):
    """Q (Eq. Qparam), lambda_p and PO deficit (Eq. POcriterion), V_- (Eq. generalVminus),
    and the moments divided by norm2 (keys a, M, A, n_modes), all from fh_derive."""
    a = np.ascontiguousarray(a, np.complex128)
    Mij = np.ascontiguousarray(Mij, np.complex128)
    Akl = np.ascontiguousarray(Akl, np.complex128)
    s = fh_obs_scalars()
    xi = np.zeros(M, np.complex128)
    vm = np.zeros(M)
    an = np.zeros(M, np.complex128)
    Mn = np.zeros((M, M), np.complex128)
    An = np.zeros((M, M), np.complex128)
    nm = np.zeros(M)
    st = _lib.fh_derive(int(M), float(norm2), _np_ptr(a), _np_ptr(Mij), _np_ptr(Akl), ctypes.byref(s), _np_ptr(xi),
                        _np_ptr(vm), _np_ptr(an), _np_ptr(Mn), _np_ptr(An), _np_ptr(nm))
    if st not in (FH_OK, FH_ESTATE):
        _check(st)
    out = {k: getattr(s, k) for k, _ in fh_obs_scalars._fields_}
    out.update(a=an, M=Mn, A=An, n_modes=nm, xi=xi, vminus_mode=vm)
    return out


def first_crossing(t, y, level, direction=1):
    """First time the sampled y(t) reaches `level` (direction +1 rising, -1
    falling), linearly interpolated; NaN if it never does (fh_first_crossing)."""
    t = np.ascontiguousarray(t, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    if t.shape != y.shape or t.ndim != 1:
        raise ValueError("t and y must be 1-D arrays of equal length")
    out = np.zeros(1)
    _check(_lib.fh_first_crossing(_np_ptr(t), _np_ptr(y), len(t), float(level), int(direction), _np_ptr(out)))
    return float(out[0])


BREAK_Q = 0.15      # Q(t_br) (Sec. IV.C)
BREAK_PO = 0.1      # 1 - lambda_p / n_tot at t_br (Sec. IV.D)
ONSET_VMINUS = 0.8  # V_-(t_sqz) (Sec. II.E)


def observable_series(M, res, dt, rhs=0):
    """Derived observables of every record of an evolve result: dict of arrays
    t, n_tot, Q, lambda_p, po_deficit, vminus, and n_modes [nrec, M] (the
    normalised mode occupations <a_k^+ a_k>)."""
    keys = ("n_tot", "Q", "lambda_p", "po_deficit", "vminus")
    out = {k: np.empty(len(res.records)) for k in keys}
    out["n_modes"] = np.empty((len(res.records), M))
    for r, rec in enumerate(res.records[:, rhs]):
        d = derive(M, *unpack_moments(M, rec))
        for k in keys:
            out[k][r] = d[k]
        out["n_modes"][r] = d["n_modes"]
    out["t"] = np.asarray(res.steps, np.float64) * dt
    return out


def breaktimes(series, q=BREAK_Q, po=BREAK_PO, vminus=ONSET_VMINUS):
    """The three breaktimes of the paper from an observable series: Q rising to
    0.15, the PO deficit rising to 0.1, V_- falling to 0.8 (NaN if not reached)."""
    t = series["t"]
    return {"t_Q": first_crossing(t, series["Q"], q, 1),
            "t_PO": first_crossing(t, series["po_deficit"], po, 1),
            "t_sqz": first_crossing(t, series["vminus"], vminus, -1)}


# ---------------------------------------------------------------- evolve ---
@dataclass
class EvolveResult:
    records: np.ndarray      # [nrec, nrhs, moment_doubles(M)]
    steps: np.ndarray        # step index of each record
    stage_ms: float
    stage_launches: int
    wall_ms: float


def evolve_rk4(model, basis, psi, dt, nsteps, every=0, flags=0, work=None):
    """nsteps classical RK4 steps in place on psi; moments every `every` steps."""
    torch = _torch()
    nrhs = _nrhs_of(basis, psi)
    if work is None:
        work = torch.empty((3 * basis.total * nrhs,), dtype=torch.complex128, device=psi.device)
    M = basis.M
    nrec = nsteps // every + 1 if every > 0 else 0
    rec = np.zeros((max(nrec, 1), nrhs, moment_doubles(M)))
    tm = fh_timing()
    _check(_lib.fh_evolve_rk4(model.handle, basis.handle, nrhs, _dev_ptr(psi, torch.complex128, "psi"),
                              _dev_ptr(work, torch.complex128, "work"), float(dt), int(nsteps), int(every),
                              _np_ptr(rec), rec.size if nrec else 0, int(flags), ctypes.byref(tm),
                              _stream() if not (flags & FH_GRAPH) else _stream()))
    steps = np.arange(nrec) * every if nrec else np.zeros(0, int)
    return EvolveResult(rec[:nrec], steps, tm.stage_ms, tm.stage_launches, tm.wall_ms)


def evolve_taylor2(model, basis, psi, dt, nsteps, c2=0.5, every=0, flags=0, work=None):
    """The paper's second-order step (Eq. Q_int) in place on psi: psi <- psi - i dt H psi -
    c2 dt^2 H H psi (c2 = 1/2: Taylor step; the printed equation has c2 = 1)."""
    torch = _torch()
    nrhs = _nrhs_of(basis, psi)
    if work is None:
        work = torch.empty((2 * basis.total * nrhs,), dtype=torch.complex128, device=psi.device)
    M = basis.M
    nrec = nsteps // every + 1 if every > 0 else 0
    rec = np.zeros((max(nrec, 1), nrhs, moment_doubles(M)))
    tm = fh_timing()
    _check(_lib.fh_evolve_taylor2(model.handle, basis.handle, nrhs, _dev_ptr(psi, torch.complex128, "psi"),
                                  _dev_ptr(work, torch.complex128, "work"), float(dt), float(c2), int(nsteps),
                                  int(every), _np_ptr(rec), rec.size if nrec else 0, int(flags), ctypes.byref(tm),
                                  _stream()))
    steps = np.arange(nrec) * every if nrec else np.zeros(0, int)
    return EvolveResult(rec[:nrec], steps, tm.stage_ms, tm.stage_launches, tm.wall_ms)


def spectral_radius(model, basis, iters=100):
    """Power-iteration estimate of max |E| of H on the basis (fh_spectral_radius)."""
    torch = _torch()
    work = torch.empty((2 * basis.total,), dtype=torch.complex128, device="cuda")
    rho = ctypes.c_double(0.0)
    _check(_lib.fh_spectral_radius(model.handle, basis.handle, _dev_ptr(work, torch.complex128, "work"), int(iters),
                                   ctypes.byref(rho), _stream()))
    return float(rho.value)


def chebyshev_coefficients(x, tol=1e-14, kmax=4096):
    """Series coefficients c_k of exp(-i x T) (fh_chebyshev_coefficients), complex array."""
    re = np.zeros(kmax)
    im = np.zeros(kmax)
    K = _lib.fh_chebyshev_coefficients(float(x), float(tol), int(kmax), _np_ptr(re), _np_ptr(im))
    if K < 0:
        raise ValueError("invalid arguments or too many terms")
    return re[:K] + 1j * im[:K]


def evolve_chebyshev(model, basis, psi, dt, nsteps, emin=None, emax=None, tol=1e-14, every=0, flags=0, work=None,
                     margin=1.1):
    """nsteps exact-exponential steps exp(-i H dt) in place on psi by the Chebyshev series
    (fh_evolve_chebyshev).  Without bounds, [emin, emax] = [-r, r] with r = margin times
    the power-iteration spectral radius."""
    torch = _torch()
    nrhs = _nrhs_of(basis, psi)
    if emin is None or emax is None:
        r = margin * spectral_radius(model, basis) + 1e-9
        emin, emax = -r, r
    if work is None:
        work = torch.empty((4 * basis.total * nrhs,), dtype=torch.complex128, device=psi.device)
    M = basis.M
    nrec = nsteps // every + 1 if every > 0 else 0
    rec = np.zeros((max(nrec, 1), nrhs, moment_doubles(M)))
    tm = fh_timing()
    _check(_lib.fh_evolve_chebyshev(model.handle, basis.handle, nrhs, _dev_ptr(psi, torch.complex128, "psi"),
                                    _dev_ptr(work, torch.complex128, "work"), float(dt), int(nsteps), float(emin),
                                    float(emax), float(tol), int(every), _np_ptr(rec), rec.size if nrec else 0,
                                    int(flags), ctypes.byref(tm), _stream()))
    steps = np.arange(nrec) * every if nrec else np.zeros(0, int)
    return EvolveResult(rec[:nrec], steps, tm.stage_ms, tm.stage_launches, tm.wall_ms)


# ------------------------------------------------------- classical field ---
def classical_rk4(model, alpha0, dt, nsteps, every=0):
    """Mean-field trajectories (fh_classical_rk4): alpha0 is [ntraj, M] or [M]
    complex (numpy or a CUDA complex128 tensor).  Returns (alpha_T, outputs) with
    alpha_T a [ntraj, M] tensor and outputs a [nout, ntraj, M] tensor of the
    values at steps 0, every, ... (None when every == 0)."""
    torch = _torch()
    a = torch.as_tensor(alpha0, dtype=torch.complex128, device="cuda").reshape(-1, model.M).clone()
    ntraj = a.shape[0]
    out = None
    if every > 0:
        out = torch.empty((nsteps // every + 1, ntraj, model.M), dtype=torch.complex128, device="cuda")
    _check(_lib.fh_classical_rk4(model.handle, ntraj, _dev_ptr(a, torch.complex128, "alpha"), float(dt), int(nsteps),
                                 int(every), None if out is None else _dev_ptr(out, torch.complex128, "out"),
                                 _stream()))
    return a, out


# --------------------------------------------------------------- adjoint ---
def adjoint_rk4(model, basis, psi0, dt, nsteps, ckpt_every, objective=FH_J_Q, mode=0, work=None,
                keep_stage_inputs=True):
    """Discrete adjoint of nsteps RK4 steps: J, dJ/dLambda, dJ/dV and lambda0 = 2 dJ/d conj(psi0).
    With keep_stage_inputs (and work=None) the work buffer is sized so that the stage inputs of a
    segment are kept (fh_adjoint_work_states_kept) rather than recomputed."""
    torch = _torch()
    nrhs = _nrhs_of(basis, psi0)
    size_fn = _lib.fh_adjoint_work_states_kept if keep_stage_inputs else _lib.fh_adjoint_work_states
    need = int(size_fn(int(nsteps), int(ckpt_every)))
    if need < 0:
        raise ValueError("nsteps and ckpt_every must be >= 1")
    if work is None:
        work = torch.empty((need * basis.total * nrhs,), dtype=torch.complex128, device=psi0.device)
    lam0 = torch.empty_like(psi0)
    M = basis.M
    J = np.zeros(nrhs)
    dL = np.zeros(nrhs)
    dV = np.zeros((nrhs, M, M, M, M))
    _check(_lib.fh_adjoint_rk4(model.handle, basis.handle, nrhs, _dev_ptr(psi0, torch.complex128, "psi0"), float(dt),
                               int(nsteps), int(ckpt_every), int(objective), int(mode),
                               _dev_ptr(work, torch.complex128, "work"), work.numel() // (basis.total * nrhs),
                               _dev_ptr(lam0, torch.complex128, "lambda0"), _np_ptr(J), _np_ptr(dL), _np_ptr(dV),
                               _stream()))
    return {"J": J, "dLambda": dL, "dV": dV, "lambda0": lam0}


def tangent_rk4(model, basis, psi0, dt, nsteps, objective=FH_J_Q, mode=0, dpsi0=None, work=None):
    """Forward-mode tangent d psi/d Lambda along nsteps RK4 steps (fh_tangent_rk4).
    psi0 is not modified.  Returns {"J", "dLambda", "psi", "dpsi"}."""
    torch = _torch()
    nrhs = _nrhs_of(basis, psi0)
    psi = psi0.clone()
    dpsi = torch.zeros_like(psi0) if dpsi0 is None else dpsi0.clone()
    if work is None:
        work = torch.empty((8 * basis.total * nrhs,), dtype=torch.complex128, device=psi0.device)
    J = np.zeros(nrhs)
    dL = np.zeros(nrhs)
    _check(_lib.fh_tangent_rk4(model.handle, basis.handle, nrhs, _dev_ptr(psi, torch.complex128, "psi"),
                               _dev_ptr(dpsi, torch.complex128, "dpsi"), _dev_ptr(work, torch.complex128, "work"),
                               float(dt), int(nsteps), int(objective), int(mode), _np_ptr(J), _np_ptr(dL), _stream()))
    return {"J": J, "dLambda": dL, "psi": psi, "dpsi": dpsi}


def coherent_vjp(basis, alpha, lambda0):
    torch = _torch()
    a = _amps(basis, alpha)
    nrhs = a.shape[0]
    dre = np.zeros((nrhs, basis.M))
    dim = np.zeros((nrhs, basis.M))
    _check(_lib.fh_coherent_vjp(basis.handle, nrhs, _np_ptr(a), _dev_ptr(lambda0, torch.complex128, "lambda0"),
                                _np_ptr(dre), _np_ptr(dim), _stream()))
    return dre, dim


from .autograd import QEvolve, q_of_coherent  # noqa: E402,F401
