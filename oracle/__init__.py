"""CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct reference for the Fock-space evolution of
Eberhardt, Zamora, Kopp & Abel (arXiv:2111.00050).  Only ``tests/``, the smoke
check in ``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the GPU library (``paper_2111_00050_amd``):
the basis comes from nested-loop enumeration plus binary search (the GPU uses a
dynamic-programming rank), the Hamiltonian is applied by literal operator
action on each ordered quadruple (the GPU gathers over unordered pair classes),
and derived observables use numpy's LAPACK eigensolver (the GPU library uses
its own Jacobi sweep).

Modules:
  oracle              ctypes binding of ``fock_oracle.c`` (basis, H psi, moments)
  oracle.states       initial states of Sec. II.B
  oracle.evolve       classical RK4, the paper's second-order step, the
                      Chebyshev propagator, and the discrete adjoint of RK4
  oracle.derived      Q, Penrose-Onsager eigenvalue, squeezing V_-
  oracle.dense        dense-matrix references for sectors of <= ~500 states
  oracle.classical    mean-field (classical field) equations and their RK4

Parity pins: see tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fock_oracle.c")
_LIB = os.path.join(_HERE, "libfock_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.ora_create.restype = P
    lib.ora_create.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, dp, ctypes.c_int, ip, ip]
    lib.ora_destroy.argtypes = [P]
    lib.ora_count_sector.restype = i64
    lib.ora_count_sector.argtypes = [ctypes.c_int] * 4
    for f in ("ora_total",):
        getattr(lib, f).restype = i64
        getattr(lib, f).argtypes = [P]
    for f in ("ora_dim", "ora_offset"):
        getattr(lib, f).restype = i64
        getattr(lib, f).argtypes = [P, ctypes.c_int]
    lib.ora_occupations.argtypes = [P, ctypes.c_int, P]
    lib.ora_rank.argtypes = [P, ctypes.c_int, i64, P, P]
    lib.ora_apply_h.argtypes = [P, P, P]
    lib.ora_apply_h_rows.argtypes = [P, P, i64, P, P]
    lib.ora_moments.argtypes = [P, P, P, P, P, P]
    lib.ora_quartic_correlators.argtypes = [P, P, P, P]
    lib.ora_apply_onebody.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def count_sector(M: int, pmod: int, N: int, P: int) -> int:
    """Number of occupation vectors with sum N and momentum P (mod pmod), by enumeration."""
    return int(_load().ora_count_sector(M, pmod, N, P))


class Oracle:
    """Model (Eq. Ham) plus a list of retained (N, P) sectors.

    ``V`` has shape (M, M, M, M); ``V[i, j, k, l]`` multiplies
    ``a_i^+ a_j^+ a_k a_l`` and the interaction carries the prefactor
    ``Lambda / 2``.  Amplitude vectors are complex128 arrays that concatenate
    the sectors in the order given.
    """

    def __init__(self, M, pmod, omega, Lambda, V, sectors, threads=1):
        self.M, self.pmod = int(M), int(pmod)
        # threads > 1: apply_h runs the gather form (apply_h_rows) on row
        # blocks in that many threads (the C call releases the GIL); the result
        # equals the scatter form up to summation order (pin P3).
        self.threads = max(1, int(threads))
        self.omega = np.ascontiguousarray(omega, dtype=np.float64).reshape(M)
        self.Lambda = float(Lambda)
        self.V = np.ascontiguousarray(V, dtype=np.float64).reshape(M, M, M, M)
        self.sectors = [(int(n), int(p)) for n, p in sectors]
        Ns = np.array([s[0] for s in self.sectors], dtype=np.intc)
        Ps = np.array([s[1] for s in self.sectors], dtype=np.intc)
        lib = _load()
        self._lib = lib
        h = lib.ora_create(
            self.M, self.pmod,
            self.omega.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            self.Lambda,
            self.V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            len(self.sectors),
            Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            Ps.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        )
        if not h:
            raise ValueError("oracle: invalid model or sector list")
        self._h = h
        self.total = int(lib.ora_total(h))
        self.dims = [int(lib.ora_dim(h, s)) for s in range(len(self.sectors))]
        self.offsets = [int(lib.ora_offset(h, s)) for s in range(len(self.sectors))]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ora_destroy(h)
            self._h = None

    # -- basis ---------------------------------------------------------------
    def occupations(self, s: int) -> np.ndarray:
        out = np.empty((self.dims[s], self.M), dtype=np.uint8)
        self._lib.ora_occupations(self._h, s, _ptr(out))
        return out

    def all_occupations(self) -> np.ndarray:
        if not self.sectors:
            return np.zeros((0, self.M), np.uint8)
        return np.concatenate([self.occupations(s) for s in range(len(self.sectors))])

    def rank(self, s: int, occ: np.ndarray) -> np.ndarray:
        occ = np.ascontiguousarray(occ, dtype=np.uint8).reshape(-1, self.M)
        idx = np.empty(len(occ), dtype=np.int64)
        self._lib.ora_rank(self._h, s, len(occ), _ptr(occ), _ptr(idx))
        return idx

    # -- operators -----------------------------------------------------------
    def apply_h(self, psi: np.ndarray) -> np.ndarray:
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        assert psi.shape == (self.total,)
        if self.threads > 1 and self.total >= 4096:
            return self._apply_h_threads(psi)
        out = np.empty_like(psi)
        self._lib.ora_apply_h(self._h, _ptr(psi), _ptr(out))
        return out

    def _apply_h_threads(self, psi: np.ndarray) -> np.ndarray:
        from concurrent.futures import ThreadPoolExecutor

        rows = np.arange(self.total, dtype=np.int64)
        out = np.empty_like(psi)
        blocks = np.array_split(np.arange(self.total), 4 * self.threads)

        def run(b):
            if len(b):
                o = np.empty(len(b), np.complex128)
                r = np.ascontiguousarray(rows[b[0]:b[-1] + 1])
                self._lib.ora_apply_h_rows(self._h, _ptr(psi), len(r), _ptr(r), _ptr(o))
                out[b[0]:b[-1] + 1] = o

        with ThreadPoolExecutor(self.threads) as ex:
            list(ex.map(run, blocks))
        return out

    def apply_h_rows(self, psi: np.ndarray, rows) -> np.ndarray:
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty(len(rows), dtype=np.complex128)
        self._lib.ora_apply_h_rows(self._h, _ptr(psi), len(rows), _ptr(rows), _ptr(out))
        return out

    def moments(self, psi: np.ndarray):
        """Unnormalised (norm2, <a_i>, <a_i^+ a_j>, <a_k a_l>)."""
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        M = self.M
        n2 = np.zeros(1)
        a = np.zeros(M, np.complex128)
        Mij = np.zeros((M, M), np.complex128)
        Akl = np.zeros((M, M), np.complex128)
        self._lib.ora_moments(self._h, _ptr(psi), _ptr(n2), _ptr(a), _ptr(Mij), _ptr(Akl))
        return float(n2[0]), a, Mij, Akl

    def quartic_correlators(self, u: np.ndarray, y: np.ndarray) -> np.ndarray:
        """G[i,j,k,l] = <u| a_i^+ a_j^+ a_k a_l |y>."""
        u = np.ascontiguousarray(u, dtype=np.complex128)
        y = np.ascontiguousarray(y, dtype=np.complex128)
        M = self.M
        G = np.zeros((M, M, M, M), np.complex128)
        self._lib.ora_quartic_correlators(self._h, _ptr(u), _ptr(y), _ptr(G))
        return G

    def apply_lower(self, i, psi):
        return self._onebody(0, i, 0, psi)

    def apply_raise(self, i, psi):
        return self._onebody(1, i, 0, psi)

    def apply_hop(self, i, j, psi):
        """a_i^+ a_j psi."""
        return self._onebody(2, i, j, psi)

    def _onebody(self, kind, i, j, psi):
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        out = np.empty_like(psi)
        self._lib.ora_apply_onebody(self._h, kind, i, j, _ptr(psi), _ptr(out))
        return out

    def transposed(self) -> "Oracle":
        """The model whose Hamiltonian is the transpose (= adjoint, V real) of this one.

        (a_i^+ a_j^+ a_k a_l)^+ = a_k^+ a_l^+ a_i a_j, so H^+ has V'[i,j,k,l] = V[k,l,i,j].
        """
        return Oracle(self.M, self.pmod, self.omega, self.Lambda,
                      self.V.transpose(2, 3, 0, 1), self.sectors, self.threads)
