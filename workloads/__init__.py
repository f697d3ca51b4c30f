"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the method's arithmetic: it only draws model
parameters and initial-state parameters.  Both the GPU library and the CPU
oracle consume what it returns.

Conventions
-----------
* Modes j = 0..M-1 sit on a periodic 1D momentum grid with labels in FFT order,
  k_j = j - M [2j >= M]; the conserved momentum of an occupation vector is
  P = sum_j j n_j mod M (== sum_j k_j n_j mod M).
* ``V`` has shape (M, M, M, M); ``V[i, j, k, l]`` multiplies a_i^+ a_j^+ a_k a_l
  and is nonzero only if i + j == k + l (mod pmod), so that H conserves number
  and momentum (Eq. Lambda's Kronecker delta).
* Contact interaction: V = 1 on every conserving quadruple (Lambda_0 term of
  Eq. Lambda).
* Long-range interaction: V = 1/q^2 with q the minimal-image momentum transfer
  between the first created mode i and the first annihilated mode k
  (q = signed representative of (k - i) mod M); the zero-transfer term
  (k == i) is removed.  Summing over all orderings reproduces the symmetric
  pair of 1/(p - p')^2 terms of Eq. (Lambda).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------- model ---
def k_labels(M: int) -> np.ndarray:
    j = np.arange(M)
    return j - M * (2 * j >= M)


def omega_quadratic(M: int) -> np.ndarray:
    return 0.5 * k_labels(M).astype(np.float64) ** 2


def omega_linear(M: int) -> np.ndarray:
    return np.abs(k_labels(M)).astype(np.float64)


def _conserving(M: int, pmod: int):
    i, j, k, l = np.meshgrid(*(np.arange(M),) * 4, indexing="ij")
    return ((i + j - k - l) % pmod) == 0, i, k


def V_contact(M: int, pmod: int | None = None) -> np.ndarray:
    pmod = M if pmod is None else pmod
    cons, _, _ = _conserving(M, pmod)
    return cons.astype(np.float64)


def minimal_image(d, M: int):
    d = np.mod(d, M)
    return np.where(2 * d > M, d - M, d)


def V_longrange(M: int, pmod: int | None = None) -> np.ndarray:
    pmod = M if pmod is None else pmod
    cons, i, k = _conserving(M, pmod)
    q = minimal_image(k - i, M).astype(np.float64)
    V = np.zeros((M, M, M, M))
    nz = cons & (q != 0)
    V[nz] = 1.0 / q[nz] ** 2
    return V


def V_random_symmetric(M: int, seed: int, pmod: int | None = None) -> np.ndarray:
    """Random real V on conserving quadruples, symmetric under V[ijkl] = V[klij]
    (so that H is Hermitian).  For operator tests only."""
    pmod = M if pmod is None else pmod
    rng = np.random.default_rng(seed)
    cons, _, _ = _conserving(M, pmod)
    V = rng.uniform(-1.0, 1.0, size=(M, M, M, M)) * cons
    return 0.5 * (V + V.transpose(2, 3, 0, 1))


def V_random(M: int, seed: int, pmod: int | None = None) -> np.ndarray:
    """Random real V on conserving quadruples with no symmetry (H not Hermitian)."""
    pmod = M if pmod is None else pmod
    rng = np.random.default_rng(seed)
    cons, _, _ = _conserving(M, pmod)
    return rng.uniform(-1.0, 1.0, size=(M, M, M, M)) * cons


# ------------------------------------------- exact momentum (paper grid) ---
# The paper's own model (Sec. II.A, Eq. Lambda; Sec. IV.A): mode j carries
# momentum p_j = j on a non-periodic grid and the interaction conserves
# sum_j j n_j exactly (i + j == k + l).  Such a V also conserves it modulo M,
# so the periodic sectors (N, P mod M) of the GPU path are unions of exact
# sectors that the dynamics never couples.
def _exact(M: int):
    i, j, k, l = np.meshgrid(*(np.arange(M),) * 4, indexing="ij")
    return (i + j) == (k + l), i, k


def V_contact_exact(M: int) -> np.ndarray:
    cons, _, _ = _exact(M)
    return cons.astype(np.float64)


def V_longrange_exact(M: int) -> np.ndarray:
    """1/(p_k - p_i)^2 per ordered term, p_j = j, zero transfer removed."""
    cons, i, k = _exact(M)
    q = (k - i).astype(np.float64)
    V = np.zeros((M, M, M, M))
    nz = cons & (q != 0)
    V[nz] = 1.0 / q[nz] ** 2
    return V


# ---------------------------------------------------------------- inputs ---
def momentum(occ, pmod: int) -> int:
    occ = np.asarray(occ)
    return int((np.arange(len(occ)) * occ).sum() % pmod)


def random_composition(rng, N: int, M: int) -> np.ndarray:
    """Uniform composition of N into M nonnegative parts (stars and bars)."""
    bars = np.sort(rng.choice(N + M - 1, size=M - 1, replace=False))
    edges = np.concatenate([[-1], bars, [N + M - 1]])
    return (np.diff(edges) - 1).astype(np.int64)


def random_occupations_in_sector(seed: int, N: int, M: int, P: int, pmod: int | None = None):
    pmod = M if pmod is None else pmod
    rng = np.random.default_rng(seed)
    while True:
        n = random_composition(rng, N, M)
        if momentum(n, pmod) == P:
            return n


def random_bounded_occupations(seed: int, M: int, lo: int, hi: int, total: int):
    """n_k iid uniform on {lo..hi}, redrawn until sum == total."""
    rng = np.random.default_rng(seed)
    while True:
        n = rng.integers(lo, hi + 1, size=M)
        if int(n.sum()) == total:
            return n.astype(np.int64)


def coherent_amplitudes(seed: int, M: int, mean_total: float) -> np.ndarray:
    """|alpha_k|^2 = mean_total u_k / sum(u), u ~ U[0,1]; phases ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=M)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=M)
    mag = np.sqrt(mean_total * u / u.sum())
    return mag * np.exp(1j * theta)


def phase_draws(n, seeds) -> np.ndarray:
    """z^(d)_k = sqrt(n_k) exp(i theta^(d)_k), one row per seed."""
    n = np.asarray(n, dtype=np.float64)
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        th = rng.uniform(0.0, 2.0 * np.pi, size=len(n))
        out.append(np.sqrt(n) * np.exp(1j * th))
    return np.array(out)


def random_psi(total: int, seed: int, nrhs: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    shape = (total,) if nrhs == 1 else (total, nrhs)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def periodic_psi(total: int, seed: int, chunk: int = 1 << 24) -> np.ndarray:
    """A cheap full-size test vector: x[i] = T1[i mod p1] + 1j T2[i mod p2] with
    Gaussian tables and the primes p1 = 1,000,003, p2 = 999,983, so two indices
    share a value only if they agree mod p1 p2 (~1e12, beyond every sector)."""
    rng = np.random.default_rng(seed)
    p1, p2 = 1_000_003, 999_983
    t1, t2 = rng.standard_normal(p1), rng.standard_normal(p2)
    x = np.empty(total, np.complex128)
    for lo in range(0, total, chunk):
        i = np.arange(lo, min(total, lo + chunk), dtype=np.int64)
        x.real[lo:lo + len(i)] = t1[i % p1]
        x.imag[lo:lo + len(i)] = t2[i % p2]
    return x


def occupation_psi(occ: np.ndarray, seed: int, chunk: int = 1 << 24) -> np.ndarray:
    """A test vector that is a function of the occupation vector alone, so that
    two bases ordering the same states differently hold the same state:
    x(n) from a 64-bit mix (splitmix64 finaliser) of n's base-256 digits and the
    seed, real and imaginary parts uniform in [-1, 1)."""
    occ = np.asarray(occ, dtype=np.uint8)
    out = np.empty(len(occ), np.complex128)
    m1, m2 = np.uint64(0xBF58476D1CE4E5B9), np.uint64(0x94D049BB133111EB)
    for lo in range(0, len(occ), chunk):
        o = occ[lo:lo + chunk].astype(np.uint64)
        z = np.full(len(o), (seed * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF, np.uint64)
        for m in range(o.shape[1]):
            z = z * np.uint64(257) + o[:, m]
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * m1
        z = (z ^ (z >> np.uint64(27))) * m2
        z = z ^ (z >> np.uint64(31))
        re = (z >> np.uint64(32)).astype(np.float64) / 2.0 ** 31 - 1.0
        im = (z & np.uint64(0xFFFFFFFF)).astype(np.float64) / 2.0 ** 31 - 1.0
        out.real[lo:lo + len(o)] = re
        out.imag[lo:lo + len(o)] = im
    return out


def all_sectors(M: int, Nmax: int, pmod: int | None = None, Nmin: int = 0):
    pmod = M if pmod is None else pmod
    return [(N, P) for N in range(Nmin, Nmax + 1) for P in range(pmod)]


def poisson_cut(mean_total: float, sigmas: float = 8.0) -> int:
    return int(math.floor(mean_total + sigmas * math.sqrt(mean_total)))


# --------------------------------------------------------------- configs ---
@dataclass
class Workload:
    name: str
    M: int
    omega: np.ndarray
    V: np.ndarray
    Lambda: float
    sectors: list
    dt: float
    nsteps: int
    every: int
    init: str                      # "number" | "coherent" | "fieldnumber"
    init_params: np.ndarray        # occupations, or amplitudes [nrhs, M]
    pmod: int = 0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if not self.pmod:
            self.pmod = self.M


def tiny_number() -> Workload:
    """M=5, w=k^2/2, contact V=1, Lambda=0.1; |4,2,1,1,0> (N=8, P=2: 99 states)."""
    M = 5
    n = np.array([4, 2, 1, 1, 0])
    return Workload("tiny number state M=5 N=8", M, omega_quadratic(M), V_contact(M), 0.1,
                    [(8, momentum(n, M))], 1e-3, 1000, 10, "number", n)


def large_sector(N: int = 48, nsteps: int = 2000) -> Workload:
    """M=8, w=k^2/2, long-range V, Lambda=0.02; random occupations of N=48 with P=0
    (25,366,335 states)."""
    M = 8
    n = random_occupations_in_sector(2, N, M, 0)
    return Workload(f"one large sector M=8 N={N} P=0", M, omega_quadratic(M), V_longrange(M), 0.02,
                    [(N, 0)], 5e-4, nsteps, 50, "number", n)


def batched_coherent(mean_total: float = 40.0, nsteps: int = 5000) -> Workload:
    """M=6, w=k^2/2, contact V, Lambda=0.05; coherent state with sum |alpha|^2 = 40,
    sectors N in [0, 40 + 8 sqrt(40)] x all P."""
    M = 6
    alpha = coherent_amplitudes(3, M, mean_total)
    return Workload(f"batched coherent M=6 nbar={mean_total:g}", M, omega_quadratic(M), V_contact(M),
                    0.05, all_sectors(M, poisson_cut(mean_total)), 1e-3, nsteps, 50, "coherent",
                    alpha[None, :])


def adjoint_number(N: int = 30) -> Workload:
    M = 6
    n = random_composition(np.random.default_rng(4), N, M)
    return Workload(f"adjoint number state M=6 N={N}", M, omega_quadratic(M), V_longrange(M), 0.03,
                    [(N, momentum(n, M))], 1e-3, 3000, 100, "number", n)


def adjoint_coherent(mean_total: float = 20.0) -> Workload:
    M = 6
    alpha = coherent_amplitudes(41, M, mean_total)
    return Workload(f"adjoint coherent M=6 nbar={mean_total:g}", M, omega_quadratic(M), V_longrange(M),
                    0.03, all_sectors(M, poisson_cut(mean_total)), 1e-3, 3000, 100, "coherent",
                    alpha[None, :])


def fieldnumber_draws(ndraws: int = 16, N: int = 30) -> Workload:
    """M=10, w=|k|, contact V, Lambda=0.01; n_k ~ U{0..6} with sum 30; field-number
    states with 16 random phase draws, all 10 P sectors of N=30."""
    M = 10
    n = random_bounded_occupations(5, M, 0, 6, N)
    z = phase_draws(n, range(500, 500 + ndraws))
    return Workload(f"field-number draws M=10 N={N} x{ndraws}", M, omega_linear(M), V_contact(M), 0.01,
                    [(N, P) for P in range(M)], 2e-4, 2000, 50, "fieldnumber", z)


def paper_phases(seed: int | None = None) -> np.ndarray:
    """theta_1..3 ~ U[0, 2 pi) for the Sec. IV.A states.  The paper does not print
    its seed but prints n_tot |chi| = 0.242 for its long-range draw (Sec. IV.E);
    for z = (0, sqrt(2r) e^{i t1}, sqrt(2r) e^{i t2}, sqrt(r) e^{i t3}, 0) that value
    is |0.13 + 0.08 sqrt(2) cos(t1 + t3 - 2 t2)| for every r.  Without a seed the
    first seed 0, 1, 2, ... whose draw rounds to 0.242 is used."""
    if seed is not None:
        return np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi, size=3)
    for s in range(10000):
        th = np.random.default_rng(s).uniform(0.0, 2.0 * np.pi, size=3)
        if round(abs(0.13 + 0.08 * math.sqrt(2.0) * math.cos(th[0] + th[2] - 2.0 * th[1])), 3) == 0.242:
            return th
    raise RuntimeError("no seed reproduces n_tot |chi| = 0.242")


def paper_problem(init: str, interaction: str, r: int, seed: int | None = None) -> Workload:
    """The test problems of Sec. IV.A on M = 5 modes with exact momentum:
    initial state |0, 2r, 2r, r, 0> (init "number") or z = (0, sqrt(2r) e^{i t1},
    sqrt(2r) e^{i t2}, sqrt(r) e^{i t3}, 0) (init "coherent" / "fieldnumber",
    phases from paper_phases(seed)); interaction "longrange": w_j = j^2/2, C = -0.1/r
    (Lambda = C with V = V_longrange_exact), or "contact+" / "contact-":
    w_j = j/r, Lambda_0 = +-0.1/r (Lambda = Lambda_0 with V = V_contact_exact).
    Sectors: periodic (N, P mod 5) covering the state (see above)."""
    M = 5
    j = np.arange(M, dtype=np.float64)
    if interaction == "longrange":
        omega, V, Lam = 0.5 * j ** 2, V_longrange_exact(M), -0.1 / r
    elif interaction in ("contact+", "contact-"):
        omega, V = j / r, V_contact_exact(M)
        Lam = (0.1 if interaction == "contact+" else -0.1) / r
    else:
        raise ValueError(interaction)
    n = np.array([0, 2 * r, 2 * r, r, 0])
    N = int(n.sum())
    if init == "number":
        return Workload(f"paper number state r={r} {interaction}", M, omega, V, Lam,
                        [(N, momentum(n, M))], 1e-3, 0, 0, "number", n, meta={"P_exact": int(j @ n)})
    th = paper_phases(seed)
    z = np.array([0.0, np.sqrt(2 * r) * np.exp(1j * th[0]), np.sqrt(2 * r) * np.exp(1j * th[1]),
                  np.sqrt(r) * np.exp(1j * th[2]), 0.0])
    if init == "fieldnumber":
        return Workload(f"paper field-number state r={r} {interaction}", M, omega, V, Lam,
                        [(N, P) for P in range(M)], 1e-3, 0, 0, "fieldnumber", z[None, :])
    if init == "coherent":
        return Workload(f"paper coherent state r={r} {interaction}", M, omega, V, Lam,
                        all_sectors(M, poisson_cut(float(N))), 1e-3, 0, 0, "coherent", z[None, :])
    raise ValueError(init)
