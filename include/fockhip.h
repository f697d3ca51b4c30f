/*
 * fockhip.h -- C ABI of the MI355X (gfx950) Fock-sector evolution library.
 *
 * Method: Eberhardt, Zamora, Kopp & Abel, "On the single classical field
 * description of interacting scalar fields", arXiv:2111.00050.
 *
 *   H = sum_j omega_j a_j^+ a_j + (Lambda/2) sum_{ijkl} V[i][j][k][l] a_i^+ a_j^+ a_k a_l
 *                                                     (Sec. II.A, Eq. Ham / Eq. Lambda)
 *   d|phi>/dt = -i H |phi>                            (Sec. II.A; Sec. III.B, Eq. Schr)
 *
 * States are expanded in the occupation-number basis (Sec. II.B, Eq.
 * numEigenstate).  H conserves particle number N = sum_j n_j and momentum
 * P = sum_j j n_j (mod pmod), so the basis splits into independent "special
 * Hilbert spaces" (Sec. III.B) -- here called sectors (N, P).  A state is the
 * concatenation of the amplitude vectors of a chosen list of sectors.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Modes j = 0..M-1 (1 <= M <= 10 on the GPU path); pmod must equal M
 *    (periodic momentum grid).  Occupations are uint8 (N <= 255).  The
 *    paper's exact momentum (sum_j j n_j, no wrap-around) is covered by an
 *    interaction that conserves it exactly (nonzero V only where
 *    i + j == k + l): every periodic sector is then a union of exact sectors
 *    that H never couples, and a state inside one exact sector stays there.
 *  - Inside a sector, basis states are ordered lexicographically ascending
 *    with n_0 the most significant entry; a state's index in that order is its
 *    rank.  State vectors concatenate sectors in the order given to
 *    fh_basis_create; fh_basis_sizes returns each sector's dimension and
 *    offset.
 *  - Amplitudes are complex FP64 (fh_c64, the layout of torch.complex128).
 *    With nrhs > 1 right-hand sides the layout is [state][rhs], rhs fastest.
 *  - Device pointers are HIP device memory owned by the caller (e.g. torch
 *    tensors); host pointers are plain host memory, copied before return.
 *  - 'stream' is a hipStream_t (NULL = the default stream).  Device work is
 *    enqueued on it; entry points that return host results synchronise it.
 *  - Every entry point returns an fh_status; no C++ exception crosses the ABI.
 *    On failure fh_last_error() returns a thread-local message.  Arguments
 *    are validated before any device work is enqueued.
 *  - Handles are immutable after creation.  Calls that reduce over states
 *    (fh_moments, fh_evolve_rk4 with observables, fh_adjoint_rk4,
 *    fh_coherent_vjp) use scratch owned by the fh_basis: such calls on one
 *    basis must not overlap on different streams.
 */
#ifndef FOCKHIP_H
#define FOCKHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif
/* The library is built with hidden visibility; exactly the entry points
 * declared here are exported. */
#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

typedef enum {
    FH_OK = 0,
    FH_EINVAL = -1,       /* invalid argument */
    FH_ENOMEM = -2,       /* allocation failed / caller buffer too small */
    FH_EOVERFLOW = -3,    /* a count or index exceeds the supported integer range */
    FH_EHIP = -4,         /* a HIP runtime call failed */
    FH_ESTATE = -5,       /* non-finite result (e.g. NaN observable) */
    FH_EUNSUPPORTED = -6  /* valid request outside what this build implements */
} fh_status;

typedef struct { double re, im; } fh_c64;
typedef struct fh_model fh_model;
typedef struct fh_basis fh_basis;

/* Thread-local description of the last non-OK status returned on this thread. */
const char* fh_last_error(void);
/* Library version, 100*major + minor. */
int fh_version(void);

/* ------------------------------------------------------------------ model --
 * Eq. (Ham) with the interaction tensor of Eq. (Lambda) given entrywise:
 * V[((i*M + j)*M + k)*M + l] multiplies a_i^+ a_j^+ a_k a_l; the sum runs over
 * all ordered quadruples with prefactor Lambda/2.  Every nonzero entry must
 * conserve momentum, (i + j - k - l) mod pmod == 0, else FH_EINVAL.  V need
 * not be symmetric; H is Hermitian iff V[i][j][k][l] summed over the
 * orderings of {i,j} and of {k,l} is symmetric under {i,j} <-> {k,l}.
 * omega[M], V[M^4] are host arrays, copied. */
fh_status fh_model_create(int M, int pmod, const double* omega, double Lambda, const double* V,
                          fh_model** out);
/* The model of H^T (== H^+ for real V): V'[i][j][k][l] = V[k][l][i][j]. */
fh_status fh_model_transpose(const fh_model* m, fh_model** out);
fh_status fh_model_destroy(fh_model* m);

/* ------------------------------------------------------------------ basis --
 * Sector list (N[s], P[s]), s < nsec, host arrays; duplicates are EINVAL.
 * Empty sectors (dimension 0) are allowed.  Builds the counting tables of the
 * lexicographic rank (Sec. III.B; sizes as in App. A) on the host with
 * overflow checks (FH_EOVERFLOW if a sector has 2^28 or more states: gathers
 * inside a sector use 32-bit byte offsets) and uploads them. */
fh_status fh_basis_create(int M, int pmod, int nsec, const int32_t* N, const int32_t* P,
                          fh_basis** out);
fh_status fh_basis_destroy(fh_basis* b);
/* M, pmod, number of sectors, total states (any output pointer may be NULL). */
fh_status fh_basis_info(const fh_basis* b, int* M, int* pmod, int* nsec, int64_t* total);
/* dim[nsec], offset[nsec + 1] (host). */
fh_status fh_basis_sizes(const fh_basis* b, int64_t* dim, int64_t* offset);
/* Rank of count occupation vectors occ[count*M] (device, uint8) in sector
 * sec -> idx[count] (device int64); -1 for vectors not in that sector.
 * Bit-exact integer work. */
fh_status fh_basis_rank(const fh_basis* b, int sec, int64_t count, const uint8_t* occ,
                        int64_t* idx, void* stream);
/* Inverse: idx[count] (device, each in [0, dim)) -> occ[count*M] (device). */
fh_status fh_basis_unrank(const fh_basis* b, int sec, int64_t count, const int64_t* idx,
                          uint8_t* occ, void* stream);
/* Occupations of the whole state vector, occ[total*M] (device). */
fh_status fh_basis_occupations(const fh_basis* b, uint8_t* occ, void* stream);

/* --------------------------------------------------------- initial states --
 * Sec. II.B.  psi is device memory of total*nrhs fh_c64.
 *  number     : occ[M] (host) -> one basis vector (every rhs); EINVAL if the
 *               vector lies in no retained sector.
 *  coherent   : alpha[nrhs*M] (host), Eq. (coherentStates):
 *               psi(n) = prod_k exp(-|a_k|^2/2) a_k^n_k / sqrt(n_k!), truncated to
 *               the retained sectors without renormalisation.
 *  fieldnumber: z[nrhs*M] (host), Eq. (fieldNumState) read as
 *               psi(n) ~ prod_k z_k^n_k / sqrt(n_k!), normalised to 1 over the
 *               retained sectors. */
fh_status fh_init_number(const fh_basis* b, const uint8_t* occ, int nrhs, fh_c64* psi, void* stream);
fh_status fh_init_coherent(const fh_basis* b, const fh_c64* alpha, int nrhs, fh_c64* psi, void* stream);
fh_status fh_init_fieldnumber(const fh_basis* b, const fh_c64* z, int nrhs, fh_c64* psi, void* stream);

/* ---------------------------------------------------------------- H apply --
 * out = H psi on every sector (the projected Hamiltonians H^j of Sec. III.B,
 * applied matrix-free).  psi, out: device, total*nrhs; must not alias.
 * nrhs in {1, 2, 4, 8, 16}. */
fh_status fh_apply_h(const fh_model* m, const fh_basis* b, int nrhs, const fh_c64* psi, fh_c64* out,
                     void* stream);

/* ---------------------------------------------------------- observables --
 * Moments of one right-hand side (rhs < nrhs), unnormalised:
 *   norm2 = <psi|psi>, a[i] = <psi|a_i|psi>, Mij[i*M+j] = <psi|a_i^+ a_j|psi>,
 *   Akl[k*M+l] = <psi|a_k a_l|psi>   (host outputs; NULL to skip a group).
 * Matrix elements into sectors that are not retained count as zero.
 * Used by Eq. (Qparam), Eq. (POcriterion), Eq. (generalVminus). */
fh_status fh_moments(const fh_basis* b, int nrhs, int rhs, const fh_c64* psi, double* norm2,
                     fh_c64* a, fh_c64* Mij, fh_c64* Akl, void* stream);

/* Allocation-free variant of fh_moments, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, same results (bitwise: same launch grid
 * and summation order); the per-workgroup partial sums and the reduced values
 * live in a static device array of 2^20 doubles (8 MiB) that every GPU the
 * library runs on holds until the process ends, instead of the basis's
 * scratch.  The call allocates nothing (no hipMalloc, hipFree or other
 * allocating routine; host staging is on the stack).  Every call on one GPU
 * shares that array and overwrites it, so calls that overlap on one GPU race
 * (and so do calls on different streams); every word read is written first
 * by the same call, so nothing needs clearing.  FH_EUNSUPPORTED if the
 * reduction of this basis on this device needs more than 2^20 doubles
 * ((M + 1) * workgroups * 42 + (M + 1) * 2 * (2M + 1); MI355X: at most
 * 946,638); FH_EINVAL if the basis was created on another device. */
fh_status fh_moments_noalloc(const fh_basis* b, int nrhs, int rhs, const fh_c64* psi, double* norm2,
                             fh_c64* a, fh_c64* Mij, fh_c64* Akl, void* stream);

typedef struct {
    double norm2;      /* <psi|psi> */
    double n_tot;      /* sum_i <a_i^+ a_i> / norm2 */
    double Q;          /* Eq. (Qparam) */
    double lambda_p;   /* largest eigenvalue of M_ij / norm2 (Eq. POcriterion) */
    double po_deficit; /* 1 - lambda_p / n_tot */
    double vminus;     /* Eq. (generalVminus) for O = a^p of Eq. (a_op); NaN if the
                          top eigenvalue is degenerate to 1e-8 relative */
} fh_obs_scalars;
/* Derived observables from the unnormalised moments of fh_moments (host
 * only; no device work).  Every expectation value is divided by norm2 =
 * <psi|psi> (truncated coherent states are not normalised).
 * Outputs (host; each array may be NULL):
 *   s              the scalars above;
 *   xi[M]          principal eigenvector of M_ij (Eq. POcriterion, Eq. a_op),
 *                  phase arbitrary;
 *   vminus_mode[M] per-mode V_- of Eq. (generalVminus) with O = a_i;
 *   a_n[M], Mij_n[M*M], Akl_n[M*M]  the normalised <a_i>, <a_i^+ a_j>,
 *                  <a_k a_l> (row-major, like the inputs);
 *   n_modes[M]     the mode occupations <a_i^+ a_i> (Sec. II.B), whose sum
 *                  is n_tot.
 * FH_ESTATE (every output NaN) when norm2 is not positive and finite, or when
 * n_tot or lambda_p is not finite; FH_EINVAL for a null input or s. */
fh_status fh_derive(int M, double norm2, const fh_c64* a, const fh_c64* Mij, const fh_c64* Akl,
                    fh_obs_scalars* s, fh_c64* xi, double* vminus_mode, fh_c64* a_n, fh_c64* Mij_n,
                    fh_c64* Akl_n, double* n_modes);

/* ------------------------------------------------------------ breaktimes --
 * First time a sampled observable reaches a level: the quantum breaktimes
 * Q(t) = 0.15 (Sec. IV.C), 1 - lambda_p/n_tot = 0.1 (Sec. IV.D) and the
 * squeezing onset V_-(t) = 0.8 (Sec. II.E, Sec. IV.E).  Host only.
 * t[n], y[n]: host arrays, t strictly increasing.  direction = +1 looks for
 * y rising to the level (first y[i] >= level), -1 for y falling to it (first
 * y[i] <= level).  *out = t[i] if i is the first sample or follows a non-finite
 * one, else the linear interpolation between samples i-1 and i; NaN when the
 * level is never reached.  Non-finite samples are skipped.  FH_EINVAL for a
 * null pointer, n < 0, direction not +-1, a non-finite level or t not strictly
 * increasing (then *out = NaN). */
fh_status fh_first_crossing(const double* t, const double* y, int64_t n, double level, int direction,
                            double* out);

/* ----------------------------------------------------------------- evolve --
 * Time evolution of each retained sector under the Schroedinger equation
 * d|phi>/dt = -i H |phi> (Sec. II.A; solved sector by sector with the
 * projected H^j of Sec. III.B, where the paper's own step is Eq. Q_int):
 * nsteps classical RK4 steps of dt on d psi/dt = -i H psi, in place on psi
 * (device, total*nrhs).  work: device scratch of 3*total*nrhs fh_c64.
 * If obs_every > 0, moments of every rhs are taken at steps 0, obs_every,
 * 2*obs_every, ... <= nsteps and written to 'moments' (host) as consecutive
 * records of FH_MOMENT_DOUBLES(M) doubles per (record, rhs):
 *   [norm2, a (2M), Mij (2M^2), Akl (2M^2)]   (complex as re, im pairs).
 * moments_capacity is the number of doubles available there.
 * flags: FH_PER_SECTOR launches every stage once per sector (the plain
 *        per-sector method); default is one persistent launch per stage over
 *        all sectors.  FH_GRAPH replays each step from a captured hipGraph.
 *        FH_TIMING records HIP events around every stage launch (not
 *        compatible with FH_GRAPH) and returns kernel time in *timing. */
#define FH_PER_SECTOR 1
#define FH_GRAPH 2
#define FH_TIMING 4
#define FH_MOMENT_DOUBLES(M) (1 + 2 * (M) + 4 * (M) * (M))
typedef struct {
    double stage_ms;        /* summed duration of the H psi stage launches */
    int64_t stage_launches; /* number of such launches */
    double wall_ms;         /* host wall time of the whole call */
} fh_timing;
fh_status fh_evolve_rk4(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* work,
                        double dt, int64_t nsteps, int64_t obs_every, double* moments,
                        int64_t moments_capacity, int flags, fh_timing* timing, void* stream);

/* The paper's second-order step, Eq. (Q_int), in place on psi:
 *   psi <- psi - i dt H psi - c2 dt^2 H (H psi)
 * c2 = 1/2 makes it the second-order Taylor step of exp(-i H dt); the printed
 * equation has c2 = 1 (first order).  Two fused H psi launches per step.
 * work: device scratch of 2*total*nrhs fh_c64.  Moments, flags and timing as
 * for fh_evolve_rk4. */
fh_status fh_evolve_taylor2(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* work, double dt,
                            double c2, int64_t nsteps, int64_t obs_every, double* moments, int64_t moments_capacity,
                            int flags, fh_timing* timing, void* stream);

/* Launch configuration of the stage kernel for this basis: persistent
 * workgroups per compute unit (0 = occupancy limit) and the XCD-aware tile
 * order (0 = plain round robin, 1 = the XCDs take contiguous chunks of tiles
 * in turn, 2 = each XCD walks one contiguous eighth of the tile list, 3 = the
 * chunks of order 1, each XCD taking the tiles of its chunks in order from a
 * counter of that XCD, so that the tiles in flight on an XCD stay one compact
 * run; with order 3 the counters live in the basis, so stage and adjoint
 * launches on one basis must not overlap on different streams).  Order 3 uses
 * the counters only on launches where every workgroup takes at least 16 tiles,
 * and in the H psi stages only from M = 7 on; otherwise it walks as order 1.  With the counters, which workgroup sums
 * which tile varies between runs, so the adjoint's correlator sums (dJ/dV,
 * dJ/dLambda at M <= 7) can differ in the last bits from run to run; states
 * and moments do not.  A new basis starts at (0, 3).
 * Not thread-safe with concurrent calls on the same basis. */
fh_status fh_basis_set_launch(fh_basis* b, int blocks_per_cu, int xcd_order);
/* Tiling and schedule of each sector's rows; storage stays lexicographic and
 * results do not depend on it.  Tiles (<= 256 consecutive rows) never cross a
 * change of the occupations of the first prefix_modes modes (0 = plain 256-row
 * chunks; at most min(M-1, 8)).  order 0 visits the tiles lexicographically;
 * order 1 visits the blocks of equal prefix along a Morton (bit-interleaved)
 * curve over the prefix, so that concurrently processed tiles and the blocks
 * their neighbours live in (prefix changes of at most +-2 per mode) stay in
 * cache together.  Not thread-safe with concurrent calls on the same basis. */
fh_status fh_basis_set_tile_order(fh_basis* b, int order, int prefix_modes);
/* Autotuner: times one H psi launch (x -> out, device, total*nrhs each,
 * distinct) for every candidate launch configuration -- workgroups per CU
 * {occupancy, 1, 2, 3} x XCD order {1, 0} x tile schedule {plain, Morton
 * over 2 or 3 prefix modes} -- with HIP events on the stream, and applies the
 * fastest to the basis.  With cache_path (text file, may be NULL) a result
 * keyed by (GPU architecture, CU count, M, nrhs, sectors, states, Nmax) is
 * reused and new results are appended.  chosen[4] (host, may be NULL)
 * receives {blocks_per_cu, xcd_order, tile_order, prefix_modes}, *best_ms the
 * launch time.  Overwrites out. */
fh_status fh_basis_autotune(const fh_model* m, fh_basis* b, int nrhs, const fh_c64* x, fh_c64* out,
                            const char* cache_path, int* chosen, double* best_ms, void* stream);

/* --------------------------------------------------------- classical field --
 * Mean-field trajectories of the same model (Sec. II, Eq. clEqnMotion;
 * Sec. III.A, Eq. classicalFieldEqns): every operator of the Heisenberg
 * equation of a_p replaced by its mean,
 *   d alpha_p/dt = -i [ omega_p alpha_p
 *                       + (Lambda/2) sum_{jkl} (V_pjkl + V_jpkl) conj(alpha_j) alpha_k alpha_l ],
 * integrated with classical RK4 (step dt, nsteps steps) in one launch, one
 * GPU thread per trajectory.  alpha: device [ntraj*M] fh_c64 (trajectory-
 * major): initial values on entry (Sec. III.A uses sqrt(n_p) for a number
 * eigenstate and z_p for coherent and field-number states), values at
 * t = nsteps*dt on return.  out: device [(nsteps/every + 1)*ntraj*M] fh_c64
 * receiving the values at steps 0, every, 2 every, ... (every >= 1), or NULL.
 * Asynchronous on the stream. */
fh_status fh_classical_rk4(const fh_model* m, int ntraj, fh_c64* alpha, double dt, int64_t nsteps, int64_t every,
                           fh_c64* out, void* stream);

/* ---------------------------------------------------------------- adjoint --
 * Discrete adjoint of nsteps RK4 steps from psi0 (device), for the objective
 * J at t = nsteps*dt:
 *   FH_J_Q      : Q of Eq. (Qparam)
 *   FH_J_PO     : 1 - lambda_p / n_tot (Eq. POcriterion)
 *   FH_J_NMODE  : <a_k^+ a_k> with k = obj_mode
 * Checkpoints split the run into segments of ckpt_every steps, the first
 * segment taking the remainder; inside a segment the states are recomputed
 * forward, except in the last one, whose states (and, when kept, stage inputs)
 * the forward sweep leaves in place.  work: device scratch of at least
 * fh_adjoint_work_states(...) * total * nrhs fh_c64; with at least
 * fh_adjoint_work_states_kept(...) states the stage inputs of every step are
 * kept from that recompute instead of being computed again (three H psi per
 * step fewer; same result to rounding order).  Outputs: lambda0
 * (device, total*nrhs) = 2 dJ/d conj(psi0); J[nrhs], dJ_dLambda[nrhs],
 * dJ_dV[nrhs*M^4] (host; dJ_dV may be NULL).  Each ordered, momentum-
 * conserving V entry is an independent parameter; entries that do not conserve
 * momentum are not parameters of the model (fh_model_create rejects them) and
 * their dJ_dV is 0. */
#define FH_J_Q 0
#define FH_J_PO 1
#define FH_J_NMODE 2
/* Chebyshev propagator: nsteps steps psi <- exp(-i H dt) psi (Sec. II.A,
 * d|phi>/dt = -i H |phi>), exact up to the series truncation tol, by
 *   H = a + b T, a = (emax + emin)/2, b = (emax - emin)/2,
 *   exp(-i H dt) = exp(-i a dt) sum_k c_k T_k(T),  c_0 = J_0(b dt), c_k = 2 (-i)^k J_k(b dt),
 * with the three-term recurrence of the Chebyshev polynomials (one H psi per
 * term).  The spectrum of H on the basis must lie in [emin, emax] (see
 * fh_spectral_radius); the call fails with FH_ESTATE when the norm is not
 * conserved to 1e-8, the sign of an interval that is too small.  Time steps
 * may be far beyond RK4's stability limit.  work: device scratch of
 * 4*total*nrhs fh_c64.  Moments, FH_PER_SECTOR and FH_TIMING as for
 * fh_evolve_rk4 (FH_GRAPH is not supported). */
fh_status fh_evolve_chebyshev(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* work, double dt,
                              int64_t nsteps, double emin, double emax, double tol, int64_t obs_every,
                              double* moments, int64_t moments_capacity, int flags, fh_timing* timing,
                              void* stream);
/* Coefficients c_k (re, im; arrays of kmax) of that series for x = b dt and
 * their number K: the first k > x with 2 |J_k(x)| < tol, plus one.  Host
 * only; returns -1 if the arguments are invalid or K would exceed kmax. */
int fh_chebyshev_coefficients(double x, double tol, int kmax, double* c_re, double* c_im);
/* Estimate of the spectral radius max |E| of H on the basis by 'iters' power
 * iterations from a fixed pseudo-random vector (SplitMix64 of the index);
 * a lower bound that converges to max |E|.  work: 2*total fh_c64 (device). */
fh_status fh_spectral_radius(const fh_model* m, const fh_basis* b, fh_c64* work, int iters, double* rho,
                             void* stream);

/* Forward-mode tangent of the RK4 map with respect to Lambda: evolves psi
 * and dpsi = d psi/d Lambda together for nsteps steps (in place; dpsi is
 * usually zero at the start),
 *   d psi/dt = -i H psi,   d dpsi/dt = -i H dpsi - i G psi,   G = dH/dLambda
 * (the interaction term of Eq. Ham with Lambda = 1), differentiated step by
 * step like the discrete RK4 map, and returns J(psi_T) and
 * dJ/dLambda = Re <2 dJ/d conj(psi_T), dpsi_T> for the objectives above.
 * Needs no checkpoints: work is 8*total*nrhs fh_c64 (device).  Two H psi
 * per stage (H y gives both the psi update and G y = (H y - diag(omega.n) y)
 * / Lambda) unless |Lambda| is so small against the kinetic scale that this
 * subtraction would cost more than 1e-12 relative accuracy (eps Nmax
 * max|omega| > 1e-12 |Lambda| Nmax^2 max|V| / 2), and always at Lambda = 0:
 * then three (G y by its own application).  A memory-light cross-check of
 * fh_adjoint_rk4's dJ/dLambda. */
fh_status fh_tangent_rk4(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* dpsi, fh_c64* work,
                         double dt, int64_t nsteps, int objective, int obj_mode, double* J, double* dJ_dLambda,
                         void* stream);
int64_t fh_adjoint_work_states(int64_t nsteps, int64_t ckpt_every);       /* segments + C + 10 */
int64_t fh_adjoint_work_states_kept(int64_t nsteps, int64_t ckpt_every);  /* segments + 4 C + 10 */
fh_status fh_adjoint_rk4(const fh_model* m, const fh_basis* b, int nrhs, const fh_c64* psi0, double dt,
                         int64_t nsteps, int64_t ckpt_every, int objective, int obj_mode, fh_c64* work,
                         int64_t work_states, fh_c64* lambda0, double* J, double* dJ_dLambda,
                         double* dJ_dV, void* stream);
/* Vector-Jacobian product of the coherent initial state (Eq. coherentStates):
 * given lambda0 = 2 dJ/d conj(psi0) for psi0 = coherent(alpha), returns
 * dJ/dRe(alpha)[nrhs*M] and dJ/dIm(alpha)[nrhs*M] (host). */
fh_status fh_coherent_vjp(const fh_basis* b, int nrhs, const fh_c64* alpha, const fh_c64* lambda0,
                          double* d_re, double* d_im, void* stream);

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif
#ifdef __cplusplus
}
#endif
#endif /* FOCKHIP_H */
