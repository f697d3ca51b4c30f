/*
 * fock_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference for the truncated interacting
 * boson problem of Eberhardt, Zamora, Kopp & Abel, "On the single classical
 * field description of interacting scalar fields" (arXiv:2111.00050).
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library; the product path never does.  It shares no code, header or
 * table with the GPU library.
 *
 * Everything here is the literal definition, evaluated the obvious way:
 *   - basis: every occupation vector of a (N, P) sector, produced by nested
 *     loops in lexicographically ascending order (n_0 most significant), kept
 *     as a sorted byte array; a state's index is found by binary search
 *     (memcmp order == lexicographic order on unsigned bytes).
 *     Sectors are the "special Hilbert spaces" of Sec. III.B: fixed total
 *     number sum_j n_j = N and momentum sum_j j n_j == P (mod pmod).
 *   - Hamiltonian, Eq. (Ham): H = sum_j w_j a_j^+ a_j
 *       + (Lambda/2) sum_{ijkl} V[i][j][k][l] a_i^+ a_j^+ a_k a_l,
 *     applied by acting with a_l, a_k, a_j^+, a_i^+ on each basis state, one
 *     ordered quadruple at a time, and projecting the result back onto the
 *     retained sectors (the projectors P^j of Sec. III.B).
 *   - moments <a_i>, <a_i^+ a_j>, <a_k a_l>, used by the Q parameter
 *     (Eq. Qparam), the Penrose-Onsager matrix (Eq. POcriterion) and the
 *     squeezing variance (Eq. generalVminus), again by literal operator action.
 *
 * Complex amplitudes are interleaved (re, im) doubles.  All arithmetic is
 * IEEE binary64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int N, P;
    int64_t dim, off;
    uint8_t *occ; /* dim * M bytes, lexicographically ascending */
} ora_sector;

typedef struct {
    int M, pmod;
    double *omega;  /* [M] */
    double Lambda;
    double *V;      /* [M^4], V[((i*M+j)*M+k)*M+l] multiplies a_i^+ a_j^+ a_k a_l */
    int nsec;
    ora_sector *sec;
    int64_t total;
} ora_ctx;

static int posmod(long long a, int m) {
    long long r = a % m;
    return (int)(r < 0 ? r + m : r);
}

/* ---------------------------------------------------------------- basis -- */

/* Nested loops over n_0, n_1, ... in ascending order give lexicographic order
 * directly.  'fill' may be NULL (count only). */
static void enum_rec(int M, int pmod, int P, int m, int remaining, long long mom,
                     uint8_t *cur, uint8_t *fill, int64_t *count) {
    if (m == M - 1) {
        cur[m] = (uint8_t)remaining;
        if (posmod(mom + (long long)m * remaining, pmod) == P) {
            if (fill) memcpy(fill + (*count) * M, cur, (size_t)M);
            (*count)++;
        }
        return;
    }
    for (int v = 0; v <= remaining; ++v) {
        cur[m] = (uint8_t)v;
        enum_rec(M, pmod, P, m + 1, remaining - v, mom + (long long)m * v, cur, fill, count);
    }
}

int64_t ora_count_sector(int M, int pmod, int N, int P) {
    if (M < 1 || N < 0 || N > 255 || pmod < 1 || P < 0 || P >= pmod) return -1;
    uint8_t cur[64];
    int64_t count = 0;
    enum_rec(M, pmod, P, 0, N, 0, cur, NULL, &count);
    return count;
}

static int lexcmp(const uint8_t *a, const uint8_t *b, int M) { return memcmp(a, b, (size_t)M); }

static int64_t find_in_sector(const ora_sector *s, int M, const uint8_t *occ) {
    int64_t lo = 0, hi = s->dim - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = lexcmp(s->occ + mid * M, occ, M);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Which retained sector holds this occupation vector (or -1). */
static int sector_of(const ora_ctx *c, const uint8_t *occ) {
    int N = 0;
    long long mom = 0;
    for (int j = 0; j < c->M; ++j) { N += occ[j]; mom += (long long)j * occ[j]; }
    int P = posmod(mom, c->pmod);
    for (int s = 0; s < c->nsec; ++s)
        if (c->sec[s].N == N && c->sec[s].P == P) return s;
    return -1;
}

/* Global index of a state in the concatenated amplitude vector, -1 when the
 * state lies outside every retained sector. */
static int64_t global_index(const ora_ctx *c, const uint8_t *occ) {
    int s = sector_of(c, occ);
    if (s < 0) return -1;
    int64_t r = find_in_sector(&c->sec[s], c->M, occ);
    return r < 0 ? -1 : c->sec[s].off + r;
}

void ora_destroy(ora_ctx *c) {
    if (!c) return;
    for (int s = 0; s < c->nsec; ++s) free(c->sec[s].occ);
    free(c->sec);
    free(c->omega);
    free(c->V);
    free(c);
}

ora_ctx *ora_create(int M, int pmod, const double *omega, double Lambda, const double *V,
                    int nsec, const int *N, const int *P) {
    if (M < 1 || M > 64 || pmod < 1 || nsec < 0) return NULL;
    ora_ctx *c = (ora_ctx *)calloc(1, sizeof(ora_ctx));
    if (!c) return NULL;
    c->M = M;
    c->pmod = pmod;
    c->Lambda = Lambda;
    size_t m4 = (size_t)M * M * M * M;
    c->omega = (double *)malloc(sizeof(double) * (size_t)M);
    c->V = (double *)malloc(sizeof(double) * m4);
    c->sec = (ora_sector *)calloc((size_t)(nsec > 0 ? nsec : 1), sizeof(ora_sector));
    if (!c->omega || !c->V || !c->sec) { ora_destroy(c); return NULL; }
    memcpy(c->omega, omega, sizeof(double) * (size_t)M);
    memcpy(c->V, V, sizeof(double) * m4);
    c->nsec = nsec;
    int64_t off = 0;
    for (int s = 0; s < nsec; ++s) {
        ora_sector *S = &c->sec[s];
        S->N = N[s];
        S->P = P[s];
        S->dim = ora_count_sector(M, pmod, N[s], P[s]);
        if (S->dim < 0) { ora_destroy(c); return NULL; }
        S->off = off;
        off += S->dim;
        S->occ = (uint8_t *)malloc((size_t)(S->dim > 0 ? S->dim : 1) * (size_t)M);
        if (!S->occ) { ora_destroy(c); return NULL; }
        uint8_t cur[64];
        int64_t cnt = 0;
        enum_rec(M, pmod, P[s], 0, N[s], 0, cur, S->occ, &cnt);
    }
    c->total = off;
    return c;
}

int64_t ora_total(const ora_ctx *c) { return c->total; }
int64_t ora_dim(const ora_ctx *c, int s) { return c->sec[s].dim; }
int64_t ora_offset(const ora_ctx *c, int s) { return c->sec[s].off; }

void ora_occupations(const ora_ctx *c, int s, uint8_t *out) {
    memcpy(out, c->sec[s].occ, (size_t)c->sec[s].dim * (size_t)c->M);
}

/* Index of each occupation vector inside sector s, -1 if not a member. */
void ora_rank(const ora_ctx *c, int s, int64_t count, const uint8_t *occ, int64_t *idx) {
    for (int64_t q = 0; q < count; ++q) idx[q] = find_in_sector(&c->sec[s], c->M, occ + q * c->M);
}

/* ------------------------------------------------------------ operators -- */

/* Annihilate one boson in mode j: returns sqrt(n_j) and lowers n_j, or 0 if
 * the mode is empty. */
static double lower(uint8_t *w, int j) {
    if (w[j] == 0) return 0.0;
    double f = sqrt((double)w[j]);
    w[j]--;
    return f;
}

/* Create one boson in mode j: raises n_j and returns sqrt(new n_j), or 0 on
 * byte overflow (cannot happen for states with N <= 253). */
static double raise_(uint8_t *w, int j) {
    if (w[j] == 255) return 0.0;
    w[j]++;
    return sqrt((double)w[j]);
}

/* out = H psi, scatter form: every basis state |n> is hit by every ordered
 * term of Eq. (Ham); the image is looked up and accumulated. */
void ora_apply_h(const ora_ctx *c, const double *psi, double *out) {
    const int M = c->M;
    memset(out, 0, sizeof(double) * 2 * (size_t)c->total);
    uint8_t w[64];
    for (int s = 0; s < c->nsec; ++s) {
        const ora_sector *S = &c->sec[s];
        for (int64_t col = 0; col < S->dim; ++col) {
            const uint8_t *n = S->occ + col * M;
            int64_t gc = S->off + col;
            double xr = psi[2 * gc], xi = psi[2 * gc + 1];
            double kin = 0.0;
            for (int j = 0; j < M; ++j) kin += c->omega[j] * (double)n[j];
            out[2 * gc] += kin * xr;
            out[2 * gc + 1] += kin * xi;
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j)
                    for (int k = 0; k < M; ++k)
                        for (int l = 0; l < M; ++l) {
                            double v = c->V[((i * M + j) * M + k) * M + l];
                            if (v == 0.0) continue;
                            memcpy(w, n, (size_t)M);
                            double f = lower(w, l);
                            if (f == 0.0) continue;
                            double g = lower(w, k);
                            if (g == 0.0) continue;
                            f *= g;
                            f *= raise_(w, j);
                            f *= raise_(w, i);
                            if (f == 0.0) continue;
                            int64_t r = global_index(c, w);
                            if (r < 0) continue;
                            double a = 0.5 * c->Lambda * v * f;
                            out[2 * r] += a * xr;
                            out[2 * r + 1] += a * xi;
                        }
        }
    }
}

/* Selected rows of H psi, gather form: for output state |n> and each ordered
 * term, the only source state that can reach |n> is n + e_k + e_l - e_i - e_j;
 * the matrix element is obtained by acting on that source literally and
 * checking that it lands on |n>.  rows[] are global indices. */
void ora_apply_h_rows(const ora_ctx *c, const double *psi, int64_t nrows, const int64_t *rows,
                      double *out) {
    const int M = c->M;
    uint8_t n[64], src[64], w[64];
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t g = rows[q];
        int s = 0;
        while (s + 1 < c->nsec && c->sec[s + 1].off <= g) ++s;
        memcpy(n, c->sec[s].occ + (g - c->sec[s].off) * M, (size_t)M);
        double kin = 0.0;
        for (int j = 0; j < M; ++j) kin += c->omega[j] * (double)n[j];
        double yr = kin * psi[2 * g], yi = kin * psi[2 * g + 1];
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j)
                for (int k = 0; k < M; ++k)
                    for (int l = 0; l < M; ++l) {
                        double v = c->V[((i * M + j) * M + k) * M + l];
                        if (v == 0.0) continue;
                        int ok = 1;
                        int tmp[64];
                        for (int t = 0; t < M; ++t) tmp[t] = n[t];
                        tmp[k]++; tmp[l]++; tmp[i]--; tmp[j]--;
                        for (int t = 0; t < M; ++t) if (tmp[t] < 0 || tmp[t] > 255) ok = 0;
                        if (!ok) continue;
                        for (int t = 0; t < M; ++t) src[t] = (uint8_t)tmp[t];
                        memcpy(w, src, (size_t)M);
                        double f = lower(w, l);
                        if (f == 0.0) continue;
                        double gk = lower(w, k);
                        if (gk == 0.0) continue;
                        f *= gk;
                        f *= raise_(w, j);
                        f *= raise_(w, i);
                        if (f == 0.0 || memcmp(w, n, (size_t)M) != 0) continue;
                        int64_t r = global_index(c, src);
                        if (r < 0) continue;
                        double a = 0.5 * c->Lambda * v * f;
                        yr += a * psi[2 * r];
                        yi += a * psi[2 * r + 1];
                    }
        out[2 * q] = yr;
        out[2 * q + 1] = yi;
    }
}

/* Unnormalised moments of the state:
 *   norm2   = <psi|psi>
 *   a[i]    = <psi| a_i |psi>
 *   Mij[i][j] = <psi| a_i^+ a_j |psi>
 *   Akl[k][l] = <psi| a_k a_l |psi>
 * Each is evaluated as sum_n conj(psi(n')) <n'|O|n> psi(n), with O acting
 * literally on |n>; images outside the retained sectors contribute zero. */
void ora_moments(const ora_ctx *c, const double *psi, double *norm2, double *a, double *Mij,
                 double *Akl) {
    const int M = c->M;
    uint8_t w[64];
    double nr = 0.0;
    memset(a, 0, sizeof(double) * 2 * (size_t)M);
    memset(Mij, 0, sizeof(double) * 2 * (size_t)M * M);
    memset(Akl, 0, sizeof(double) * 2 * (size_t)M * M);
    for (int s = 0; s < c->nsec; ++s) {
        const ora_sector *S = &c->sec[s];
        for (int64_t col = 0; col < S->dim; ++col) {
            const uint8_t *n = S->occ + col * M;
            int64_t gc = S->off + col;
            double xr = psi[2 * gc], xi = psi[2 * gc + 1];
            nr += xr * xr + xi * xi;
            for (int i = 0; i < M; ++i) {
                memcpy(w, n, (size_t)M);
                double f = lower(w, i);
                if (f == 0.0) continue;
                int64_t r = global_index(c, w);
                if (r < 0) continue;
                double yr = psi[2 * r], yi = psi[2 * r + 1];
                /* conj(y) * f * x */
                a[2 * i] += f * (yr * xr + yi * xi);
                a[2 * i + 1] += f * (yr * xi - yi * xr);
            }
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j) {
                    memcpy(w, n, (size_t)M);
                    double f = lower(w, j);
                    if (f == 0.0) continue;
                    f *= raise_(w, i);
                    int64_t r = global_index(c, w);
                    if (r < 0) continue;
                    double yr = psi[2 * r], yi = psi[2 * r + 1];
                    Mij[2 * (i * M + j)] += f * (yr * xr + yi * xi);
                    Mij[2 * (i * M + j) + 1] += f * (yr * xi - yi * xr);
                }
            for (int k = 0; k < M; ++k)
                for (int l = 0; l < M; ++l) {
                    memcpy(w, n, (size_t)M);
                    double f = lower(w, l);
                    if (f == 0.0) continue;
                    double g = lower(w, k);
                    if (g == 0.0) continue;
                    f *= g;
                    int64_t r = global_index(c, w);
                    if (r < 0) continue;
                    double yr = psi[2 * r], yi = psi[2 * r + 1];
                    Akl[2 * (k * M + l)] += f * (yr * xr + yi * xi);
                    Akl[2 * (k * M + l) + 1] += f * (yr * xi - yi * xr);
                }
        }
    }
    *norm2 = nr;
}

/* G[i][j][k][l] = <u| a_i^+ a_j^+ a_k a_l |y> for every ordered quadruple
 * (those with V == 0 included), literal scatter form.  Used by the adjoint
 * reference: the derivative of the generator with respect to one entry of V
 * is (Lambda/2) times this single operator. */
void ora_quartic_correlators(const ora_ctx *c, const double *u, const double *y, double *G) {
    const int M = c->M;
    size_t m4 = (size_t)M * M * M * M;
    memset(G, 0, sizeof(double) * 2 * m4);
    uint8_t w[64];
    for (int s = 0; s < c->nsec; ++s) {
        const ora_sector *S = &c->sec[s];
        for (int64_t col = 0; col < S->dim; ++col) {
            const uint8_t *n = S->occ + col * M;
            int64_t gc = S->off + col;
            double xr = y[2 * gc], xi = y[2 * gc + 1];
            if (xr == 0.0 && xi == 0.0) continue;
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j)
                    for (int k = 0; k < M; ++k)
                        for (int l = 0; l < M; ++l) {
                            memcpy(w, n, (size_t)M);
                            double f = lower(w, l);
                            if (f == 0.0) continue;
                            double g = lower(w, k);
                            if (g == 0.0) continue;
                            f *= g;
                            f *= raise_(w, j);
                            f *= raise_(w, i);
                            int64_t r = global_index(c, w);
                            if (r < 0) continue;
                            double ur = u[2 * r], ui = u[2 * r + 1];
                            size_t q = (size_t)((i * M + j) * M + k) * M + l;
                            G[2 * q] += f * (ur * xr + ui * xi);
                            G[2 * q + 1] += f * (ur * xi - ui * xr);
                        }
        }
    }
}

/* out = O psi for the one-body operators used by the adjoint's terminal
 * condition:
 *   kind 0: a_i psi          (image projected onto retained sectors)
 *   kind 1: a_i^+ psi
 *   kind 2: a_i^+ a_j psi
 * (i, j) select the modes. */
void ora_apply_onebody(const ora_ctx *c, int kind, int i, int j, const double *psi, double *out) {
    const int M = c->M;
    uint8_t w[64];
    memset(out, 0, sizeof(double) * 2 * (size_t)c->total);
    for (int s = 0; s < c->nsec; ++s) {
        const ora_sector *S = &c->sec[s];
        for (int64_t col = 0; col < S->dim; ++col) {
            const uint8_t *n = S->occ + col * M;
            int64_t gc = S->off + col;
            memcpy(w, n, (size_t)M);
            double f;
            if (kind == 0) {
                f = lower(w, i);
            } else if (kind == 1) {
                f = raise_(w, i);
            } else {
                f = lower(w, j);
                if (f != 0.0) f *= raise_(w, i);
            }
            if (f == 0.0) continue;
            int64_t r = global_index(c, w);
            if (r < 0) continue;
            out[2 * r] += f * psi[2 * gc];
            out[2 * r + 1] += f * psi[2 * gc + 1];
        }
    }
}
