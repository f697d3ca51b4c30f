// derive.cpp -- host-side derived observables from the moments (fh_derive).
//
//   n_tot    = sum_i <a_i^+ a_i>                       (Sec. II.B)
//   Q        = (n_tot - sum_i |<a_i>|^2) / n_tot         (Eq. Qparam)
//   lambda_p = largest eigenvalue of M_ij = <a_i^+ a_j>  (Eq. POcriterion)
//   O        = sum_k xi_k a_k, xi the principal eigenvector (Eq. a_op)
//   V_-      = 1 + 2 (<O^+ O> - |<O>|^2) - 2 |<O^2> - <O>^2|   (Eq. generalVminus)
// All expectations are divided by norm2 = <psi|psi> (the state need not be
// normalised: truncated coherent states are not); the normalised moments and
// the mode occupations <a_i^+ a_i> are returned as well.  The Hermitian
// eigenproblem is solved with cyclic complex Jacobi rotations.
#include <cmath>
#include <complex>
#include <limits>
#include <vector>

#include "../../include/fockhip.h"

namespace {

using cd = std::complex<double>;

// Eigen-decomposition of a Hermitian n x n matrix A (row-major, overwritten).
// On return the diagonal of A holds the eigenvalues and the columns of V the
// eigenvectors.
void jacobi_hermitian(int n, std::vector<cd>& A, std::vector<cd>& V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto at = [&](int r, int c) -> cd& { return A[(size_t)r * n + c]; };
    double scale = 0.0;
    for (const cd& z : A) scale += std::norm(z);
    scale = std::sqrt(scale);
    if (scale == 0.0) return;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c)
                if (r != c) off += std::norm(at(r, c));
        if (std::sqrt(off) <= 1e-17 * scale) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cd apq = at(p, q);
                const double g = std::abs(apq);
                if (g <= 1e-300) continue;
                // Phase that makes the (p, q) entry real: D = diag(1, e^{-i phi}).
                const cd ph = apq / g;  // e^{i phi}
                const double alpha = at(p, p).real(), beta = at(q, q).real();
                const double tau = (beta - alpha) / (2.0 * g);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // U = D G on the (p, q) plane, G = [[c, s], [-s, c]]:
                const cd upp = c, upq = s, uqp = -s * std::conj(ph), uqq = c * std::conj(ph);
                for (int k = 0; k < n; ++k) {  // A <- A U
                    const cd akp = at(k, p), akq = at(k, q);
                    at(k, p) = akp * upp + akq * uqp;
                    at(k, q) = akp * upq + akq * uqq;
                }
                for (int k = 0; k < n; ++k) {  // A <- U^+ A
                    const cd apk = at(p, k), aqk = at(q, k);
                    at(p, k) = std::conj(upp) * apk + std::conj(uqp) * aqk;
                    at(q, k) = std::conj(upq) * apk + std::conj(uqq) * aqk;
                }
                at(p, q) = 0.0;
                at(q, p) = 0.0;
                at(p, p) = at(p, p).real();
                at(q, q) = at(q, q).real();
                for (int k = 0; k < n; ++k) {  // V <- V U
                    const cd vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = vkp * upp + vkq * uqp;
                    V[(size_t)k * n + q] = vkp * upq + vkq * uqq;
                }
            }
    }
}

}  // namespace

extern "C" fh_status fh_derive(int M, double norm2, const fh_c64* a, const fh_c64* Mij, const fh_c64* Akl,
                               fh_obs_scalars* s, fh_c64* xi_out, double* vminus_mode, fh_c64* a_norm,
                               fh_c64* Mij_norm, fh_c64* Akl_norm, double* n_modes) {
    if (M < 1 || M > 64 || !a || !Mij || !Akl || !s) return FH_EINVAL;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    s->norm2 = norm2;
    if (!(norm2 > 0.0) || !std::isfinite(norm2)) {
        s->n_tot = s->Q = s->lambda_p = s->po_deficit = s->vminus = nan;
        const fh_c64 cnan{nan, nan};
        for (int i = 0; i < M; ++i) {
            if (xi_out) xi_out[i] = cnan;
            if (vminus_mode) vminus_mode[i] = nan;
            if (a_norm) a_norm[i] = cnan;
            if (n_modes) n_modes[i] = nan;
        }
        for (int q = 0; q < M * M; ++q) {
            if (Mij_norm) Mij_norm[q] = cnan;
            if (Akl_norm) Akl_norm[q] = cnan;
        }
        return FH_ESTATE;
    }
    std::vector<cd> av(M), Mm((size_t)M * M), Am((size_t)M * M);
    for (int i = 0; i < M; ++i) av[i] = cd(a[i].re, a[i].im) / norm2;
    for (int q = 0; q < M * M; ++q) {
        Mm[q] = cd(Mij[q].re, Mij[q].im) / norm2;
        Am[q] = cd(Akl[q].re, Akl[q].im) / norm2;
    }
    auto put = [](const cd& z) { return fh_c64{z.real(), z.imag()}; };
    if (a_norm)
        for (int i = 0; i < M; ++i) a_norm[i] = put(av[i]);
    if (Mij_norm)
        for (int q = 0; q < M * M; ++q) Mij_norm[q] = put(Mm[q]);
    if (Akl_norm)
        for (int q = 0; q < M * M; ++q) Akl_norm[q] = put(Am[q]);
    if (n_modes)
        for (int i = 0; i < M; ++i) n_modes[i] = Mm[(size_t)i * M + i].real();
    double ntot = 0.0, sa = 0.0;
    for (int i = 0; i < M; ++i) {
        ntot += Mm[(size_t)i * M + i].real();
        sa += std::norm(av[i]);
    }
    s->n_tot = ntot;
    s->Q = ntot != 0.0 ? (ntot - sa) / ntot : nan;
    // Hermitian part of M and its spectrum.
    std::vector<cd> H((size_t)M * M), V;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j)
            H[(size_t)i * M + j] = 0.5 * (Mm[(size_t)i * M + j] + std::conj(Mm[(size_t)j * M + i]));
    jacobi_hermitian(M, H, V);
    int top = 0, second = -1;
    for (int i = 1; i < M; ++i)
        if (H[(size_t)i * M + i].real() > H[(size_t)top * M + top].real()) top = i;
    for (int i = 0; i < M; ++i)
        if (i != top && (second < 0 || H[(size_t)i * M + i].real() > H[(size_t)second * M + second].real())) second = i;
    const double lam = H[(size_t)top * M + top].real();
    s->lambda_p = lam;
    s->po_deficit = ntot != 0.0 ? 1.0 - lam / ntot : nan;
    std::vector<cd> xi(M);
    for (int k = 0; k < M; ++k) xi[k] = V[(size_t)k * M + top];
    // <O> = sum xi_k <a_k>; <O^+ O> = xi^+ M xi; <O^2> = sum xi_k xi_l <a_k a_l>.
    cd O = 0.0, O2 = 0.0, OdO = 0.0;
    for (int k = 0; k < M; ++k) O += xi[k] * av[k];
    for (int k = 0; k < M; ++k)
        for (int l = 0; l < M; ++l) {
            O2 += xi[k] * xi[l] * Am[(size_t)k * M + l];
            OdO += std::conj(xi[k]) * xi[l] * Mm[(size_t)k * M + l];
        }
    double vm = 1.0 + 2.0 * (OdO.real() - std::norm(O)) - 2.0 * std::abs(O2 - O * O);
    if (second >= 0 && lam - H[(size_t)second * M + second].real() <= 1e-8 * std::fabs(lam)) vm = nan;
    s->vminus = vm;
    if (xi_out)
        for (int k = 0; k < M; ++k) xi_out[k] = fh_c64{xi[k].real(), xi[k].imag()};
    if (vminus_mode)
        for (int i = 0; i < M; ++i) {
            const cd ai = av[i];
            vminus_mode[i] = 1.0 + 2.0 * (Mm[(size_t)i * M + i].real() - std::norm(ai)) -
                             2.0 * std::abs(Am[(size_t)i * M + i] - ai * ai);
        }
    if (!std::isfinite(ntot) || !std::isfinite(lam)) return FH_ESTATE;
    return FH_OK;
}

extern "C" fh_status fh_first_crossing(const double* t, const double* y, int64_t n, double level, int direction,
                                       double* out) {
    if (!out) return FH_EINVAL;
    *out = std::numeric_limits<double>::quiet_NaN();
    if (n < 0 || (n > 0 && (!t || !y)) || (direction != 1 && direction != -1) || !std::isfinite(level))
        return FH_EINVAL;
    for (int64_t i = 1; i < n; ++i)
        if (!(t[i] > t[i - 1])) return FH_EINVAL;
    // past(v): the sample lies at or beyond the level in the crossing direction
    auto past = [&](double v) { return direction > 0 ? v >= level : v <= level; };
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(y[i]) || !past(y[i])) continue;
        if (i == 0 || !std::isfinite(y[i - 1])) {
            *out = t[i];
        } else {
            const double f = (level - y[i - 1]) / (y[i] - y[i - 1]);
            *out = t[i - 1] + f * (t[i] - t[i - 1]);
        }
        return FH_OK;
    }
    return FH_OK;
}
