// fh_launch.hpp -- per-M kernel sets (one translation unit per M) and the
// generic utility kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fh_common.hpp"

namespace fh {

constexpr int kNrhsVariants = 5;  // nrhs = 1, 2, 4, 8, 16
inline int nrhs_slot(int nrhs) {
    switch (nrhs) {
        case 1: return 0;
        case 2: return 1;
        case 4: return 2;
        case 8: return 3;
        case 16: return 4;
        default: return -1;
    }
}

using StageLaunch = void (*)(const StageArgs&, int grid, size_t lds, hipStream_t);
struct StageEntry {
    const void* fn;
    StageLaunch launch;
};

struct KernelSet {
    int M;
    const void* stage_fn[kNrhsVariants];
    StageLaunch stage[kNrhsVariants];
    const void* moments_fn;
    void (*moments)(const MomArgs&, int grid, int groups, size_t lds, hipStream_t);
    const void* onebody_fn;
    void (*onebody)(const OneBodyArgs&, int grid, size_t lds, hipStream_t);
    const void* corr_fn;
    void (*corr)(const CorrArgs&, int grid, int classes, size_t lds, hipStream_t);
    void (*occ_table)(const OccArgs&, int grid, size_t lds, hipStream_t);
    void (*classical)(const ClassicalArgs&, hipStream_t);
    void (*init_product)(const InitArgs&, int grid, size_t lds, hipStream_t);
    void (*vjp)(const VjpArgs&, int grid, size_t lds, hipStream_t);
    void (*rank)(const RankArgs&, hipStream_t);
    void (*unrank)(const RankArgs&, hipStream_t);
};

const KernelSet* kernel_set_M1();
const KernelSet* kernel_set_M2();
const KernelSet* kernel_set_M3();
const KernelSet* kernel_set_M4();
const KernelSet* kernel_set_M5();
const KernelSet* kernel_set_M6();
const KernelSet* kernel_set_M7();
const KernelSet* kernel_set_M8();
const KernelSet* kernel_set_M9();
const KernelSet* kernel_set_M10();

inline const KernelSet* kernel_set(int M) {
    switch (M) {
        case 1: return kernel_set_M1();
        case 2: return kernel_set_M2();
        case 3: return kernel_set_M3();
        case 4: return kernel_set_M4();
        case 5: return kernel_set_M5();
        case 6: return kernel_set_M6();
        case 7: return kernel_set_M7();
        case 8: return kernel_set_M8();
        case 9: return kernel_set_M9();
        case 10: return kernel_set_M10();
        default: return nullptr;
    }
}

// Generic kernels (util.hip).
void launch_fill(double* p, long long n, double v, hipStream_t s);
void launch_set_c64(double* p, long long idx, double re, double im, hipStream_t s);
// out[g*nvals + o] (+)= sum_{b<G} part[(g*G + b)*stride + o], fixed order.
void launch_reduce_partials(const double* part, int ngroups, int G, int stride, int nvals, double* out,
                            int accumulate, hipStream_t s);
// One RK4 stage of the tangent d psi/d Lambda (n complex entries; see util.hip).
void launch_tangent_stage(const double* hz, const double* gy, const double* base, double* acc, double* next,
                          double* baseout, long long n, int mode, double a, double c0, double b, hipStream_t s);
// RK4 stage update as a separate pass (h = H y, may be next or baseout).
void launch_rk4_update(const double* h, const double* base, double* acc, double* next, double* baseout, long long n,
                       int mode, double ks_re, double ks_im, double a, double c0, double b, hipStream_t s);
// G y = (H y - diag(omega . n) y) / Lambda from h = H y (see util.hip).
void launch_interaction_part(const double* h, const double* y, const unsigned char* occ, int stride, int M,
                             const double* omega, double inv_lambda, long long nstates, int nrhs, double* gy,
                             hipStream_t s);
// Re sum conj(g) z over column rhs: writes per-block partials, returns their count.
int launch_dot_re(const double* g, const double* z, long long total, int nrhs, int rhs, double* partial,
                  hipStream_t s);
// Chebyshev term, complex scale and deterministic start vector (see util.hip).
void launch_cheb_term(const double* h, const double* x, const double* prev, double* next, double* acc, long long n,
                      double alpha, double beta, double gamma, double c_re, double c_im, int init, double c0_re,
                      double c0_im, hipStream_t s);
void launch_cscale(double* out, const double* in, long long n, double re, double im, hipStream_t s);
void launch_hash_fill(double* x, long long n, unsigned long long seed, hipStream_t s);
// psi[i*nrhs + q] *= scale[q]
void launch_scale_rhs(double* psi, long long total, int nrhs, const double* scale, hipStream_t s);
// out = column q of the total x nrhs complex vector in, contiguous (total complex).
void launch_take_column(const double* in, double* out, long long total, int nrhs, int q, hipStream_t s);

}  // namespace fh
