// util.hip -- small generic kernels: fills, element set, fixed-order partial
// reductions and per-rhs scaling.
#include <hip/hip_runtime.h>

#include "fh_launch.hpp"

namespace fh {

__global__ void fill_kernel(double* p, long long n, double v) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void set_c64_kernel(double* p, long long idx, double re, double im) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        p[2 * idx] = re;
        p[2 * idx + 1] = im;
    }
}

// One thread per (group, value): a sequential sum over the G partials, so the
// result does not depend on scheduling.
__global__ void reduce_partials_kernel(const double* part, int ngroups, int G, int stride, int nvals, double* out,
                                       int accumulate) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ngroups * nvals) return;
    const int g = q / nvals, o = q % nvals;
    double s = 0.0;
    for (int b = 0; b < G; ++b) s += part[((size_t)g * G + b) * stride + o];
    out[q] = accumulate ? out[q] + s : s;
}

__global__ void scale_rhs_kernel(double* psi, long long total, int nrhs, const double* scale) {
    const long long n = total * nrhs;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double s = scale[i % nrhs];
        psi[2 * i] *= s;
        psi[2 * i + 1] *= s;
    }
}

static unsigned grid_for(long long n) {
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_fill(double* p, long long n, double v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}
void launch_set_c64(double* p, long long idx, double re, double im, hipStream_t s) {
    hipLaunchKernelGGL(set_c64_kernel, dim3(1), dim3(64), 0, s, p, idx, re, im);
}
void launch_reduce_partials(const double* part, int ngroups, int G, int stride, int nvals, double* out,
                            int accumulate, hipStream_t s) {
    const int n = ngroups * nvals;
    if (n > 0)
        hipLaunchKernelGGL(reduce_partials_kernel, dim3((n + 63) / 64), dim3(64), 0, s, part, ngroups, G, stride,
                           nvals, out, accumulate);
}
void launch_scale_rhs(double* psi, long long total, int nrhs, const double* scale, hipStream_t s) {
    if (total > 0)
        hipLaunchKernelGGL(scale_rhs_kernel, dim3(grid_for(total * nrhs)), dim3(256), 0, s, psi, total, nrhs, scale);
}

}  // namespace fh
