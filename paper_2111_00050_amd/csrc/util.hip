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

// out[i] = in[i * nrhs + q], i < total (complex): one column of a
// several-column vector, contiguous.
__global__ void take_column_kernel(const double2* __restrict__ in, double2* __restrict__ out, long long total,
                                   int nrhs, int q) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
        out[i] = in[i * nrhs + q];
}

// RK4 stage of the tangent z = d psi / d Lambda:  k = -i (hz + gy) with
// hz = H z_s and gy = G y_s already applied; epilogue as in the fused stage:
//   FIRST: acc = base + a k, next = c0 base + b k;  MID: acc += a k,
//   next = c0 base + b k;  LAST: baseout = acc + a k.   (n complex entries)
__global__ void tangent_stage_kernel(const double* hz, const double* gy, const double* base, double* acc,
                                     double* next, double* baseout, long long n, int mode, double a, double c0,
                                     double b) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double kr = hz[2 * i + 1] + gy[2 * i + 1];      // -i (x + i y) = y - i x
        const double ki = -(hz[2 * i] + gy[2 * i]);
        if (mode == kLast) {
            baseout[2 * i] = fma(a, kr, acc[2 * i]);
            baseout[2 * i + 1] = fma(a, ki, acc[2 * i + 1]);
            continue;
        }
        const double br = base[2 * i], bi = base[2 * i + 1];
        const double ar = mode == kFirst ? br : acc[2 * i], ai = mode == kFirst ? bi : acc[2 * i + 1];
        acc[2 * i] = fma(a, kr, ar);
        acc[2 * i + 1] = fma(a, ki, ai);
        next[2 * i] = fma(b, kr, c0 * br);
        next[2 * i + 1] = fma(b, ki, c0 * bi);
    }
}

// The RK4 update of a stage as its own pass over n complex entries, for the
// mode counts where the stage kernel runs without its fused epilogue: h = H y
// on entry (h may be the destination, next or baseout, and is read before it
// is written); k = ks h; FIRST: acc = base + a k, next = c0 base + b k;
// MID: acc += a k, next = c0 base + b k; LAST: baseout = acc + a k.  Same
// arithmetic as the fused epilogue.
__global__ void rk4_update_kernel(const double* h, const double* base, double* acc, double* next, double* baseout,
                                  long long n, int mode, double ks_re, double ks_im, double a, double c0, double b) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double hr = h[2 * i], hi = h[2 * i + 1];
        const double kr = ks_re * hr - ks_im * hi;
        const double ki = ks_re * hi + ks_im * hr;
        if (mode == kLast) {
            const double ar = acc[2 * i], ai = acc[2 * i + 1];
            baseout[2 * i] = fma(a, kr, ar);
            baseout[2 * i + 1] = fma(a, ki, ai);
            continue;
        }
        const double br = base[2 * i], bi = base[2 * i + 1];
        const double ar = mode == kFirst ? br : acc[2 * i], ai = mode == kFirst ? bi : acc[2 * i + 1];
        acc[2 * i] = fma(a, kr, ar);
        acc[2 * i + 1] = fma(a, ki, ai);
        next[2 * i] = fma(b, kr, c0 * br);
        next[2 * i + 1] = fma(b, ki, c0 * bi);
    }
}

// The interaction part of H applied to y from h = H y: G y = (h - diag(omega . n) y) / Lambda,
// over nstates * nrhs complex entries ([state][rhs]); occupations from the basis's records
// (stride bytes per state).  The kinetic diagonal is summed in the stage kernel's order.
__global__ void interaction_part_kernel(const double* h, const double* y, const unsigned char* occ, int stride, int M,
                                        const double* omega, double inv_lambda, long long nstates, int nrhs,
                                        double* gy) {
    const long long n = nstates * nrhs;
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const unsigned char* r = occ + (i / nrhs) * stride;
        double kin = 0.0;
        for (int j = 0; j < M; ++j) kin = fma(omega[j], (double)r[j], kin);
        gy[2 * i] = (h[2 * i] - kin * y[2 * i]) * inv_lambda;
        gy[2 * i + 1] = (h[2 * i + 1] - kin * y[2 * i + 1]) * inv_lambda;
    }
}

// Per-block partial sums of Re sum_i conj(g_i) z_i over column rhs of a
// [total][nrhs] complex layout; partial[blockIdx.x] (fixed-order tree in the block).
__global__ void dot_re_kernel(const double* g, const double* z, long long total, int nrhs, int rhs, double* partial) {
    __shared__ double red[256];
    double s = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const long long e = i * nrhs + rhs;
        s = fma(g[2 * e], z[2 * e], fma(g[2 * e + 1], z[2 * e + 1], s));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One Chebyshev term (n complex entries): next = alpha h + beta x + gamma prev
// (prev may be NULL when gamma == 0; next may alias prev), then
// acc = (init ? c0 x : acc) + c next, with complex c0, c.
__global__ void cheb_term_kernel(const double* h, const double* x, const double* prev, double* next, double* acc,
                                 long long n, double alpha, double beta, double gamma, double c_re, double c_im,
                                 int init, double c0_re, double c0_im) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xr = x[2 * i], xi = x[2 * i + 1];
        double nr = fma(alpha, h[2 * i], beta * xr), ni = fma(alpha, h[2 * i + 1], beta * xi);
        if (prev) {
            nr = fma(gamma, prev[2 * i], nr);
            ni = fma(gamma, prev[2 * i + 1], ni);
        }
        double ar, ai;
        if (init) {
            ar = c0_re * xr - c0_im * xi;
            ai = c0_re * xi + c0_im * xr;
        } else {
            ar = acc[2 * i];
            ai = acc[2 * i + 1];
        }
        acc[2 * i] = ar + (c_re * nr - c_im * ni);
        acc[2 * i + 1] = ai + (c_re * ni + c_im * nr);
        next[2 * i] = nr;
        next[2 * i + 1] = ni;
    }
}

// out = (re + i im) * in   (n complex entries; out may alias in)
__global__ void cscale_kernel(double* out, const double* in, long long n, double re, double im) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xr = in[2 * i], xi = in[2 * i + 1];
        out[2 * i] = re * xr - im * xi;
        out[2 * i + 1] = re * xi + im * xr;
    }
}

// Deterministic start vector: entry i from the SplitMix64 finaliser of (seed, i),
// real and imaginary parts uniform in [-1, 1).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__global__ void hash_fill_kernel(double* x, long long n, unsigned long long seed) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const unsigned long long r = splitmix64(seed ^ (0x632BE59BD9B4E019ull * (unsigned long long)(i + 1)));
        x[2 * i] = (double)(r >> 11) * 0x1.0p-52 - 1.0;
        x[2 * i + 1] = (double)(splitmix64(r) >> 11) * 0x1.0p-52 - 1.0;
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
void launch_tangent_stage(const double* hz, const double* gy, const double* base, double* acc, double* next,
                          double* baseout, long long n, int mode, double a, double c0, double b, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(tangent_stage_kernel, dim3(grid_for(n)), dim3(256), 0, s, hz, gy, base, acc, next, baseout,
                           n, mode, a, c0, b);
}
void launch_rk4_update(const double* h, const double* base, double* acc, double* next, double* baseout, long long n,
                       int mode, double ks_re, double ks_im, double a, double c0, double b, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(rk4_update_kernel, dim3(grid_for(n)), dim3(256), 0, s, h, base, acc, next, baseout, n, mode,
                           ks_re, ks_im, a, c0, b);
}
void launch_interaction_part(const double* h, const double* y, const unsigned char* occ, int stride, int M,
                             const double* omega, double inv_lambda, long long nstates, int nrhs, double* gy,
                             hipStream_t s) {
    if (nstates > 0)
        hipLaunchKernelGGL(interaction_part_kernel, dim3(grid_for(nstates * nrhs)), dim3(256), 0, s, h, y, occ, stride,
                           M, omega, inv_lambda, nstates, nrhs, gy);
}
int launch_dot_re(const double* g, const double* z, long long total, int nrhs, int rhs, double* partial,
                  hipStream_t s) {
    const int G = 1024;
    hipLaunchKernelGGL(dot_re_kernel, dim3(G), dim3(256), 0, s, g, z, total, nrhs, rhs, partial);
    return G;
}
void launch_cheb_term(const double* h, const double* x, const double* prev, double* next, double* acc, long long n,
                      double alpha, double beta, double gamma, double c_re, double c_im, int init, double c0_re,
                      double c0_im, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(cheb_term_kernel, dim3(grid_for(n)), dim3(256), 0, s, h, x, prev, next, acc, n, alpha, beta,
                           gamma, c_re, c_im, init, c0_re, c0_im);
}
void launch_cscale(double* out, const double* in, long long n, double re, double im, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cscale_kernel, dim3(grid_for(n)), dim3(256), 0, s, out, in, n, re, im);
}
void launch_hash_fill(double* x, long long n, unsigned long long seed, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(hash_fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, seed);
}
void launch_take_column(const double* in, double* out, long long total, int nrhs, int q, hipStream_t s) {
    if (total > 0)
        hipLaunchKernelGGL(take_column_kernel, dim3(grid_for(total)), dim3(256), 0, s,
                           reinterpret_cast<const double2*>(in), reinterpret_cast<double2*>(out), total, nrhs, q);
}
void launch_scale_rhs(double* psi, long long total, int nrhs, const double* scale, hipStream_t s) {
    if (total > 0)
        hipLaunchKernelGGL(scale_rhs_kernel, dim3(grid_for(total * nrhs)), dim3(256), 0, s, psi, total, nrhs, scale);
}

}  // namespace fh
