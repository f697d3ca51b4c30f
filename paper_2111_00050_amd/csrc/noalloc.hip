// noalloc.hip -- fh_moments_noalloc: the moment reductions of fh_moments with
// their scratch (per-workgroup partial sums and the reduced values) in a
// file-scope device array instead of the basis's buffers, for callers that
// cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <array>
#include <mutex>

#include "fh_host.hpp"

namespace {

// Scratch of the allocation-free moments: 2^20 doubles (8 MiB) on every device
// the library runs on, held until the process ends.  Host code never uses the
// symbol's name as a device address: it uses the address that
// hipGetSymbolAddress returns for the current device (scratch_on_device).
constexpr size_t kScratchDoubles = size_t(1) << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::array<double*, kMaxDevices> g_scratch_ptr{};

// Device address of 'scratch' on the current device, looked up once per
// device with that device current.
fh_status scratch_on_device(double** out) {
    int dev = -1;
    FH_HIP(hipGetDevice(&dev));
    FH_REQUIRE(dev >= 0 && dev < kMaxDevices, FH_EUNSUPPORTED, "fh_moments_noalloc: device id out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        FH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        FH_REQUIRE(p != nullptr, FH_EHIP, "fh_moments_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return FH_OK;
}

}  // namespace

using namespace fh;

extern "C" __attribute__((visibility("default"))) fh_status fh_moments_noalloc(const fh_basis* b, int nrhs,
                                                                               int rhs, const fh_c64* psi,
                                                                               double* norm2, fh_c64* a,
                                                                               fh_c64* Mij, fh_c64* Akl,
                                                                               void* stream) {
    try {
        FH_REQUIRE(b != nullptr && psi != nullptr, FH_EINVAL, "fh_moments_noalloc: NULL argument");
        FH_REQUIRE(nrhs == 1 || nrhs == 2 || nrhs == 4 || nrhs == 8 || nrhs == 16, FH_EINVAL,
                   "nrhs must be 1, 2, 4, 8 or 16");
        FH_REQUIRE(rhs >= 0 && rhs < nrhs, FH_EINVAL, "fh_moments_noalloc: rhs out of range");
        const int M = b->M, NO = momentsOut(M);
        int cur = -1;
        FH_HIP(hipGetDevice(&cur));
        FH_REQUIRE(cur == b->device, FH_EINVAL, "fh_moments_noalloc: the basis lives on another device");
        const int groups = (Mij || Akl) ? M + 1 : 1;
        size_t lds = 0;
        const int G = moments_grid(b, &lds);
        const size_t npart = (size_t)groups * G * 2 * kMomOutMax, nred = (size_t)groups * 2 * NO;
        FH_REQUIRE(npart + nred <= kScratchDoubles, FH_EUNSUPPORTED,
                   "fh_moments_noalloc: the reduction needs more than the 2^20 doubles of static scratch "
                   "(too many workgroups on this device)");
        double* sc = nullptr;
        fh_status st = scratch_on_device(&sc);
        if (st != FH_OK) return st;
        // host staging on the stack: no allocation on any path
        std::array<double, (size_t)(kMaxM + 1) * 2 * (2 * kMaxM + 1)> v;
        std::array<double, FH_MOMENT_DOUBLES(kMaxM)> rec;
        st = moments_core(b, nrhs, rhs, reinterpret_cast<const double*>(psi), rec.data(),
                          static_cast<hipStream_t>(stream), groups, sc, sc + npart, v.data());
        if (st != FH_OK) return st;
        if (norm2) *norm2 = rec[0];
        for (int i = 0; i < M && a; ++i) a[i] = fh_c64{rec[1 + 2 * i], rec[2 + 2 * i]};
        for (int q = 0; q < M * M && Mij; ++q) Mij[q] = fh_c64{rec[1 + 2 * M + 2 * q], rec[2 + 2 * M + 2 * q]};
        for (int q = 0; q < M * M && Akl; ++q)
            Akl[q] = fh_c64{rec[1 + 2 * M + 2 * M * M + 2 * q], rec[2 + 2 * M + 2 * M * M + 2 * q]};
        return FH_OK;
    } catch (...) {
        set_error("fh_moments_noalloc: unexpected exception");
        return FH_EHIP;
    }
}
