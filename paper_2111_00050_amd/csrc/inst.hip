// inst.hip -- instantiates every kernel of fh_device.hpp for one mode count.
// Compiled once per M with -DFH_INST_M=<M>.
#include "fh_device.hpp"
#include "fh_launch.hpp"

#ifndef FH_INST_M
#error "FH_INST_M must be defined"
#endif

#define FH_CAT2(a, b) a##b
#define FH_CAT(a, b) FH_CAT2(a, b)

namespace fh {
namespace {
constexpr int kM = FH_INST_M;

template <int NR>
void stage_nr(const StageArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((stage_kernel<kM, NR>), dim3(grid), dim3(kTileRows), lds, s, a);
}

void stage_any(int slot, const StageArgs& a, int grid, size_t lds, hipStream_t s) {
    switch (slot) {
        case 0: stage_nr<1>(a, grid, lds, s); break;
        case 1: stage_nr<2>(a, grid, lds, s); break;
        case 2: stage_nr<4>(a, grid, lds, s); break;
        case 3: stage_nr<8>(a, grid, lds, s); break;
        case 4: stage_nr<16>(a, grid, lds, s); break;
        default: break;
    }
}

void moments_l(const MomArgs& a, int grid, int groups, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((moments_kernel<kM>), dim3(grid, groups), dim3(kTileRows), lds, s, a);
}
void onebody_l(const OneBodyArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((onebody_kernel<kM>), dim3(grid), dim3(kTileRows), lds, s, a);
}
void corr_l(const CorrArgs& a, int grid, int classes, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((corr_kernel<kM>), dim3(grid, classes), dim3(kTileRows), lds, s, a);
}
void init_l(const InitArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((init_product_kernel<kM>), dim3(grid), dim3(kTileRows), lds, s, a);
}
void vjp_l(const VjpArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((vjp_kernel<kM>), dim3(grid), dim3(kTileRows), lds, s, a);
}
void rank_l(const RankArgs& a, hipStream_t s) {
    const long long nb = (a.count + 255) / 256;
    if (nb > 0) hipLaunchKernelGGL((rank_kernel<kM>), dim3((unsigned)nb), dim3(256), 0, s, a);
}
void unrank_l(const RankArgs& a, hipStream_t s) {
    const long long nb = (a.count + 255) / 256;
    if (nb > 0) hipLaunchKernelGGL((unrank_kernel<kM>), dim3((unsigned)nb), dim3(256), 0, s, a);
}
}  // namespace

const KernelSet* FH_CAT(kernel_set_M, FH_INST_M)() {
    static const KernelSet ks = {
        kM,
        {reinterpret_cast<const void*>(&stage_kernel<kM, 1>), reinterpret_cast<const void*>(&stage_kernel<kM, 2>),
         reinterpret_cast<const void*>(&stage_kernel<kM, 4>), reinterpret_cast<const void*>(&stage_kernel<kM, 8>),
         reinterpret_cast<const void*>(&stage_kernel<kM, 16>)},
        &stage_any,
        reinterpret_cast<const void*>(&moments_kernel<kM>),
        &moments_l,
        reinterpret_cast<const void*>(&onebody_kernel<kM>),
        &onebody_l,
        reinterpret_cast<const void*>(&corr_kernel<kM>),
        &corr_l,
        &init_l,
        &vjp_l,
        &rank_l,
        &unrank_l,
    };
    return &ks;
}

}  // namespace fh
