// inst_aux.hip -- instantiates every kernel of fh_device.hpp except the
// stage kernel (inst_stage.hip) for one mode count, and assembles the kernel
// set of that M.  Compiled once per M with -DFH_INST_M=<M>.
// The stage kernel template is only declared here, never instantiated.
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

void moments_l(const MomArgs& a, int grid, int groups, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((moments_kernel<kM>), dim3(grid, groups), dim3(kTileRows), lds, s, a);
}
void onebody_l(const OneBodyArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((onebody_kernel<kM>), dim3(grid), dim3(kTileRows), lds, s, a);
}
void corr_l(const CorrArgs& a, int grid, int classes, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((corr_kernel<kM>), dim3(grid, classes), dim3(kTileRows), lds, s, a);
}
void classical_l(const ClassicalArgs& a, hipStream_t s) {
    const int nb = (a.ntraj + 255) / 256;
    if (nb > 0) hipLaunchKernelGGL((classical_kernel<kM>), dim3(nb), dim3(256), 0, s, a);
}
void occ_l(const OccArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((occ_table_kernel<kM>), dim3(grid), dim3(kTileRows), lds, s, a);
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

#define FH_STAGE(r) FH_CAT(FH_CAT(FH_CAT(stage_entry_M, FH_INST_M), _R), r)()
StageEntry FH_CAT(FH_CAT(stage_entry_M, FH_INST_M), _R1)();
StageEntry FH_CAT(FH_CAT(stage_entry_M, FH_INST_M), _R2)();
StageEntry FH_CAT(FH_CAT(stage_entry_M, FH_INST_M), _R4)();
StageEntry FH_CAT(FH_CAT(stage_entry_M, FH_INST_M), _R8)();
StageEntry FH_CAT(FH_CAT(stage_entry_M, FH_INST_M), _R16)();

const KernelSet* FH_CAT(kernel_set_M, FH_INST_M)() {
    static const StageEntry st[kNrhsVariants] = {FH_STAGE(1), FH_STAGE(2), FH_STAGE(4), FH_STAGE(8), FH_STAGE(16)};
    static const KernelSet ks = {
        kM,
        {st[0].fn, st[1].fn, st[2].fn, st[3].fn, st[4].fn},
        {st[0].launch, st[1].launch, st[2].launch, st[3].launch, st[4].launch},
        reinterpret_cast<const void*>(&moments_kernel<kM>),
        &moments_l,
        reinterpret_cast<const void*>(&onebody_kernel<kM>),
        &onebody_l,
        reinterpret_cast<const void*>(&corr_kernel<kM>),
        &corr_l,
        &occ_l,
        &classical_l,
        &init_l,
        &vjp_l,
        &rank_l,
        &unrank_l,
    };
    return &ks;
}

}  // namespace fh
