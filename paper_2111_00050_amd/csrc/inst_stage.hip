// inst_stage.hip -- instantiates the H psi stage kernel for one (M, nrhs):
// the static-walk variant and, from M = 7 on, the per-XCD counter variant.
// Compiled once per pair with -DFH_INST_M=<M> -DFH_INST_R=<nrhs>.
#include "fh_device.hpp"
#include "fh_launch.hpp"

#if !defined(FH_INST_M) || !defined(FH_INST_R)
#error "FH_INST_M and FH_INST_R must be defined"
#endif

#define FH_CAT4_(a, b, c, d) a##b##c##d
#define FH_CAT4(a, b, c, d) FH_CAT4_(a, b, c, d)

namespace fh {
namespace {
void launch(const StageArgs& a, int grid, size_t lds, hipStream_t s) {
    if constexpr (FH_INST_M >= kStageCounterMinM) {
        if (a.queue) {
            hipLaunchKernelGGL((stage_kernel<FH_INST_M, FH_INST_R, true>), dim3(grid), dim3(kTileRows), lds, s, a);
            return;
        }
    }
    hipLaunchKernelGGL((stage_kernel<FH_INST_M, FH_INST_R, false>), dim3(grid), dim3(kTileRows), lds, s, a);
}
}  // namespace

StageEntry FH_CAT4(stage_entry_M, FH_INST_M, _R, FH_INST_R)() {
    return StageEntry{reinterpret_cast<const void*>(&stage_kernel<FH_INST_M, FH_INST_R, false>), &launch};
}
}  // namespace fh
