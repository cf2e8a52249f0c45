// 32-row instances of the fused scale-space pass (kernel in pyramid_kernel.h).
#include "pyramid_kernel.h"

namespace s3d {

hipError_t launch_blur_tall(const FusedLaunch &a, int r, bool dog, bool pb, hipStream_t st)
{
    return fused::launch_ty<kBlurTYTall>(a, r, dog, pb, st);
}

int fused_blocks_per_cu_tall(int r, bool dog, bool pb) { return fused::occupancy_ty<kBlurTYTall>(r, dog, pb); }

}  // namespace s3d
