// Fused scale-space pass for gfx950: one launch computes
//   G_i = G_{i-1} blurred by a separable Gaussian (x, then y, then z),
//   D_{i-1} = G_{i-1} - G_i                     (optional),
//   the 2x2x2 mean of G_i into the next octave's G_0 (optional),
//   B_{i-1} = the BRIEF pre-blur of G_{i-1}      (optional),
// reading G_{i-1} from HBM once (Section 3.2.2: Gaussian Convolution,
// Difference-of-Gaussian and Sub-sampling, fused here into one pass).
//
// Work decomposition: a workgroup owns a 32 x TY (x, y) tile (TY = 16, or
// 32 for launches over >= 24M voxels) and a slab of L output planes in z.
// It streams the input planes of its slab plus R halo planes on each side
// through LDS: each plane's (TY+2R) x (32+2R) halo tile is staged in LDS (coalesced row loads, clamp-to-edge), blurred
// along x into a second LDS tile, then along y into registers. The z pass
// keeps the last 2R+1 y-blurred values of each output column in a
// per-thread register ring. The plane loop is unrolled by 2R+1, so each
// step writes and reads ring slots that are compile-time constants: the
// ring stays in fixed registers with no copies between steps. The kernel
// template is in pyramid_kernel.h; this file holds the 16-row instances and
// the dispatch, pyramid_tall.hip the 32-row instances.
#include "pyramid_kernel.h"

namespace s3d {

// 32-row instances live in pyramid_tall.hip.
hipError_t launch_blur_tall(const FusedLaunch &a, int r, bool dog, bool pb, hipStream_t st);
int fused_blocks_per_cu_tall(int r, bool dog, bool pb);

hipError_t launch_blur(const FusedLaunch &a, int r, bool dog, bool pb, int ty, hipStream_t st)
{
    if (a.n_blocks <= 0) return hipSuccess;
    if (ty == kBlurTYTall) return launch_blur_tall(a, r, dog, pb, st);
    if (ty == kBlurTYSmall) return fused::launch_ty<kBlurTYSmall>(a, r, dog, pb, st);
    return hipErrorInvalidValue;
}

// Workgroups of the fused pass at radius r and tile height ty that one CU
// holds at once (registers and LDS), 0 on error or for a combination that
// has no instance.
int fused_blocks_per_cu(int r, bool dog, bool pb, int ty)
{
    if (ty == kBlurTYTall) return fused_blocks_per_cu_tall(r, dog, pb);
    if (ty == kBlurTYSmall) return fused::occupancy_ty<kBlurTYSmall>(r, dog, pb);
    return 0;
}

}  // namespace s3d
