// stage_kernel.hip -- one (precision, order) instance of the stage kernel
// and its companions (energy, halo publication, upwind adjoint gradient).
// Built once per pair with -DMDG_R=<float|double> -DMDG_P=<order>, so the
// instances compile in parallel; the device code is in stage_kernel.hpp.
#include "stage_kernel.hpp"

#if !defined(MDG_R) || !defined(MDG_P)
#error "build with -DMDG_R=float|double -DMDG_P=1..4"
#endif

namespace mdg {
template void launch_p<MDG_R, MDG_P>(const DevArgs&, bool, bool, bool, int, size_t, bool, bool, bool, hipStream_t);
template void launch_energy_rp<MDG_R, MDG_P>(const void*, const void*, int64_t, double*, double*, int, hipStream_t);
template void launch_publish_rp<MDG_R, MDG_P>(const void*, uint32_t, int, const int32_t*, void*, uint32_t, int, int,
                                               const int64_t*, int, hipStream_t);
template void launch_grad_upw_rp<MDG_R, MDG_P>(double*, const void*, const void*, const void*, double, const void*,
                                                const int32_t*, int64_t, double, int, hipStream_t);
}  // namespace mdg
