// Instances of the 3D single-precision-evaluation block advect kernels.
#include <hip/hip_runtime.h>
#include "pic_advect.h"

namespace pic {
namespace {
template <int S, bool F> BlockFn pick(bool ode, bool ti)
{
    constexpr int X = BLK3_F32[0], Y = BLK3_F32[1], Z = BLK3_F32[2];
    if (ode && ti) return k_advect_blk<3, S, float, X, Y, Z, F, true, true>;
    if (ode) return k_advect_blk<3, S, float, X, Y, Z, F, true, false>;
    if (ti) return k_advect_blk<3, S, float, X, Y, Z, F, false, true>;
    return k_advect_blk<3, S, float, X, Y, Z, F, false, false>;
}
template <int S> BlockFn pick_f(bool fused, bool ode, bool ti) { return fused ? pick<S, true>(ode, ti) : pick<S, false>(ode, ti); }
}  // namespace

BlockFn block_kernel_3f(int scheme, bool fused, bool ode, bool ti)
{
    switch (scheme) {
    case PIC_EULER: return pick_f<1>(fused, ode, ti);
    case PIC_RK2: return pick_f<2>(fused, ode, ti);
    case PIC_RK4: return pick_f<4>(fused, ode, ti);
    }
    return nullptr;
}
}  // namespace pic
