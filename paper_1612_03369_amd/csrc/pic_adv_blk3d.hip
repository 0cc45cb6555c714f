// Instances of the 3D double-precision block advect kernels, including the
// cell-block shapes the batch autotuner chooses from.
#include <hip/hip_runtime.h>
#include "pic_advect.h"

namespace pic {
namespace {
template <int S, bool F> BlockFn pick(bool ode, bool ti)
{
    constexpr int X = BLK3_F64[0], Y = BLK3_F64[1], Z = BLK3_F64[2];
    if (ode && ti) return k_advect_blk<3, S, double, X, Y, Z, F, true, true>;
    if (ode) return k_advect_blk<3, S, double, X, Y, Z, F, true, false>;
    if (ti) return k_advect_blk<3, S, double, X, Y, Z, F, false, true>;
    return k_advect_blk<3, S, double, X, Y, Z, F, false, false>;
}
template <int S> BlockFn pick_f(bool fused, bool ode, bool ti) { return fused ? pick<S, true>(ode, ti) : pick<S, false>(ode, ti); }
template <int S, int V> BlockFn shape(bool fused)
{
    if (fused) return k_advect_blk<3, S, double, SHAPES3[V][0], SHAPES3[V][1], SHAPES3[V][2], true>;
    return k_advect_blk<3, S, double, SHAPES3[V][0], SHAPES3[V][1], SHAPES3[V][2], false>;
}
template <int S> BlockFn shape_v(int variant, bool fused)
{
    switch (variant) {
    case 0: return shape<S, 0>(fused);
    case 1: return shape<S, 1>(fused);
    case 2: return shape<S, 2>(fused);
    }
    return nullptr;
}
}  // namespace

BlockFn block_kernel_3d(int scheme, bool fused, bool ode, bool ti)
{
    switch (scheme) {
    case PIC_EULER: return pick_f<1>(fused, ode, ti);
    case PIC_RK2: return pick_f<2>(fused, ode, ti);
    case PIC_RK4: return pick_f<4>(fused, ode, ti);
    }
    return nullptr;
}

BlockFn batch_block_kernel_3(int scheme, int variant, bool fused)
{
    switch (scheme) {
    case PIC_EULER: return shape_v<1>(variant, fused);
    case PIC_RK2: return shape_v<2>(variant, fused);
    case PIC_RK4: return shape_v<4>(variant, fused);
    }
    return nullptr;
}
}  // namespace pic
