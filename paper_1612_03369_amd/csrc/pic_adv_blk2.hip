// Instances of the 2D block advect kernels (both evaluation precisions),
// including the cell-block shapes the batch autotuner chooses from.
#include <hip/hip_runtime.h>
#include "pic_advect.h"

namespace pic {
namespace {
template <int S, typename T, bool F> BlockFn pick(bool ode, bool ti)
{
    constexpr int X = BLK2[0], Y = BLK2[1];
    if (ode && ti) return k_advect_blk<2, S, T, X, Y, 1, F, true, true>;
    if (ode) return k_advect_blk<2, S, T, X, Y, 1, F, true, false>;
    if (ti) return k_advect_blk<2, S, T, X, Y, 1, F, false, true>;
    return k_advect_blk<2, S, T, X, Y, 1, F, false, false>;
}
template <int S> BlockFn pick_f(int prec, bool fused, bool ode, bool ti)
{
    if (prec == PIC_F32) return fused ? pick<S, float, true>(ode, ti) : pick<S, float, false>(ode, ti);
    return fused ? pick<S, double, true>(ode, ti) : pick<S, double, false>(ode, ti);
}
template <int S, int V> BlockFn shape(bool fused)
{
    if (fused) return k_advect_blk<2, S, double, SHAPES2[V][0], SHAPES2[V][1], 1, true>;
    return k_advect_blk<2, S, double, SHAPES2[V][0], SHAPES2[V][1], 1, false>;
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

BlockFn block_kernel_2(int scheme, int prec, bool fused, bool ode, bool ti)
{
    switch (scheme) {
    case PIC_EULER: return pick_f<1>(prec, fused, ode, ti);
    case PIC_RK2: return pick_f<2>(prec, fused, ode, ti);
    case PIC_RK4: return pick_f<4>(prec, fused, ode, ti);
    }
    return nullptr;
}

BlockFn batch_block_kernel_2(int scheme, int variant, bool fused)
{
    switch (scheme) {
    case PIC_EULER: return shape_v<1>(variant, fused);
    case PIC_RK2: return shape_v<2>(variant, fused);
    case PIC_RK4: return shape_v<4>(variant, fused);
    }
    return nullptr;
}
}  // namespace pic
