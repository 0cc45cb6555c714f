// Instances of the 3D per-tile advect kernels (displaced and octree meshes; uniform
// meshes when a combination has no block kernel).
#include <hip/hip_runtime.h>
#include "pic_advect.h"

#ifndef PIC_OCT_LDS
#define PIC_OCT_LDS 1       // octree advect with the tile's leaf nodes staged in LDS
#endif

namespace pic {
namespace {
constexpr int DIM = 3;
template <int S, typename T, bool O, bool TI> AdvectFn pick_kind(int kind)
{
    switch (kind) {
    case MESH_UNIFORM: return k_advect<DIM, S, T, MESH_UNIFORM, O, TI>;
    case MESH_DISPLACED: return k_advect<DIM, S, T, MESH_DISPLACED, O, TI>;
    default:
        if constexpr (DIM == 3) {
            if constexpr (O || TI) return k_advect<DIM, S, T, MESH_OCTREE, O, TI>;
            else return PIC_OCT_LDS ? k_advect_oct<S, T> : k_advect<DIM, S, T, MESH_OCTREE>;
        }
        return nullptr;
    }
}
template <int S, typename T> AdvectFn pick(int kind, bool ode, bool ti)
{
    if (ode && ti) return pick_kind<S, T, true, true>(kind);
    if (ode) return pick_kind<S, T, true, false>(kind);
    if (ti) return pick_kind<S, T, false, true>(kind);
    return pick_kind<S, T, false, false>(kind);
}
template <int S> AdvectFn pick_p(int prec, int kind, bool ode, bool ti)
{
    return prec == PIC_F32 ? pick<S, float>(kind, ode, ti) : pick<S, double>(kind, ode, ti);
}
}  // namespace

AdvectFn advect_kernel_3(int scheme, int prec, int kind, bool ode, bool ti)
{
    switch (scheme) {
    case PIC_EULER: return pick_p<1>(prec, kind, ode, ti);
    case PIC_RK2: return pick_p<2>(prec, kind, ode, ti);
    case PIC_RK4: return pick_p<4>(prec, kind, ode, ti);
    }
    return nullptr;
}
}  // namespace pic
