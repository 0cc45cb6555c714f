// Structures shared by the host launcher code and the kernels.
#pragma once
#include "pic_common.h"

namespace pic {

// Everything a kernel needs about one problem; lives in device memory so that
// the current-buffer index can be flipped by a kernel (graph replays need no
// host involvement).
struct ProblemDev {
    MeshDev mesh;
    StoreDev store[2];
    int cur;                 // index of the current buffer
    int n_prop, prop_f64;
    int pop_min, pop_max;
    // property equations integrated with the positions (off unless odes != 0):
    // damage in prop[ode_dmg], deformation gradient in prop[ode_F .. ode_F + dim^2)
    int odes, ode_dmg, ode_F;
    double ode_alpha, ode_beta;
    int64_t cap;
    double dt;
    const void *u64;         // repacked field, double
    const void *u32;         // repacked field, float
    // field that changes in time (Sec. 2.3; off unless ti != 0): u^{n+1}
    // repacked as u1_64 / u1_32, the field step dt_u, and the time elapsed
    // since t^n in *tau (device memory, advanced by dt on every counted step)
    int ti;
    double dt_u;
    const void *u1_64;
    const void *u1_32;
    double *tau;
    ScratchDev scr;
    // adjoint: arrays of the segment being replayed
    const double *adj_lam_in;  // [dim][cap] lambda of the next step, in that step's order
    double *adj_lam_out;       // [dim][cap] lambda of this step, in this step's order
    double *adj_dU;            // [dim][n_nodes]
    const int32_t *adj_src;    // [cap] gather sources of the step
};

struct WorkItem {
    int32_t problem;
    int32_t c0, c1;          // cells [c0, c1)
};
// Block of cells [i0, i0+BX) x [j0, j0+BY) x [k0, k0+BZ) of a uniform mesh
// (clipped to the mesh); its particles are BY*BZ runs of consecutive cells.
struct BlockItem {
    int32_t problem;         // -1: empty slot (no work)
    int32_t i0, j0, k0;
};
struct ScanItem {
    int32_t problem;
    int32_t chunk;
};
struct RangeItem {
    int32_t problem;
    int32_t pad;
    int64_t begin, end;      // [begin, end) in particles or cells; one workgroup of BLOCK each
};

}  // namespace pic
