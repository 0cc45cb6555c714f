// Adjoint of the multi-step RK advection with respect to the nodal field.
//
// Forward step (classical RK4; RK2 and Euler analogously):
//   y1 = x, y2 = x + k1/2, y3 = x + k2/2, y4 = x + k3, k_s = dt u_h(y_s),
//   x+ = x + k1/6 + k2/3 + k3/3 + k4/6.
// Reverse step with lam' = dL/dx+:
//   kb1 = lam'/6, kb2 = kb3 = lam'/3, kb4 = lam'/6;
//   for s = 4,3,2,1: yb_s = dt grad(u_h)(y_s)^T kb_s,
//                    dU_c[node_i(K_s)] += dt phi_i(yhat_s) kb_s,c,
//   with kb3 += yb4 after stage 4, kb2 += yb3/2 after stage 3, kb1 += yb2/2
//   after stage 2;  lam = lam' + yb1 + yb2 + yb3 + yb4.
// The gradient of u_h is taken in the cell the stage point was located in.
#pragma once
#include "pic_common.h"
#include "pic_internal.h"

namespace pic {

// physical gradient G[c][j] = d u_c / d x_j at (K, t)
template <int D, int KIND>
__device__ __forceinline__ void grad_phys(const MeshDev &m, const typename NodeVec<D, double>::type *U, int64_t K,
                                          const double *t, double G[3][3])
{
    double Gr[3][3];
    eval_q2_refgrad<D, KIND>(m, U, K, t, Gr);
    if constexpr (KIND == MESH_DISPLACED) {
        double J[3][3];
        map_jacobian<D, KIND>(m, K, t, J);
        // G = Gr J^{-1}: row c solves J^T g = Gr[c]
        double JT[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) JT[a][b] = J[b][a];
        for (int c = 0; c < D; ++c) {
            double s[3];
            solve_small<D>(JT, Gr[c], s);
            for (int j = 0; j < D; ++j) G[c][j] = s[j];
        }
    } else {
        double x0[3], h[3];
        cell_box<KIND>(m, K, x0, h);
        for (int c = 0; c < D; ++c)
            for (int j = 0; j < D; ++j) G[c][j] = Gr[c][j] / h[j];
    }
}

// dU_c[node_i(K)] += w phi_i(t) kb_c with hardware FP64 atomics
template <int D, int KIND>
__device__ __forceinline__ void scatter_field(const MeshDev &m, double *dU, int64_t K, const double *t, double w,
                                              const double *kb)
{
    double l[3][3];
    for (int a = 0; a < D; ++a) lag3(t[a], l[a]);
    const int nc3 = D == 3 ? 3 : 1;
    const int64_t nn = m.n_nodes;
    for (int c3 = 0; c3 < nc3; ++c3)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                double phi = l[0][a] * l[1][b] * (D == 3 ? l[2][c3] : 1.0);
                int64_t g = q2_node<D, KIND>(m, K, a, b, c3);
                double f = w * phi;
                for (int c = 0; c < D; ++c) unsafeAtomicAdd(&dU[c * nn + g], f * kb[c]);
            }
}

/*
 * One reverse step.  Thread per particle p of the step's output order
 * (src[p] = its index s in the step's input order).  Recomputes the stage
 * points from the saved input state (same code as the forward, so the same
 * cells), applies the reverse sweep, writes lam_out[s].  Particles lost in the
 * step keep lam_out = 0 (cleared beforehand).
 */
template <int D, int S, int KIND>
__global__ __launch_bounds__(BLOCK) void k_adjoint_step(const ProblemDev *__restrict__ probs, const double *__restrict__ x_in,
                                                        const double *__restrict__ xr_in, const int32_t *__restrict__ cell_in,
                                                        const int32_t *__restrict__ src, const int32_t *__restrict__ n_out_ptr,
                                                        const double *__restrict__ lam_next, double *__restrict__ lam_out,
                                                        double *__restrict__ dU)
{
    const ProblemDev &P = probs[0];
    const MeshDev &m = P.mesh;
    const auto *U = reinterpret_cast<const typename NodeVec<D, double>::type *>(P.u64);
    const int64_t cap = P.cap;
    const double dt = P.dt;
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= (int64_t)*n_out_ptr) return;
    const int64_t s = src[p];
    double x[3], y[D > 0 ? 4 : 1][3], ty[4][3], k[4][3], u[3];
    int32_t Ky[4];
    for (int a = 0; a < D; ++a) {
        x[a] = x_in[a * cap + s];
        y[0][a] = x[a];
        ty[0][a] = xr_in[a * cap + s];
    }
    Ky[0] = cell_in[s];
    LocStats ls = {0, 0, 0, 0};
    constexpr int NS = S == 4 ? 4 : S;
    for (int st = 0; st < NS; ++st) {
        if (st > 0) {
            double f = (S == 4 && st == 3) ? 1.0 : 0.5;
            for (int a = 0; a < D; ++a) y[st][a] = x[a] + f * k[st - 1][a];
            locate<D, KIND>(m, y[st], Ky[st - 1 > 0 ? st - 1 : 0], Ky[st], ty[st], ls);
        }
        eval_q2<D, double, KIND>(m, U, Ky[st], ty[st], u);
        for (int a = 0; a < D; ++a) k[st][a] = dt * u[a];
    }
    double lam[3], kb[4][3], yb[4][3];
    for (int a = 0; a < D; ++a) lam[a] = lam_next[a * cap + p];
    if constexpr (S == 1) {
        for (int a = 0; a < D; ++a) kb[0][a] = lam[a];
    } else if constexpr (S == 2) {
        for (int a = 0; a < D; ++a) {
            kb[1][a] = lam[a];
            kb[0][a] = 0.0;
        }
    } else {
        for (int a = 0; a < D; ++a) {
            kb[0][a] = lam[a] / 6.0;
            kb[1][a] = lam[a] / 3.0;
            kb[2][a] = lam[a] / 3.0;
            kb[3][a] = lam[a] / 6.0;
        }
    }
    for (int st = NS - 1; st >= 0; --st) {
        double G[3][3];
        grad_phys<D, KIND>(m, U, Ky[st], ty[st], G);
        for (int j = 0; j < D; ++j) {
            double acc = 0.0;
            for (int c = 0; c < D; ++c) acc += G[c][j] * kb[st][c];
            yb[st][j] = dt * acc;
        }
        scatter_field<D, KIND>(m, dU, Ky[st], ty[st], dt, kb[st]);
        if constexpr (S == 2) {
            if (st == 1)
                for (int a = 0; a < D; ++a) kb[0][a] = 0.5 * yb[1][a];
        } else if constexpr (S == 4) {
            if (st == 3)
                for (int a = 0; a < D; ++a) kb[2][a] += yb[3][a];
            if (st == 2)
                for (int a = 0; a < D; ++a) kb[1][a] += 0.5 * yb[2][a];
            if (st == 1)
                for (int a = 0; a < D; ++a) kb[0][a] += 0.5 * yb[1][a];
        }
    }
    for (int a = 0; a < D; ++a) {
        double v = lam[a];
        for (int st = 0; st < NS; ++st) v += yb[st][a];
        lam_out[a * cap + s] = v;
    }
}

__global__ void k_fill_f64(double *p, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

// Copy the live part of the current buffer's (x, xr, cell, cs) to flat arrays
// (dir = 0) or from flat arrays into the current buffer (dir = 1).  The
// current buffer is selected on the device.
__global__ __launch_bounds__(BLOCK) void k_state_copy(const ProblemDev *__restrict__ probs, double *x, double *xr,
                                                      int32_t *cell, int32_t *cs, int dir)
{
    const ProblemDev &P = probs[0];
    const StoreDev b = P.store[P.cur];
    const int64_t cap = P.cap, nc = P.mesh.n_cells;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t n = dir == 0 ? b.cs[nc] : cs[nc];
    const int D = P.mesh.dim;
    if (i <= nc && cs) {
        if (dir == 0) cs[i] = b.cs[i];
        else b.cs[i] = cs[i];
    }
    if (i >= n) return;
    for (int a = 0; a < D; ++a) {
        if (dir == 0) {
            x[a * cap + i] = b.x[a * cap + i];
            xr[a * cap + i] = b.xr[a * cap + i];
        } else {
            b.x[a * cap + i] = x[a * cap + i];
            b.xr[a * cap + i] = xr[a * cap + i];
        }
    }
    if (dir == 0) cell[i] = b.cell[i];
    else b.cell[i] = cell[i];
}

__global__ void k_copy_i32(int32_t *dst, const int32_t *src, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace pic
