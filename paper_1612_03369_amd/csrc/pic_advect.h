// Advection + location kernels (Sec. 2.3, 2.4): the generic per-tile kernel,
// the octree kernel with LDS-staged leaf nodes and the uniform-mesh kernel
// with an LDS window of the node lattice.  Templates only: each combination
// is instantiated in exactly one of the pic_adv_*.hip units, which return
// them through the selector functions declared at the end.
#pragma once
#include "pic.h"
#include "pic_common.h"
#include "pic_internal.h"

namespace pic {

// Cell-block shapes of the LDS-staged advect (uniform meshes) per (dim, precision).
#ifndef PIC_BLK3_F32
#define PIC_BLK3_F32 4, 4, 4
#endif
constexpr int BLK3_F32[3] = {PIC_BLK3_F32};
constexpr int BLK3_F64[3] = {4, 4, 4};
constexpr int BLK2[3] = {8, 8, 1};
// Cell blocks of the reverse step: smaller in 3D, so that its two LDS windows
// (field and dU accumulators, double precision) leave room for two workgroups
// per CU.
constexpr int ADJ3[3] = {4, 2, 2};
constexpr int ADJ2[3] = {8, 8, 1};
inline const int *block_shape(int dim, int prec)
{
    return dim == 2 ? BLK2 : (prec == PIC_F32 ? BLK3_F32 : BLK3_F64);
}

// Candidate cell-block shapes of the batched (double-precision) advect, one
// of which pic_batch_tune picks per (dim, scheme) group; shape 0 is the
// default above.
constexpr int N_SHAPES = 3;
constexpr int SHAPES2[N_SHAPES][3] = {{8, 8, 1}, {8, 4, 1}, {16, 8, 1}};
constexpr int SHAPES3[N_SHAPES][3] = {{4, 4, 4}, {4, 2, 2}, {4, 4, 2}};
static_assert(SHAPES2[0][0] == BLK2[0] && SHAPES2[0][1] == BLK2[1], "shape 0 is the default");
static_assert(SHAPES3[0][0] == BLK3_F64[0] && SHAPES3[0][1] == BLK3_F64[1] && SHAPES3[0][2] == BLK3_F64[2],
              "shape 0 is the default");
inline const int *batch_shape(int dim, int variant) { return dim == 2 ? SHAPES2[variant] : SHAPES3[variant]; }

// ===========================================================================
// advect + locate (Sec. 2.3 and 2.4)
// ===========================================================================
// ev(c, K, t, u): the field at reference point t of cell K at the stage time
// code c (0: the step's start, 1: its midpoint, 2: its end; a steady field
// ignores it).
template <int D, int S, int KIND, class Eval>
__device__ __forceinline__ uint32_t advect_one_e(const MeshDev &m, Eval &&ev, double dt, double *x, double *t,
                                                 int32_t K, bool &near, LocStats &ls)
{
    double u[3], k1[3], y[3], ty[3];
    int32_t Ky;
    ev(0, K, t, u);                          // stage 1: stored (K, xhat), no location needed
#pragma unroll
    for (int a = 0; a < D; ++a) k1[a] = dt * u[a];
    double xn[3];
    if constexpr (S == 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + k1[a];
    } else if constexpr (S == 2) {
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = x[a] + 0.5 * k1[a];
        near |= near_boundary<D>(m, y);
        if (!locate<D, KIND>(m, y, K, Ky, ty, ls)) return LOST;
        ev(1, Ky, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + dt * u[a];
    } else {
        double k2[3], k3[3];
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = x[a] + 0.5 * k1[a];
        near |= near_boundary<D>(m, y);
        if (!locate<D, KIND>(m, y, K, Ky, ty, ls)) return LOST;
        ev(1, Ky, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) k2[a] = dt * u[a];
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = x[a] + 0.5 * k2[a];
        near |= near_boundary<D>(m, y);
        if (!locate<D, KIND>(m, y, Ky, Ky, ty, ls)) return LOST;
        ev(1, Ky, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) k3[a] = dt * u[a];
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = x[a] + k3[a];
        near |= near_boundary<D>(m, y);
        if (!locate<D, KIND>(m, y, Ky, Ky, ty, ls)) return LOST;
        ev(2, Ky, ty, u);
        const double s6 = 1.0 / 6.0, s3 = 1.0 / 3.0;
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + k1[a] * s6 + k2[a] * s3 + k3[a] * s3 + (dt * u[a]) * s6;
    }
    near |= near_boundary<D>(m, xn);
    int32_t Kn;
    double tn[3];
    if (!locate<D, KIND>(m, xn, K, Kn, tn, ls)) return LOST;
    near |= face_dist<D>(tn) < NEAR_TOL;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        x[a] = xn[a];
        t[a] = tn[a];
    }
    return (uint32_t)Kn;
}

template <int D, int S, typename T, int KIND>
__device__ __forceinline__ uint32_t advect_one(const MeshDev &m, const typename NodeVec<D, T>::type *__restrict__ U,
                                               double dt, double *x, double *t, int32_t K, bool &near, LocStats &ls)
{
    auto ev = [&](int, int32_t Kc, const double *tc, double *uc) { eval_q2<D, T, KIND>(m, U, Kc, tc, uc); };
    return advect_one_e<D, S, KIND>(m, ev, dt, x, t, K, near, ls);
}

// The same step for the position and the property equations as one system
// (damage and deformation gradient, Pp = [d, F_00, F_01, ...]): every stage
// evaluates u and grad u at its point; gr(c, K, t, G) gives the physical
// gradient in cell K at stage time code c.  Positions take exactly the operations of advect_one_e.
template <int D, int S, int KIND, class Eval, class Grad>
__device__ __forceinline__ uint32_t advect_one_e_ode(const MeshDev &m, Eval &&ev, Grad &&gr, double dt, double alpha,
                                                     double beta, double *x, double *t, double *Pp, int32_t K,
                                                     bool &near, LocStats &ls)
{
    constexpr int NP = 1 + D * D;
    constexpr int NS = S == 1 ? 1 : (S == 2 ? 2 : 4);
    double u[3], G[3][3], kx[4][3], kP[4][NP], y[3], ty[3], Ps[NP];
    int32_t Ky = K;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (s == 0) {
            ev(0, K, t, u);
            gr(0, K, t, G);
#pragma unroll
            for (int q = 0; q < NP; ++q) Ps[q] = Pp[q];
        } else {
            const double c = (S == 4 && s == 3) ? 1.0 : 0.5;
#pragma unroll
            for (int a = 0; a < D; ++a) y[a] = x[a] + c * kx[s - 1][a];
#pragma unroll
            for (int q = 0; q < NP; ++q) Ps[q] = Pp[q] + c * kP[s - 1][q];
            near |= near_boundary<D>(m, y);
            if (!locate<D, KIND>(m, y, s == 1 ? K : Ky, Ky, ty, ls)) return LOST;
            ev(S == 4 && s == 3 ? 2 : 1, Ky, ty, u);
            gr(S == 4 && s == 3 ? 2 : 1, Ky, ty, G);
        }
        double dd, dF[D * D];
        prop_rates<D>(G, alpha, beta, Ps[0], Ps + 1, dd, dF);
#pragma unroll
        for (int a = 0; a < D; ++a) kx[s][a] = dt * u[a];
        kP[s][0] = dt * dd;
#pragma unroll
        for (int q = 0; q < D * D; ++q) kP[s][1 + q] = dt * dF[q];
    }
    double xn[3], Pn[NP];
    if constexpr (S == 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + kx[0][a];
#pragma unroll
        for (int q = 0; q < NP; ++q) Pn[q] = Pp[q] + kP[0][q];
    } else if constexpr (S == 2) {
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + kx[1][a];
#pragma unroll
        for (int q = 0; q < NP; ++q) Pn[q] = Pp[q] + kP[1][q];
    } else {
        const double s6 = 1.0 / 6.0, s3 = 1.0 / 3.0;
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + kx[0][a] * s6 + kx[1][a] * s3 + kx[2][a] * s3 + kx[3][a] * s6;
#pragma unroll
        for (int q = 0; q < NP; ++q) Pn[q] = Pp[q] + kP[0][q] * s6 + kP[1][q] * s3 + kP[2][q] * s3 + kP[3][q] * s6;
    }
    near |= near_boundary<D>(m, xn);
    int32_t Kn;
    double tn[3];
    if (!locate<D, KIND>(m, xn, K, Kn, tn, ls)) return LOST;
    near |= face_dist<D>(tn) < NEAR_TOL;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        x[a] = xn[a];
        t[a] = tn[a];
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) Pp[q] = Pn[q];
    return (uint32_t)Kn;
}

// Uniform meshes: the same step with (i,j,k) carried along (no index division
// after the first) and the closed-form location.
template <int D, int S, typename T>
__device__ __forceinline__ uint32_t advect_one_uniform(const MeshDev &m, gptr<typename NodeVec<D, T>::type> U, double dt,
                                                       double *x, double *t, uint32_t K, bool &near)
{
    int ijk[3], jk[3];
    double u[3], k1[3], y[3], ty[3], xn[3];
    ijk_of<D>(m, K, ijk);
    eval_q2_ijk<D, T>(U, m.nnx, m.nny, ijk, t, u);
#pragma unroll
    for (int a = 0; a < D; ++a) k1[a] = dt * u[a];
    bool in = true;
    if constexpr (S == 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + k1[a];
    } else if constexpr (S == 2) {
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = x[a] + 0.5 * k1[a];
        near |= in & near_boundary<D>(m, y);
        in &= locate_uniform<D>(m, y, jk, ty);
        eval_q2_ijk<D, T>(U, m.nnx, m.nny, jk, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + dt * u[a];
    } else {
        double k2[3], k3[3];
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = x[a] + 0.5 * k1[a];
        near |= in & near_boundary<D>(m, y);
        in &= locate_uniform<D>(m, y, jk, ty);
        eval_q2_ijk<D, T>(U, m.nnx, m.nny, jk, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            k2[a] = dt * u[a];
            y[a] = x[a] + 0.5 * k2[a];
        }
        near |= in & near_boundary<D>(m, y);
        in &= locate_uniform<D>(m, y, jk, ty);
        eval_q2_ijk<D, T>(U, m.nnx, m.nny, jk, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            k3[a] = dt * u[a];
            y[a] = x[a] + k3[a];
        }
        near |= in & near_boundary<D>(m, y);
        in &= locate_uniform<D>(m, y, jk, ty);
        eval_q2_ijk<D, T>(U, m.nnx, m.nny, jk, ty, u);
        const double s6 = 1.0 / 6.0, s3 = 1.0 / 3.0;
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + k1[a] * s6 + k2[a] * s3 + k3[a] * s3 + (dt * u[a]) * s6;
    }
    near |= in & near_boundary<D>(m, xn);
    double tn[3];
    in &= locate_uniform<D>(m, xn, jk, tn);
    if (!in) return LOST;
    near |= face_dist<D>(tn) < NEAR_TOL;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        x[a] = xn[a];
        t[a] = tn[a];
    }
    return cell_of<D>(m, jk);
}

// Field interpolated linearly in time between u^n and u^{n+1} (Sec. 2.3):
// the two fields are evaluated at the point and combined with the weight
// theta = (time since t^n) / dt_u of the stage; th[c] holds theta at the
// step's start (c = 0), midpoint (1) and end (2).
struct StageTheta {
    double th[3];
    __device__ __forceinline__ void init(double since, double dt, double dt_u)
    {
        th[0] = since / dt_u;
        th[1] = (since + 0.5 * dt) / dt_u;
        th[2] = (since + dt) / dt_u;
    }
    __device__ __forceinline__ double operator()(int c) const { return c == 0 ? th[0] : (c == 1 ? th[1] : th[2]); }
};
template <int N> __device__ __forceinline__ void lerp_time(double *u0, const double *u1, double th)
{
#pragma unroll
    for (int a = 0; a < N; ++a) u0[a] = u0[a] + th * (u1[a] - u0[a]);
}

// Accumulate per-thread counters into the device statistics: wavefront sum,
// then one atomic per wavefront into the stripe of this workgroup.
__device__ __forceinline__ void flush_stats(unsigned long long *stats, int slot, int v, int *)
{
    const int w = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && w)
        atomicAdd(&stats[(blockIdx.x % STAT_STRIPES) * ST_COUNT + slot], (unsigned long long)w);
}

/*
 * Work item = tile of consecutive cells [c0, c1) of one problem; its
 * particles are contiguous in the store.  For every particle: advance +
 * locate, write the new location and reference location in place and the
 * key (new cell or LOST).  Stayers are counted per cell in LDS, arrivals with
 * global atomics on the destination cell.
 */
#ifndef PIC_ADVECT_MIN_WAVES
#define PIC_ADVECT_MIN_WAVES 0      // 0: compiler's choice; N: cap registers for N waves per SIMD
#endif
#if PIC_ADVECT_MIN_WAVES > 0
#define PIC_ADVECT_ATTR __attribute__((amdgpu_waves_per_eu(PIC_ADVECT_MIN_WAVES)))
#else
#define PIC_ADVECT_ATTR
#endif
template <int D, int S, typename T, int KIND, bool ODE = false, bool TI = false>
__global__ __launch_bounds__(BLOCK) PIC_ADVECT_ATTR void k_advect(const ProblemDev *__restrict__ probs,
                                                                  const WorkItem *__restrict__ work, int n_work)
{
    __shared__ int s_cnt[MAX_TILE];
    for (int wb = blockIdx.x; wb < xcd_span(n_work); wb += gridDim.x) {
        const int w = xcd_item(wb, n_work);
        if (w >= n_work) continue;
        const WorkItem wi = work[w];
        const ProblemDev &P = probs[wi.problem];
        const MeshDev &m = P.mesh;
        const StoreDev cur = P.store[P.cur];
        const int64_t cap = P.cap;
        const double dt = P.dt;
        const int c0 = wi.c0, nt = wi.c1 - wi.c0;
        const int p0 = cur.cs[c0], p1 = cur.cs[wi.c1];
        StageTheta th;
        if constexpr (TI) th.init(*P.tau, dt, P.dt_u);
        for (int k = threadIdx.x; k < nt; k += BLOCK) s_cnt[k] = 0;
        __syncthreads();
        int st_lost = 0, st_moved = 0, st_near = 0;
        LocStats ls = {0, 0, 0, 0, 0};
        for (int i = p0 + threadIdx.x; i < p1; i += BLOCK) {
            const int32_t K = cur.cell[i];
            double x[3], t[3];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                x[a] = cur.x[a * cap + i];
                t[a] = cur.xr[a * cap + i];
            }
            bool near = false;
            uint32_t key;
            double Pp[1 + D * D];
            if constexpr (ODE || TI) {
                using VT = typename NodeVec<D, T>::type;
                using VD = typename NodeVec<D, double>::type;
                const auto *U = reinterpret_cast<const VT *>(sizeof(T) == 4 ? P.u32 : P.u64);
                const auto *U1 = reinterpret_cast<const VT *>(sizeof(T) == 4 ? P.u1_32 : P.u1_64);
                auto ev = [&](int c, int32_t Kc, const double *tc, double *uc) {
                    eval_q2<D, T, KIND>(m, U, Kc, tc, uc);
                    if constexpr (TI) {
                        double u1[3];
                        eval_q2<D, T, KIND>(m, U1, Kc, tc, u1);
                        lerp_time<D>(uc, u1, th(c));
                    }
                };
                if constexpr (ODE) {
                    auto pin = (gptr<double>)cur.prop;
                    Pp[0] = pin[P.ode_dmg * cap + i];
#pragma unroll
                    for (int q = 0; q < D * D; ++q) Pp[1 + q] = pin[(P.ode_F + q) * cap + i];
                    const auto *U64 = reinterpret_cast<const VD *>(P.u64);
                    const auto *U164 = reinterpret_cast<const VD *>(P.u1_64);
                    auto gr = [&](int c, int32_t Kc, const double *tc, double G[3][3]) {
                        grad_phys<D, KIND>(m, U64, Kc, tc, G);
                        if constexpr (TI) {
                            double G1[3][3];
                            grad_phys<D, KIND>(m, U164, Kc, tc, G1);
#pragma unroll
                            for (int r = 0; r < D; ++r) lerp_time<D>(G[r], G1[r], th(c));
                        }
                    };
                    key = advect_one_e_ode<D, S, KIND>(m, ev, gr, dt, P.ode_alpha, P.ode_beta, x, t, Pp, K, near, ls);
                    if (key != LOST) {
                        auto po = (gptr_mut<double>)cur.prop;
                        po[P.ode_dmg * cap + i] = Pp[0];
#pragma unroll
                        for (int q = 0; q < D * D; ++q) po[(P.ode_F + q) * cap + i] = Pp[1 + q];
                    }
                } else {
                    key = advect_one_e<D, S, KIND>(m, ev, dt, x, t, K, near, ls);
                }
            } else if constexpr (KIND == MESH_UNIFORM) {
                using V = typename NodeVec<D, T>::type;
                auto U = (gptr<V>)(sizeof(T) == 4 ? P.u32 : P.u64);
                key = advect_one_uniform<D, S, T>(m, U, dt, x, t, (uint32_t)K, near);
            } else {
                const auto *U = reinterpret_cast<const typename NodeVec<D, T>::type *>(sizeof(T) == 4 ? P.u32 : P.u64);
                key = advect_one<D, S, T, KIND>(m, U, dt, x, t, K, near, ls);
            }
            if (key != LOST) {
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    cur.x[a * cap + i] = x[a];
                    cur.xr[a * cap + i] = t[a];
                }
            }
            P.scr.key[P.cur][i] = key;
            const bool stay = key == (uint32_t)K;
            if (stay) atomicAdd(&s_cnt[K - c0], 1);
            else if (key != LOST) atomicAdd(&P.scr.n_arrive[key], 1);
            st_lost += key == LOST;
            st_moved += (key != LOST) && !stay;
            st_near += near;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nt; k += BLOCK) P.scr.n_stay[c0 + k] = s_cnt[k];
        flush_stats(P.scr.stats, ST_PSTEPS, threadIdx.x == 0 ? p1 - p0 : 0, nullptr);
        flush_stats(P.scr.stats, ST_LOST, st_lost, nullptr);
        flush_stats(P.scr.stats, ST_MOVED, st_moved, nullptr);
        flush_stats(P.scr.stats, ST_NEAR, st_near, nullptr);
        if constexpr (KIND != MESH_UNIFORM) {
            flush_stats(P.scr.stats, ST_FIRST_TRY, ls.first_try, nullptr);
            flush_stats(P.scr.stats, ST_FALLBACK, ls.fallback, nullptr);
            flush_stats(P.scr.stats, ST_NEWTON_FAIL, ls.newton_fail, nullptr);
            flush_stats(P.scr.stats, ST_SEARCHED, ls.searched, nullptr);
            flush_stats(P.scr.stats, ST_SEARCHES, ls.searches, nullptr);
        }
        __syncthreads();
    }
}

// Octree meshes: the 27 node values of every leaf of the tile are copied to
// LDS once (leaves of a tile are consecutive, so their node lists are one
// contiguous run of the cell -> node map); particles evaluate stage points in
// the tile's leaves from LDS and elsewhere from the global field, with the
// same arithmetic (identical rounding).
constexpr int OCT_TILE = 64;
#ifndef PIC_OCT_WAVES
#define PIC_OCT_WAVES 3     // single precision, Euler/RK2: cap registers for this many waves per SIMD
#endif
template <int S, typename T>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && S <= 2 ? PIC_OCT_WAVES : 1))) void
k_advect_oct(const ProblemDev *__restrict__ probs,
                                                      const WorkItem *__restrict__ work, int n_work)
{
    using V = typename NodeVec<3, T>::type;
    __shared__ V s_nodes[OCT_TILE * 27];
    __shared__ int s_cnt[OCT_TILE];
    for (int wb = blockIdx.x; wb < xcd_span(n_work); wb += gridDim.x) {
        const int w = xcd_item(wb, n_work);
        if (w >= n_work) continue;
        const WorkItem wi = work[w];
        const ProblemDev &P = probs[wi.problem];
        const MeshDev &m = P.mesh;
        const StoreDev cur = P.store[P.cur];
        const int64_t cap = P.cap;
        const double dt = P.dt;
        const int c0 = wi.c0, nt = wi.c1 - wi.c0;     // nt <= OCT_TILE (work lists of octree meshes)
        const int p0 = cur.cs[c0], p1 = cur.cs[wi.c1];
        const V *U = reinterpret_cast<const V *>(sizeof(T) == 4 ? P.u32 : P.u64);
        const int32_t *cn = m.cell_nodes + (int64_t)c0 * 27;
        for (int q = threadIdx.x; q < nt * 27; q += BLOCK) s_nodes[q] = U[cn[q]];
        for (int k = threadIdx.x; k < nt; k += BLOCK) s_cnt[k] = 0;
        __syncthreads();
        auto ev = [&](int, int32_t Kc, const double *tc, double *uc) {
            if ((unsigned)(Kc - c0) < (unsigned)nt)
                eval_q2_local<3, T>(s_nodes + (Kc - c0) * 27, tc, uc);
            else
                eval_q2<3, T, MESH_OCTREE>(m, U, Kc, tc, uc);
        };
        int st_lost = 0, st_moved = 0, st_near = 0;
        LocStats ls = {0, 0, 0, 0, 0};
        for (int i = p0 + threadIdx.x; i < p1; i += BLOCK) {
            const int32_t K = cur.cell[i];
            double x[3], t[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                x[a] = cur.x[a * cap + i];
                t[a] = cur.xr[a * cap + i];
            }
            bool near = false;
            const uint32_t key = advect_one_e<3, S, MESH_OCTREE>(m, ev, dt, x, t, K, near, ls);
            if (key != LOST) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    cur.x[a * cap + i] = x[a];
                    cur.xr[a * cap + i] = t[a];
                }
            }
            P.scr.key[P.cur][i] = key;
            const bool stay = key == (uint32_t)K;
            if (stay) atomicAdd(&s_cnt[K - c0], 1);
            else if (key != LOST) atomicAdd(&P.scr.n_arrive[key], 1);
            st_lost += key == LOST;
            st_moved += (key != LOST) && !stay;
            st_near += near;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nt; k += BLOCK) P.scr.n_stay[c0 + k] = s_cnt[k];
        flush_stats(P.scr.stats, ST_PSTEPS, threadIdx.x == 0 ? p1 - p0 : 0, nullptr);
        flush_stats(P.scr.stats, ST_LOST, st_lost, nullptr);
        flush_stats(P.scr.stats, ST_MOVED, st_moved, nullptr);
        flush_stats(P.scr.stats, ST_NEAR, st_near, nullptr);
        flush_stats(P.scr.stats, ST_FIRST_TRY, ls.first_try, nullptr);
        flush_stats(P.scr.stats, ST_FALLBACK, ls.fallback, nullptr);
        flush_stats(P.scr.stats, ST_NEWTON_FAIL, ls.newton_fail, nullptr);
        flush_stats(P.scr.stats, ST_SEARCHED, ls.searched, nullptr);
        flush_stats(P.scr.stats, ST_SEARCHES, ls.searches, nullptr);
        __syncthreads();
    }
}

// ===========================================================================
// advect + locate on uniform meshes with the field of a block of cells staged
// in LDS
// ===========================================================================
// Block of BX x BY x BZ cells; the LDS window holds the Q2 nodes of the
// block's cells plus a one-cell halo: (2(BX+2)+1) x (2(BY+2)+1) x (2(BZ+2)+1)
// nodes, node (wx, wy, wz) = global node (2(i0-1)+wx, 2(j0-1)+wy, 2(k0-1)+wz).
// Neighbouring cells share their face nodes, so the window holds about 8
// nodes per cell instead of the 27 a per-cell layout would need.
template <int D, int BX, int BY, int BZ> struct BlockShape {
    static constexpr int CX = BX + 2;
    static constexpr int CY = BY + 2;
    static constexpr int CZ = D == 3 ? BZ + 2 : 1;
    static constexpr int WX = 2 * CX + 1;
    static constexpr int WY = 2 * CY + 1;
    static constexpr int WZ = D == 3 ? 2 * CZ + 1 : 1;
    static constexpr int NODES = WX * WY * WZ;
    static constexpr int CELLS = BX * BY * (D == 3 ? BZ : 1);
    static constexpr int ROWS = BY * (D == 3 ? BZ : 1);
};

// Field at the reference point t of cell ijk: from the LDS window when the
// cell lies in the block or its halo, else from the global node array (same
// arithmetic, same rounding).
template <int D, typename T, int BX, int BY, int BZ>
__device__ __forceinline__ void eval_blk(const MeshDev &m, gptr<typename NodeVec<D, T>::type> Ug,
                                         const typename NodeVec<D, T>::type *W, const int *b0, const int ijk[3],
                                         const double *t, double *u)
{
    using Sh = BlockShape<D, BX, BY, BZ>;
    const int di = ijk[0] - b0[0] + 1, dj = ijk[1] - b0[1] + 1, dk = ijk[2] - b0[2] + 1;
    bool in = ((unsigned)di < (unsigned)Sh::CX) & ((unsigned)dj < (unsigned)Sh::CY);
    if constexpr (D == 3) in &= (unsigned)dk < (unsigned)Sh::CZ;
    if (in) {
        const int base = 2 * di + Sh::WX * (2 * dj + (D == 3 ? Sh::WY * 2 * dk : 0));
        eval_q2_at<D, T>(W, base, (int)Sh::WX, (int)(Sh::WX * Sh::WY), t, u);
    } else {
        eval_q2_ijk<D, T>(Ug, m.nnx, m.nny, ijk, t, u);
    }
}

// x-Horner form of the single-precision 3D evaluation.  Along x, the Q2 row
// through nodes u0, u1, u2 (reference x = 0, 1/2, 1) is the quadratic
// a + t (b + t c) with a = u0, b = 4 u1 - 3 u0 - u2, c = 2 (u0 - 2 u1 + u2):
// two FMAs per row and component instead of three plus the x basis.  The
// y and z directions keep the Lagrange sum.  The coefficients are computed by
// these functions only, whether staged in LDS or formed from the global node
// array, so both give the same rounding.
__device__ __forceinline__ float xh_b(float u0, float u1, float u2) { return __builtin_fmaf(4.f, u1, -__builtin_fmaf(3.f, u0, u2)); }
__device__ __forceinline__ float xh_c(float u0, float u1, float u2) { return 2.f * __builtin_fmaf(-2.f, u1, u0 + u2); }
__device__ __forceinline__ float xh_row(float a, float b, float c, float t)
{
    return __builtin_fmaf(__builtin_fmaf(c, t, b), t, a);
}
// Coefficients of one cell row (three float4: a, b, c; the fourth lanes unused).
__device__ __forceinline__ void xh_coef(const float4 &u0, const float4 &u1, const float4 &u2, float4 &a, float4 &b,
                                        float4 &c)
{
    a = u0;
    b = make_float4(xh_b(u0.x, u1.x, u2.x), xh_b(u0.y, u1.y, u2.y), xh_b(u0.z, u1.z, u2.z), 0.f);
    c = make_float4(xh_c(u0.x, u1.x, u2.x), xh_c(u0.y, u1.y, u2.y), xh_c(u0.z, u1.z, u2.z), 0.f);
}
// Sum over the nine rows of a cell given row(b, c3, A, B, C) loading the
// coefficients of row (b, c3); the rows of a plane are all loaded before use.
template <class Row> __device__ __forceinline__ void eval_xh(Row &&row, const double *tr, double *u)
{
    const float t0 = (float)tr[0];
    float lb[3], lc[3];
    lag3((float)tr[1], lb);
    lag3((float)tr[2], lc);
    float a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) {
        float4 A[3], B[3], C[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) row(b, c3, A[b], B[b], C[b]);
        __builtin_amdgcn_sched_barrier(0);
        float r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            r0 = __builtin_fmaf(lb[b], xh_row(A[b].x, B[b].x, C[b].x, t0), r0);
            r1 = __builtin_fmaf(lb[b], xh_row(A[b].y, B[b].y, C[b].y, t0), r1);
            r2 = __builtin_fmaf(lb[b], xh_row(A[b].z, B[b].z, C[b].z, t0), r2);
        }
        a0 = __builtin_fmaf(lc[c3], r0, a0);
        a1 = __builtin_fmaf(lc[c3], r1, a1);
        a2 = __builtin_fmaf(lc[c3], r2, a2);
    }
    u[0] = (double)a0;
    u[1] = (double)a1;
    u[2] = (double)a2;
}
// The x-Horner window of a block: cell rows of the block's cells plus a
// one-cell halo, CX cells along x by WY x WZ node rows, three float4 each.
template <int BX, int BY, int BZ> struct XhShape {
    using Sh = BlockShape<3, BX, BY, BZ>;
    static constexpr int ROWS = Sh::CX * Sh::WY * Sh::WZ;
    static constexpr int VEC = 3 * ROWS;
};
// Field at (ijk, t) from the x-Horner window when the cell lies in the block
// or its halo, else from coefficients formed from the global node array.
template <int BX, int BY, int BZ>
__device__ __forceinline__ void eval_blk_xh(const MeshDev &m, gptr<float4> Ug, const float4 *W, const int *b0,
                                            const int ijk[3], const double *t, double *u)
{
    using Sh = BlockShape<3, BX, BY, BZ>;
    const int di = ijk[0] - b0[0] + 1, dj = ijk[1] - b0[1] + 1, dk = ijk[2] - b0[2] + 1;
    const bool in = ((unsigned)di < (unsigned)Sh::CX) & ((unsigned)dj < (unsigned)Sh::CY) & ((unsigned)dk < (unsigned)Sh::CZ);
    if (in) {
        const int base = 3 * (di + Sh::CX * (2 * dj + Sh::WY * 2 * dk));
        eval_xh([&](int b, int c3, float4 &A, float4 &B, float4 &C) {
            const int q = base + 3 * Sh::CX * (b + Sh::WY * c3);
            A = W[q];
            B = W[q + 1];
            C = W[q + 2];
        }, t, u);
    } else {
        const int64_t sy = m.nnx, sz = (int64_t)m.nnx * m.nny;
        const int64_t base = 2 * ijk[0] + sy * (2 * ijk[1]) + sz * (2 * ijk[2]);
        eval_xh([&](int b, int c3, float4 &A, float4 &B, float4 &C) {
            const int64_t r = base + sy * b + sz * c3;
            xh_coef(Ug[r], Ug[r + 1], Ug[r + 2], A, B, C);
        }, t, u);
    }
}

// One step of one particle on a uniform mesh; ev(c, ijk, t, u) evaluates the
// field in cell ijk at stage time code c (as advect_one_e).
template <int D, int S, class Eval>
__device__ __forceinline__ uint32_t advect_one_blk(const MeshDev &m, Eval &&ev, double dt, double *x, double *t,
                                                   const int ijk[3], bool &near)
{
    int jk[3];
    double u[3], y[3], ty[3], xn[3];
    ev(0, ijk, t, u);
    bool in = true;
    if constexpr (S == 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + dt * u[a];
    } else if constexpr (S == 2) {
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = x[a] + 0.5 * (dt * u[a]);
        in &= locate_stage<D>(m, y, jk, ty, near, in);
        ev(1, jk, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + dt * u[a];
    } else {
        // xn accumulates x + k1/6 + k2/3 + k3/3 + k4/6 left to right as each
        // stage slope becomes known, so no slope is kept beyond its stage
        const double s6 = 1.0 / 6.0, s3 = 1.0 / 3.0;
        double k[3];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            k[a] = dt * u[a];
            xn[a] = x[a] + k[a] * s6;
            y[a] = x[a] + 0.5 * k[a];
        }
        in &= locate_stage<D>(m, y, jk, ty, near, in);
        ev(1, jk, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            k[a] = dt * u[a];
            xn[a] = xn[a] + k[a] * s3;
            y[a] = x[a] + 0.5 * k[a];
        }
        in &= locate_stage<D>(m, y, jk, ty, near, in);
        ev(1, jk, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            k[a] = dt * u[a];
            xn[a] = xn[a] + k[a] * s3;
            y[a] = x[a] + k[a];
        }
        in &= locate_stage<D>(m, y, jk, ty, near, in);
        ev(2, jk, ty, u);
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = xn[a] + (dt * u[a]) * s6;
    }
    near |= in & near_boundary<D>(m, xn);
    double tn[3];
    in &= locate_uniform<D>(m, xn, jk, tn);
    if (!in) return LOST;
    near |= face_dist<D>(tn) < NEAR_TOL;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        x[a] = xn[a];
        t[a] = tn[a];
    }
    return cell_of<D>(m, jk);
}

/*
 * Work item = block of cells of a uniform mesh.  The workgroup stages a window
 * of the field over the block's cells plus a one-cell halo in LDS once (the
 * x-Horner rows or the Q2 node lattice), then advances every particle of the
 * block's cells; stage points in the halo read LDS, the rare ones farther away
 * read global memory.  A particle's cell is the cell of its block row whose
 * range holds its slot, and its reference coordinates the closed form of its
 * position in that cell: neither is read, and neither is stored (the
 * re-sort's gather writes both when it forms the final store).
 *
 * FUSED = false: the particles are those of the current buffer; the new
 * location and the key are written in place.
 * FUSED = true: the particles are the destination slots p of the re-sort in
 * progress (cells of the other buffer, whose cell_start the scan produced);
 * slot p takes particle src[p] of the current buffer, advances it by the next
 * step and writes its location, id, properties and new key to the other
 * buffer.  A fused step is thus "finish the previous step's permutation and
 * compute the next step's keys" in one pass over the particle state.
 */
// Physical gradient of the field at the reference point t of cell ijk, from
// the LDS window or the global node array (as eval_blk).
template <int D, typename T, int BX, int BY, int BZ>
__device__ __forceinline__ void grad_blk(const MeshDev &m, gptr<typename NodeVec<D, T>::type> Ug,
                                         const typename NodeVec<D, T>::type *W, const int *b0, const int ijk[3],
                                         const double *t, double G[3][3])
{
    using Sh = BlockShape<D, BX, BY, BZ>;
    const int di = ijk[0] - b0[0] + 1, dj = ijk[1] - b0[1] + 1, dk = ijk[2] - b0[2] + 1;
    bool in = ((unsigned)di < (unsigned)Sh::CX) & ((unsigned)dj < (unsigned)Sh::CY);
    if constexpr (D == 3) in &= (unsigned)dk < (unsigned)Sh::CZ;
    double Gr[3][3];
    if (in) {
        const int base = 2 * di + Sh::WX * (2 * dj + (D == 3 ? Sh::WY * 2 * dk : 0));
        grad_q2_at<D, T>(W, base, (int)Sh::WX, (int)(Sh::WX * Sh::WY), t, Gr);
    } else {
        const int64_t sz = (int64_t)m.nnx * m.nny;
        const int64_t base = 2 * ijk[0] + (int64_t)m.nnx * (2 * ijk[1]) + (D == 3 ? sz * (2 * ijk[2]) : 0);
        grad_q2_at<D, T>(Ug, base, (int64_t)m.nnx, sz, t, Gr);
    }
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
        for (int j = 0; j < D; ++j) G[c][j] = Gr[c][j] * m.inv_h[j];
}

// advect_one_blk with the property equations (Pp = [d, F_00, F_01, ...]):
// positions take exactly the operations of advect_one_blk; every stage also
// evaluates grad u at its point and the property rates at its property values.
template <int D, int S, class Eval, class Grad>
__device__ __forceinline__ uint32_t advect_one_blk_ode(const MeshDev &m, Eval &&ev, Grad &&gr, double dt,
                                                       double alpha, double beta, double *x, double *t, double *Pp,
                                                       const int ijk0[3], bool &near)
{
    constexpr int NP = 1 + D * D;
    constexpr int NS = S == 1 ? 1 : (S == 2 ? 2 : 4);
    const double s6 = 1.0 / 6.0, s3 = 1.0 / 3.0;
    int jk[3] = {ijk0[0], ijk0[1], ijk0[2]};
    double u[3], G[3][3], y[3], ty[3], xn[3], k[3], Ps[NP], kP[4][NP];
    bool in = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (s == 0) {
            ev(0, jk, t, u);
            gr(0, jk, t, G);
#pragma unroll
            for (int q = 0; q < NP; ++q) Ps[q] = Pp[q];
        } else {
            const double c = (S == 4 && s == 3) ? 1.0 : 0.5;
            in &= locate_stage<D>(m, y, jk, ty, near, in);
            ev(S == 4 && s == 3 ? 2 : 1, jk, ty, u);
            gr(S == 4 && s == 3 ? 2 : 1, jk, ty, G);
#pragma unroll
            for (int q = 0; q < NP; ++q) Ps[q] = Pp[q] + c * kP[s - 1][q];
        }
        double dd, dF[D * D];
        prop_rates<D>(G, alpha, beta, Ps[0], Ps + 1, dd, dF);
        kP[s][0] = dt * dd;
#pragma unroll
        for (int q = 0; q < D * D; ++q) kP[s][1 + q] = dt * dF[q];
        // positions: the operations of advect_one_blk
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if constexpr (S == 1) {
                xn[a] = x[a] + dt * u[a];
            } else if constexpr (S == 2) {
                if (s == 0) y[a] = x[a] + 0.5 * (dt * u[a]);
                else xn[a] = x[a] + dt * u[a];
            } else {
                if (s < 3) {
                    k[a] = dt * u[a];
                    xn[a] = s == 0 ? x[a] + k[a] * s6 : xn[a] + k[a] * s3;
                    y[a] = s < 2 ? x[a] + 0.5 * k[a] : x[a] + k[a];
                } else {
                    xn[a] = xn[a] + (dt * u[a]) * s6;
                }
            }
        }
    }
    double Pn[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        if constexpr (S == 1) Pn[q] = Pp[q] + kP[0][q];
        else if constexpr (S == 2) Pn[q] = Pp[q] + kP[1][q];
        else Pn[q] = Pp[q] + kP[0][q] * s6 + kP[1][q] * s3 + kP[2][q] * s3 + kP[3][q] * s6;
    }
    near |= in & near_boundary<D>(m, xn);
    double tn[3];
    in &= locate_uniform<D>(m, xn, jk, tn);
    if (!in) return LOST;
    near |= face_dist<D>(tn) < NEAR_TOL;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        x[a] = xn[a];
        t[a] = tn[a];
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) Pp[q] = Pn[q];
    return cell_of<D>(m, jk);
}

#ifndef PIC_ADV_THREADS
#define PIC_ADV_THREADS 256         // threads per workgroup of the block kernels
#endif
#ifndef PIC_BLK_MIN_WAVES
#define PIC_BLK_MIN_WAVES 3         // 3D single-precision kernels: cap registers for this many waves per SIMD
#endif
// Register cap of the block kernels, as waves per SIMD (1 = compiler's choice).
// The 3D single-precision kernels run at three waves with no spills; the
// double-precision ones would spill under that cap and get two.
template <int D, typename T> struct BlkWaves {
    static constexpr int value = D == 2 ? 1 : (sizeof(T) == 4 ? (PIC_BLK_MIN_WAVES > 0 ? PIC_BLK_MIN_WAVES : 1) : 2);
};
#ifndef PIC_XH
#define PIC_XH 1                    // 3D single-precision block kernels: x-Horner window (0: node window)
#endif
#ifndef PIC_BLK_PREFETCH
#define PIC_BLK_PREFETCH 2          // 1: load the next particle's state while advancing this one; 2: also its gather source one step earlier
#endif
constexpr int ADV_BLOCK = PIC_ADV_THREADS;
#ifndef PIC_ODE_WAVES
#define PIC_ODE_WAVES 2             // single-precision kernels with the property equations: registers for two waves per SIMD
#endif
#ifndef PIC_BLK_EARLY
#define PIC_BLK_EARLY 1             // fused kernels: read id and the first properties before the step (0: after it)
#endif
constexpr int PF_PROPS = 4;         // single-precision properties carried in registers by the fused kernels
template <int D, int S, typename T, int BX, int BY, int BZ, bool FUSED, bool ODE = false, bool TI = false>
__global__ __launch_bounds__(ADV_BLOCK) __attribute__((amdgpu_waves_per_eu(ODE ? (sizeof(T) == 4 ? PIC_ODE_WAVES : 1) : TI ? 1 : BlkWaves<D, T>::value))) void k_advect_blk(const ProblemDev *__restrict__ probs,
                                                                      const BlockItem *__restrict__ work, int n_work)
{
    using Sh = BlockShape<D, BX, BY, BZ>;
    using V = typename NodeVec<D, T>::type;
    // single-precision 3D evaluation of a steady field reads the x-Horner
    // window; the other forms read the node window
    constexpr bool XH = PIC_XH && D == 3 && sizeof(T) == 4 && !ODE && !TI;
    using Xh = XhShape<BX, BY, D == 3 ? BZ : 1>;
    __shared__ V s_w[XH ? 1 : Sh::NODES * (TI ? 2 : 1)];   // u^n window, then the u^{n+1} window
    __shared__ float4 s_xh[XH ? Xh::VEC : 1];
    __shared__ int s_cnt[Sh::CELLS];
    static_assert(Sh::ROWS <= 64, "one wave scans the rows of a block");
    __shared__ int s_pre_w[ADV_BLOCK / 64][Sh::ROWS + 1];
    __shared__ int s_beg_w[ADV_BLOCK / 64][Sh::ROWS];
    __shared__ int s_cs_w[ADV_BLOCK / 64][Sh::ROWS][BX + 1];
    int *s_pre = s_pre_w[threadIdx.x >> 6];      // each wave keeps its own copy of the row runs
    int *s_beg = s_beg_w[threadIdx.x >> 6];
    int(*s_cs)[BX + 1] = s_cs_w[threadIdx.x >> 6];   // and of the cell starts within each row
    for (int wb = blockIdx.x; wb < xcd_span(n_work); wb += gridDim.x) {
        const int w = xcd_item(wb, n_work);
        if (w >= n_work) continue;
        const BlockItem bi = work[w];
        if (bi.problem < 0) continue;            // empty slot of a padded list
        const ProblemDev &P = probs[bi.problem];
        const MeshDev &m = P.mesh;
        const StoreDev cur = P.store[P.cur];
        const StoreDev out = P.store[FUSED ? 1 - P.cur : P.cur];
        uint32_t *key_out = P.scr.key[FUSED ? 1 - P.cur : P.cur];
        const int64_t cap = P.cap;
        const double dt = P.dt;
        auto Ug = (gptr<V>)(sizeof(T) == 4 ? P.u32 : P.u64);
        auto Ug1 = (gptr<V>)(sizeof(T) == 4 ? P.u1_32 : P.u1_64);
        const int b0[3] = {bi.i0, bi.j0, D == 3 ? bi.k0 : 0};
        // a fused launch advances the step after the one whose re-sort it
        // completes: that step starts dt later than the time counter says
        StageTheta th;
        if constexpr (TI) th.init(FUSED ? *P.tau + dt : *P.tau, dt, P.dt_u);
        auto ev = [&](int c, const int *ijk, const double *tc, double *uc) {
            if constexpr (XH)
                eval_blk_xh<BX, BY, BZ>(m, (gptr<float4>)P.u32, s_xh, b0, ijk, tc, uc);
            else
                eval_blk<D, T, BX, BY, BZ>(m, Ug, s_w, b0, ijk, tc, uc);
            if constexpr (TI) {
                double u1[3];
                eval_blk<D, T, BX, BY, BZ>(m, Ug1, s_w + Sh::NODES, b0, ijk, tc, u1);
                lerp_time<D>(uc, u1, th(c));
            }
        };
        auto gr = [&](int c, const int *ijk, const double *tc, double G[3][3]) {
            grad_blk<D, T, BX, BY, BZ>(m, Ug, s_w, b0, ijk, tc, G);
            if constexpr (TI) {
                double G1[3][3];
                grad_blk<D, T, BX, BY, BZ>(m, Ug1, s_w + Sh::NODES, b0, ijk, tc, G1);
#pragma unroll
                for (int r = 0; r < D; ++r) lerp_time<D>(G[r], G1[r], th(c));
            }
        };
        const int nx = min(BX, m.n[0] - bi.i0), ny = min(BY, m.n[1] - bi.j0);
        const int nz = D == 3 ? min(BZ, m.n[2] - bi.k0) : 1;
        {
            // particle runs of the block's rows (in the buffer being written)
            // and their prefix, computed by every wave for itself so that the
            // first particles can be fetched before the window is complete
            const int r = threadIdx.x & 63;
            int len = 0, beg = 0;
            if (r < Sh::ROWS) {
                const int rj = r % BY, rk = r / BY;
                if (rj < ny && rk < nz) {
                    const int K = bi.i0 + m.n[0] * ((bi.j0 + rj) + m.n[1] * (D == 3 ? bi.k0 + rk : 0));
                    beg = out.cs[K];
                    len = out.cs[K + nx] - beg;
                    // starts of the row's cells; columns beyond the mesh never match
#pragma unroll
                    for (int c = 1; c < BX; ++c) s_cs[r][c] = c < nx ? out.cs[K + c] : 0x7fffffff;
                }
                s_beg[r] = beg;
            }
            int inc = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(inc, o, 64);
                if (r >= o) inc += v;
            }
            if (r < Sh::ROWS) s_pre[r + 1] = inc;
            if (r == 0) s_pre[0] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int total = s_pre[Sh::ROWS];
        int st_lost = 0, st_moved = 0, st_near = 0;
        // particle f of the block -> its row and position in the buffer written
        auto locate_f = [&](int f, int &r) {
            r = 0;
#pragma unroll
            for (int step = Sh::ROWS / 2; step >= 1; step >>= 1)
                if (r + step < Sh::ROWS && s_pre[r + step] <= f) r += step;
            return s_beg[r] + (f - s_pre[r]);
        };
        // The cell of the particle at position p of row r is the row's cell
        // whose range holds p: the particle's current cell (in a fused step,
        // the key that placed it there), so neither key nor cell is read.
        auto column_of = [&](int r, int p) {
            int c = 0;
#pragma unroll
            for (int q = 1; q < BX; ++q) c += p >= s_cs[r][q];
            return c;
        };
        // one-deep software prefetch of the next particle's state
        int rn = 0, pn = 0, sn = 0, cn = 0;
        double xn_[3] = {0, 0, 0};
        auto fetch = [&](int f) {
            pn = locate_f(f, rn);
            sn = FUSED ? P.scr.src[pn] : pn;
            cn = column_of(rn, pn);
#pragma unroll
            for (int a = 0; a < D; ++a) xn_[a] = cur.x[a * cap + sn];
        };
        // two-deep variant: the gather source of particle f + 2 BLOCK is loaded
        // one iteration ahead of its state
        int pA = 0, rA = 0, sA = 0;
        auto stage_a = [&](int f) {
            pA = locate_f(f, rA);
            sA = FUSED ? P.scr.src[pA] : pA;
        };
        auto stage_b = [&]() {
            pn = pA;
            rn = rA;
            sn = sA;
            cn = column_of(rn, pn);
#pragma unroll
            for (int a = 0; a < D; ++a) xn_[a] = cur.x[a * cap + sn];
        };
        if (PIC_BLK_PREFETCH == 2) {
            if ((int)threadIdx.x < total) {
                stage_a(threadIdx.x);
                stage_b();
            }
            if ((int)threadIdx.x + ADV_BLOCK < total) stage_a(threadIdx.x + ADV_BLOCK);
        } else if (PIC_BLK_PREFETCH && (int)threadIdx.x < total) {
            fetch(threadIdx.x);
        }
        // stage the window (its loads overlap the first fetch); nodes beyond
        // the mesh are never read (stage points are clamped to mesh cells)
        // and are left unset.  Every thread requests all its nodes before it
        // stores the first one to LDS, so that the loads are in flight
        // together (entries beyond the mesh load node 0 and are dropped).
        if constexpr (XH) {
            // x-Horner window: cell row q = (cell cx of the row, node row wy,
            // node plane wz) from the three nodes 2 (i0 - 1 + cx) + {0, 1, 2}
            constexpr int NQ = (Xh::ROWS + ADV_BLOCK - 1) / ADV_BLOCK;
            const int nnx = m.nnx, nny = m.nny, nnz = m.nnz;
            float4 v0[NQ], v1[NQ], v2[NQ];
            uint32_t ok = 0;
            int tq = threadIdx.x;
            asm volatile("" : "+v"(tq));
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = tq + u * ADV_BLOCK;
                const int cx = q % Sh::CX, wy = (q / Sh::CX) % Sh::WY, wz = q / (Sh::CX * Sh::WY);
                const int gi = 2 * (bi.i0 - 1 + cx), gj = 2 * (bi.j0 - 1) + wy, gk = 2 * (bi.k0 - 1) + wz;
                const bool in = q < Xh::ROWS && gi >= 0 && gi + 2 < nnx && gj >= 0 && gj < nny && gk >= 0 && gk < nnz;
                const int64_t g = in ? gi + (int64_t)nnx * (gj + (int64_t)nny * gk) : 0;
                ok |= (uint32_t)in << u;
                const gptr<float4> U32 = (gptr<float4>)P.u32;
                v0[u] = U32[g];
                v1[u] = U32[in ? g + 1 : 0];
                v2[u] = U32[in ? g + 2 : 0];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = tq + u * ADV_BLOCK;
                if ((ok >> u) & 1u) {
                    float4 A, B, C;
                    xh_coef(v0[u], v1[u], v2[u], A, B, C);
                    s_xh[3 * q] = A;
                    s_xh[3 * q + 1] = B;
                    s_xh[3 * q + 2] = C;
                }
            }
        } else {
            constexpr int NQ = (Sh::NODES + ADV_BLOCK - 1) / ADV_BLOCK;
            const int nnx = m.nnx, nny = m.nny, nnz = D == 3 ? m.nnz : 1;
            using E = decltype(V{}.x);
            E a0[NQ], a1[NQ], a2[NQ], b0_[TI ? NQ : 1], b1_[TI ? NQ : 1], b2_[TI ? NQ : 1];
            uint32_t ok = 0;
            // (the index arithmetic stays inside the work-item loop: hoisted
            // out of it, its NQ results would be spilled)
            int tq = threadIdx.x;
            asm volatile("" : "+v"(tq));
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = tq + u * ADV_BLOCK;
                const int wx = q % Sh::WX, wy = (q / Sh::WX) % Sh::WY, wz = q / (Sh::WX * Sh::WY);
                const int gi = 2 * (bi.i0 - 1) + wx, gj = 2 * (bi.j0 - 1) + wy, gk = D == 3 ? 2 * (bi.k0 - 1) + wz : 0;
                const bool in = q < Sh::NODES && gi >= 0 && gi < nnx && gj >= 0 && gj < nny && gk >= 0 && gk < nnz;
                const int64_t g = in ? gi + (int64_t)nnx * (gj + (int64_t)nny * gk) : 0;
                ok |= (uint32_t)in << u;
                const V v = Ug[g];
                a0[u] = v.x;
                a1[u] = v.y;
                a2[u] = nv_z(v);
                if constexpr (TI) {
                    const V v1 = Ug1[g];
                    b0_[u] = v1.x;
                    b1_[u] = v1.y;
                    b2_[u] = nv_z(v1);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int q = tq + u * ADV_BLOCK;
                if ((ok >> u) & 1u) {
                    s_w[q] = node_of<V>(a0[u], a1[u], a2[u]);
                    if constexpr (TI) s_w[Sh::NODES + q] = node_of<V>(b0_[u], b1_[u], b2_[u]);
                }
            }
        }
        for (int q = threadIdx.x; q < Sh::CELLS; q += ADV_BLOCK) s_cnt[q] = 0;
        __syncthreads();
        for (int f = threadIdx.x; f < total; f += ADV_BLOCK) {
            if (!PIC_BLK_PREFETCH) fetch(f);
            const int r = rn, p = pn, sidx = sn, col = cn;
            // the particle's cell, and its reference coordinates there by the
            // closed form that located it (on a uniform mesh they are a function
            // of the position and the cell, so they are not read)
            const int ijk[3] = {bi.i0 + col, bi.j0 + r % BY, D == 3 ? bi.k0 + r / BY : 0};
            const int32_t K = (int32_t)cell_of<D>(m, ijk);
            double x[3], t[3];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                x[a] = xn_[a];
                t[a] = (x[a] - fma((double)ijk[a], m.h[a], m.lo[a])) * m.inv_h[a];
            }
            if (PIC_BLK_PREFETCH == 2) {
                if (f + ADV_BLOCK < total) stage_b();
                if (f + 2 * ADV_BLOCK < total) stage_a(f + 2 * ADV_BLOCK);
            } else if (PIC_BLK_PREFETCH && f + ADV_BLOCK < total) {
                fetch(f + ADV_BLOCK);
            }
            // The id and the first single-precision properties of the particle
            // are read now: their latency then hides behind the step, whereas a
            // load issued after the step's stores would wait for those stores
            // too (one memory counter serves loads and stores).  Loads past the
            // last property re-read the first one, so that no load sits behind
            // a branch.
            uint32_t idv = 0;
            uint32_t pv[PF_PROPS];
            const int npf = FUSED && PIC_BLK_EARLY && !P.prop_f64 ? min(P.n_prop, PF_PROPS) : 0;
            auto read_early = [&]() {
                if constexpr (FUSED && PIC_BLK_EARLY) {
                    idv = cur.id[sidx];
                    if (npf > 0) {
#pragma unroll
                        for (int j = 0; j < PF_PROPS; ++j)
                            pv[j] = ((const uint32_t PIC_G *)cur.prop)[(j < npf ? j : 0) * cap + sidx];
                    }
                }
            };
            read_early();
            bool near = false;
            uint32_t key;
            double Pp[1 + D * D];
            if constexpr (ODE) {
                auto pin = (gptr<double>)cur.prop;
                Pp[0] = pin[P.ode_dmg * cap + sidx];
#pragma unroll
                for (int q = 0; q < D * D; ++q) Pp[1 + q] = pin[(P.ode_F + q) * cap + sidx];
                key = advect_one_blk_ode<D, S>(m, ev, gr, dt, P.ode_alpha, P.ode_beta, x, t, Pp, ijk, near);
            } else {
                key = advect_one_blk<D, S>(m, ev, dt, x, t, ijk, near);
            }
            // The new position and key are stored; the reference coordinates
            // and the cell array are not: until the re-sort's gather writes
            // them (the cell from the key, the reference coordinates by the
            // closed form), no kernel of the step sequence reads either.
            if (key != LOST || FUSED) {
#pragma unroll
                for (int a = 0; a < D; ++a) out.x[a * cap + p] = x[a];
            }
            if constexpr (FUSED) {
                if constexpr (PIC_BLK_EARLY) {
                    out.id[p] = idv;
#pragma unroll
                    for (int j = 0; j < PF_PROPS; ++j)
                        if (j < npf) ((uint32_t PIC_G *)out.prop)[j * cap + p] = pv[j];
                } else {
                    out.id[p] = cur.id[sidx];
                }
                // the rest one by one (the integrated properties are written below)
                if (P.prop_f64) {
                    for (int j = npf; j < P.n_prop; ++j) {
                        if constexpr (ODE)
                            if (j == P.ode_dmg || (unsigned)(j - P.ode_F) < (unsigned)(D * D)) continue;
                        ((double *)out.prop)[j * cap + p] = ((const double *)cur.prop)[j * cap + sidx];
                    }
                } else {
                    for (int j = npf; j < P.n_prop; ++j)
                        ((float *)out.prop)[j * cap + p] = ((const float *)cur.prop)[j * cap + sidx];
                }
            }
            if constexpr (ODE) {
                // the integrated properties (double precision; in place when not fused)
                if (key != LOST || FUSED) {
                    auto po = (gptr_mut<double>)out.prop;
                    po[P.ode_dmg * cap + p] = Pp[0];
#pragma unroll
                    for (int q = 0; q < D * D; ++q) po[(P.ode_F + q) * cap + p] = Pp[1 + q];
                }
            }
            key_out[p] = key;
            const bool stay = key == (uint32_t)K;
            if (stay) {
                atomicAdd(&s_cnt[col + BX * r], 1);
            } else if (key != LOST) {
                atomicAdd(&P.scr.n_arrive[key], 1);
            }
            st_lost += key == LOST;
            st_moved += (key != LOST) && !stay;
            st_near += near;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < Sh::CELLS; q += ADV_BLOCK) {
            const int ci = q % BX, r = q / BX, cj = r % BY, ck = r / BY;
            if (ci < nx && cj < ny && ck < nz)
                P.scr.n_stay[(bi.i0 + ci) + m.n[0] * ((bi.j0 + cj) + m.n[1] * (D == 3 ? bi.k0 + ck : 0))] = s_cnt[q];
        }
        flush_stats(P.scr.stats, ST_PSTEPS, threadIdx.x == 0 ? total : 0, nullptr);
        flush_stats(P.scr.stats, ST_LOST, st_lost, nullptr);
        flush_stats(P.scr.stats, ST_MOVED, st_moved, nullptr);
        flush_stats(P.scr.stats, ST_NEAR, st_near, nullptr);
        __syncthreads();
    }
}


using BlockFn = void (*)(const ProblemDev *, const BlockItem *, int);
using AdvectFn = void (*)(const ProblemDev *, const WorkItem *, int);

// Uniform-mesh block kernels of the default shapes (ode: with the property
// equations; ti: field interpolated in time), per unit.
BlockFn block_kernel_2(int scheme, int prec, bool fused, bool ode, bool ti);
BlockFn block_kernel_3f(int scheme, bool fused, bool ode, bool ti);
BlockFn block_kernel_3d(int scheme, bool fused, bool ode, bool ti);
// Double-precision block kernels of batch shape `variant` (fused: the
// gather + advect form, as block_kernel).
BlockFn batch_block_kernel_2(int scheme, int variant, bool fused);
BlockFn batch_block_kernel_3(int scheme, int variant, bool fused);
// Generic per-tile kernels (any mesh kind).
AdvectFn advect_kernel_2(int scheme, int prec, int kind, bool ode, bool ti);
AdvectFn advect_kernel_3(int scheme, int prec, int kind, bool ode, bool ti);
inline AdvectFn advect_kernel(int dim, int scheme, int prec, int kind, bool ode, bool ti)
{
    return dim == 2 ? advect_kernel_2(scheme, prec, kind, ode, ti) : advect_kernel_3(scheme, prec, kind, ode, ti);
}

inline BlockFn block_kernel(int dim, int scheme, int prec, bool fused, bool ode, bool ti)
{
    if (dim == 2) return block_kernel_2(scheme, prec, fused, ode, ti);
    return prec == PIC_F32 ? block_kernel_3f(scheme, fused, ode, ti) : block_kernel_3d(scheme, fused, ode, ti);
}
inline BlockFn batch_block_kernel(int dim, int scheme, int variant, bool fused)
{
    return dim == 2 ? batch_block_kernel_2(scheme, variant, fused) : batch_block_kernel_3(scheme, variant, fused);
}

}  // namespace pic
