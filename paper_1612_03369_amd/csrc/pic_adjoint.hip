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

// ---------------------------------------------------------------------------
// uniform meshes: blocks of cells of the step's input state, dU pre-reduced
// in an LDS window of the block's Q2 nodes plus a one-cell halo
// ---------------------------------------------------------------------------
template <int D, int BX, int BY, int BZ> struct NodeWin {
    static constexpr int WX = 2 * BX + 5;
    static constexpr int WY = 2 * BY + 5;
    static constexpr int WZ = D == 3 ? 2 * BZ + 5 : 1;
    static constexpr int NODES = WX * WY * WZ;
    static constexpr int ROWS = BY * (D == 3 ? BZ : 1);
};

// reference gradient Gr[c][r] = d u_c / d t_r of the nodal field at (ijk, t)
// and the 1D basis values l[axis][0..2] (the nodal basis values are their
// products)
// base = index of local node (0,0,0) of the cell in the grid U, sy / sz = the
// grid's row strides (global node array or the block's LDS window)
template <int D, typename Ptr, typename I>
__device__ __forceinline__ void grad_basis_at(Ptr U, I base, I sy, I sz, const double *t, double Gr[3][3],
                                              double l[3][3])
{
    // sum-factorised: along x the value and derivative sums of each node row,
    // then along y, then along z (value sums carry the other axes' weights)
    double dl[3][3];
    for (int a = 0; a < D; ++a) {
        lag3(t[a], l[a]);
        dlag3(t[a], dl[a]);
    }
    if constexpr (D == 2) {
        double sx[2] = {0, 0}, sy_[2] = {0, 0};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double r0[2] = {0, 0}, rd[2] = {0, 0};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const auto v = U[base + a + sy * b];
                const double vc[2] = {(double)nv_x(v), (double)nv_y(v)};
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    r0[c] = fma(vc[c], l[0][a], r0[c]);
                    rd[c] = fma(vc[c], dl[0][a], rd[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                sx[c] = fma(rd[c], l[1][b], sx[c]);
                sy_[c] = fma(r0[c], dl[1][b], sy_[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) Gr[c][0] = Gr[c][1] = Gr[c][2] = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            Gr[c][0] = sx[c];
            Gr[c][1] = sy_[c];
        }
    } else {
        double gx[3] = {0, 0, 0}, gy[3] = {0, 0, 0}, gz[3] = {0, 0, 0};
#pragma unroll 1
        for (int c3 = 0; c3 < 3; ++c3) {
            double p0[3] = {0, 0, 0}, px[3] = {0, 0, 0}, py[3] = {0, 0, 0};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double r0[3] = {0, 0, 0}, rd[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const auto v = U[base + a + sy * b + sz * c3];
                    const double vc[3] = {(double)nv_x(v), (double)nv_y(v), (double)nv_z(v)};
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        r0[c] = fma(vc[c], l[0][a], r0[c]);
                        rd[c] = fma(vc[c], dl[0][a], rd[c]);
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    p0[c] = fma(r0[c], l[1][b], p0[c]);
                    px[c] = fma(rd[c], l[1][b], px[c]);
                    py[c] = fma(r0[c], dl[1][b], py[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                gx[c] = fma(px[c], l[2][c3], gx[c]);
                gy[c] = fma(py[c], l[2][c3], gy[c]);
                gz[c] = fma(p0[c], dl[2][c3], gz[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Gr[c][0] = gx[c];
            Gr[c][1] = gy[c];
            Gr[c][2] = gz[c];
        }
    }
}

// v[k] for k in {0, 1, 2} by selects (no run-time indexing of a register array)
__device__ __forceinline__ double sel3(const double *v, int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

/*
 * One reverse step on a uniform mesh.  Work item = block of cells of the
 * step's input state (its particles are runs of consecutive cells); dst[i] is
 * the output position of input particle i (-1 if it was lost).  Stage points
 * are recomputed with the forward's own location and evaluation, the reverse
 * sweep is applied, lam_out[i] is written, and the dU contributions of the
 * block are summed in LDS before one atomic per window node.
 */
template <int D, int S, int BX, int BY, int BZ>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_adjoint_blk(const ProblemDev *__restrict__ probs,
                                                       const BlockItem *__restrict__ work, int n_work,
                                                       const double *__restrict__ x_in, const double *__restrict__ xr_in,
                                                       const int32_t *__restrict__ cell_in, const int32_t *__restrict__ cs_in,
                                                       const int32_t *__restrict__ dst, const double *__restrict__ lam_next,
                                                       double *__restrict__ lam_out, double *__restrict__ dU)
{
    using Wn = NodeWin<D, BX, BY, BZ>;
    using V = typename NodeVec<D, double>::type;
    __shared__ double s_acc[Wn::NODES * D];
    __shared__ V s_u[Wn::NODES];                  // the field on the same window
    __shared__ int s_pre[Wn::ROWS + 1];
    __shared__ int s_beg[Wn::ROWS];
    const ProblemDev &P = probs[0];
    const MeshDev &m = P.mesh;
    const int64_t cap = P.cap;
    const double dt = P.dt;
    auto Ug = (gptr<V>)P.u64;
    const int64_t nn = m.n_nodes;
    // the lane's digit offsets of the dU walk (see below): rotated local
    // indices along each axis and the window offsets of the (b, c) rows
    int rot_a[3], rot_b[3], rot_c[3], off_bc[3][3];
    {
        const int rot = (threadIdx.x & 63) % (D == 3 ? 27 : 9);
        const int oa = rot % 3, ob = (rot / 3) % 3, oc = D == 3 ? rot / 9 : 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            rot_a[i] = (i + oa) % 3;
            rot_b[i] = (i + ob) % 3;
            rot_c[i] = (i + oc) % 3;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) off_bc[i][j] = Wn::WX * (rot_b[i] + (D == 3 ? Wn::WY * rot_c[j] : 0));
    }
    for (int wb = blockIdx.x; wb < xcd_span(n_work); wb += gridDim.x) {
        const int w = xcd_item(wb, n_work);
        if (w >= n_work) continue;
        const BlockItem bi = work[w];
        const int b0[3] = {bi.i0, bi.j0, D == 3 ? bi.k0 : 0};
        const int nx = min(BX, m.n[0] - bi.i0), ny = min(BY, m.n[1] - bi.j0);
        const int nz = D == 3 ? min(BZ, m.n[2] - bi.k0) : 1;
        for (int q = threadIdx.x; q < Wn::NODES * D; q += BLOCK) s_acc[q] = 0.0;
        for (int q = threadIdx.x; q < Wn::NODES; q += BLOCK) {
            const int wx = q % Wn::WX, wy = (q / Wn::WX) % Wn::WY, wz = q / (Wn::WX * Wn::WY);
            const int gx = 2 * b0[0] - 2 + wx, gy = 2 * b0[1] - 2 + wy, gz = D == 3 ? 2 * b0[2] - 2 + wz : 0;
            if (gx >= 0 && gx < m.nnx && gy >= 0 && gy < m.nny && gz >= 0 && gz < m.nnz)
                s_u[q] = Ug[gx + (int64_t)m.nnx * (gy + (int64_t)m.nny * gz)];
        }
        if (threadIdx.x < 64) {
            const int r = threadIdx.x;
            int len = 0, beg = 0;
            if (r < Wn::ROWS) {
                const int rj = r % BY, rk = r / BY;
                if (rj < ny && rk < nz) {
                    const int K = bi.i0 + m.n[0] * ((bi.j0 + rj) + m.n[1] * (D == 3 ? bi.k0 + rk : 0));
                    beg = cs_in[K];
                    len = cs_in[K + nx] - beg;
                }
                s_beg[r] = beg;
            }
            int inc = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(inc, o, 64);
                if (r >= o) inc += v;
            }
            if (r < Wn::ROWS) s_pre[r + 1] = inc;
            if (r == 0) s_pre[0] = 0;
        }
        __syncthreads();
        const int total = s_pre[Wn::ROWS];
        for (int f = threadIdx.x; f < total; f += BLOCK) {
            int r = 0;
#pragma unroll
            for (int step = Wn::ROWS / 2; step >= 1; step >>= 1)
                if (r + step < Wn::ROWS && s_pre[r + step] <= f) r += step;
            const int i = s_beg[r] + (f - s_pre[r]);
            const int p = dst[i];
            if (p < 0) {
                for (int a = 0; a < D; ++a) lam_out[a * cap + i] = 0.0;
                continue;
            }
            double x[3], ty[4][3], k[4][3], u[3], y[3];
            int jk[4][3];
            bool near = false;
            ijk_of<D>(m, (uint32_t)cell_in[i], jk[0]);
            // the first stage point is the particle: its reference coordinates
            // by the closed form, as the forward's block kernels take them
            for (int a = 0; a < D; ++a) {
                x[a] = x_in[a * cap + i];
                ty[0][a] = (x[a] - fma((double)jk[0][a], m.h[a], m.lo[a])) * m.inv_h[a];
            }
            // window node index of local node (0,0,0) of cell ijk, or -1 outside the window
            auto wbase = [&](const int *ijk) {
                const int di = ijk[0] - b0[0] + 1, dj = ijk[1] - b0[1] + 1, dk = ijk[2] - b0[2] + 1;
                bool inw = ((unsigned)di < (unsigned)(BX + 2)) & ((unsigned)dj < (unsigned)(BY + 2));
                if constexpr (D == 3) inw &= (unsigned)dk < (unsigned)(BZ + 2);
                return inw ? 2 * di + Wn::WX * (2 * dj + (D == 3 ? Wn::WY * 2 * dk : 0)) : -1;
            };
            const int64_t gsz = (int64_t)m.nnx * m.nny;
            auto gbase = [&](const int *ijk) {
                return 2 * ijk[0] + (int64_t)m.nnx * (2 * ijk[1]) + (D == 3 ? gsz * (2 * ijk[2]) : 0);
            };
            constexpr int NS = S == 4 ? 4 : S;
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                if (st > 0) {
                    const double fct = (S == 4 && st == 3) ? 1.0 : 0.5;
                    for (int a = 0; a < D; ++a) y[a] = x[a] + fct * k[st - 1][a];
                    locate_stage<D>(m, y, jk[st], ty[st], near, true);
                }
                const int wq = wbase(jk[st]);
                if (wq >= 0)
                    eval_q2_at<D, double>((const V *)s_u, wq, (int)Wn::WX, (int)(Wn::WX * Wn::WY), ty[st], u);
                else
                    eval_q2_at<D, double>(Ug, gbase(jk[st]), (int64_t)m.nnx, gsz, ty[st], u);
                for (int a = 0; a < D; ++a) k[st][a] = dt * u[a];
            }
            double lam[3], kb[4][3], yb[4][3];
            for (int a = 0; a < D; ++a) lam[a] = lam_next[a * cap + p];
            for (int a = 0; a < D; ++a) {
                if constexpr (S == 1) {
                    kb[0][a] = lam[a];
                } else if constexpr (S == 2) {
                    kb[1][a] = lam[a];
                    kb[0][a] = 0.0;
                } else {
                    kb[0][a] = lam[a] / 6.0;
                    kb[1][a] = lam[a] / 3.0;
                    kb[2][a] = lam[a] / 3.0;
                    kb[3][a] = lam[a] / 6.0;
                }
            }
#pragma unroll
            for (int st = NS - 1; st >= 0; --st) {
                double Gr[3][3], l[3][3];
                const int wq = wbase(jk[st]);
                if (wq >= 0)
                    grad_basis_at<D>((const V *)s_u, wq, (int)Wn::WX, (int)(Wn::WX * Wn::WY), ty[st], Gr, l);
                else
                    grad_basis_at<D>(Ug, gbase(jk[st]), (int64_t)m.nnx, gsz, ty[st], Gr, l);
                for (int j = 0; j < D; ++j) {
                    double acc = 0.0;
                    for (int c = 0; c < D; ++c) acc += Gr[c][j] * kb[st][c];
                    yb[st][j] = dt * acc / m.h[j];
                }
                // dU_c[node] += dt phi_node kb_c : LDS window if the cell's nodes are in it
                const int di = jk[st][0] - b0[0] + 1, dj = jk[st][1] - b0[1] + 1, dk = jk[st][2] - b0[2] + 1;
                bool inw = ((unsigned)di < (unsigned)(BX + 2)) & ((unsigned)dj < (unsigned)(BY + 2));
                if constexpr (D == 3) inw &= (unsigned)dk < (unsigned)(BZ + 2);
                // Lanes holding particles of one cell would add to the same
                // node at the same time (serialised LDS atomics); each lane
                // walks the cell's nodes from its own start: step (ra, rb, rc)
                // visits node ((ra + oa) mod 3, (rb + ob) mod 3, (rc + oc) mod 3)
                // with the lane's digit offsets, so lanes with different
                // offsets never meet.  The rotated basis values, node offsets
                // and weights are formed once per stage; the walk is unrolled.
                constexpr int NB = D == 3 ? 27 : 9;
                if (inw) {
                    const int base = 2 * di + Wn::WX * (2 * dj + (D == 3 ? Wn::WY * 2 * dk : 0));
                    double LA[3], LBC[3][3], dk3[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        LA[i] = sel3(l[0], rot_a[i]);
                        const double lbi = sel3(l[1], rot_b[i]);
#pragma unroll
                        for (int j = 0; j < 3; ++j) LBC[i][j] = D == 3 ? lbi * sel3(l[2], rot_c[j]) : (j == 0 ? lbi : 0.0);
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) dk3[c] = c < D ? dt * kb[st][c] : 0.0;
#pragma unroll
                    for (int rc = 0; rc < (D == 3 ? 3 : 1); ++rc)
#pragma unroll
                        for (int rb = 0; rb < 3; ++rb) {
                            const int qbc = base + off_bc[rb][rc];
#pragma unroll
                            for (int ra = 0; ra < 3; ++ra) {
                                const double ph = LA[ra] * LBC[rb][rc];
                                const int q = qbc + rot_a[ra];
#pragma unroll
                                for (int c = 0; c < D; ++c) atomicAdd(&s_acc[c * Wn::NODES + q], ph * dk3[c]);
                            }
                        }
                }
                const int rot = (threadIdx.x & 63) % NB;
                for (int r = 0; r < NB && !inw; ++r) {
                    const int nq = r + rot >= NB ? r + rot - NB : r + rot;
                    const int a = nq % 3, b = (nq / 3) % 3, c3 = D == 3 ? nq / 9 : 0;
                    const double la = a == 0 ? l[0][0] : (a == 1 ? l[0][1] : l[0][2]);
                    const double lb = b == 0 ? l[1][0] : (b == 1 ? l[1][1] : l[1][2]);
                    double ph = la * lb;
                    if constexpr (D == 3) ph *= c3 == 0 ? l[2][0] : (c3 == 1 ? l[2][1] : l[2][2]);
                    const double f = dt * ph;
                    {
                        const int64_t g = (2 * jk[st][0] + a) + (int64_t)m.nnx * ((2 * jk[st][1] + b) +
                                          (int64_t)m.nny * (D == 3 ? 2 * jk[st][2] + c3 : 0));
                        for (int c = 0; c < D; ++c) unsafeAtomicAdd(&dU[c * nn + g], f * kb[st][c]);
                    }
                }
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
                lam_out[a * cap + i] = v;
            }
        }
        __syncthreads();
        // flush the window: window node (wx, wy, wz) = global node 2*b0 - 2 + w
        for (int q = threadIdx.x; q < Wn::NODES; q += BLOCK) {
            const int wx = q % Wn::WX, wy = (q / Wn::WX) % Wn::WY, wz = q / (Wn::WX * Wn::WY);
            const int gx = 2 * b0[0] - 2 + wx, gy = 2 * b0[1] - 2 + wy, gz = D == 3 ? 2 * b0[2] - 2 + wz : 0;
            if (gx < 0 || gx > 2 * m.n[0] || gy < 0 || gy > 2 * m.n[1] || gz < 0 || gz > (D == 3 ? 2 * m.n[2] : 0))
                continue;
            const int64_t g = gx + (int64_t)m.nnx * (gy + (int64_t)m.nny * gz);
            for (int c = 0; c < D; ++c) {
                const double v = s_acc[c * Wn::NODES + q];
                if (v != 0.0) unsafeAtomicAdd(&dU[c * nn + g], v);
            }
        }
        __syncthreads();
    }
}

// dst[i] = output position of input particle i (or -1): inverse of src
__global__ void k_invert(const int32_t *__restrict__ src, const int32_t *__restrict__ cs_in,
                         const int32_t *__restrict__ cs_out, int64_t nc, int32_t *__restrict__ dst, int64_t cap)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < cap && q < cs_in[nc]) dst[q] = -1;
}
__global__ void k_invert_scatter(const int32_t *__restrict__ src, const int32_t *__restrict__ cs_out, int64_t nc,
                                 int32_t *__restrict__ dst, int64_t cap)
{
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p < cap && p < cs_out[nc]) dst[src[p]] = (int32_t)p;
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
    LocStats ls = {0, 0, 0, 0, 0};
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
