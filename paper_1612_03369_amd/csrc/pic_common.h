// Device-side types and helpers of the particle hot path (gfx950).
//
// Q2 field evaluation (Sec. 2.3: the velocity is evaluated through the shape
// functions on the reference cell at the stored reference location), the
// cell maps Phi_K and their inverses, and point location (Sec. 2.4: in-cell
// test via xhat in Khat, vertex-neighbour search ordered by a.b, global
// search as the last resort).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr uint32_t LOST = 0xFFFFFFFFu;
constexpr double NEAR_TOL = 1e-10;   // near-face band in reference coordinates
constexpr int BLOCK = 256;           // threads per workgroup of the per-tile kernels
// Cells per thread of the scan's chunks (BLOCK threads per chunk): meshes of up
// to 2^19 cells take short chunks (more workgroups, shorter load chains), larger
// ones long chunks, so that the sum over the preceding chunks' totals that each
// workgroup of the down-sweep forms stays short.
constexpr int SCAN_PT_MAX = 8;
__host__ __device__ inline int scan_per_thread(int64_t n_cells) { return n_cells <= (int64_t(1) << 19) ? 2 : SCAN_PT_MAX; }
__host__ __device__ inline int64_t scan_chunk_cells(int64_t n_cells) { return (int64_t)BLOCK * scan_per_thread(n_cells); }
constexpr int MAX_TILE = 1024;       // cells per work item (LDS arrays are sized by it)
constexpr int MAX_NBR = 64;          // vertex neighbours of one cell (octree upper bound)
#ifndef PIC_EVAL_BATCH
#define PIC_EVAL_BATCH 1                // 3D evaluation: load a plane of nodes before summing it
#endif
#ifndef PIC_EVAL_UNROLL
#define PIC_EVAL_UNROLL 3               // unroll of the outermost sum-factorisation loop
#endif

enum MeshKind : int { MESH_UNIFORM = 0, MESH_DISPLACED = 1, MESH_OCTREE = 2 };

// Counter slots in the device statistics array.
enum StatSlot : int {
    ST_LOST = 0, ST_MOVED, ST_NEAR, ST_FIRST_TRY, ST_FALLBACK, ST_NEWTON_FAIL, ST_ADDED, ST_DELETED,
    ST_STEPS, ST_SEARCHED, ST_PSTEPS, ST_SEARCHES, ST_COUNT = 16
};
// Counters are spread over STAT_STRIPES copies (one 128-byte line each),
// picked by workgroup index, so that no address sees more than a sliver of
// the atomics; readers sum the stripes.
constexpr int STAT_STRIPES = 256;

struct MeshDev {
    int dim, kind;
    int n[3];                 // structured: cells per axis
    int nnx, nny, nnz;        // structured Q2 node grid extents 2n+1 (nnz = 1 in 2D)
    int nvx, nvy;             // structured vertex grid extents n+1
    int64_t n_cells, n_nodes, n_vert;
    double lo[3], hi[3], h[3], inv_h[3];
    double bnd_tol[3];        // near-boundary band per axis (1e-10 * smallest cell edge)
    const double *vert;       // displaced: [dim][n_vert]
    // octree
    int max_level;
    double fine_h[3], inv_fine_h[3];
    const int32_t *anchor;    // [3][n_cells] finest-cell units
    const uint8_t *level;     // [n_cells]
    const int32_t *fine;      // [(2^L)^3] finest cell -> leaf
    const int32_t *cell_nodes;// [n_cells][27]
    // vertex-neighbour lists (displaced, octree)
    const int32_t *nbr_off;   // [n_cells + 1]
    const int32_t *nbr;       // [nbr_off[n_cells]]
};

// Pointers into device memory that kernels read from structures: in device
// code they carry the global address space, so that their loads and stores
// are global (not flat) accesses, which do not hold up waits on LDS.
#ifdef __HIP_DEVICE_COMPILE__
#define PIC_G __attribute__((address_space(1)))
#else
#define PIC_G
#endif

// One buffer of the particle store.
struct StoreDev {
    double PIC_G *x;       // [dim][cap]
    double PIC_G *xr;      // [dim][cap]
    int32_t PIC_G *cell;   // [cap]
    uint32_t PIC_G *id;    // [cap]
    void PIC_G *prop;      // [n_prop][cap]
    int32_t PIC_G *cs;     // [n_cells + 1]
};

inline StoreDev make_store(double *x, double *xr, int32_t *cell, uint32_t *id, void *prop, int32_t *cs)
{
    StoreDev s;
    s.x = (double PIC_G *)x;
    s.xr = (double PIC_G *)xr;
    s.cell = (int32_t PIC_G *)cell;
    s.id = (uint32_t PIC_G *)id;
    s.prop = (void PIC_G *)prop;
    s.cs = (int32_t PIC_G *)cs;
    return s;
}

// Per-context scratch (carved out of the caller's workspace).
struct ScratchDev {
    uint32_t PIC_G *key[2];     // [cap] per buffer: new cell (or LOST) of the particle at that position
    int32_t PIC_G *src;         // [cap] gather source of each destination slot
    int32_t PIC_G *n_stay;      // [nc]
    int32_t PIC_G *n_arrive;    // [nc]
    int32_t PIC_G *cursor;      // [nc]
    int64_t PIC_G *chunk;       // [n_chunks + 1]
    unsigned long long *stats;  // [STAT_STRIPES][ST_COUNT]
    unsigned long long *next_id;// [1 + STAT_STRIPES]: next_id[0], then striped maxima written by seeding
    int32_t *flags;       // [4]
};

// ---------------------------------------------------------------------------
// node value vectors: 3D fields padded to 4 components, 2D to 2
// ---------------------------------------------------------------------------
template <int D, typename T> struct NodeVec;
template <> struct NodeVec<3, float> { using type = float4; };
template <> struct NodeVec<3, double> { using type = double4; };
template <> struct NodeVec<2, float> { using type = float2; };
template <> struct NodeVec<2, double> { using type = double2; };

template <typename V> __device__ __forceinline__ auto nv_x(const V &v) { return v.x; }
template <typename V> __device__ __forceinline__ auto nv_y(const V &v) { return v.y; }
__device__ __forceinline__ float nv_z(const float4 &v) { return v.z; }
__device__ __forceinline__ double nv_z(const double4 &v) { return v.z; }
__device__ __forceinline__ float nv_z(const float2 &) { return 0.f; }
__device__ __forceinline__ double nv_z(const double2 &) { return 0.0; }
// node value from its components (z ignored in 2D; the fourth lane of a 3D node is padding)
template <typename V, typename E> __device__ __forceinline__ V node_of(E x, E y, E z)
{
    V v;
    v.x = x;
    v.y = y;
    if constexpr (sizeof(V) == 4 * sizeof(E)) {
        v.z = z;
        v.w = E(0);
    }
    return v;
}

// ---------------------------------------------------------------------------
// rounding-pinned building blocks of the sum-factorised evaluation: every
// evaluation path (global memory, LDS window, octree node map) combines node
// values with exactly these fused multiply-adds, so they agree bit for bit
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// s = la0 v0 + la1 v1 + la2 v2 along x, then acc += w * s
template <typename T>
__device__ __forceinline__ T row3(const T *la, T v0, T v1, T v2)
{
    return fma_t(la[2], v2, fma_t(la[1], v1, la[0] * v0));
}

// ---------------------------------------------------------------------------
// 1D quadratic Lagrange basis on the nodes {0, 1/2, 1} and its derivative
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ void lag3(T t, T l[3])
{
    const T u = T(1) - t;
    l[0] = u * fma_t(T(-2), t, T(1));
    l[1] = (T(4) * t) * u;
    l[2] = t * fma_t(T(2), t, T(-1));
}
template <typename T> __device__ __forceinline__ void dlag3(T t, T d[3])
{
    d[0] = T(4) * t - T(3);
    d[1] = T(4) - T(8) * t;
    d[2] = T(4) * t - T(1);
}

// Node index of local node (0,0,0) of structured cell K and its (i,j,k).
__device__ __forceinline__ void cell_ijk(const MeshDev &m, int64_t K, int ijk[3])
{
    ijk[0] = (int)(K % m.n[0]);
    ijk[1] = (int)((K / m.n[0]) % m.n[1]);
    ijk[2] = m.dim == 3 ? (int)(K / ((int64_t)m.n[0] * m.n[1])) : 0;
}

// Global node of local node (a,b,c) in cell K.
template <int D, int KIND>
__device__ __forceinline__ int64_t q2_node(const MeshDev &m, int64_t K, int a, int b, int c)
{
    if constexpr (KIND == MESH_OCTREE) {
        return m.cell_nodes[K * 27 + a + 3 * b + 9 * c];
    } else {
        int ijk[3];
        cell_ijk(m, K, ijk);
        return (2 * ijk[0] + a) + (int64_t)m.nnx * ((2 * ijk[1] + b) + (int64_t)m.nny * (2 * ijk[2] + c));
    }
}

// ---------------------------------------------------------------------------
// Q2 evaluation, sum-factorised: u = sum_c lc sum_b lb sum_a la U[a,b,c]
// ---------------------------------------------------------------------------
template <int D, typename T, int KIND>
__device__ __forceinline__ void eval_q2(const MeshDev &m, const typename NodeVec<D, T>::type *__restrict__ U,
                                        int64_t K, const double *tr, double *u)
{
    T t0 = (T)tr[0], t1 = (T)tr[1];
    T la[3], lb[3];
    lag3(t0, la);
    lag3(t1, lb);
    if constexpr (D == 2) {
        T a0 = 0, a1 = 0;
        if constexpr (KIND == MESH_OCTREE) {
            // not used: octree meshes are 3D
        } else {
            int ijk[3];
            cell_ijk(m, K, ijk);
            const auto *base = U + (2 * ijk[0]) + (int64_t)m.nnx * (2 * ijk[1]);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const auto *row = base + (int64_t)m.nnx * b;
                auto v0 = row[0], v1 = row[1], v2 = row[2];
                a0 = fma_t(lb[b], row3(la, (T)v0.x, (T)v1.x, (T)v2.x), a0);
                a1 = fma_t(lb[b], row3(la, (T)v0.y, (T)v1.y, (T)v2.y), a1);
            }
        }
        u[0] = (double)a0;
        u[1] = (double)a1;
    } else {
        T lc[3];
        lag3((T)tr[2], lc);
        T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll PIC_EVAL_UNROLL
        for (int c = 0; c < 3; ++c) {
            T r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                typename NodeVec<D, T>::type v0, v1, v2;
                if constexpr (KIND == MESH_OCTREE) {
                    const int32_t *cn = m.cell_nodes + K * 27 + 3 * b + 9 * c;
                    v0 = U[cn[0]];
                    v1 = U[cn[1]];
                    v2 = U[cn[2]];
                } else {
                    int ijk[3];
                    cell_ijk(m, K, ijk);
                    const auto *row = U + (2 * ijk[0]) +
                                      (int64_t)m.nnx * ((2 * ijk[1] + b) + (int64_t)m.nny * (2 * ijk[2] + c));
                    v0 = row[0];
                    v1 = row[1];
                    v2 = row[2];
                }
                r0 = fma_t(lb[b], row3(la, (T)v0.x, (T)v1.x, (T)v2.x), r0);
                r1 = fma_t(lb[b], row3(la, (T)v0.y, (T)v1.y, (T)v2.y), r1);
                r2 = fma_t(lb[b], row3(la, (T)v0.z, (T)v1.z, (T)v2.z), r2);
            }
            a0 = fma_t(lc[c], r0, a0);
            a1 = fma_t(lc[c], r1, a1);
            a2 = fma_t(lc[c], r2, a2);
        }
        u[0] = (double)a0;
        u[1] = (double)a1;
        u[2] = (double)a2;
    }
}

// The same sum over the 27 node values of one cell held contiguously in
// local order a + 3b + 9c (an LDS copy of an octree leaf's nodes); the
// arithmetic matches eval_q2 on the global field.
template <int D, typename T>
__device__ __forceinline__ void eval_q2_local(const typename NodeVec<D, T>::type *W, const double *tr, double *u)
{
    static_assert(D == 3, "octree leaves are 3D");
    T la[3], lb[3], lc[3];
    lag3((T)tr[0], la);
    lag3((T)tr[1], lb);
    lag3((T)tr[2], lc);
    T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll PIC_EVAL_UNROLL
    for (int c = 0; c < 3; ++c) {
        T r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const auto v0 = W[3 * b + 9 * c], v1 = W[3 * b + 9 * c + 1], v2 = W[3 * b + 9 * c + 2];
            r0 = fma_t(lb[b], row3(la, (T)v0.x, (T)v1.x, (T)v2.x), r0);
            r1 = fma_t(lb[b], row3(la, (T)v0.y, (T)v1.y, (T)v2.y), r1);
            r2 = fma_t(lb[b], row3(la, (T)v0.z, (T)v1.z, (T)v2.z), r2);
        }
        a0 = fma_t(lc[c], r0, a0);
        a1 = fma_t(lc[c], r1, a1);
        a2 = fma_t(lc[c], r2, a2);
    }
    u[0] = (double)a0;
    u[1] = (double)a1;
    u[2] = (double)a2;
}

// Reference gradient G[c][r] = d u_c / d xhat_r (double precision).
template <int D, int KIND>
__device__ __forceinline__ void eval_q2_refgrad(const MeshDev &m, const typename NodeVec<D, double>::type *__restrict__ U,
                                                int64_t K, const double *tr, double G[3][3])
{
    double l[3][3], dl[3][3];
    for (int a = 0; a < D; ++a) {
        lag3(tr[a], l[a]);
        dlag3(tr[a], dl[a]);
    }
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) G[c][r] = 0.0;
    const int nc = D == 3 ? 3 : 1;
    for (int c3 = 0; c3 < nc; ++c3)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                auto v = U[q2_node<D, KIND>(m, K, a, b, c3)];
                double w0, w1, w2 = 0.0;
                if constexpr (D == 2) {
                    w0 = dl[0][a] * l[1][b];
                    w1 = l[0][a] * dl[1][b];
                } else {
                    w0 = dl[0][a] * l[1][b] * l[2][c3];
                    w1 = l[0][a] * dl[1][b] * l[2][c3];
                    w2 = l[0][a] * l[1][b] * dl[2][c3];
                }
                double vc[3] = {(double)nv_x(v), (double)nv_y(v), (double)nv_z(v)};
                for (int c = 0; c < D; ++c) {
                    G[c][0] += vc[c] * w0;
                    G[c][1] += vc[c] * w1;
                    if constexpr (D == 3) G[c][2] += vc[c] * w2;
                }
            }
}

// ---------------------------------------------------------------------------
// uniform meshes: (i,j,k) carried through location and evaluation
// ---------------------------------------------------------------------------
// global-address-space pointer (global_load instead of flat_load); the host
// pass of the compiler sees a plain pointer
#if defined(__HIP_DEVICE_COMPILE__)
template <typename V> using gptr = const V __attribute__((address_space(1))) *;
template <typename V> using gptr_mut = V __attribute__((address_space(1))) *;
#else
template <typename V> using gptr = const V *;
template <typename V> using gptr_mut = V *;
#endif

// (i,j,k) of cell K with 32-bit arithmetic (cells < 2^31)
template <int D>
__device__ __forceinline__ void ijk_of(const MeshDev &m, uint32_t K, int ijk[3])
{
    const uint32_t n0 = (uint32_t)m.n[0];
    const uint32_t q = K / n0;
    ijk[0] = (int)(K - q * n0);
    if constexpr (D == 3) {
        const uint32_t n1 = (uint32_t)m.n[1];
        const uint32_t r = q / n1;
        ijk[1] = (int)(q - r * n1);
        ijk[2] = (int)r;
    } else {
        ijk[1] = (int)q;
        ijk[2] = 0;
    }
}

template <int D> __device__ __forceinline__ uint32_t cell_of(const MeshDev &m, const int ijk[3])
{
    uint32_t K = (uint32_t)ijk[0] + (uint32_t)m.n[0] * (uint32_t)ijk[1];
    if constexpr (D == 3) K += (uint32_t)m.n[0] * (uint32_t)m.n[1] * (uint32_t)ijk[2];
    return K;
}

// Owning cell of y by the closed form floor((y - lo)/h) with the half-open
// rule (upper domain faces closed); false outside the closed box.
template <int D>
__device__ __forceinline__ bool locate_uniform(const MeshDev &m, const double *y, int ijk[3], double *t)
{
    bool inside = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        inside &= (y[a] >= m.lo[a]) & (y[a] <= m.hi[a]);
        const double s = (y[a] - m.lo[a]) * m.inv_h[a];
        int i = (int)floor(s);
        i = i >= m.n[a] ? m.n[a] - 1 : (i < 0 ? 0 : i);
        t[a] = (y[a] - fma((double)i, m.h[a], m.lo[a])) * m.inv_h[a];
        ijk[a] = i;
    }
    if constexpr (D == 2) ijk[2] = 0;
    return inside;
}

// Q2 evaluation on a structured node grid, sum-factorised.  base = index of
// local node (0,0,0) of the cell, sy / sz = index strides of the grid's y and
// z rows.  The grid may be the global node array or a window of it in LDS:
// the arithmetic, and hence the rounding, is the same for both.
template <int D, typename T, typename Ptr, typename I>
__device__ __forceinline__ void eval_q2_at(Ptr U, I base, I sy, I sz, const double *tr, double *u)
{
    T la[3], lb[3];
    lag3((T)tr[0], la);
    lag3((T)tr[1], lb);
    if constexpr (D == 2) {
        const I nnx = sy;
        T a0 = 0, a1 = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const I r = base + nnx * b;
            const auto v0 = U[r], v1 = U[r + 1], v2 = U[r + 2];
            a0 = fma_t(lb[b], row3(la, (T)v0.x, (T)v1.x, (T)v2.x), a0);
            a1 = fma_t(lb[b], row3(la, (T)v0.y, (T)v1.y, (T)v2.y), a1);
        }
        u[0] = (double)a0;
        u[1] = (double)a1;
    } else {
        T lc[3];
        lag3((T)tr[2], lc);
        const I nnx = sy;
        T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll PIC_EVAL_UNROLL
        for (int c = 0; c < 3; ++c) {
#if PIC_EVAL_BATCH
            // the nine nodes of plane c are all requested before the first is
            // used, so that their load latencies overlap (the scheduler would
            // otherwise interleave loads and uses to save registers)
            T vx[3][3], vy[3][3], vz[3][3];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const auto w = U[base + nnx * b + sz * c + i];
                    vx[b][i] = (T)w.x;
                    vy[b][i] = (T)w.y;
                    vz[b][i] = (T)w.z;
                }
            __builtin_amdgcn_sched_barrier(0);
#endif
            T r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
#if PIC_EVAL_BATCH
                r0 = fma_t(lb[b], row3(la, vx[b][0], vx[b][1], vx[b][2]), r0);
                r1 = fma_t(lb[b], row3(la, vy[b][0], vy[b][1], vy[b][2]), r1);
                r2 = fma_t(lb[b], row3(la, vz[b][0], vz[b][1], vz[b][2]), r2);
#else
                const I r = base + nnx * b + sz * c;
                const auto v0 = U[r], v1 = U[r + 1], v2 = U[r + 2];
                r0 = fma_t(lb[b], row3(la, (T)v0.x, (T)v1.x, (T)v2.x), r0);
                r1 = fma_t(lb[b], row3(la, (T)v0.y, (T)v1.y, (T)v2.y), r1);
                r2 = fma_t(lb[b], row3(la, (T)v0.z, (T)v1.z, (T)v2.z), r2);
#endif
            }
            a0 = fma_t(lc[c], r0, a0);
            a1 = fma_t(lc[c], r1, a1);
            a2 = fma_t(lc[c], r2, a2);
        }
        u[0] = (double)a0;
        u[1] = (double)a1;
        u[2] = (double)a2;
    }
}

// The same on the global node array of a structured mesh, cell (i,j,k).
template <int D, typename T>
__device__ __forceinline__ void eval_q2_ijk(gptr<typename NodeVec<D, T>::type> U, int nnx, int nny, const int ijk[3],
                                            const double *tr, double *u)
{
    const int64_t sz = (int64_t)nnx * nny;
    const int64_t base = 2 * ijk[0] + (int64_t)nnx * (2 * ijk[1]) + (D == 3 ? sz * (2 * ijk[2]) : 0);
    eval_q2_at<D, T>(U, base, (int64_t)nnx, sz, tr, u);
}

// Stage-point location on a uniform mesh: cell and reference coordinates from
// s = (y - lo)/h; inside = 0 <= s <= n per axis.  `live` says whether every
// earlier point of the step was inside the domain: only then is the point
// tested for the near-boundary band (|y - lo| or |y - hi| below 1e-10 h on
// some axis, inside or outside), as a step that stops at its first point
// outside the domain would test it.  The band test runs only for points with
// s below NEAR_PRE or above n - NEAR_PRE on some axis, which every point in
// the band is (|s| and |s - n| exceed the band by at most a few ulps of n),
// so the common case costs two comparisons per axis.  Reference coordinates
// s - i are accurate to a few ulps of s, which only feeds the field
// evaluation; stored locations use locate_uniform.
constexpr double NEAR_PRE = 1e-6;
template <int D> __device__ __forceinline__ bool near_boundary(const MeshDev &m, const double *y);
template <int D>
__device__ __forceinline__ bool locate_stage(const MeshDev &m, const double *y, int ijk[3], double *t, bool &near,
                                             bool live)
{
    bool inside = true, maybe = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double s = (y[a] - m.lo[a]) * m.inv_h[a];
        const double n = (double)m.n[a];
        inside &= (s >= 0.0) & (s <= n);
        maybe |= (s < NEAR_PRE) | (s > n - NEAR_PRE);
        int i = (int)floor(s);
        i = i >= m.n[a] ? m.n[a] - 1 : (i < 0 ? 0 : i);
        t[a] = s - (double)i;
        ijk[a] = i;
    }
    if constexpr (D == 2) ijk[2] = 0;
    if (maybe & live) near |= near_boundary<D>(m, y);
    return inside;
}

// ---------------------------------------------------------------------------
// cell maps
// ---------------------------------------------------------------------------
// Axis-aligned box of a uniform or octree cell.
template <int KIND>
__device__ __forceinline__ void cell_box(const MeshDev &m, int64_t K, double x0[3], double h[3])
{
    if constexpr (KIND == MESH_OCTREE) {
        int s = 1 << (m.max_level - (int)m.level[K]);
        for (int a = 0; a < 3; ++a) {
            x0[a] = m.lo[a] + (double)m.anchor[a * m.n_cells + K] * m.fine_h[a];
            h[a] = (double)s * m.fine_h[a];
        }
    } else {
        int ijk[3];
        cell_ijk(m, K, ijk);
        for (int a = 0; a < 3; ++a) {
            x0[a] = m.lo[a] + (double)ijk[a] * m.h[a];
            h[a] = m.h[a];
        }
    }
}

// Vertices of a displaced structured cell, X[v][a], v = va + 2 vb + 4 vc.
template <int D>
__device__ __forceinline__ void cell_vertices(const MeshDev &m, int64_t K, double X[8][3])
{
    int ijk[3];
    cell_ijk(m, K, ijk);
    for (int v = 0; v < (1 << D); ++v) {
        int va = v & 1, vb = (v >> 1) & 1, vc = (v >> 2) & 1;
        int64_t g = (ijk[0] + va) + (int64_t)m.nvx * ((ijk[1] + vb) + (int64_t)m.nvy * (ijk[2] + vc));
        for (int a = 0; a < D; ++a) X[v][a] = m.vert[a * m.n_vert + g];
    }
}

// Multilinear map and Jacobian J[a][r] of a displaced cell.
template <int D>
__device__ __forceinline__ void q1_map(const double X[8][3], const double *t, double *x, double J[3][3])
{
    for (int a = 0; a < D; ++a) {
        x[a] = 0.0;
        for (int r = 0; r < D; ++r) J[a][r] = 0.0;
    }
    for (int v = 0; v < (1 << D); ++v) {
        double f[3], df[3];
        for (int a = 0; a < D; ++a) {
            int bit = (v >> a) & 1;
            f[a] = bit ? t[a] : 1.0 - t[a];
            df[a] = bit ? 1.0 : -1.0;
        }
        double N = f[0] * f[1] * (D == 3 ? f[2] : 1.0);
        double g[3];
        g[0] = df[0] * f[1] * (D == 3 ? f[2] : 1.0);
        g[1] = f[0] * df[1] * (D == 3 ? f[2] : 1.0);
        g[2] = D == 3 ? f[0] * f[1] * df[2] : 0.0;
        for (int a = 0; a < D; ++a) {
            x[a] += N * X[v][a];
            for (int r = 0; r < D; ++r) J[a][r] += g[r] * X[v][a];
        }
    }
}

template <int D> __device__ __forceinline__ bool solve_small(const double J[3][3], const double *r, double *s)
{
    if constexpr (D == 2) {
        double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (det == 0.0) return false;
        double inv = 1.0 / det;
        s[0] = (r[0] * J[1][1] - J[0][1] * r[1]) * inv;
        s[1] = (J[0][0] * r[1] - r[0] * J[1][0]) * inv;
        return true;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        if (det == 0.0) return false;
        double inv = 1.0 / det;
        double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        // s = J^{-1} r = adj(J) r / det, adj(J)[r][c] = cofactor[c][r]
        s[0] = (c00 * r[0] + c10 * r[1] + c20 * r[2]) * inv;
        s[1] = (c01 * r[0] + c11 * r[1] + c21 * r[2]) * inv;
        s[2] = (c02 * r[0] + c12 * r[1] + c22 * r[2]) * inv;
        return true;
    }
}

// Phi_K(t) for any mesh kind.
template <int D, int KIND>
__device__ __forceinline__ void map_to_real(const MeshDev &m, int64_t K, const double *t, double *x)
{
    if constexpr (KIND == MESH_DISPLACED) {
        double X[8][3], J[3][3];
        cell_vertices<D>(m, K, X);
        q1_map<D>(X, t, x, J);
    } else {
        double x0[3], h[3];
        cell_box<KIND>(m, K, x0, h);
        for (int a = 0; a < D; ++a) x[a] = x0[a] + t[a] * h[a];
    }
}

// Jacobian of Phi_K at t (for gradients on displaced cells).
template <int D, int KIND>
__device__ __forceinline__ void map_jacobian(const MeshDev &m, int64_t K, const double *t, double J[3][3])
{
    if constexpr (KIND == MESH_DISPLACED) {
        double X[8][3], x[3];
        cell_vertices<D>(m, K, X);
        q1_map<D>(X, t, x, J);
    } else {
        double x0[3], h[3];
        cell_box<KIND>(m, K, x0, h);
        for (int a = 0; a < 3; ++a)
            for (int r = 0; r < 3; ++r) J[a][r] = (a == r) ? h[a] : 0.0;
    }
}

// Inverse map: Newton from the cell centre (1 exact step on affine cells).
template <int D, int KIND>
__device__ __forceinline__ bool map_to_ref(const MeshDev &m, int64_t K, const double *x, double *t)
{
    if constexpr (KIND == MESH_DISPLACED) {
        double X[8][3];
        cell_vertices<D>(m, K, X);
        for (int a = 0; a < D; ++a) t[a] = 0.5;
        for (int it = 0; it < 12; ++it) {
            double y[3], J[3][3], r[3], s[3];
            q1_map<D>(X, t, y, J);
            for (int a = 0; a < D; ++a) r[a] = y[a] - x[a];
            if (!solve_small<D>(J, r, s)) return false;
            double dmax = 0.0;
            for (int a = 0; a < D; ++a) {
                t[a] -= s[a];
                dmax = fmax(dmax, fabs(s[a]));
            }
            if (dmax < 1e-14) return true;
        }
        return false;
    } else {
        double x0[3], h[3];
        cell_box<KIND>(m, K, x0, h);
        for (int a = 0; a < D; ++a) t[a] = (x[a] - x0[a]) / h[a];
        return true;
    }
}

// Is axis a of cell K on the upper face of the domain?
template <int KIND>
__device__ __forceinline__ bool on_upper_face(const MeshDev &m, int64_t K, int a)
{
    if constexpr (KIND == MESH_OCTREE) {
        int s = 1 << (m.max_level - (int)m.level[K]);
        return m.anchor[a * m.n_cells + K] + s == (1 << m.max_level);
    } else {
        int ijk[3];
        cell_ijk(m, K, ijk);
        return ijk[a] == m.n[a] - 1;
    }
}

// Half-open in-cell test of reference coordinates.
template <int D, int KIND>
__device__ __forceinline__ bool ref_inside(const MeshDev &m, int64_t K, const double *t)
{
    for (int a = 0; a < D; ++a) {
        if (!(t[a] >= 0.0)) return false;
        if (t[a] < 1.0) continue;
        if (t[a] == 1.0 && on_upper_face<KIND>(m, K, a)) continue;
        return false;
    }
    return true;
}

template <int D> __device__ __forceinline__ double face_dist(const double *t)
{
    double d = fmin(t[0], 1.0 - t[0]);
    for (int a = 1; a < D; ++a) d = fmin(d, fmin(t[a], 1.0 - t[a]));
    return d;
}

template <int D> __device__ __forceinline__ bool in_box_domain(const MeshDev &m, const double *y)
{
    for (int a = 0; a < D; ++a)
        if (!(y[a] >= m.lo[a] && y[a] <= m.hi[a])) return false;
    return true;
}

template <int D> __device__ __forceinline__ bool near_boundary(const MeshDev &m, const double *y)
{
    bool nb = false;
    for (int a = 0; a < D; ++a)
        nb |= (int)(fabs(y[a] - m.lo[a]) < m.bnd_tol[a]) | (int)(fabs(y[a] - m.hi[a]) < m.bnd_tol[a]);
    return nb;
}

// Location statistics gathered per thread.
// first_try: searches whose first candidate held the point; fallback:
// searches that ended in the global search; searched: candidate cells tried;
// searches: points not in their hint cell (each starts one search).
struct LocStats {
    int first_try, fallback, newton_fail, searched, searches;
};

// Global search of a displaced mesh: every cell whose bounding box (+1e-10)
// holds y; first pass half-open, second pass closed with tolerance 1e-12,
// taking the most interior candidate (ties: lowest index).
template <int D>
__device__ bool global_search_displaced(const MeshDev &m, const double *y, int32_t &K, double *t, LocStats &ls)
{
    for (int pass = 0; pass < 2; ++pass) {
        int64_t best = -1;
        double best_d = -1.0, bt[3] = {0, 0, 0};
        for (int64_t c = 0; c < m.n_cells; ++c) {
            double X[8][3];
            cell_vertices<D>(m, c, X);
            bool inbox = true;
            for (int a = 0; a < D; ++a) {
                double mn = X[0][a], mx = X[0][a];
                for (int v = 1; v < (1 << D); ++v) {
                    mn = fmin(mn, X[v][a]);
                    mx = fmax(mx, X[v][a]);
                }
                inbox &= (y[a] >= mn - 1e-10) && (y[a] <= mx + 1e-10);
            }
            if (!inbox) continue;
            double tt[3];
            if (!map_to_ref<D, MESH_DISPLACED>(m, c, y, tt)) {
                ls.newton_fail++;
                continue;
            }
            if (pass == 0) {
                if (ref_inside<D, MESH_DISPLACED>(m, c, tt)) {
                    K = (int32_t)c;
                    for (int a = 0; a < D; ++a) t[a] = tt[a];
                    return true;
                }
            } else {
                bool ok = true;
                for (int a = 0; a < D; ++a) ok &= (tt[a] >= -1e-12) && (tt[a] <= 1.0 + 1e-12);
                double fd = face_dist<D>(tt);
                if (ok && fd > best_d) {
                    best = c;
                    best_d = fd;
                    for (int a = 0; a < D; ++a) bt[a] = tt[a];
                }
            }
        }
        if (pass == 1 && best >= 0) {
            K = (int32_t)best;
            for (int a = 0; a < D; ++a) t[a] = bt[a];
            return true;
        }
    }
    return false;
}

// Octree global search: lookup on the finest-level grid.
__device__ __forceinline__ int32_t octree_lookup(const MeshDev &m, const double *y)
{
    const int fine = 1 << m.max_level;
    int64_t f[3];
    for (int a = 0; a < 3; ++a) {
        int64_t i = (int64_t)floor((y[a] - m.lo[a]) * m.inv_fine_h[a]);
        f[a] = i < 0 ? 0 : (i >= fine ? fine - 1 : i);
    }
    return m.fine[f[0] + (int64_t)fine * (f[1] + (int64_t)fine * f[2])];
}

// Cell centre (for the a.b search order).
template <int D, int KIND>
__device__ __forceinline__ void cell_centre(const MeshDev &m, int64_t K, double *c)
{
    double t[3] = {0.5, 0.5, 0.5};
    map_to_real<D, KIND>(m, K, t, c);
}

// Closest vertex of cell K to y.
template <int D, int KIND>
__device__ __forceinline__ int closest_vertex(const MeshDev &m, int64_t K, const double *y, double *v)
{
    double best = 1e300;
    int corner = 0;
    for (int q = 0; q < (1 << D); ++q) {
        double t[3] = {(double)(q & 1), (double)((q >> 1) & 1), (double)((q >> 2) & 1)};
        double p[3];
        map_to_real<D, KIND>(m, K, t, p);
        double d = 0.0;
        for (int a = 0; a < D; ++a) d += (p[a] - y[a]) * (p[a] - y[a]);
        if (d < best) {
            best = d;
            corner = q;
            for (int a = 0; a < D; ++a) v[a] = p[a];
        }
    }
    return corner;
}

/*
 * Locate y starting from cell `hint`.  Uniform meshes: closed form (the cell is
 * floor((y - lo)/h); the result equals what the neighbour search would find
 * since the owning cell is unique).  Displaced and octree meshes: in-cell test
 * of the hint; then the cells that share the hint's vertex v closest to y, in
 * descending order of (y - v).(c_K' - v); then the global search (brute force
 * on displaced meshes, the finest-level lookup table on octrees).  Returns
 * false when y is outside the closed domain.
 */
template <int D, int KIND>
__device__ __forceinline__ bool locate(const MeshDev &m, const double *y, int32_t hint, int32_t &K, double *t,
                                       LocStats &ls)
{
    if (!in_box_domain<D>(m, y)) return false;
    if constexpr (KIND == MESH_UNIFORM) {
        int64_t c = 0, stride = 1;
        for (int a = 0; a < D; ++a) {
            double s = (y[a] - m.lo[a]) * m.inv_h[a];
            int i = (int)floor(s);
            i = i >= m.n[a] ? m.n[a] - 1 : (i < 0 ? 0 : i);
            double x0 = m.lo[a] + (double)i * m.h[a];
            t[a] = (y[a] - x0) * m.inv_h[a];
            c += (int64_t)i * stride;
            stride *= m.n[a];
        }
        K = (int32_t)c;
        return true;
    } else {
        double tt[3];
        bool conv = map_to_ref<D, KIND>(m, hint, y, tt);
        if (!conv) ls.newton_fail++;
        if (conv && ref_inside<D, KIND>(m, hint, tt)) {
            K = hint;
            for (int a = 0; a < D; ++a) t[a] = tt[a];
            return true;
        }
        ls.searches++;
        // Cells sharing the hint's vertex v closest to y, in descending order
        // of a.b with a = y - v and b = c_K' - v (ties: lower cell index
        // first), then the global search.  The order is walked without a
        // candidate list: each try takes the best candidate after the
        // previous one.
        double v[3], av[3];
        const int corner = closest_vertex<D, KIND>(m, hint, y, v);
        for (int a = 0; a < D; ++a) av[a] = y[a] - v[a];
        double ps = 0.0;
        int32_t pc = -1;
        for (int tried = 0; tried < (1 << D); ++tried) {
            int32_t bc = -1;
            double bs = 0.0;
            auto consider = [&](int32_t c) {
                double cc[3];
                cell_centre<D, KIND>(m, c, cc);
                double sc = 0.0;
                for (int a = 0; a < D; ++a) sc += av[a] * (cc[a] - v[a]);
                const bool after = pc < 0 || sc < ps || (sc == ps && c > pc);
                if (after && (bc < 0 || sc > bs || (sc == bs && c < bc))) {
                    bc = c;
                    bs = sc;
                }
            };
            if constexpr (KIND == MESH_OCTREE) {
                // v on the finest lattice; the leaves sharing v are those
                // holding the (up to) eight finest cells around it
                const int n = (int)m.n_cells, fine = 1 << m.max_level;
                const int sh = 1 << (m.max_level - (int)m.level[hint]);
                int vi[3];
                for (int a = 0; a < 3; ++a) vi[a] = m.anchor[a * n + hint] + ((corner >> a) & 1) * sh;
                for (int o = 0; o < 8; ++o) {
                    const int f0 = vi[0] - 1 + (o & 1), f1 = vi[1] - 1 + ((o >> 1) & 1), f2 = vi[2] - 1 + (o >> 2);
                    if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= fine || f1 >= fine || f2 >= fine) continue;
                    const int32_t c = m.fine[f0 + (int64_t)fine * (f1 + (int64_t)fine * f2)];
                    if (c != hint) consider(c);
                }
            } else {
                // structured: the neighbours across v are offset by 0 or by
                // the direction of v's corner along each axis
                int ijk[3];
                cell_ijk(m, hint, ijk);
                for (int pat = 1; pat < (1 << D); ++pat) {
                    int q[3] = {ijk[0], ijk[1], ijk[2]};
                    bool ok = true;
                    for (int a = 0; a < D; ++a) {
                        if ((pat >> a) & 1) q[a] += ((corner >> a) & 1) ? 1 : -1;
                        ok &= (q[a] >= 0) & (q[a] < m.n[a]);
                    }
                    if (ok) consider((int32_t)(q[0] + (int64_t)m.n[0] * (q[1] + (int64_t)m.n[1] * q[2])));
                }
            }
            if (bc < 0) break;
            ls.searched++;
            if (!map_to_ref<D, KIND>(m, bc, y, tt)) {
                ls.newton_fail++;
            } else if (ref_inside<D, KIND>(m, bc, tt)) {
                if (tried == 0) ls.first_try++;
                K = bc;
                for (int a = 0; a < D; ++a) t[a] = tt[a];
                return true;
            }
            ps = bs;
            pc = bc;
        }
        ls.fallback++;
        if constexpr (KIND == MESH_OCTREE) {
            const int32_t c = octree_lookup(m, y);
            map_to_ref<D, KIND>(m, c, y, tt);
            K = c;
            for (int a = 0; a < D; ++a) t[a] = tt[a];
            return true;
        } else {
            return global_search_displaced<D>(m, y, K, t, ls);
        }
    }
}

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

// Reference gradient Gr[c][r] = d u_c / d xhat_r of the Q2 field on a node
// grid (base / sy / sz as in eval_q2_at), accumulated in T.
template <int D, typename T, typename Ptr, typename I>
__device__ __forceinline__ void grad_q2_at(Ptr U, I base, I sy, I sz, const double *tr, double Gr[3][3])
{
    T l[3][3], dl[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        lag3((T)tr[a], l[a]);
        dlag3((T)tr[a], dl[a]);
    }
    T g[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) g[c][r] = T(0);
#pragma unroll 1
    for (int c3 = 0; c3 < (D == 3 ? 3 : 1); ++c3) {
#if PIC_EVAL_BATCH
        // the plane's nine nodes are requested before the first is used
        T px[3][3], py[3][3], pz[3][3];
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const auto v = U[base + a + sy * b + sz * c3];
                px[b][a] = (T)nv_x(v);
                py[b][a] = (T)nv_y(v);
                pz[b][a] = D == 3 ? (T)nv_z(v) : T(0);
            }
        __builtin_amdgcn_sched_barrier(0);
#endif
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
#if !PIC_EVAL_BATCH
                const auto v = U[base + a + sy * b + sz * c3];
#endif
                T w[3];
                if constexpr (D == 2) {
                    w[0] = dl[0][a] * l[1][b];
                    w[1] = l[0][a] * dl[1][b];
                    w[2] = T(0);
                } else {
                    w[0] = dl[0][a] * l[1][b] * l[2][c3];
                    w[1] = l[0][a] * dl[1][b] * l[2][c3];
                    w[2] = l[0][a] * l[1][b] * dl[2][c3];
                }
#if PIC_EVAL_BATCH
                const T vc[3] = {px[b][a], py[b][a], pz[b][a]};
#else
                const T vc[3] = {(T)nv_x(v), (T)nv_y(v), D == 3 ? (T)nv_z(v) : T(0)};
#endif
#pragma unroll
                for (int c = 0; c < D; ++c)
#pragma unroll
                    for (int r = 0; r < D; ++r) g[c][r] = fma_t(vc[c], w[r], g[c][r]);
            }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) Gr[c][r] = (double)g[c][r];
}

// Property equations integrated along the trajectory (Sec. 2.6), at a point
// with velocity gradient G[i][j] = d u_i / d x_j:
//   damage d' = alpha |eps| - beta d, eps = (G + G^T)/2, |.| Frobenius norm;
//   deformation gradient F' = G F (F row-major, D x D).
template <int D>
__device__ __forceinline__ void prop_rates(const double G[3][3], double alpha, double beta, double dmg, const double *F,
                                           double &ddmg, double *dF)
{
    double e2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double e = 0.5 * (G[i][j] + G[j][i]);
            e2 = fma(e, e, e2);
        }
    ddmg = alpha * sqrt(e2) - beta * dmg;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) acc = fma(G[i][k], F[k * D + j], acc);
            dF[i * D + j] = acc;
        }
}

// ---------------------------------------------------------------------------
// XCD-aware work mapping.  Workgroups are dealt to the eight XCDs round robin
// (workgroup b runs on XCD b mod 8) and each XCD has its own L2.  Workgroup b
// takes item (b mod 8) * ceil(n/8) + b / 8, so every XCD walks one contiguous
// eighth of a spatially ordered work list: neighbouring items (shared halo
// nodes, particles moving between neighbouring cells, cache lines split
// between neighbouring segments) meet in the same L2.  Launch xcd_span(n)
// workgroups; items >= n are skipped.
// ---------------------------------------------------------------------------
constexpr int N_XCD = 8;
__host__ __device__ inline int xcd_span(int n) { return N_XCD * ((n + N_XCD - 1) / N_XCD); }
__device__ __forceinline__ int xcd_item(int b, int n) { return (b % N_XCD) * ((n + N_XCD - 1) / N_XCD) + b / N_XCD; }

// ---------------------------------------------------------------------------
// workgroup helpers
// ---------------------------------------------------------------------------
// Sum of an int over a wavefront.
__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace pic
