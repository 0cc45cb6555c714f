/*
 * Plain FP64 CPU oracle of the particle-in-cell hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: it exists so that tests, the smoke check and the CPU-baseline
 * leg of the benchmark can compare the GPU library against an independent,
 * obviously correct implementation.  It shares no code, header or table with
 * the GPU library.
 *
 * Everything is double precision and written as plain loops in the order the
 * method states them (Gassmoeller, Heien, Puckett, Bangerth, "Flexible and
 * scalable particle-in-cell methods for massively parallel computations"):
 *
 *   - particle = (id, location, reference location, properties)       Sec. 2.1
 *   - stored reference location kept in sync with the location         Sec. 2.1, remark on reference coordinates
 *   - reference-local generation: x = Phi_K(xhat), only Phi_K needed   Sec. 2.2, remark on local generation
 *   - forward Euler / RK2 / RK4                                        Sec. 2.3 (readings below)
 *   - field interpolated linearly in time between u^n and u^{n+1},
 *     particle steps that sub-divide the field step                   Sec. 2.3
 *   - field evaluation through the shape functions on the reference cell  Sec. 2.3
 *   - in-cell test after every (sub)step via xhat in Khat              Sec. 2.4
 *   - discard particles leaving the domain (option 3)                  Sec. 2.4
 *   - batched re-insertion of movers (order: stayers, then arrivals)   Sec. 2.4
 *   - population management (add in sparse, remove in dense cells)     Sec. 2.5
 *   - properties of new particles from existing ones                   Sec. 2.6
 *   - particle -> cell interpolation: arithmetic average               Sec. 2.7 (ii)
 *
 * Readings where the paper is garbled or silent (each is listed with its
 * justification in the design notes of the repository):
 *   RK2: explicit midpoint, k1 = dt u(x), x+ = x + dt u(x + k1/2)
 *        (the printed form halves the step twice and would be first order).
 *   RK4: classical RK4 with every k_i = dt u(.) (the printed k2, k3 carry an
 *        extra 1/2 which breaks consistency under a constant field).
 *   Any stage point or end point outside the closed domain: particle lost.
 *   Owning cell: half-open rule 0 <= xhat_i < 1, with xhat_i <= 1 allowed on
 *        the upper faces of the domain.
 *   Order within a cell: stable sort of the pre-step order by (new cell, moved).
 *   Inverse map on displaced (bilinear/trilinear) cells: Newton from the cell
 *        centre, stop at |dxhat|_inf < 1e-14 or 12 iterations.
 *   Population: delete the largest ids above max; add min-n particles at
 *        SplitMix64-hashed reference coordinates; new ids by a scan over cells
 *        in index order; new properties = mean of the cell's survivors, or the
 *        initial function (initial position) for an empty cell.
 *   Adjoint: reverse sweep of the RK stages for L = (1/Nv) sum |x(T) - x*|^2.
 *   Time interpolation: the two fields are evaluated at the point and combined,
 *        u~(x, t) = u^n(x) + theta (u^{n+1}(x) - u^n(x)), theta = (t - t^n) / dt_u;
 *        stage times t + 0, dt/2 (RK2; RK4 stages 2 and 3), dt (RK4 stage 4),
 *        with t the particle step's start; theta > 1 extrapolates.
 *
 * Meshes:
 *   kind 0: uniform box mesh, closed-form locate by floor.
 *   kind 1: displaced structured grid (bi/trilinear cells), brute-force locate
 *           over all cells with Newton inversion (small meshes only).
 *   kind 2: 2:1-balanced octree of axis-aligned boxes on the unit cube, locate
 *           by a lookup on the finest-level grid.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LOST 0xFFFFFFFFu
#define NEAR_FACE_TOL 1e-10

typedef struct {
    int dim;
    int kind;               /* 0 uniform, 1 displaced structured, 2 octree */
    int n[3];               /* structured: cells per axis */
    double lo[3], hi[3];
    const double *vert;     /* kind 1: vertex coordinates [dim][n_vertices] */
    /* kind 2 */
    int64_t n_cells;
    int max_level;
    const uint8_t *level;   /* [n_cells] */
    const int32_t *anchor;  /* [3][n_cells], finest-level units */
    const int32_t *fine_to_leaf;   /* [(2^max_level)^3] */
    const int32_t *cell_nodes;     /* [n_cells][27] global Q2 node index */
} orc_mesh;

/* ------------------------------------------------------------------ */
/* mesh helpers                                                        */
/* ------------------------------------------------------------------ */
static int nloc(int dim) { return dim == 2 ? 9 : 27; }
static int nvert(int dim) { return dim == 2 ? 4 : 8; }

int64_t orc_n_cells(const orc_mesh *m)
{
    if (m->kind == 2) return m->n_cells;
    int64_t c = 1;
    for (int a = 0; a < m->dim; ++a) c *= m->n[a];
    return c;
}

static void cell_ijk(const orc_mesh *m, int64_t c, int ijk[3])
{
    ijk[0] = (int)(c % m->n[0]);
    ijk[1] = (int)((c / m->n[0]) % m->n[1]);
    ijk[2] = m->dim == 3 ? (int)(c / ((int64_t)m->n[0] * m->n[1])) : 0;
}

/* global index of local Q2 node (a,b,c) of cell K (structured numbering) */
static int64_t q2_node(const orc_mesh *m, int64_t K, int loc)
{
    if (m->kind == 2) return m->cell_nodes[K * 27 + loc];
    int ijk[3];
    cell_ijk(m, K, ijk);
    int a = loc % 3, b = (loc / 3) % 3, c = loc / 9;
    int64_t nx = 2 * m->n[0] + 1, ny = 2 * m->n[1] + 1;
    return (2 * ijk[0] + a) + nx * ((2 * ijk[1] + b) + ny * (int64_t)(2 * ijk[2] + c));
}

/* box of an axis-aligned cell (uniform or octree): lower corner and edge lengths */
static void cell_box(const orc_mesh *m, int64_t K, double x0[3], double h[3])
{
    if (m->kind == 2) {
        double fine = (double)(1 << m->max_level);
        double sz = (double)(1 << (m->max_level - m->level[K])) / fine;
        for (int a = 0; a < 3; ++a) {
            double L = m->hi[a] - m->lo[a];
            x0[a] = m->lo[a] + L * (m->anchor[a * m->n_cells + K] / fine);
            h[a] = L * sz;
        }
        return;
    }
    int ijk[3];
    cell_ijk(m, K, ijk);
    for (int a = 0; a < 3; ++a) {
        h[a] = (m->hi[a] - m->lo[a]) / m->n[a];
        x0[a] = m->lo[a] + ijk[a] * h[a];
    }
}

/* vertices of a displaced structured cell: X[v][axis], v = va + 2 vb + 4 vc */
static void cell_vertices(const orc_mesh *m, int64_t K, double X[8][3])
{
    int ijk[3];
    cell_ijk(m, K, ijk);
    int64_t nvx = m->n[0] + 1, nvy = m->n[1] + 1;
    int64_t nv = nvx * nvy * (m->dim == 3 ? (m->n[2] + 1) : 1);
    for (int v = 0; v < nvert(m->dim); ++v) {
        int va = v & 1, vb = (v >> 1) & 1, vc = (v >> 2) & 1;
        int64_t g = (ijk[0] + va) + nvx * ((ijk[1] + vb) + nvy * (int64_t)(ijk[2] + vc));
        for (int a = 0; a < m->dim; ++a) X[v][a] = m->vert[a * nv + g];
    }
}

/* bilinear/trilinear shape function of vertex v and its gradient */
static double q1_shape(int dim, int v, const double *t, double *grad)
{
    double f[3], df[3];
    for (int a = 0; a < dim; ++a) {
        int bit = (v >> a) & 1;
        f[a] = bit ? t[a] : 1.0 - t[a];
        df[a] = bit ? 1.0 : -1.0;
    }
    double val = 1.0;
    for (int a = 0; a < dim; ++a) val *= f[a];
    if (grad)
        for (int r = 0; r < dim; ++r) {
            double g = df[r];
            for (int a = 0; a < dim; ++a)
                if (a != r) g *= f[a];
            grad[r] = g;
        }
    return val;
}

/* Phi_K(xhat) and its Jacobian J[axis][ref] */
static void map_to_real(const orc_mesh *m, int64_t K, const double *xr, double *x, double J[3][3])
{
    int d = m->dim;
    if (m->kind != 1) {
        double x0[3], h[3];
        cell_box(m, K, x0, h);
        for (int a = 0; a < d; ++a) {
            x[a] = x0[a] + xr[a] * h[a];
            if (J)
                for (int r = 0; r < d; ++r) J[a][r] = (a == r) ? h[a] : 0.0;
        }
        return;
    }
    double X[8][3];
    cell_vertices(m, K, X);
    for (int a = 0; a < d; ++a) {
        x[a] = 0.0;
        if (J)
            for (int r = 0; r < d; ++r) J[a][r] = 0.0;
    }
    for (int v = 0; v < nvert(d); ++v) {
        double g[3];
        double N = q1_shape(d, v, xr, g);
        for (int a = 0; a < d; ++a) {
            x[a] += N * X[v][a];
            if (J)
                for (int r = 0; r < d; ++r) J[a][r] += g[r] * X[v][a];
        }
    }
}

void orc_map_to_real(const orc_mesh *m, int64_t K, const double *xr, double *x)
{
    map_to_real(m, K, xr, x, NULL);
}

/* solve J s = r for 2x2 or 3x3 by Cramer's rule; returns 0 if singular */
static int solve_small(int d, double J[3][3], const double *r, double *s)
{
    if (d == 2) {
        double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (det == 0.0) return 0;
        s[0] = (r[0] * J[1][1] - J[0][1] * r[1]) / det;
        s[1] = (J[0][0] * r[1] - r[0] * J[1][0]) / det;
        return 1;
    }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (det == 0.0) return 0;
    for (int c = 0; c < 3; ++c) {
        double M[3][3];
        memcpy(M, J, sizeof(M));
        for (int a = 0; a < 3; ++a) M[a][c] = r[a];
        s[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
              - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
              + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
    }
    return 1;
}

/* Newton inversion of Phi_K: returns 1 on convergence */
static int map_to_ref(const orc_mesh *m, int64_t K, const double *x, double *xr)
{
    int d = m->dim;
    if (m->kind != 1) {
        double x0[3], h[3];
        cell_box(m, K, x0, h);
        for (int a = 0; a < d; ++a) xr[a] = (x[a] - x0[a]) / h[a];
        return 1;
    }
    for (int a = 0; a < d; ++a) xr[a] = 0.5;
    for (int it = 0; it < 12; ++it) {
        double y[3], J[3][3], r[3], s[3];
        map_to_real(m, K, xr, y, J);
        for (int a = 0; a < d; ++a) r[a] = y[a] - x[a];
        if (!solve_small(d, J, r, s)) return 0;
        double dmax = 0.0;
        for (int a = 0; a < d; ++a) {
            xr[a] -= s[a];
            if (fabs(s[a]) > dmax) dmax = fabs(s[a]);
        }
        if (dmax < 1e-14) return 1;
    }
    return 0;
}

/* is axis a of cell K on the upper face of the domain? */
static int on_upper_face(const orc_mesh *m, int64_t K, int a)
{
    if (m->kind == 2) {
        int fine = 1 << m->max_level;
        int sz = 1 << (m->max_level - m->level[K]);
        return m->anchor[a * m->n_cells + K] + sz == fine;
    }
    int ijk[3];
    cell_ijk(m, K, ijk);
    return ijk[a] == m->n[a] - 1;
}

/* half-open in-cell test of a reference point */
static int ref_inside(const orc_mesh *m, int64_t K, const double *xr)
{
    for (int a = 0; a < m->dim; ++a) {
        if (!(xr[a] >= 0.0)) return 0;
        if (xr[a] < 1.0) continue;
        if (xr[a] == 1.0 && on_upper_face(m, K, a)) continue;
        return 0;
    }
    return 1;
}

static double face_distance(int dim, const double *xr)
{
    double d = 1.0;
    for (int a = 0; a < dim; ++a) {
        double t = fmin(xr[a], 1.0 - xr[a]);
        if (t < d) d = t;
    }
    return d;
}

/* Locate x: returns 1 and sets (cell, xr) if x is in the closed domain, else 0. */
int orc_locate(const orc_mesh *m, const double *x, int32_t *cell, double *xr)
{
    int d = m->dim;
    if (m->kind == 0 || m->kind == 2) {
        for (int a = 0; a < d; ++a)
            if (!(x[a] >= m->lo[a] && x[a] <= m->hi[a])) return 0;
    }
    if (m->kind == 0) {
        int64_t K = 0, stride = 1;
        for (int a = 0; a < d; ++a) {
            double h = (m->hi[a] - m->lo[a]) / m->n[a];
            int64_t i = (int64_t)floor((x[a] - m->lo[a]) / h);
            if (i >= m->n[a]) i = m->n[a] - 1;      /* upper face of the domain */
            if (i < 0) i = 0;
            K += i * stride;
            stride *= m->n[a];
        }
        *cell = (int32_t)K;
        map_to_ref(m, K, x, xr);
        return 1;
    }
    if (m->kind == 2) {
        int fine = 1 << m->max_level;
        int64_t f[3];
        for (int a = 0; a < 3; ++a) {
            double L = m->hi[a] - m->lo[a];
            int64_t i = (int64_t)floor((x[a] - m->lo[a]) / L * fine);
            if (i >= fine) i = fine - 1;
            if (i < 0) i = 0;
            f[a] = i;
        }
        int64_t K = m->fine_to_leaf[f[0] + fine * (f[1] + (int64_t)fine * f[2])];
        *cell = (int32_t)K;
        map_to_ref(m, K, x, xr);
        return 1;
    }
    /* kind 1: brute force over every cell, bounding boxes enlarged by 1e-10 */
    int64_t nc = orc_n_cells(m);
    int64_t best = -1;
    double best_dist = -1.0, best_xr[3] = {0, 0, 0};
    for (int pass = 0; pass < 2 && best < 0; ++pass) {
        for (int64_t K = 0; K < nc; ++K) {
            double X[8][3], bmin[3], bmax[3];
            cell_vertices(m, K, X);
            for (int a = 0; a < d; ++a) {
                bmin[a] = bmax[a] = X[0][a];
                for (int v = 1; v < nvert(d); ++v) {
                    if (X[v][a] < bmin[a]) bmin[a] = X[v][a];
                    if (X[v][a] > bmax[a]) bmax[a] = X[v][a];
                }
            }
            int inbox = 1;
            for (int a = 0; a < d; ++a)
                if (x[a] < bmin[a] - 1e-10 || x[a] > bmax[a] + 1e-10) inbox = 0;
            if (!inbox) continue;
            double t[3];
            if (!map_to_ref(m, K, x, t)) continue;
            if (pass == 0) {
                if (ref_inside(m, K, t)) {
                    best = K;
                    memcpy(best_xr, t, sizeof(t));
                    break;
                }
            } else {
                int ok = 1;
                for (int a = 0; a < d; ++a)
                    if (t[a] < -1e-12 || t[a] > 1.0 + 1e-12) ok = 0;
                double fd = face_distance(d, t);
                if (ok && fd > best_dist) {
                    best = K;
                    best_dist = fd;
                    memcpy(best_xr, t, sizeof(t));
                }
            }
        }
    }
    if (best < 0) return 0;
    *cell = (int32_t)best;
    memcpy(xr, best_xr, sizeof(double) * d);
    return 1;
}

/* distance of x to the boundary of the box domain relative to the smallest h */
static int near_boundary(const orc_mesh *m, const double *x)
{
    for (int a = 0; a < m->dim; ++a) {
        double h = (m->kind == 2) ? (m->hi[a] - m->lo[a]) / (1 << m->max_level)
                                  : (m->hi[a] - m->lo[a]) / m->n[a];
        if (fabs(x[a] - m->lo[a]) < NEAR_FACE_TOL * h || fabs(x[a] - m->hi[a]) < NEAR_FACE_TOL * h)
            return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Q2 field                                                            */
/* ------------------------------------------------------------------ */
static void lagrange_q2(double t, double l[3], double dl[3])
{
    l[0] = (1.0 - t) * (1.0 - 2.0 * t);
    l[1] = 4.0 * t * (1.0 - t);
    l[2] = t * (2.0 * t - 1.0);
    if (dl) {
        dl[0] = 4.0 * t - 3.0;
        dl[1] = 4.0 - 8.0 * t;
        dl[2] = 4.0 * t - 1.0;
    }
}

/* value of local basis function loc at xr, and optionally its reference gradient */
static double q2_basis(int dim, int loc, const double *xr, double *grad)
{
    double l[3][3], dl[3][3];
    for (int a = 0; a < dim; ++a) lagrange_q2(xr[a], l[a], dl[a]);
    int idx[3] = {loc % 3, (loc / 3) % 3, loc / 9};
    double v = 1.0;
    for (int a = 0; a < dim; ++a) v *= l[a][idx[a]];
    if (grad)
        for (int r = 0; r < dim; ++r) {
            double g = dl[r][idx[r]];
            for (int a = 0; a < dim; ++a)
                if (a != r) g *= l[a][idx[a]];
            grad[r] = g;
        }
    return v;
}

/* u(x) = sum over the 3^d local nodes of U[node] * phi(xhat): naive sum */
void orc_eval(const orc_mesh *m, const double *U, int64_t n_nodes, int64_t K, const double *xr, double *u)
{
    int d = m->dim;
    for (int c = 0; c < d; ++c) u[c] = 0.0;
    for (int loc = 0; loc < nloc(d); ++loc) {
        double phi = q2_basis(d, loc, xr, NULL);
        int64_t g = q2_node(m, K, loc);
        for (int c = 0; c < d; ++c) u[c] += U[c * n_nodes + g] * phi;
    }
}

/* physical gradient G[c][j] = d u_c / d x_j = (d u_c / d xhat) J^{-1} */
static void eval_grad(const orc_mesh *m, const double *U, int64_t n_nodes, int64_t K, const double *xr,
                      double G[3][3])
{
    int d = m->dim;
    double Gr[3][3] = {{0}};
    for (int loc = 0; loc < nloc(d); ++loc) {
        double g[3];
        q2_basis(d, loc, xr, g);
        int64_t node = q2_node(m, K, loc);
        for (int c = 0; c < d; ++c)
            for (int r = 0; r < d; ++r) Gr[c][r] += U[c * n_nodes + node] * g[r];
    }
    double x[3], J[3][3];
    map_to_real(m, K, xr, x, J);
    /* G = Gr J^{-1}: solve J^T G^T = Gr^T row by row */
    for (int c = 0; c < d; ++c) {
        double JT[3][3], s[3];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) JT[a][b] = J[b][a];
        solve_small(d, JT, Gr[c], s);
        for (int j = 0; j < d; ++j) G[c][j] = s[j];
    }
}

/*
 * Velocity over one field step (Sec. 2.3): u^n = U0 and, when the field
 * changes in time, u^{n+1} = U1 (NULL: steady field).  `since` is the time
 * elapsed since t^n; the two fields are evaluated at the point and combined
 * linearly in time.
 */
typedef struct {
    const double *U0, *U1;
    int64_t nn;
    double dt_u;
} orc_field;

static void field_eval(const orc_mesh *m, const orc_field *f, double since, int64_t K, const double *xr, double *u)
{
    orc_eval(m, f->U0, f->nn, K, xr, u);
    if (!f->U1) return;
    double u1[3];
    orc_eval(m, f->U1, f->nn, K, xr, u1);
    double theta = since / f->dt_u;
    for (int a = 0; a < m->dim; ++a) u[a] = u[a] + theta * (u1[a] - u[a]);
}

static void field_grad(const orc_mesh *m, const orc_field *f, double since, int64_t K, const double *xr,
                       double G[3][3])
{
    eval_grad(m, f->U0, f->nn, K, xr, G);
    if (!f->U1) return;
    double G1[3][3];
    eval_grad(m, f->U1, f->nn, K, xr, G1);
    double theta = since / f->dt_u;
    for (int c = 0; c < m->dim; ++c)
        for (int j = 0; j < m->dim; ++j) G[c][j] = G[c][j] + theta * (G1[c][j] - G[c][j]);
}

/* ------------------------------------------------------------------ */
/* store                                                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n, cap;
    int dim, n_prop;
    double *x;      /* [dim][cap] */
    double *xr;     /* [dim][cap] */
    int32_t *cell;  /* [cap] */
    uint32_t *id;   /* [cap] */
    double *prop;   /* [n_prop][cap] */
} orc_store;

typedef struct {
    int64_t live, lost, moved, near_face;
} orc_stats;

/* Reference-local generation: particles listed cell by cell; x = Phi_K(xhat).
   Property j of a new particle is its initial coordinate j (if init_position). */
int orc_seed(const orc_mesh *m, const int32_t *counts, const double *xr_in, int64_t n_in,
             const uint32_t *ids, int init_position, orc_store *s)
{
    int d = m->dim;
    int64_t nc = orc_n_cells(m), p = 0;
    if (n_in > s->cap) return -1;
    for (int64_t K = 0; K < nc; ++K)
        for (int32_t k = 0; k < counts[K]; ++k, ++p) {
            double t[3], x[3];
            for (int a = 0; a < d; ++a) t[a] = xr_in[a * n_in + p];
            map_to_real(m, K, t, x, NULL);
            for (int a = 0; a < d; ++a) {
                s->x[a * s->cap + p] = x[a];
                s->xr[a * s->cap + p] = t[a];
            }
            s->cell[p] = (int32_t)K;
            s->id[p] = ids[p];
            if (init_position)
                for (int j = 0; j < s->n_prop; ++j) s->prop[j * s->cap + p] = x[j % d];
        }
    s->n = p;
    return 0;
}

/* u at an arbitrary point and time: locate, then evaluate.  Returns 0 if outside. */
static int velocity_at(const orc_mesh *m, const orc_field *f, double since, const double *y, double *u,
                       int32_t *cell_out, double *xr_out)
{
    int32_t K;
    double t[3];
    if (!orc_locate(m, y, &K, t)) return 0;
    field_eval(m, f, since, K, t, u);
    if (cell_out) *cell_out = K;
    if (xr_out) memcpy(xr_out, t, sizeof(double) * m->dim);
    return 1;
}

/*
 * Advance one particle by one step of length dt that starts `since` after
 * t^n.  Stage 1 uses the stored (K, xhat) without a locate.  Returns 1 if the
 * particle survives; sets *near if any stage point or the end point is within
 * the near-face band.
 */
static int advect_one(const orc_mesh *m, const orc_field *f, double since, double dt, int scheme,
                      const double *x, int32_t K, const double *xr,
                      double *xn, int32_t *Kn, double *xrn, int *near)
{
    int d = m->dim;
    double k1[3], k2[3], k3[3], k4[3], y[3], u[3];
    *near = 0;
    field_eval(m, f, since, K, xr, u);
    for (int a = 0; a < d; ++a) k1[a] = dt * u[a];
    if (scheme == 1) {
        for (int a = 0; a < d; ++a) xn[a] = x[a] + k1[a];
    } else if (scheme == 2) {
        for (int a = 0; a < d; ++a) y[a] = x[a] + 0.5 * k1[a];
        if (near_boundary(m, y)) *near = 1;
        if (!velocity_at(m, f, since + 0.5 * dt, y, u, NULL, NULL)) return 0;
        for (int a = 0; a < d; ++a) xn[a] = x[a] + dt * u[a];
    } else {
        for (int a = 0; a < d; ++a) y[a] = x[a] + 0.5 * k1[a];
        if (near_boundary(m, y)) *near = 1;
        if (!velocity_at(m, f, since + 0.5 * dt, y, u, NULL, NULL)) return 0;
        for (int a = 0; a < d; ++a) k2[a] = dt * u[a];
        for (int a = 0; a < d; ++a) y[a] = x[a] + 0.5 * k2[a];
        if (near_boundary(m, y)) *near = 1;
        if (!velocity_at(m, f, since + 0.5 * dt, y, u, NULL, NULL)) return 0;
        for (int a = 0; a < d; ++a) k3[a] = dt * u[a];
        for (int a = 0; a < d; ++a) y[a] = x[a] + k3[a];
        if (near_boundary(m, y)) *near = 1;
        if (!velocity_at(m, f, since + dt, y, u, NULL, NULL)) return 0;
        for (int a = 0; a < d; ++a) k4[a] = dt * u[a];
        for (int a = 0; a < d; ++a)
            xn[a] = x[a] + k1[a] / 6.0 + k2[a] / 3.0 + k3[a] / 3.0 + k4[a] / 6.0;
    }
    if (near_boundary(m, xn)) *near = 1;
    if (!orc_locate(m, xn, Kn, xrn)) return 0;
    if (face_distance(d, xrn) < NEAR_FACE_TOL) *near = 1;
    return 1;
}

/*
 * Advection + location for every particle of the store (no reordering).
 * Writes the new location and reference location in place and the new cell
 * (or ORC_LOST) into key[i]; near[i] = 1 for near-face particles.
 */
static void advect_all(const orc_mesh *m, const orc_field *f, double since, double dt, int scheme,
                       orc_store *s, uint32_t *key, uint8_t *near)
{
    int d = m->dim;
    int64_t cap = s->cap;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->n; ++i) {
        double x[3], t[3], xn[3], tn[3];
        int32_t Kn;
        int nf;
        for (int a = 0; a < d; ++a) {
            x[a] = s->x[a * cap + i];
            t[a] = s->xr[a * cap + i];
        }
        int alive = advect_one(m, f, since, dt, scheme, x, s->cell[i], t, xn, &Kn, tn, &nf);
        near[i] = (uint8_t)nf;
        if (!alive) {
            key[i] = ORC_LOST;
            continue;
        }
        for (int a = 0; a < d; ++a) {
            s->x[a * cap + i] = xn[a];
            s->xr[a * cap + i] = tn[a];
        }
        key[i] = (uint32_t)Kn;
    }
}

void orc_advect(const orc_mesh *m, const double *U, int64_t nn, double dt, int scheme,
                orc_store *s, uint32_t *key, uint8_t *near)
{
    orc_field f = {U, NULL, nn, 1.0};
    advect_all(m, &f, 0.0, dt, scheme, s, key, near);
}

/*
 * orc_advect in a field that changes in time (Sec. 2.3): u^n = U0 at t^n,
 * u^{n+1} = U1 at t^n + dt_u, the particle step [t^n + since, t^n + since + dt]
 * (a sub-step when dt < dt_u).
 */
void orc_advect_t(const orc_mesh *m, const double *U0, const double *U1, int64_t nn, double dt_u, double since,
                  double dt, int scheme, orc_store *s, uint32_t *key, uint8_t *near)
{
    orc_field f = {U0, U1, nn, dt_u};
    advect_all(m, &f, since, dt, scheme, s, key, near);
}

/* ------------------------------------------------------------------ */
/* property equations integrated along the trajectory (Sec. 2.6)        */
/* ------------------------------------------------------------------ */
/*
 * Right-hand sides of the two property equations of Sec. 2.6 at one point
 * with velocity gradient G[i][j] = d u_i / d x_j:
 *   damage       d' = alpha |eps| - beta d,  eps = (G + G^T) / 2,
 *                |eps| the Frobenius norm sqrt(sum_ij eps_ij^2);
 *   deformation  F' = G F  (F row-major, dim x dim).
 */
static void prop_rhs(int dim, const double G[3][3], double alpha, double beta, double dmg, const double *F,
                     double *ddmg, double *dF)
{
    double e2 = 0.0;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double e = 0.5 * (G[i][j] + G[j][i]);
            e2 += e * e;
        }
    *ddmg = alpha * sqrt(e2) - beta * dmg;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double acc = 0.0;
            for (int k = 0; k < dim; ++k) acc += G[i][k] * F[k * dim + j];
            dF[i * dim + j] = acc;
        }
}

/*
 * One step of the coupled system (x, d, F) with the explicit RK scheme of
 * the positions: every stage evaluates u and grad u at the stage point (in
 * the cell the point was located in) and the property right-hand sides at
 * the stage's property values.  Stage 1 uses the stored (K, xhat).
 * P = [d, F_00, F_01, ...] (1 + dim^2 values).
 */
static int advect_one_odes(const orc_mesh *m, const orc_field *f, double since, double dt, int scheme, double alpha,
                           double beta, const double *x, int32_t K, const double *xr, const double *P,
                           double *xn, int32_t *Kn, double *xrn, double *Pn, int *near)
{
    int d = m->dim, np = 1 + d * d;
    int ns = scheme == 1 ? 1 : (scheme == 2 ? 2 : 4);
    double kx[4][3], kP[4][10], y[3], Ps[10], u[3], G[3][3], yr[3];
    int32_t Ky;
    *near = 0;
    for (int s = 0; s < ns; ++s) {
        if (s == 0) {
            field_eval(m, f, since, K, xr, u);
            field_grad(m, f, since, K, xr, G);
            for (int q = 0; q < np; ++q) Ps[q] = P[q];
        } else {
            /* RK2: midpoint; RK4: x + k1/2, x + k2/2, x + k3; the stage's time is t + c dt */
            double c = (scheme == 4 && s == 3) ? 1.0 : 0.5;
            for (int a = 0; a < d; ++a) y[a] = x[a] + c * kx[s - 1][a];
            for (int q = 0; q < np; ++q) Ps[q] = P[q] + c * kP[s - 1][q];
            if (near_boundary(m, y)) *near = 1;
            if (!velocity_at(m, f, since + c * dt, y, u, &Ky, yr)) return 0;
            field_grad(m, f, since + c * dt, Ky, yr, G);
        }
        double dd, dF[9];
        prop_rhs(d, G, alpha, beta, Ps[0], Ps + 1, &dd, dF);
        for (int a = 0; a < d; ++a) kx[s][a] = dt * u[a];
        kP[s][0] = dt * dd;
        for (int q = 0; q < d * d; ++q) kP[s][1 + q] = dt * dF[q];
    }
    if (scheme == 1) {
        for (int a = 0; a < d; ++a) xn[a] = x[a] + kx[0][a];
        for (int q = 0; q < np; ++q) Pn[q] = P[q] + kP[0][q];
    } else if (scheme == 2) {
        for (int a = 0; a < d; ++a) xn[a] = x[a] + kx[1][a];
        for (int q = 0; q < np; ++q) Pn[q] = P[q] + kP[1][q];
    } else {
        for (int a = 0; a < d; ++a) xn[a] = x[a] + kx[0][a] / 6.0 + kx[1][a] / 3.0 + kx[2][a] / 3.0 + kx[3][a] / 6.0;
        for (int q = 0; q < np; ++q) Pn[q] = P[q] + kP[0][q] / 6.0 + kP[1][q] / 3.0 + kP[2][q] / 3.0 + kP[3][q] / 6.0;
    }
    if (near_boundary(m, xn)) *near = 1;
    if (!orc_locate(m, xn, Kn, xrn)) return 0;
    if (face_distance(d, xrn) < NEAR_FACE_TOL) *near = 1;
    return 1;
}

/*
 * orc_advect with the property equations: damage in property damage_prop,
 * the deformation gradient in properties deform_prop .. deform_prop + dim^2 - 1
 * (row-major).  Both must be given (>= 0).
 */
static void advect_odes_all(const orc_mesh *m, const orc_field *f, double since, double dt, int scheme, double alpha,
                            double beta, int damage_prop, int deform_prop, orc_store *s, uint32_t *key, uint8_t *near)
{
    int d = m->dim, np = 1 + d * d;
    int64_t cap = s->cap;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->n; ++i) {
        double x[3], t[3], xn[3], tn[3], P[10], Pn[10];
        int32_t Kn;
        int nf;
        for (int a = 0; a < d; ++a) {
            x[a] = s->x[a * cap + i];
            t[a] = s->xr[a * cap + i];
        }
        P[0] = s->prop[damage_prop * cap + i];
        for (int q = 0; q < d * d; ++q) P[1 + q] = s->prop[(deform_prop + q) * cap + i];
        int alive = advect_one_odes(m, f, since, dt, scheme, alpha, beta, x, s->cell[i], t, P, xn, &Kn, tn, Pn, &nf);
        near[i] = (uint8_t)nf;
        if (!alive) {
            key[i] = ORC_LOST;
            continue;
        }
        for (int a = 0; a < d; ++a) {
            s->x[a * cap + i] = xn[a];
            s->xr[a * cap + i] = tn[a];
        }
        s->prop[damage_prop * cap + i] = Pn[0];
        for (int q = 0; q < d * d; ++q) s->prop[(deform_prop + q) * cap + i] = Pn[1 + q];
        (void)np;
        key[i] = (uint32_t)Kn;
    }
}

void orc_advect_odes(const orc_mesh *m, const double *U, int64_t nn, double dt, int scheme, double alpha, double beta,
                     int damage_prop, int deform_prop, orc_store *s, uint32_t *key, uint8_t *near)
{
    orc_field f = {U, NULL, nn, 1.0};
    advect_odes_all(m, &f, 0.0, dt, scheme, alpha, beta, damage_prop, deform_prop, s, key, near);
}

/* orc_advect_odes in a field that changes in time (as orc_advect_t) */
void orc_advect_odes_t(const orc_mesh *m, const double *U0, const double *U1, int64_t nn, double dt_u, double since,
                       double dt, int scheme, double alpha, double beta, int damage_prop, int deform_prop,
                       orc_store *s, uint32_t *key, uint8_t *near)
{
    orc_field f = {U0, U1, nn, dt_u};
    advect_odes_all(m, &f, since, dt, scheme, alpha, beta, damage_prop, deform_prop, s, key, near);
}

/*
 * Stable counting sort of the surviving particles by (new cell, moved).
 * perm[j] = pre-step index of the particle that lands at position j.
 * cell_start[K] = first position of cell K; returns the new count.
 */
int64_t orc_sort_perm(int64_t n_cells, int64_t n, const int32_t *old_cell, const uint32_t *key,
                      int64_t *perm, int64_t *cell_start)
{
    int64_t nb = 2 * n_cells;
    int64_t *bucket = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (key[i] == ORC_LOST) continue;
        int64_t b = 2 * (int64_t)key[i] + (key[i] != (uint32_t)old_cell[i]);
        bucket[b + 1]++;
    }
    for (int64_t b = 0; b < nb; ++b) bucket[b + 1] += bucket[b];
    for (int64_t K = 0; K <= n_cells; ++K) cell_start[K] = bucket[2 * K];
    int64_t total = bucket[nb];
    for (int64_t i = 0; i < n; ++i) {
        if (key[i] == ORC_LOST) continue;
        int64_t b = 2 * (int64_t)key[i] + (key[i] != (uint32_t)old_cell[i]);
        perm[bucket[b]++] = i;
    }
    free(bucket);
    return total;
}

/* apply a permutation to the store: new[j] = old[perm[j]] */
static void permute_store(orc_store *s, const int64_t *perm, int64_t n_new, const uint32_t *key)
{
    int d = s->dim;
    int64_t cap = s->cap;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n_new > 0 ? n_new : 1));
    for (int a = 0; a < d; ++a) {
        for (int64_t j = 0; j < n_new; ++j) tmp[j] = s->x[a * cap + perm[j]];
        memcpy(s->x + a * cap, tmp, sizeof(double) * (size_t)n_new);
        for (int64_t j = 0; j < n_new; ++j) tmp[j] = s->xr[a * cap + perm[j]];
        memcpy(s->xr + a * cap, tmp, sizeof(double) * (size_t)n_new);
    }
    for (int p = 0; p < s->n_prop; ++p) {
        for (int64_t j = 0; j < n_new; ++j) tmp[j] = s->prop[p * cap + perm[j]];
        memcpy(s->prop + p * cap, tmp, sizeof(double) * (size_t)n_new);
    }
    uint32_t *ti = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_new > 0 ? n_new : 1));
    for (int64_t j = 0; j < n_new; ++j) ti[j] = s->id[perm[j]];
    memcpy(s->id, ti, sizeof(uint32_t) * (size_t)n_new);
    for (int64_t j = 0; j < n_new; ++j) ti[j] = key[perm[j]];
    memcpy(s->cell, ti, sizeof(uint32_t) * (size_t)n_new);
    free(ti);
    free(tmp);
    s->n = n_new;
}

/* One full step: advect + locate every particle, drop the lost, re-sort by cell. */
int orc_step(const orc_mesh *m, const double *U, int64_t nn, double dt, int scheme, orc_store *s,
             int64_t *cell_start, orc_stats *st)
{
    int64_t n = s->n, nc = orc_n_cells(m);
    uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *near = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    orc_advect(m, U, nn, dt, scheme, s, key, near);
    int64_t lost = 0, moved = 0, nf = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (key[i] == ORC_LOST) ++lost;
        else if (key[i] != (uint32_t)s->cell[i]) ++moved;
        nf += near[i];
    }
    int64_t n_new = orc_sort_perm(nc, n, s->cell, key, perm, cell_start);
    permute_store(s, perm, n_new, key);
    if (st) {
        st->lost += lost;
        st->moved += moved;
        st->near_face += nf;
        st->live = n_new;
    }
    free(key);
    free(near);
    free(perm);
    return 0;
}

/*
 * Particles after mesh refinement or coarsening (Sec. 2.5): every particle of
 * store `src` (on the old mesh) goes to the cell of the new mesh m that holds
 * its location -- a child of its old cell when that was refined, the parent
 * when it was coarsened -- with its reference location recomputed there;
 * location, id and properties are kept, particles outside m are dropped.
 * The result is stored in dst sorted by new cell, in the old store order
 * within a cell (a stable sort).  dst->n_prop must equal src->n_prop; returns
 * -1 if dst is too small.  cell_start [n_cells(m)+1] receives the new offsets.
 */
int orc_transfer(const orc_mesh *m, const orc_store *src, orc_store *dst, int64_t *cell_start)
{
    int d = m->dim;
    int64_t n = src->n, nc = orc_n_cells(m);
    if (n > dst->cap) return -1;
    int32_t *key = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *xr = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double x[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) x[a] = src->x[a * src->cap + i];
        if (!orc_locate(m, x, &key[i], xr + 3 * i)) key[i] = -1;
    }
    /* counting sort by new cell, stable */
    for (int64_t K = 0; K <= nc; ++K) cell_start[K] = 0;
    for (int64_t i = 0; i < n; ++i)
        if (key[i] >= 0) cell_start[key[i] + 1]++;
    for (int64_t K = 0; K < nc; ++K) cell_start[K + 1] += cell_start[K];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc > 0 ? nc : 1));
    for (int64_t K = 0; K < nc; ++K) fill[K] = cell_start[K];
    for (int64_t i = 0; i < n; ++i) {
        if (key[i] < 0) continue;
        int64_t p = fill[key[i]]++;
        for (int a = 0; a < d; ++a) {
            dst->x[a * dst->cap + p] = src->x[a * src->cap + i];
            dst->xr[a * dst->cap + p] = xr[3 * i + a];
        }
        dst->cell[p] = key[i];
        dst->id[p] = src->id[i];
        for (int j = 0; j < src->n_prop; ++j) dst->prop[j * dst->cap + p] = src->prop[j * src->cap + i];
    }
    dst->n = cell_start[nc];
    free(key);
    free(xr);
    free(fill);
    return 0;
}

/* Threads of the OpenMP loops (timing of the oracle only; results do not
 * depend on it).  Returns the number in use afterwards. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* counter-based random numbers: SplitMix64 (Steele, Lea, Flood 2014)   */
/* ------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t state)
{
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double orc_uniform01(uint64_t seed, uint64_t step, uint64_t cell, uint64_t slot, uint64_t coord)
{
    uint64_t h = orc_splitmix64(seed);
    h = orc_splitmix64(h ^ step);
    h = orc_splitmix64(h ^ cell);
    h = orc_splitmix64(h ^ slot);
    h = orc_splitmix64(h ^ coord);
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* Reference-local generation with the counter hash (Sec. 2.2, remark on
 * generating particles in the reference cell): particle j of cell K, listed
 * cell by cell, gets xhat_a = uniform01(seed, 2^64 - 1, K, j, a) (the step slot
 * holds the all-ones tag of this stream), x = Phi_K(xhat), id = first_id +
 * its position in the listing, property j = coordinate j mod dim of x if
 * init_position. */
int orc_seed_per_cell(const orc_mesh *m, const int32_t *counts, uint64_t seed, uint32_t first_id, int init_position,
                      orc_store *s)
{
    int d = m->dim;
    int64_t nc = orc_n_cells(m), p = 0;
    for (int64_t K = 0; K < nc; ++K) {
        if (counts[K] < 0) return -2;
        p += counts[K];
    }
    if (p > s->cap) return -1;
    p = 0;
    for (int64_t K = 0; K < nc; ++K)
        for (int32_t j = 0; j < counts[K]; ++j, ++p) {
            double t[3], x[3];
            for (int a = 0; a < d; ++a) t[a] = orc_uniform01(seed, ~0ull, (uint64_t)K, (uint64_t)j, (uint64_t)a);
            map_to_real(m, K, t, x, NULL);
            for (int a = 0; a < d; ++a) {
                s->x[a * s->cap + p] = x[a];
                s->xr[a * s->cap + p] = t[a];
            }
            s->cell[p] = (int32_t)K;
            s->id[p] = first_id + (uint32_t)p;
            if (init_position)
                for (int q = 0; q < s->n_prop; ++q) s->prop[q * s->cap + p] = x[q % d];
        }
    s->n = p;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Metropolis-Hastings generation (Sec. 2.2)                           */
/* ------------------------------------------------------------------ */
/* rho^(xhat) = max(0, rho_h(Phi_K(xhat))) |det grad Phi_K(xhat)|, rho_h the
 * Q2 interpolant of the nodal density (naive 27-term sum) */
static double mh_density(const orc_mesh *m, const double *rho, int64_t K, const double *t)
{
    int d = m->dim;
    double r = 0.0;
    for (int loc = 0; loc < nloc(d); ++loc) r += rho[q2_node(m, K, loc)] * q2_basis(d, loc, t, NULL);
    double x[3], J[3][3];
    map_to_real(m, K, t, x, J);
    double det = d == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                        : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                              J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    return (r > 0.0 ? r : 0.0) * fabs(det);
}

/*
 * For every cell K a Metropolis-Hastings chain in the reference cell with a
 * proposal uniform in Khat: it starts at the centre of Khat; state i
 * (i = 0 .. J counts[K] - 1) proposes xhat' with coordinates
 * uniform01(seed, 1, K, i, axis) and moves there when
 * uniform01(seed, 2, K, i, 0) * rho^(current) < rho^(xhat'), else repeats the
 * current state.  States J-1, 2J-1, ... become the cell's particles, stored
 * cell by cell with ids first_id + store position and properties = initial
 * position.  *longest_run = the longest run of equal consecutive states over
 * all chains (J must exceed it for the thinned samples to be distinct).
 * Returns -1 if the store is too small.
 */
int orc_seed_mh(const orc_mesh *m, const int32_t *counts, const double *rho, int J, uint64_t seed,
                uint32_t first_id, orc_store *s, int64_t *longest_run)
{
    int d = m->dim;
    int64_t nc = orc_n_cells(m), total = 0, longest = 0;
    for (int64_t K = 0; K < nc; ++K) total += counts[K];
    if (total > s->cap) return -1;
    int64_t p = 0;
    for (int64_t K = 0; K < nc; ++K) {
        double cur[3] = {0.5, 0.5, 0.5};
        double rcur = mh_density(m, rho, K, cur);
        int64_t run = 0;                     /* runs count chain states; the start is not one */
        int64_t n_states = (int64_t)J * counts[K];
        for (int64_t i = 0; i < n_states; ++i) {
            double prop[3] = {0, 0, 0};
            for (int a = 0; a < d; ++a) prop[a] = orc_uniform01(seed, 1, (uint64_t)K, (uint64_t)i, (uint64_t)a);
            double rprop = mh_density(m, rho, K, prop);
            double u = orc_uniform01(seed, 2, (uint64_t)K, (uint64_t)i, 0);
            if (u * rcur < rprop) {
                for (int a = 0; a < d; ++a) cur[a] = prop[a];
                rcur = rprop;
                run = 1;
            } else {
                ++run;
            }
            if (run > longest) longest = run;
            if ((i + 1) % J == 0) {
                double x[3];
                map_to_real(m, K, cur, x, NULL);
                for (int a = 0; a < d; ++a) {
                    s->x[a * s->cap + p] = x[a];
                    s->xr[a * s->cap + p] = cur[a];
                }
                s->cell[p] = (int32_t)K;
                s->id[p] = first_id + (uint32_t)p;
                for (int j = 0; j < s->n_prop; ++j) s->prop[j * s->cap + p] = x[j % d];
                ++p;
            }
        }
    }
    s->n = p;
    *longest_run = longest;
    return 0;
}

/* ------------------------------------------------------------------ */
/* population management                                               */
/* ------------------------------------------------------------------ */
/*
 * For every cell (index order): more than max particles -> delete the
 * n - max with the largest ids; fewer than min -> append min - n new
 * particles at hashed reference coordinates.  New ids are next_id plus an
 * exclusive scan of the per-cell additions.  A new particle's properties are
 * the mean over the cell's survivors, or its initial position if the cell is
 * empty.  The store must be sorted by cell with cell_start valid.
 */
int orc_population(const orc_mesh *m, orc_store *s, int64_t *cell_start, int min_pc, int max_pc,
                   uint64_t seed, uint64_t step, uint64_t *next_id, int64_t *added, int64_t *deleted)
{
    int d = m->dim, np = s->n_prop;
    int64_t nc = orc_n_cells(m), cap = s->cap;
    int64_t n_out = 0;
    for (int64_t K = 0; K < nc; ++K) {
        int64_t n = cell_start[K + 1] - cell_start[K];
        int64_t keep = n > max_pc ? max_pc : n;
        int64_t add = n < min_pc ? min_pc - n : 0;
        n_out += keep + add;
    }
    if (n_out > cap) return -1;
    orc_store o = *s;
    o.x = (double *)malloc(sizeof(double) * (size_t)(d * cap));
    o.xr = (double *)malloc(sizeof(double) * (size_t)(d * cap));
    o.cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    o.id = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    o.prop = (double *)malloc(sizeof(double) * (size_t)((np > 0 ? np : 1) * cap));
    int64_t *new_start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
    uint64_t id_base = *next_id;
    int64_t q = 0, tot_add = 0, tot_del = 0;
    for (int64_t K = 0; K < nc; ++K) {
        new_start[K] = q;
        int64_t b = cell_start[K], n = cell_start[K + 1] - b;
        int64_t del = n > max_pc ? n - max_pc : 0;
        /* a particle is deleted if at least n - del - ... : it is among the del largest ids */
        double mean[64];
        for (int j = 0; j < np; ++j) mean[j] = 0.0;
        int64_t kept = 0;
        for (int64_t i = b; i < b + n; ++i) {
            int64_t larger = 0;
            for (int64_t k = b; k < b + n; ++k)
                if (s->id[k] > s->id[i]) ++larger;
            if (larger < del) continue;          /* one of the del largest ids */
            for (int a = 0; a < d; ++a) {
                o.x[a * cap + q] = s->x[a * cap + i];
                o.xr[a * cap + q] = s->xr[a * cap + i];
            }
            for (int j = 0; j < np; ++j) {
                o.prop[j * cap + q] = s->prop[j * cap + i];
                mean[j] += s->prop[j * cap + i];
            }
            o.cell[q] = (int32_t)K;
            o.id[q] = s->id[i];
            ++q;
            ++kept;
        }
        tot_del += del;
        int64_t add = kept < min_pc ? min_pc - kept : 0;
        for (int j = 0; j < np; ++j) mean[j] = kept > 0 ? mean[j] / (double)kept : 0.0;
        for (int64_t slot = 0; slot < add; ++slot) {
            double t[3], x[3];
            for (int a = 0; a < d; ++a) t[a] = orc_uniform01(seed, step, (uint64_t)K, (uint64_t)slot, (uint64_t)a);
            map_to_real(m, K, t, x, NULL);
            for (int a = 0; a < d; ++a) {
                o.x[a * cap + q] = x[a];
                o.xr[a * cap + q] = t[a];
            }
            for (int j = 0; j < np; ++j) o.prop[j * cap + q] = kept > 0 ? mean[j] : x[j % d];
            o.cell[q] = (int32_t)K;
            o.id[q] = (uint32_t)(id_base + tot_add + slot);
            ++q;
        }
        tot_add += add;
    }
    new_start[nc] = q;
    memcpy(s->x, o.x, sizeof(double) * (size_t)(d * cap));
    memcpy(s->xr, o.xr, sizeof(double) * (size_t)(d * cap));
    memcpy(s->cell, o.cell, sizeof(int32_t) * (size_t)q);
    memcpy(s->id, o.id, sizeof(uint32_t) * (size_t)q);
    if (np > 0) memcpy(s->prop, o.prop, sizeof(double) * (size_t)(np * cap));
    for (int64_t K = 0; K <= nc; ++K) cell_start[K] = new_start[K];
    s->n = q;
    *next_id = id_base + (uint64_t)tot_add;
    *added = tot_add;
    *deleted = tot_del;
    free(o.x);
    free(o.xr);
    free(o.cell);
    free(o.id);
    free(o.prop);
    free(new_start);
    return 0;
}

/* ------------------------------------------------------------------ */
/* particle -> cell: arithmetic average                                */
/* ------------------------------------------------------------------ */
void orc_cell_average(int64_t n_cells, const int64_t *cell_start, const orc_store *s,
                      double *out /* [n_cells][n_prop] */, int32_t *count)
{
    int np = s->n_prop;
    for (int64_t K = 0; K < n_cells; ++K) {
        int64_t b = cell_start[K], e = cell_start[K + 1];
        count[K] = (int32_t)(e - b);
        for (int j = 0; j < np; ++j) {
            if (e == b) {
                out[K * np + j] = NAN;
                continue;
            }
            double sum = 0.0;
            for (int64_t i = b; i < e; ++i) sum += s->prop[j * s->cap + i];
            out[K * np + j] = sum / (double)(e - b);
        }
    }
}

/*
 * Geometric (mode 1) and harmonic (mode 2) averages of each property over the
 * particles of each cell (Sec. 2.7 (ii)):
 *   geometric  exp( (1/n) sum_k log p_k )   (0 if a value is 0, NaN if one is negative)
 *   harmonic   n / sum_k (1 / p_k)          (0 if a value is 0)
 * Empty cells give NaN.
 */
void orc_cell_mean(int64_t n_cells, const int64_t *cell_start, const orc_store *s, int mode,
                   double *out /* [n_cells][n_prop] */, int32_t *count)
{
    int np = s->n_prop;
    for (int64_t K = 0; K < n_cells; ++K) {
        int64_t b = cell_start[K], e = cell_start[K + 1];
        count[K] = (int32_t)(e - b);
        for (int j = 0; j < np; ++j) {
            if (e == b) {
                out[K * np + j] = NAN;
                continue;
            }
            double sum = 0.0;
            for (int64_t i = b; i < e; ++i) {
                double v = s->prop[j * s->cap + i];
                sum += mode == 1 ? log(v) : 1.0 / v;
            }
            out[K * np + j] = mode == 1 ? exp(sum / (double)(e - b)) : (double)(e - b) / sum;
        }
    }
}

/*
 * Particle -> evaluation points of each cell (Sec. 2.7 (i), (iii), (iv)).  The
 * points are given in reference coordinates qhat [dim][n_q], the same for
 * every cell; only the particles of the point's own cell take part.
 *   kind 0, nearest neighbour: the property of the particle with the smallest
 *           physical distance |Phi_K(qhat) - x_k| (ties: first in store order);
 *   kind 1, distance weighted: weights 1 / |Phi_K(qhat) - x_k|^2; particles at
 *           the point itself (distance 0) take the whole weight, equally;
 *   kind 2, shape-function weighted: weights w_k = sum_v N_v(qhat) N_v(xhat_k)
 *           over the d-linear vertex shape functions N_v of the reference cell.
 * out [n_cells][n_q][n_prop]; empty cells give NaN.
 */
static double q1_vertex_sum(int dim, const double *a, const double *b)
{
    /* sum_v N_v(a) N_v(b), written out as the sum over the 2^dim vertices */
    double sum = 0.0;
    for (int v = 0; v < nvert(dim); ++v) {
        double na = q1_shape(dim, v, a, NULL), nb = q1_shape(dim, v, b, NULL);
        sum += na * nb;
    }
    return sum;
}

void orc_interp_points(const orc_mesh *m, const int64_t *cell_start, const orc_store *s, int kind, int n_q,
                       const double *qhat, double *out)
{
    int d = m->dim, np = s->n_prop;
    int64_t nc = orc_n_cells(m);
    for (int64_t K = 0; K < nc; ++K) {
        int64_t b = cell_start[K], e = cell_start[K + 1];
        for (int q = 0; q < n_q; ++q) {
            double qr[3] = {0, 0, 0}, xq[3], J[3][3];
            for (int a = 0; a < d; ++a) qr[a] = qhat[a * n_q + q];
            map_to_real(m, K, qr, xq, J);
            double *o = out + (K * n_q + q) * np;
            if (e == b) {
                for (int j = 0; j < np; ++j) o[j] = NAN;
                continue;
            }
            if (kind == 0) {
                int64_t best = b;
                double bd = INFINITY;
                for (int64_t i = b; i < e; ++i) {
                    double d2 = 0.0;
                    for (int a = 0; a < d; ++a) {
                        double r = s->x[a * s->cap + i] - xq[a];
                        d2 += r * r;
                    }
                    if (d2 < bd) {
                        bd = d2;
                        best = i;
                    }
                }
                for (int j = 0; j < np; ++j) o[j] = s->prop[j * s->cap + best];
                continue;
            }
            /* weights: distance (with the exact-hit limit) or shape-function products */
            int n_hit = 0;
            for (int64_t i = b; i < e && kind == 1; ++i) {
                double d2 = 0.0;
                for (int a = 0; a < d; ++a) {
                    double r = s->x[a * s->cap + i] - xq[a];
                    d2 += r * r;
                }
                n_hit += d2 == 0.0;
            }
            for (int j = 0; j < np; ++j) {
                double sw = 0.0, swp = 0.0;
                for (int64_t i = b; i < e; ++i) {
                    double w;
                    if (kind == 1) {
                        double d2 = 0.0;
                        for (int a = 0; a < d; ++a) {
                            double r = s->x[a * s->cap + i] - xq[a];
                            d2 += r * r;
                        }
                        if (n_hit) w = d2 == 0.0 ? 1.0 : 0.0;
                        else w = 1.0 / d2;
                    } else {
                        double xr[3] = {0, 0, 0};
                        for (int a = 0; a < d; ++a) xr[a] = s->xr[a * s->cap + i];
                        w = q1_vertex_sum(d, qr, xr);
                    }
                    sw += w;
                    swp += w * s->prop[j * s->cap + i];
                }
                o[j] = swp / sw;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* adjoint of the multi-step RK map with respect to the nodal field    */
/* ------------------------------------------------------------------ */
/* scatter-add dU_c[node_i(K)] += w * phi_i(xhat) * kb_c */
static void scatter_dU(const orc_mesh *m, double *dU, int64_t nn, int64_t K, const double *xr, double w,
                       const double *kb)
{
    int d = m->dim;
    for (int loc = 0; loc < nloc(d); ++loc) {
        double phi = q2_basis(d, loc, xr, NULL);
        int64_t g = q2_node(m, K, loc);
        for (int c = 0; c < d; ++c) dU[c * nn + g] += w * phi * kb[c];
    }
}

/* ybar = dt * G^T kb with G[c][j] = d u_c / d x_j at the stage point */
static void vjp(const orc_mesh *m, const double *U, int64_t nn, int64_t K, const double *xr, double dt,
                const double *kb, double *yb)
{
    int d = m->dim;
    double G[3][3];
    eval_grad(m, U, nn, K, xr, G);
    for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int c = 0; c < d; ++c) s += G[c][j] * kb[c];
        yb[j] = dt * s;
    }
}

/*
 * Loss and gradient for particles given by their initial (x, K, xhat).
 * target[a*n + i] is the target of particle i, mask[i] selects the valid
 * ones (the caller fixes the mask, e.g. particles that survive in both the
 * base and the target run).  Returns L; dU [dim][nn] is overwritten.
 * Particles that get lost in this run contribute nothing (counted in *n_lost).
 */
double orc_adjoint(const orc_mesh *m, const double *U, int64_t nn, double dt, int scheme, int n_steps,
                   int64_t n, const double *x0, const int32_t *K0, const double *xr0,
                   const double *target, const uint8_t *mask, double *dU, int64_t *n_lost)
{
    int d = m->dim;
    int64_t nv = 0;
    for (int64_t i = 0; i < n; ++i) nv += mask[i] ? 1 : 0;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *buf = (double *)calloc((size_t)nthreads * (size_t)(d * nn), sizeof(double));
    double loss = 0.0;
    int64_t lost_total = 0;
    int nstage = scheme == 4 ? 4 : scheme;
#pragma omp parallel reduction(+ : loss, lost_total)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g = buf + (size_t)tid * (size_t)(d * nn);
        /* per particle trajectory: stage points of every step */
        double *Ys = (double *)malloc(sizeof(double) * (size_t)n_steps * 4 * 3);
        double *Ts = (double *)malloc(sizeof(double) * (size_t)n_steps * 4 * 3);
        int32_t *Ks = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_steps * 4);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (!mask[i]) continue;
            double x[3], t[3];
            int32_t K = K0[i];
            for (int a = 0; a < d; ++a) {
                x[a] = x0[a * n + i];
                t[a] = xr0[a * n + i];
            }
            int alive = 1;
            for (int st = 0; st < n_steps && alive; ++st) {
                double k[4][3], y[3], u[3];
                int32_t Ky = K;
                double ty[3];
                memcpy(ty, t, sizeof(ty));
                for (int s = 0; s < nstage; ++s) {
                    if (s == 0) {
                        memcpy(y, x, sizeof(y));
                    } else {
                        double f = (scheme == 4 && s == 3) ? 1.0 : 0.5;
                        for (int a = 0; a < d; ++a) y[a] = x[a] + f * k[s - 1][a];
                        if (!orc_locate(m, y, &Ky, ty)) { alive = 0; break; }
                    }
                    orc_eval(m, U, nn, Ky, ty, u);
                    for (int a = 0; a < d; ++a) {
                        k[s][a] = dt * u[a];
                        Ys[(st * 4 + s) * 3 + a] = y[a];
                        Ts[(st * 4 + s) * 3 + a] = ty[a];
                    }
                    Ks[st * 4 + s] = Ky;
                }
                if (!alive) break;
                if (scheme == 1)
                    for (int a = 0; a < d; ++a) x[a] = x[a] + k[0][a];
                else if (scheme == 2)
                    for (int a = 0; a < d; ++a) x[a] = x[a] + k[1][a];
                else
                    for (int a = 0; a < d; ++a)
                        x[a] = x[a] + k[0][a] / 6.0 + k[1][a] / 3.0 + k[2][a] / 3.0 + k[3][a] / 6.0;
                if (!orc_locate(m, x, &K, t)) alive = 0;
            }
            if (!alive) { lost_total += 1; continue; }
            double lam[3];
            for (int a = 0; a < d; ++a) {
                double r = x[a] - target[a * n + i];
                loss += r * r / (double)nv;
                lam[a] = 2.0 * r / (double)nv;
            }
            for (int st = n_steps - 1; st >= 0; --st) {
                double kb[4][3], yb[4][3];
                const double *T;
                int32_t Kst;
                if (scheme == 1) {
                    memcpy(kb[0], lam, sizeof(lam));
                    T = Ts + (st * 4 + 0) * 3; Kst = Ks[st * 4 + 0];
                    vjp(m, U, nn, Kst, T, dt, kb[0], yb[0]);
                    scatter_dU(m, g, nn, Kst, T, dt, kb[0]);
                    for (int a = 0; a < d; ++a) lam[a] += yb[0][a];
                } else if (scheme == 2) {
                    memcpy(kb[1], lam, sizeof(lam));
                    T = Ts + (st * 4 + 1) * 3; Kst = Ks[st * 4 + 1];
                    vjp(m, U, nn, Kst, T, dt, kb[1], yb[1]);
                    scatter_dU(m, g, nn, Kst, T, dt, kb[1]);
                    for (int a = 0; a < d; ++a) kb[0][a] = 0.5 * yb[1][a];
                    T = Ts + (st * 4 + 0) * 3; Kst = Ks[st * 4 + 0];
                    vjp(m, U, nn, Kst, T, dt, kb[0], yb[0]);
                    scatter_dU(m, g, nn, Kst, T, dt, kb[0]);
                    for (int a = 0; a < d; ++a) lam[a] += yb[0][a] + yb[1][a];
                } else {
                    for (int a = 0; a < d; ++a) {
                        kb[0][a] = lam[a] / 6.0;
                        kb[1][a] = lam[a] / 3.0;
                        kb[2][a] = lam[a] / 3.0;
                        kb[3][a] = lam[a] / 6.0;
                    }
                    for (int s = 3; s >= 0; --s) {
                        T = Ts + (st * 4 + s) * 3; Kst = Ks[st * 4 + s];
                        vjp(m, U, nn, Kst, T, dt, kb[s], yb[s]);
                        scatter_dU(m, g, nn, Kst, T, dt, kb[s]);
                        if (s == 3) for (int a = 0; a < d; ++a) kb[2][a] += yb[3][a];
                        if (s == 2) for (int a = 0; a < d; ++a) kb[1][a] += 0.5 * yb[2][a];
                        if (s == 1) for (int a = 0; a < d; ++a) kb[0][a] += 0.5 * yb[1][a];
                    }
                    for (int a = 0; a < d; ++a) lam[a] += yb[0][a] + yb[1][a] + yb[2][a] + yb[3][a];
                }
            }
        }
        free(Ys);
        free(Ts);
        free(Ks);
    }
    for (int64_t j = 0; j < d * nn; ++j) {
        double s = 0.0;
        for (int t = 0; t < nthreads; ++t) s += buf[(size_t)t * (size_t)(d * nn) + (size_t)j];
        dU[j] = s;
    }
    free(buf);
    if (n_lost) *n_lost = lost_total;
    return loss;
}

/* ------------------------------------------------------------------ */
/* octree: finest-grid lookup, Q2 node numbering, hanging constraints  */
/* ------------------------------------------------------------------ */
/*
 * Fill fine_to_leaf [(2^L)^3] for leaves given by (level, anchor).
 * Returns 0 if the leaves tile the cube exactly, -1 otherwise.
 */
int orc_octree_fine_table(int64_t n_cells, int max_level, const uint8_t *level, const int32_t *anchor,
                          int32_t *table)
{
    int64_t fine = 1 << max_level;
    int64_t total = fine * fine * fine;
    for (int64_t f = 0; f < total; ++f) table[f] = -1;
    for (int64_t K = 0; K < n_cells; ++K) {
        int64_t sz = (int64_t)1 << (max_level - level[K]);
        int64_t ax = anchor[K], ay = anchor[n_cells + K], az = anchor[2 * n_cells + K];
        for (int64_t k = az; k < az + sz; ++k)
            for (int64_t j = ay; j < ay + sz; ++j)
                for (int64_t i = ax; i < ax + sz; ++i) {
                    int64_t f = i + fine * (j + fine * k);
                    if (table[f] != -1) return -1;
                    table[f] = (int32_t)K;
                }
    }
    for (int64_t f = 0; f < total; ++f)
        if (table[f] < 0) return -1;
    return 0;
}
