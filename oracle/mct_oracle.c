/*
 * Plain FP64 CPU oracle of the MCT-2D-CEM explicit dynamic step
 * (two-dimensional Crack Element Model with Multiple Crack-tips Tracking,
 * arXiv 2509.01827).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * is loaded by tests/, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The product library (include/mct2d.h) neither links nor calls
 * it, and the two share no source, header, table or helper.
 *
 * It is deliberately slow and literal: generic mesh tables (element
 * connectivity, an edge list sorted by node pair, edge->element adjacency),
 * one loop per formula, one candidate at a time.
 *
 * Where each part comes from:
 *   - ES-FEM edge displacement / smoothed strain: Sec. 2.1, Eq. (disp_ES_FEM)
 *     and Eq. (strain_discretization); Q4 strain matrix: Eq.
 *     (QUAD_strain_discretization).
 *   - Q4 internal force: Eq. (QUAD_fint_discretization), f = B~^T sigma *
 *     sum_j A_j/4; plane Cauchy stress (Sec. 2.1, text after that equation).
 *   - Energy release rate of a split elementary topology: Sec. 2.2, the
 *     unnumbered equation for G_{Gk-G0} = delta_d . sigma_perp / 2 with the
 *     Heaviside edge-stretch gate, and its Q4 form with three candidate paths.
 *   - Q4 per-element decision (none / one / two / three candidates over Gc,
 *     split ratio gamma): Sec. 2.2, itemised rules after Fig. 2-3.
 *   - Crack patterns I (adjacent edge) and II (opposite edge): Fig. 2-3.
 *   - Multiple Crack-tips Tracking: Sec. 3 and its pick criterion (the
 *     unnumbered inequalities G2 > gamma (G2 - Gi)), Fig. 3-1(b).
 *   - Single crack-tip tracking (the SCT mode): Sec. 3 first paragraph and
 *     Fig. 3-1(a): only the current tip quadrature point is evaluated; when
 *     its element splits the tip moves to the exit edge.
 *   - Explicit formulation: Sec. 2 opening sentence.
 *
 * Readings where the paper is silent (the same readings as the library's):
 *   - B of element j at edge g_s is the isoparametric Q4 gradient evaluated
 *     at the midpoint of that edge in j's natural coordinates (reference
 *     configuration, small strain).
 *   - Linear elastic plane stress, engineering shear strain.
 *   - Central differences with lumped mass m_i = sum rho A_e / 4, first step
 *     half a time step, prescribed velocities override v.
 *   - A split element takes no part in edge smoothing; its pieces carry
 *     reduced elements (3 nodes: CST, 2 nodes: bar, 1 node: nothing).
 *   - Candidates are edges with exactly one intact neighbour; the crack-path
 *     normal orients toward node N2; one split per step; gamma test exactly
 *     as printed.
 *
 * FP contract (binds the HIP library as well): IEEE binary64, round to
 * nearest, compiled with -ffp-contract=off; fma() only where written.
 *
 * Binary32 build (ORC_FP32 defined; liboracle32.so): the set-up (areas,
 * lumped masses, equivalent nodal forces, D, dt, the tables) stays binary64
 * exactly as above; the step reads every set-up value rounded once to
 * binary32 and computes in binary32 (state, strains, stresses, forces, G,
 * the element rule and the pick); times t_k and the load factor are
 * evaluated in binary64 and rounded; a split adds its Gc * L (a binary32
 * product) to U_d in binary64.  `real` is the step's type; R() makes a
 * constant a real.
 *
 * Loops whose iterations write disjoint outputs (edges, elements, elements
 * of one colour, nodes, candidate evaluation) may run on several OpenMP
 * threads; every value is still computed by one thread in the order written
 * here, so results do not depend on the thread count.
 */
#include <math.h>
#include <omp.h>
#include <float.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ESTATE (-2)
#define ORC_ECAPACITY (-3)

#define SPLIT_FLAG 0x80u

#ifdef ORC_FP32
typedef float real;
#define rfma fmaf
#define rsqrt sqrtf
#else
typedef double real;
#define rfma fma
#define rsqrt sqrt
#endif
#define R(x) ((real)(x))

typedef struct {
    int step, elem, entry, exit;
    double G;
} orc_split_t;

/* One near-threshold decision (the floating-point contract asks for every
 * decision whose margin is within a relative tolerance to be recorded, so
 * that a divergence between two runs can be traced to it).  kind: 1 a path
 * G against Gc (element rule threshold, Sec. 2.2); 2 the gap between the two
 * largest paths above Gc of one element (the rule's argmax); 3 the element
 * rule's split-ratio margin against one other path above Gc; 4 the gap
 * between the two largest accepted candidates of a step (the MCT pick's
 * argmax, Sec. 3); 5 the pick's split-ratio margin (against the smallest
 * accepted G).  k is the exit edge of the path concerned (kinds 1, 3: that
 * path; 2, 4, 5: the chosen one); G the chosen (or the path's) value, ref
 * the value it was compared with. */
typedef struct {
    int step, elem, a, kind, k;
    double G, ref;
} orc_near_t;

typedef struct {
    /* mesh: nv = 4 (Q4, structured grid) or 3 (CST, unstructured) */
    int nv, nx, ny, nn, ne, ns;
    double *X, *Y;
    int *conn;       /* nv per element at stride 4, counter-clockwise */
    int *edge_node;  /* 2 per edge: (smaller node id, larger node id) */
    int *edge_elem;  /* 2 per edge: smaller element id first, -1 = none */
    int *edge_loc;   /* 2 per edge: local edge index inside that element */
    int *elem_edge;  /* nv per element at stride 4: global edge id of local edge k */
    int *color;
    int ncolor;
    double *area;
    /* material */
    double E, nu, rho, D11, D12, D33;
    double *Gc;
    double gamma;
    /* loads */
    double *edge_trac; /* 2 per edge */
    unsigned char *edge_loaded;
    unsigned char *vmask; /* per node: bit0 = x prescribed, bit1 = y */
    double *v0;           /* 2 per node */
    double t_ramp;
    /* traction load curve: phi(t) piecewise linear through (curve_t[i],
     * curve_phi[i]), constant beyond the ends; ncurve = 0: phi = 1 */
    int ncurve;
    double *curve_t, *curve_phi;
    double dt_in, cfl;
    /* derived */
    double *mass, *minv, *fext;
    double dt;
    int finalized;
    /* state */
    unsigned char *split;
    real *ux, *uy, *vx, *vy;
    long step;
    orc_split_t *log;
    int nlog, caplog;
    double Ud;
    /* tracking: 0 = multiple crack tips, 1 = single crack tip; tip =
     * element * 4 + local edge of the intact element at the current tip, or
     * -1 (start tip: -2 = derive from the pre-notch at finalize) */
    int sct, tip;
    /* per-front pick (a variant of the Sec. 3 pick): front_r2 = rho^2 > 0
     * enables it; 0 = the global pick */
    double front_r2;
    /* Q4 edge smoothing: 0 = the point rule (B of element j at the midpoint
     * of the edge), 1 = sub-cells (the triangle edge + centroid of j) */
    int subcell;
    /* near-threshold decision log: tolerance (0 = off) and records */
    double near_tol;
    orc_near_t *near;
    int nnear, capnear;
    /* scratch */
    real *sig;              /* 3 per edge */
    real *eps;              /* 3 per edge: smoothed strain */
    unsigned char *sig_ok;  /* edge has >= 1 intact neighbour */
    real *fe;               /* 8 per element */
    real *fx, *fy, *ax, *ay;
} orc_model_t;

/* set-up values as the step reads them (binary64 rounded once to real) */
static real rX(const orc_model_t *m, int n) { return (real)m->X[n]; }
static real rY(const orc_model_t *m, int n) { return (real)m->Y[n]; }
static real r_area(const orc_model_t *m, int e) { return (real)m->area[e]; }
static real r_gc(const orc_model_t *m, int e) { return (real)m->Gc[e]; }

/* natural coordinates of the Q4 nodes and of the four edge midpoints */
static const real XI_N[4] = {-1.0, 1.0, 1.0, -1.0};
static const real ETA_N[4] = {-1.0, -1.0, 1.0, 1.0};
static const real XI_M[4] = {0.0, 1.0, 0.0, -1.0};
static const real ETA_M[4] = {-1.0, 0.0, 1.0, 0.0};

/* ------------------------------------------------------------------ */
/* element kinematics                                                   */
/* ------------------------------------------------------------------ */

/* Gradients dN_n/dx, dN_n/dy of the bilinear Q4 shape functions of an
 * element with node coordinates (x[4], y[4]) at the midpoint of its local
 * edge k (Eq. QUAD_strain_discretization evaluated at the edge quadrature
 * point). */
static void q4_grad_at_edge(const real x[4], const real y[4], int k,
                            real dndx[4], real dndy[4]) {
    real dxi[4], deta[4];
    for (int n = 0; n < 4; ++n) {
        dxi[n] = R(0.25) * XI_N[n] * (R(1.0) + ETA_M[k] * ETA_N[n]);
        deta[n] = R(0.25) * ETA_N[n] * (R(1.0) + XI_M[k] * XI_N[n]);
    }
    real j11 = 0.0, j12 = 0.0, j21 = 0.0, j22 = 0.0;
    for (int n = 0; n < 4; ++n) {
        j11 = rfma(dxi[n], x[n], j11);
        j12 = rfma(dxi[n], y[n], j12);
        j21 = rfma(deta[n], x[n], j21);
        j22 = rfma(deta[n], y[n], j22);
    }
    real det = j11 * j22 - j12 * j21;
    real inv = R(1.0) / det;
    for (int n = 0; n < 4; ++n) {
        dndx[n] = (j22 * dxi[n] - j12 * deta[n]) * inv;
        dndy[n] = (j11 * deta[n] - j21 * dxi[n]) * inv;
    }
}

/* Gradients of the linear shape functions of a triangle (x[3], y[3]),
 * constant over the element (Eq. CST_strain_discretization). */
static void tri_grad(const real x[3], const real y[3], real dndx[3], real dndy[3]) {
    real twoA = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    real inv = R(1.0) / twoA;
    dndx[0] = (y[1] - y[2]) * inv;
    dndx[1] = (y[2] - y[0]) * inv;
    dndx[2] = (y[0] - y[1]) * inv;
    dndy[0] = (x[2] - x[1]) * inv;
    dndy[1] = (x[0] - x[2]) * inv;
    dndy[2] = (x[1] - x[0]) * inv;
}

/* strain (exx, eyy, gxy) = B u for an element with nn nodes */
static void strain_from_grad(int nn, const real *dndx, const real *dndy,
                             const real *ux, const real *uy, real eps[3]) {
    real exx = 0.0, eyy = 0.0, gxy = 0.0;
    for (int n = 0; n < nn; ++n) {
        exx = rfma(dndx[n], ux[n], exx);
        eyy = rfma(dndy[n], uy[n], eyy);
        gxy = rfma(dndy[n], ux[n], gxy);
        gxy = rfma(dndx[n], uy[n], gxy);
    }
    eps[0] = exx;
    eps[1] = eyy;
    eps[2] = gxy;
}

/* plane-stress Hooke law, engineering shear strain */
static void stress_from_strain(const orc_model_t *m, const real eps[3], real sig[3]) {
    const real D11 = (real)m->D11, D12 = (real)m->D12, D33 = (real)m->D33;
    sig[0] = rfma(D12, eps[1], D11 * eps[0]);
    sig[1] = rfma(D12, eps[0], D11 * eps[1]);
    sig[2] = D33 * eps[2];
}

static void elem_coords(const orc_model_t *m, int e, real x[4], real y[4]) {
    for (int n = 0; n < m->nv; ++n) {
        x[n] = rX(m, m->conn[4 * e + n]);
        y[n] = rY(m, m->conn[4 * e + n]);
    }
}

/* binary64 corner coordinates (set-up: areas) */
static void elem_coords_d(const orc_model_t *m, int e, double x[4], double y[4]) {
    for (int n = 0; n < m->nv; ++n) {
        x[n] = m->X[m->conn[4 * e + n]];
        y[n] = m->Y[m->conn[4 * e + n]];
    }
}

static void elem_disp(const orc_model_t *m, int e, real ux[4], real uy[4]) {
    for (int n = 0; n < m->nv; ++n) {
        ux[n] = m->ux[m->conn[4 * e + n]];
        uy[n] = m->uy[m->conn[4 * e + n]];
    }
}

/* triangle area: half the cross product of two edges from node 0 (the
 * step's sub-cells, in real; tri_area_d: set-up, binary64) */
static real tri_area(const real x[3], const real y[3]) {
    return R(0.5) * ((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]));
}

static double tri_area_d(const double x[3], const double y[3]) {
    return 0.5 * ((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]));
}

/* quadrilateral area: half the cross product of the diagonals (set-up) */
static double quad_area(const double x[4], const double y[4]) {
    return 0.5 * ((x[2] - x[0]) * (y[3] - y[1]) - (x[3] - x[1]) * (y[2] - y[0]));
}

/* polygon area by a fan from the first vertex */
static real polygon_area(int nv, const real *px, const real *py) {
    real s = 0.0;
    for (int i = 1; i + 1 < nv; ++i)
        s += (px[i] - px[0]) * (py[i + 1] - py[0]) - (px[i + 1] - px[0]) * (py[i] - py[0]);
    return R(0.5) * s;
}

static int is_intact(const orc_model_t *m, int e) { return e >= 0 && m->split[e] == 0; }

/* B of element e at the quadrature point of its local edge k: the Q4
 * gradient at the edge midpoint, or the constant CST gradient */
static void elem_grad_at_edge(const orc_model_t *m, int e, int k, real dndx[4], real dndy[4]) {
    real x[4], y[4];
    elem_coords(m, e, x, y);
    if (m->nv == 4)
        q4_grad_at_edge(x, y, k, dndx, dndy);
    else
        tri_grad(x, y, dndx, dndy);
}

/* ------------------------------------------------------------------ */
/* a1: ES-FEM smoothed strain and stress at every edge                  */
/* ------------------------------------------------------------------ */

/* Sub-cell of Q4 element e at its local edge k: the triangle (n_k, n_k+1,
 * c) with c the vertex centroid of e; the displacement at c is the mean of
 * the four nodal displacements.  Fills the three corner coordinates and
 * displacements (corner order n_k, n_k+1, c) and returns the area.  This is
 * the smoothing-domain part of standard edge-based smoothing over triangular
 * sub-cells (divergence theorem with a linear displacement along the
 * sub-cell boundary), the alternative to the point rule. */
static real subcell(const orc_model_t *m, int e, int k, const real *ux_all, const real *uy_all,
                    real x[3], real y[3], real ux[3], real uy[3]) {
    real ex[4], ey[4];
    elem_coords(m, e, ex, ey);
    int a = m->conn[4 * e + k], b = m->conn[4 * e + ((k + 1) & 3)];
    x[0] = ex[k];
    y[0] = ey[k];
    x[1] = ex[(k + 1) & 3];
    y[1] = ey[(k + 1) & 3];
    x[2] = R(0.25) * (((ex[0] + ex[1]) + ex[2]) + ex[3]);
    y[2] = R(0.25) * (((ey[0] + ey[1]) + ey[2]) + ey[3]);
    if (ux_all) {
        const int *cn = &m->conn[4 * e];
        ux[0] = ux_all[a];
        uy[0] = uy_all[a];
        ux[1] = ux_all[b];
        uy[1] = uy_all[b];
        ux[2] = R(0.25) * (((ux_all[cn[0]] + ux_all[cn[1]]) + ux_all[cn[2]]) + ux_all[cn[3]]);
        uy[2] = R(0.25) * (((uy_all[cn[0]] + uy_all[cn[1]]) + uy_all[cn[2]]) + uy_all[cn[3]]);
    }
    return tri_area(x, y);
}

static void edge_stresses(orc_model_t *m) {
#pragma omp parallel for schedule(static)
    for (int s = 0; s < m->ns; ++s) {
        real q[2][3], A[2];
        int cnt = 0;
        for (int side = 0; side < 2; ++side) {
            int e = m->edge_elem[2 * s + side];
            if (!is_intact(m, e)) continue;
            if (m->nv == 4 && m->subcell) {
                real x[3], y[3], ux[3], uy[3], dndx[3], dndy[3];
                A[cnt] = subcell(m, e, m->edge_loc[2 * s + side], m->ux, m->uy, x, y, ux, uy);
                tri_grad(x, y, dndx, dndy);
                strain_from_grad(3, dndx, dndy, ux, uy, q[cnt]);
                cnt++;
                continue;
            }
            real ux[4], uy[4], dndx[4], dndy[4];
            elem_disp(m, e, ux, uy);
            elem_grad_at_edge(m, e, m->edge_loc[2 * s + side], dndx, dndy);
            strain_from_grad(m->nv, dndx, dndy, ux, uy, q[cnt]);
            A[cnt] = r_area(m, e);
            cnt++;
        }
        real eps[3];
        if (cnt == 0) {
            m->sig_ok[s] = 0;
            m->sig[3 * s] = m->sig[3 * s + 1] = m->sig[3 * s + 2] = 0.0;
            m->eps[3 * s] = m->eps[3 * s + 1] = m->eps[3 * s + 2] = 0.0;
            continue;
        }
        if (cnt == 1) {
            /* one intact neighbour: w = A/A = 1 */
            eps[0] = q[0][0];
            eps[1] = q[0][1];
            eps[2] = q[0][2];
        } else {
            /* w_j = A_j / sum A, lower element id first */
            real sum = A[0] + A[1];
            real w0 = A[0] / sum, w1 = A[1] / sum;
            for (int c = 0; c < 3; ++c) eps[c] = rfma(w1, q[1][c], w0 * q[0][c]);
        }
        stress_from_strain(m, eps, &m->sig[3 * s]);
        for (int c = 0; c < 3; ++c) m->eps[3 * s + c] = eps[c];
        m->sig_ok[s] = 1;
    }
}

/* ------------------------------------------------------------------ */
/* a2: element internal forces (intact Q4 and split pieces)             */
/* ------------------------------------------------------------------ */

/* CST (Eq. CST_fint_discretization): element e receives (A_e/3) B_e^T
 * sigma_s from each of its three edges; B_e is constant, so the three edge
 * stresses are summed first (local edge order). */
static void intact_force_tri(const orc_model_t *m, int e, real f[8]) {
    real dndx[4], dndy[4], S[3];
    elem_grad_at_edge(m, e, 0, dndx, dndy);
    const real *s0 = &m->sig[3 * m->elem_edge[4 * e]];
    const real *s1 = &m->sig[3 * m->elem_edge[4 * e + 1]];
    const real *s2 = &m->sig[3 * m->elem_edge[4 * e + 2]];
    for (int c = 0; c < 3; ++c) S[c] = (s0[c] + s1[c]) + s2[c];
    real coef = r_area(m, e) / R(3.0);
    for (int n = 0; n < 3; ++n) {
        f[2 * n] = coef * rfma(dndy[n], S[2], dndx[n] * S[0]);
        f[2 * n + 1] = coef * rfma(dndx[n], S[2], dndy[n] * S[1]);
    }
}

/* Q4 element force with sub-cells: each local edge k contributes
 * A_T B_T^T sigma_k of its sub-cell; the centroid corner's share goes a
 * quarter to each node.  Per node n and edge k the bracket is
 * t_a + t_c / 4 (n = k), t_b + t_c / 4 (n = k + 1) or t_c / 4, scaled by
 * A_T and summed over k = 0..3. */
static void intact_force_subcell(const orc_model_t *m, int e, real f[8]) {
    for (int k = 0; k < 4; ++k) {
        real x[3], y[3], b[3], c[3];
        real AT = subcell(m, e, k, NULL, NULL, x, y, NULL, NULL);
        tri_grad(x, y, b, c);
        const real *sg = &m->sig[3 * m->elem_edge[4 * e + k]];
        real tx[3], ty[3];
        for (int i = 0; i < 3; ++i) {
            tx[i] = rfma(c[i], sg[2], b[i] * sg[0]);
            ty[i] = rfma(b[i], sg[2], c[i] * sg[1]);
        }
        for (int n = 0; n < 4; ++n) {
            real gx = R(0.25) * tx[2], gy = R(0.25) * ty[2];
            if (n == k) {
                gx = tx[0] + R(0.25) * tx[2];
                gy = ty[0] + R(0.25) * ty[2];
            } else if (n == ((k + 1) & 3)) {
                gx = tx[1] + R(0.25) * tx[2];
                gy = ty[1] + R(0.25) * ty[2];
            }
            real vx = AT * gx, vy = AT * gy;
            if (k == 0) {
                f[2 * n] = vx;
                f[2 * n + 1] = vy;
            } else {
                f[2 * n] = f[2 * n] + vx;
                f[2 * n + 1] = f[2 * n + 1] + vy;
            }
        }
    }
}

static void intact_force(const orc_model_t *m, int e, real f[8]) {
    if (m->nv == 3) {
        intact_force_tri(m, e, f);
        return;
    }
    if (m->subcell) {
        intact_force_subcell(m, e, f);
        return;
    }
    real x[4], y[4];
    elem_coords(m, e, x, y);
    real sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k) {
        real dndx[4], dndy[4];
        q4_grad_at_edge(x, y, k, dndx, dndy);
        const real *sg = &m->sig[3 * m->elem_edge[4 * e + k]];
        for (int n = 0; n < 4; ++n) {
            real tx = rfma(dndy[n], sg[2], dndx[n] * sg[0]);
            real ty = rfma(dndx[n], sg[2], dndy[n] * sg[1]);
            if (k == 0) {
                sx[n] = tx;
                sy[n] = ty;
            } else {
                sx[n] = sx[n] + tx;
                sy[n] = sy[n] + ty;
            }
        }
    }
    real c = R(0.25) * r_area(m, e);
    for (int n = 0; n < 4; ++n) {
        f[2 * n] = c * sx[n];
        f[2 * n + 1] = c * sy[n];
    }
}

/* Piece of a split element: local nodes first..last going CCW, closed by
 * the crack midpoints of edges `exit_edge` (after last) and `entry_edge`
 * (before first).  Adds its nodal forces into f[8] (each node belongs to one
 * piece only).  Returns the piece strain energy. */
static real piece_force(const orc_model_t *m, int e, int entry_edge, int exit_edge,
                        real f[8]) {
    const int *cn = &m->conn[4 * e];
    const int nvert = m->nv;
    int loc[3];
    int np = 0;
    for (int k = (entry_edge + 1) % nvert;; k = (k + 1) % nvert) {
        loc[np++] = k;
        if (k == exit_edge) break;
    }
    /* polygon: M_entry, nodes..., M_exit */
    real px[5], py[5];
    int nv = 0;
    int a0 = cn[entry_edge], a1 = cn[(entry_edge + 1) % nvert];
    int b0 = cn[exit_edge], b1 = cn[(exit_edge + 1) % nvert];
    px[nv] = R(0.5) * (rX(m, a0) + rX(m, a1));
    py[nv++] = R(0.5) * (rY(m, a0) + rY(m, a1));
    for (int i = 0; i < np; ++i) {
        px[nv] = rX(m, cn[loc[i]]);
        py[nv++] = rY(m, cn[loc[i]]);
    }
    px[nv] = R(0.5) * (rX(m, b0) + rX(m, b1));
    py[nv++] = R(0.5) * (rY(m, b0) + rY(m, b1));
    real Ap = polygon_area(nv, px, py);

    if (np == 3) {
        /* constant-strain triangle over the three nodes */
        real b[3], c[3];
        tri_grad(&px[1], &py[1], b, c);
        real ux[3], uy[3];
        for (int i = 0; i < 3; ++i) {
            ux[i] = m->ux[cn[loc[i]]];
            uy[i] = m->uy[cn[loc[i]]];
        }
        real eps[3], sg[3];
        strain_from_grad(3, b, c, ux, uy, eps);
        stress_from_strain(m, eps, sg);
        for (int i = 0; i < 3; ++i) {
            real tx = rfma(c[i], sg[2], b[i] * sg[0]);
            real ty = rfma(b[i], sg[2], c[i] * sg[1]);
            f[2 * loc[i]] = Ap * tx;
            f[2 * loc[i] + 1] = Ap * ty;
        }
        return R(0.5) * Ap * (sg[0] * eps[0] + sg[1] * eps[1] + sg[2] * eps[2]);
    }
    if (np == 2) {
        /* bar along the two nodes, cross-section Ap / L */
        int p = cn[loc[0]], q = cn[loc[1]];
        real dx = rX(m, q) - rX(m, p), dy = rY(m, q) - rY(m, p);
        real L2 = dx * dx + dy * dy;
        real dux = m->ux[q] - m->ux[p], duy = m->uy[q] - m->uy[p];
        real strain = (dx * dux + dy * duy) / L2;
        real stress = (real)m->E * strain;
        real coef = Ap * stress / L2;
        f[2 * loc[1]] = coef * dx;
        f[2 * loc[1] + 1] = coef * dy;
        f[2 * loc[0]] = -(coef * dx);
        f[2 * loc[0] + 1] = -(coef * dy);
        return R(0.5) * Ap * stress * strain;
    }
    /* one node: a free corner carries no stiffness */
    f[2 * loc[0]] = 0.0;
    f[2 * loc[0] + 1] = 0.0;
    return 0.0;
}

static real split_force(const orc_model_t *m, int e, real f[8]) {
    int a = (m->split[e] >> 2) & 3, b = m->split[e] & 3;
    real w = piece_force(m, e, a, b, f);
    w += piece_force(m, e, b, a, f);
    return w;
}

/* a1 + a2 + a3: internal nodal forces of the current displacement */
static void internal_forces(orc_model_t *m) {
    edge_stresses(m);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->ne; ++e) {
        if (m->split[e] == 0)
            intact_force(m, e, &m->fe[8 * e]);
        else
            split_force(m, e, &m->fe[8 * e]);
    }
    /* graph-coloured scatter: colour 0, 1, ... ; inside a colour no two
     * elements share a node, so the per-node summation order is the colour
     * order */
    for (int i = 0; i < m->nn; ++i) m->fx[i] = m->fy[i] = 0.0;
    for (int c = 0; c < m->ncolor; ++c)
#pragma omp parallel for schedule(static)
        for (int e = 0; e < m->ne; ++e) {
            if (m->color[e] != c) continue;
            for (int n = 0; n < m->nv; ++n) {
                int g = m->conn[4 * e + n];
                m->fx[g] = m->fx[g] + m->fe[8 * e + 2 * n];
                m->fy[g] = m->fy[g] + m->fe[8 * e + 2 * n + 1];
            }
        }
}

/* ------------------------------------------------------------------ */
/* a5: energy release rate of the split elementary topologies           */
/* ------------------------------------------------------------------ */

/* Unit normal and length of the crack path from the midpoint G0 of local
 * edge a to the midpoint Gk of local edge k, oriented toward node N2 = n_{a+1}
 * (reference configuration). */
static void path_normal(const orc_model_t *m, int e, int a, int k, real *nx,
                        real *ny, real *len) {
    const int *cn = &m->conn[4 * e];
    int p0 = cn[a], p1 = cn[(a + 1) % m->nv], q0 = cn[k], q1 = cn[(k + 1) % m->nv];
    real g0x = R(0.5) * (rX(m, p0) + rX(m, p1)), g0y = R(0.5) * (rY(m, p0) + rY(m, p1));
    real gkx = R(0.5) * (rX(m, q0) + rX(m, q1)), gky = R(0.5) * (rY(m, q0) + rY(m, q1));
    real dx = gkx - g0x, dy = gky - g0y;
    real L = rsqrt(dx * dx + dy * dy);
    real cx = dy / L, cy = -dx / L;
    if (cx * (rX(m, p1) - g0x) + cy * (rY(m, p1) - g0y) < R(0.0)) {
        cx = -cx;
        cy = -cy;
    }
    *nx = cx;
    *ny = cy;
    *len = L;
}

/* G of the paths of candidate (element e, crack-tip edge a): k = a+1, a+2,
 * a+3 (CCW) for Q4, k = a+1, a+2 for CST (then G[2] = 0).  Returns the
 * Heaviside gate H. */
static int candidate_G(const orc_model_t *m, int e, int a, real G[3]) {
    const int *cn = &m->conn[4 * e];
    int n1 = cn[a], n2 = cn[(a + 1) % m->nv];
    real dux = m->ux[n2] - m->ux[n1], duy = m->uy[n2] - m->uy[n1];
    /* H(|x2-x1|/|X2-X1| - 1) as a comparison of squared lengths */
    real x1 = rX(m, n1) + m->ux[n1], y1 = rY(m, n1) + m->uy[n1];
    real x2 = rX(m, n2) + m->ux[n2], y2 = rY(m, n2) + m->uy[n2];
    real lx = x2 - x1, ly = y2 - y1;
    real Lx = rX(m, n2) - rX(m, n1), Ly = rY(m, n2) - rY(m, n1);
    int H = (lx * lx + ly * ly) > (Lx * Lx + Ly * Ly);
    G[2] = 0.0;
    for (int j = 0; j < m->nv - 1; ++j) {
        if (!H) {
            G[j] = 0.0;
            continue;
        }
        int k = (a + 1 + j) % m->nv;
        const real *sg = &m->sig[3 * m->elem_edge[4 * e + k]];
        real nx, ny, len;
        path_normal(m, e, a, k, &nx, &ny, &len);
        real spx = rfma(sg[2], ny, sg[0] * nx);
        real spy = rfma(sg[1], ny, sg[2] * nx);
        G[j] = R(0.5) * rfma(duy, spy, dux * spx);
    }
    return H;
}

/* Element decision over the n candidate paths (Sec. 2.2: n = 2 for CST,
 * the list after Fig. 2-2; n = 3 for Q4, the list after Fig. 2-3).  Returns
 * the chosen path index j (k = a+1+j) or -1. */
static int element_rule(int n, const real *G, real Gc, real gamma) {
    int best = -1;
    for (int j = 0; j < n; ++j)
        if (G[j] > Gc && (best < 0 || G[j] > G[best])) best = j;
    if (best < 0) return -1;
    for (int j = 0; j < n; ++j) {
        if (j == best || !(G[j] > Gc)) continue;
        if (!(G[best] > gamma * (G[best] - G[j]))) return -1;
    }
    return best;
}

/* exported form (values rounded to real) */
int orc_element_rule_n(int n, const double *G, double Gc, double gamma) {
    real g[3] = {0, 0, 0};
    if (n < 1 || n > 3) return -1;
    for (int j = 0; j < n; ++j) g[j] = (real)G[j];
    return element_rule(n, g, (real)Gc, (real)gamma);
}

int orc_element_rule(const double G[3], double Gc, double gamma) {
    return orc_element_rule_n(3, G, Gc, gamma);
}

/* Near-threshold records (see orc_near_t).  A decision is near when its
 * margin is within near_tol relative to the value that decides it:
 * |G - Gc| <= tol Gc, G1 - G2 <= tol G1, |G1 - gamma (G1 - Gj)| <= tol G1,
 * each evaluated in the step's precision. */
static void near_push(orc_model_t *m, int elem, int a, int kind, int k, real G, real ref) {
    if (m->nnear == m->capnear) {
        m->capnear = m->capnear ? 2 * m->capnear : 256;
        m->near = realloc(m->near, sizeof(orc_near_t) * (size_t)m->capnear);
    }
    orc_near_t r = {(int)m->step, elem, a, kind, k, (double)G, (double)ref};
    m->near[m->nnear++] = r;
}

/* Records of one evaluated candidate (element f, tip edge a; its n path
 * values G, gate open): every path near Gc; with two or more paths above Gc
 * the gap between the largest two and every split-ratio margin of the
 * element rule. */
static void near_candidate(orc_model_t *m, int f, int a, int n, const real *G, real Gc) {
    const real tol = (real)m->near_tol, gamma = (real)m->gamma;
    for (int j = 0; j < n; ++j)
        if (fabs(G[j] - Gc) <= tol * Gc) near_push(m, f, a, 1, (a + 1 + j) % m->nv, G[j], Gc);
    int best = -1, nS = 0;
    for (int j = 0; j < n; ++j)
        if (G[j] > Gc) {
            nS++;
            if (best < 0 || G[j] > G[best]) best = j;
        }
    if (nS < 2) return;
    real second = R(-1.0);
    for (int j = 0; j < n; ++j)
        if (j != best && G[j] > Gc && G[j] > second) second = G[j];
    if (G[best] - second <= tol * G[best]) near_push(m, f, a, 2, (a + 1 + best) % m->nv, G[best], second);
    for (int j = 0; j < n; ++j) {
        if (j == best || !(G[j] > Gc)) continue;
        if (fabs(G[best] - gamma * (G[best] - G[j])) <= tol * G[best])
            near_push(m, f, a, 3, (a + 1 + j) % m->nv, G[best], G[j]);
    }
}

/* Records of the global pick over n >= 1 accepted candidates with best c:
 * the gap to the second largest G (n >= 2) and the split-ratio margin
 * against the smallest accepted G. */
static void near_pick(orc_model_t *m, int n, const real *G, const int *elem, const int *a, const int *k, int c) {
    const real tol = (real)m->near_tol, gamma = (real)m->gamma;
    real second = R(-1.0), gmin = G[c];
    for (int i = 0; i < n; ++i) {
        if (G[i] < gmin) gmin = G[i];
        if (i != c && G[i] > second) second = G[i];
    }
    if (n >= 2 && G[c] - second <= tol * G[c]) near_push(m, elem[c], a[c], 4, k[c], G[c], second);
    if (fabs(G[c] - gamma * (G[c] - gmin)) <= tol * G[c]) near_push(m, elem[c], a[c], 5, k[c], G[c], gmin);
}

/* MCT pick (Sec. 3): the candidate with the largest G (ties: lower element
 * id, then lower tip edge) provided it passes the split-ratio test against
 * every other candidate.  Returns its index or -1. */
static int mct_pick(int n, const real *G, const int *elem, const int *a, real gamma) {
    int best = -1;
    for (int c = 0; c < n; ++c) {
        if (best < 0 || G[c] > G[best] ||
            (G[c] == G[best] && (elem[c] < elem[best] || (elem[c] == elem[best] && a[c] < a[best]))))
            best = c;
    }
    if (best < 0) return -1;
    for (int c = 0; c < n; ++c) {
        if (c == best) continue;
        if (!(G[best] > gamma * (G[best] - G[c]))) return -1;
    }
    return best;
}

/* exported form (values rounded to real) */
int orc_mct_pick(int n, const double *G, const int *elem, const int *a, double gamma) {
    real *g = malloc(sizeof(real) * (size_t)(n > 0 ? n : 1));
    for (int c = 0; c < n; ++c) g[c] = (real)G[c];
    int r = mct_pick(n, g, elem, a, (real)gamma);
    free(g);
    return r;
}

/* Reference midpoint of the tip edge a of element e (the quadrature point
 * G0 of the candidate). */
static void tip_midpoint(const orc_model_t *m, int e, int a, double *x, double *y) {
    int p = m->conn[4 * e + a], q = m->conn[4 * e + (a + 1) % m->nv];
    *x = 0.5 * (m->X[p] + m->X[q]);
    *y = 0.5 * (m->Y[p] + m->Y[q]);
}

/* key order of the pick: larger G, then lower element id, then lower tip edge */
static int better_key(real G1, int e1, int a1, real G2, int e2, int a2) {
    if (G1 != G2) return G1 > G2;
    if (e1 != e2) return e1 < e2;
    return a1 < a2;
}

/* Per-front pick (variant): candidate c splits iff, against every other
 * accepted candidate c' it competes with -- the same element, or a tip point
 * closer than rho (squared distance < rho^2) -- it has the better key and
 * passes the split-ratio test G_c > gamma (G_c - G_c').  With rho = infinity
 * this is the global pick.  Picked candidates never compete with each
 * other, so their elements are distinct.  Writes the picked indices, in key
 * order, to out; returns their count. */
static int front_pick(int n, const real *G, const int *elem, const int *a, const double *x, const double *y,
                      real gamma, double rho2, int *out) {
    int np = 0;
    for (int c = 0; c < n; ++c) {
        int ok = 1;
        for (int d = 0; d < n && ok; ++d) {
            if (d == c) continue;
            double dx = x[c] - x[d], dy = y[c] - y[d];
            int compete = elem[c] == elem[d] || dx * dx + dy * dy < rho2;
            if (!compete) continue;
            if (!better_key(G[c], elem[c], a[c], G[d], elem[d], a[d])) ok = 0;
            if (!(G[c] > gamma * (G[c] - G[d]))) ok = 0;
        }
        if (ok) out[np++] = c;
    }
    /* key order (insertion sort, small sets) */
    for (int i = 1; i < np; ++i) {
        int v = out[i], j = i - 1;
        while (j >= 0 && better_key(G[v], elem[v], a[v], G[out[j]], elem[out[j]], a[out[j]])) {
            out[j + 1] = out[j];
            j--;
        }
        out[j + 1] = v;
    }
    return np;
}

/* exported form (values rounded to real) */
int orc_front_pick(int n, const double *G, const int *elem, const int *a, const double *x, const double *y,
                   double gamma, double rho2, int *out) {
    real *g = malloc(sizeof(real) * (size_t)(n > 0 ? n : 1));
    for (int c = 0; c < n; ++c) g[c] = (real)G[c];
    int r = front_pick(n, g, elem, a, x, y, (real)gamma, rho2, out);
    free(g);
    return r;
}

/* Free-surface candidate (R: edge with exactly one intact neighbour, i.e. a
 * domain-boundary edge of an intact element or an edge shared with a split
 * element).  Sets the intact element f and the local index a of the edge in
 * it. */
static int edge_candidate(const orc_model_t *m, int s, int *f, int *a) {
    int e0 = m->edge_elem[2 * s], e1 = m->edge_elem[2 * s + 1];
    int i0 = is_intact(m, e0), i1 = is_intact(m, e1);
    if (i0 + i1 != 1) return 0;
    *f = i0 ? e0 : e1;
    *a = i0 ? m->edge_loc[2 * s] : m->edge_loc[2 * s + 1];
    return 1;
}

/* a5 + a6: evaluate every free-surface quadrature point, pick, split. */
/* Neighbour element across local edge k of element e, or -1. */
static int neighbour(const orc_model_t *m, int e, int k) {
    int s = m->elem_edge[4 * e + k];
    int e0 = m->edge_elem[2 * s], e1 = m->edge_elem[2 * s + 1];
    return e0 == e ? e1 : e0;
}

/* The tip after element f split with exit edge k: the element across k
 * with the same edge, if it exists and is intact; else none. */
static int tip_after(const orc_model_t *m, int f, int k) {
    int nb = neighbour(m, f, k);
    if (nb < 0 || !is_intact(m, nb)) return -1;
    int s = m->elem_edge[4 * f + k];
    int loc = m->edge_elem[2 * s] == nb ? m->edge_loc[2 * s] : m->edge_loc[2 * s + 1];
    return 4 * nb + loc;
}

static void record_split(orc_model_t *m, int f, int a, int k, real G) {
    m->split[f] = (unsigned char)(SPLIT_FLAG | (unsigned)(a << 2) | (unsigned)k);
    if (m->nlog == m->caplog) {
        m->caplog = m->caplog ? 2 * m->caplog : 1024;
        m->log = realloc(m->log, sizeof(orc_split_t) * (size_t)m->caplog);
    }
    orc_split_t rec = {(int)m->step, f, a, k, (double)G};
    m->log[m->nlog++] = rec;
    real nx, ny, len;
    path_normal(m, f, a, k, &nx, &ny, &len);
    m->Ud += (double)(r_gc(m, f) * len);
}

/* Single crack-tip tracking: the element rule at the current tip only. */
static void sct_phase(orc_model_t *m) {
    if (m->tip < 0) return;
    int f = m->tip >> 2, a = m->tip & 3;
    int s = m->elem_edge[4 * f + a], ff, aa;
    if (!edge_candidate(m, s, &ff, &aa) || ff != f) return;
    real G[3];
    int H = candidate_G(m, f, a, G);
    if (H && m->near_tol > 0.0) near_candidate(m, f, a, m->nv - 1, G, r_gc(m, f));
    int j = element_rule(m->nv - 1, G, r_gc(m, f), (real)m->gamma);
    if (j < 0) return;
    int k = (a + 1 + j) % m->nv;
    record_split(m, f, a, k, G[j]);
    m->tip = tip_after(m, f, k);
}

static void fracture_phase(orc_model_t *m) {
    if (m->sct) {
        sct_phase(m);
        return;
    }
    int cap = m->ns;
    real *cG = malloc(sizeof(real) * (size_t)cap);
    int *cE = malloc(sizeof(int) * (size_t)cap), *cA = malloc(sizeof(int) * (size_t)cap);
    int *cK = malloc(sizeof(int) * (size_t)cap);
    /* per edge: accepted path index or -1 (evaluated independently) */
    int *acc = malloc(sizeof(int) * (size_t)cap);
    real *accG = malloc(sizeof(real) * (size_t)cap);
    /* near-threshold log: every candidate's gate and path values */
    const int near = m->near_tol > 0.0;
    real *allG = near ? malloc(sizeof(real) * 3 * (size_t)cap) : NULL;
    unsigned char *gate = near ? calloc((size_t)cap, 1) : NULL;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int s = 0; s < m->ns; ++s) {
        int f, a;
        acc[s] = -1;
        if (!edge_candidate(m, s, &f, &a)) continue;
        real G[3];
        int H = candidate_G(m, f, a, G);
        if (near) {
            gate[s] = (unsigned char)H;
            for (int j = 0; j < 3; ++j) allG[3 * s + j] = G[j];
        }
        int j = element_rule(m->nv - 1, G, r_gc(m, f), (real)m->gamma);
        if (j < 0) continue;
        acc[s] = j;
        accG[s] = G[j];
    }
    /* near-threshold records of the candidates, in edge-id order */
    if (near) {
        for (int s = 0; s < m->ns; ++s) {
            int f, a;
            if (!gate[s] || !edge_candidate(m, s, &f, &a)) continue;
            near_candidate(m, f, a, m->nv - 1, &allG[3 * s], r_gc(m, f));
        }
        free(allG);
        free(gate);
    }
    /* accepted candidates in edge-id order */
    int nc = 0;
    for (int s = 0; s < m->ns; ++s) {
        if (acc[s] < 0) continue;
        int f, a;
        edge_candidate(m, s, &f, &a);
        cG[nc] = accG[s];
        cE[nc] = f;
        cA[nc] = a;
        cK[nc] = (a + 1 + acc[s]) % m->nv;
        nc++;
    }
    free(acc);
    free(accG);
    if (m->front_r2 > 0.0) {
        double *px = malloc(sizeof(double) * (size_t)(nc ? nc : 1));
        double *py = malloc(sizeof(double) * (size_t)(nc ? nc : 1));
        int *pick = malloc(sizeof(int) * (size_t)(nc ? nc : 1));
        for (int i = 0; i < nc; ++i) tip_midpoint(m, cE[i], cA[i], &px[i], &py[i]);
        int np = front_pick(nc, cG, cE, cA, px, py, (real)m->gamma, m->front_r2, pick);
        for (int i = 0; i < np; ++i) record_split(m, cE[pick[i]], cA[pick[i]], cK[pick[i]], cG[pick[i]]);
        free(px);
        free(py);
        free(pick);
    } else {
        int c = mct_pick(nc, cG, cE, cA, (real)m->gamma);
        if (near && nc > 0) {
            /* the best key, whether or not it passes the split-ratio test */
            int b = 0;
            for (int i = 1; i < nc; ++i)
                if (better_key(cG[i], cE[i], cA[i], cG[b], cE[b], cA[b])) b = i;
            near_pick(m, nc, cG, cE, cA, cK, b);
        }
        if (c >= 0) record_split(m, cE[c], cA[c], cK[c], cG[c]);
    }
    free(cG);
    free(cE);
    free(cA);
    free(cK);
}

/* ------------------------------------------------------------------ */
/* a4: central-difference step                                          */
/* ------------------------------------------------------------------ */

/* v0 times the ramp factor t / t_ramp (binary64, rounded to real) */
static real prescribed(const orc_model_t *m, real v0, double t) {
    if (m->t_ramp > 0.0 && t < m->t_ramp) return v0 * (real)(t / m->t_ramp);
    return v0;
}

/* Load factor of the tractions at time t (the pressure history of Sec. 4.4
 * is supplied as such a curve). */
double orc_load_factor(const orc_model_t *m, double t) {
    if (m->ncurve == 0) return 1.0;
    if (t <= m->curve_t[0]) return m->curve_phi[0];
    int n = m->ncurve;
    if (t >= m->curve_t[n - 1]) return m->curve_phi[n - 1];
    int i = 0;
    while (m->curve_t[i + 1] <= t) i++;
    double slope = (m->curve_phi[i + 1] - m->curve_phi[i]) / (m->curve_t[i + 1] - m->curve_t[i]);
    return m->curve_phi[i] + (t - m->curve_t[i]) * slope;
}

static void one_step(orc_model_t *m) {
    internal_forces(m);
    const real phi = (real)orc_load_factor(m, (double)m->step * m->dt);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->nn; ++i) {
        const real mi = (real)m->minv[i];
        m->ax[i] = (phi * (real)m->fext[2 * i] - m->fx[i]) * mi;
        m->ay[i] = (phi * (real)m->fext[2 * i + 1] - m->fy[i]) * mi;
        if (m->vmask[i] & 1) m->ax[i] = 0.0;
        if (m->vmask[i] & 2) m->ay[i] = 0.0;
    }
    /* fracture on (u^k, sigma^k); the split acts from step k+1 */
    fracture_phase(m);
    const real dt = (real)m->dt;
    const real dtv = (m->step == 0) ? R(0.5) * dt : dt;
    const double th = ((double)m->step + 0.5) * m->dt;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->nn; ++i) {
        real vx = m->vx[i] + dtv * m->ax[i];
        real vy = m->vy[i] + dtv * m->ay[i];
        if (m->vmask[i] & 1) vx = prescribed(m, (real)m->v0[2 * i], th);
        if (m->vmask[i] & 2) vy = prescribed(m, (real)m->v0[2 * i + 1], th);
        m->vx[i] = vx;
        m->vy[i] = vy;
        m->ux[i] = m->ux[i] + dt * vx;
        m->uy[i] = m->uy[i] + dt * vy;
    }
    m->step++;
}

/* ------------------------------------------------------------------ */
/* set-up                                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int lo, hi, e, k;
} edge_rec_t;

static int cmp_edge_rec(const void *pa, const void *pb) {
    const edge_rec_t *a = pa, *b = pb;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    if (a->e != b->e) return a->e < b->e ? -1 : 1;
    return 0;
}

static void *zalloc(size_t n) { return calloc(n ? n : 1, 1); }

void orc_destroy(orc_model_t *m) {
    if (!m) return;
    void *ptrs[] = {m->X, m->Y, m->conn, m->edge_node, m->edge_elem, m->edge_loc, m->elem_edge,
                    m->color, m->area, m->Gc, m->edge_trac, m->edge_loaded, m->vmask, m->v0,
                    m->mass, m->minv, m->fext, m->split, m->ux, m->uy, m->vx, m->vy, m->log,
                    m->sig, m->eps, m->sig_ok, m->fe, m->fx, m->fy, m->ax, m->ay, m->curve_t,
                    m->curve_phi, m->near};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
    free(m);
}

/* Edge table, element->edge map, greedy colouring, areas and the per-node
 * and per-edge arrays of a model whose nv, nn, ne, X, Y and conn are set.
 * Returns 0, or ORC_EINVAL for a mesh that is not a valid 2-manifold with
 * consistently oriented elements (an edge used by more than two elements, or
 * twice in the same direction). */
static int build_tables(orc_model_t *m) {
    const int nv = m->nv;
    /* edge table: every (element, local edge) keyed by its sorted node pair */
    edge_rec_t *r = zalloc(sizeof(edge_rec_t) * 4 * m->ne);
    for (int e = 0; e < m->ne; ++e)
        for (int k = 0; k < nv; ++k) {
            int a = m->conn[4 * e + k], b = m->conn[4 * e + (k + 1) % nv];
            edge_rec_t t = {a < b ? a : b, a < b ? b : a, e, k};
            r[nv * e + k] = t;
        }
    qsort(r, (size_t)nv * m->ne, sizeof(edge_rec_t), cmp_edge_rec);
    m->edge_node = zalloc(sizeof(int) * 2 * nv * m->ne);
    m->edge_elem = zalloc(sizeof(int) * 2 * nv * m->ne);
    m->edge_loc = zalloc(sizeof(int) * 2 * nv * m->ne);
    m->elem_edge = zalloc(sizeof(int) * 4 * m->ne);
    int ns = 0, bad = 0;
    for (int i = 0; i < nv * m->ne; ++i) {
        if (i > 0 && r[i].lo == r[i - 1].lo && r[i].hi == r[i - 1].hi) {
            if (m->edge_elem[2 * (ns - 1) + 1] >= 0) bad = 1; /* third use */
            int e0 = m->edge_elem[2 * (ns - 1)], k0 = m->edge_loc[2 * (ns - 1)];
            if (m->conn[4 * e0 + k0] == m->conn[4 * r[i].e + r[i].k]) bad = 1; /* same direction */
            m->edge_elem[2 * (ns - 1) + 1] = r[i].e;
            m->edge_loc[2 * (ns - 1) + 1] = r[i].k;
        } else {
            m->edge_node[2 * ns] = r[i].lo;
            m->edge_node[2 * ns + 1] = r[i].hi;
            m->edge_elem[2 * ns] = r[i].e;
            m->edge_loc[2 * ns] = r[i].k;
            m->edge_elem[2 * ns + 1] = -1;
            m->edge_loc[2 * ns + 1] = -1;
            ns++;
        }
        m->elem_edge[4 * r[i].e + r[i].k] = ns - 1;
    }
    free(r);
    m->ns = ns;
    /* greedy colouring in element-id order: smallest colour not used by an
     * already coloured element that shares a node */
    m->color = zalloc(sizeof(int) * m->ne);
    int *node_cnt = zalloc(sizeof(int) * (m->nn + 1));
    for (int e = 0; e < m->ne; ++e)
        for (int n = 0; n < nv; ++n) node_cnt[m->conn[4 * e + n] + 1]++;
    for (int i = 0; i < m->nn; ++i) node_cnt[i + 1] += node_cnt[i];
    int *node_el = zalloc(sizeof(int) * nv * m->ne);
    int *fill = zalloc(sizeof(int) * m->nn);
    for (int e = 0; e < m->ne; ++e)
        for (int n = 0; n < nv; ++n) {
            int g = m->conn[4 * e + n];
            node_el[node_cnt[g] + fill[g]++] = e;
        }
    m->ncolor = 0;
    for (int e = 0; e < m->ne && !bad; ++e) {
        unsigned long long used = 0;
        for (int n = 0; n < nv; ++n) {
            int g = m->conn[4 * e + n];
            for (int t = node_cnt[g]; t < node_cnt[g + 1]; ++t)
                if (node_el[t] < e) used |= 1ull << m->color[node_el[t]];
        }
        int c = 0;
        while (c < 64 && (used & (1ull << c))) c++;
        if (c == 64) bad = 1;
        m->color[e] = c;
        if (c + 1 > m->ncolor) m->ncolor = c + 1;
    }
    free(node_cnt);
    free(node_el);
    free(fill);
    m->area = zalloc(sizeof(double) * m->ne);
    for (int e = 0; e < m->ne; ++e) {
        double x[4], y[4];
        elem_coords_d(m, e, x, y);
        m->area[e] = nv == 4 ? quad_area(x, y) : tri_area_d(x, y);
    }
    m->Gc = zalloc(sizeof(double) * m->ne);
    m->edge_trac = zalloc(sizeof(double) * 2 * ns);
    m->edge_loaded = zalloc(ns);
    m->vmask = zalloc(m->nn);
    m->v0 = zalloc(sizeof(double) * 2 * m->nn);
    m->mass = zalloc(sizeof(double) * m->nn);
    m->minv = zalloc(sizeof(double) * m->nn);
    m->fext = zalloc(sizeof(double) * 2 * m->nn);
    m->split = zalloc(m->ne);
    m->ux = zalloc(sizeof(real) * m->nn);
    m->uy = zalloc(sizeof(real) * m->nn);
    m->vx = zalloc(sizeof(real) * m->nn);
    m->vy = zalloc(sizeof(real) * m->nn);
    m->sig = zalloc(sizeof(real) * 3 * ns);
    m->eps = zalloc(sizeof(real) * 3 * ns);
    m->sig_ok = zalloc(ns);
    m->fe = zalloc(sizeof(real) * 8 * m->ne);
    m->fx = zalloc(sizeof(real) * m->nn);
    m->fy = zalloc(sizeof(real) * m->nn);
    m->ax = zalloc(sizeof(real) * m->nn);
    m->ay = zalloc(sizeof(real) * m->nn);
    m->gamma = 1.0;
    m->cfl = 0.5;
    return bad ? ORC_EINVAL : ORC_OK;
}

static orc_model_t *new_model(int nv, int nn, int ne, const double *X, const double *Y) {
    orc_model_t *m = zalloc(sizeof(orc_model_t));
    m->tip = -1;
    m->nv = nv;
    m->nn = nn;
    m->ne = ne;
    m->X = zalloc(sizeof(double) * nn);
    m->Y = zalloc(sizeof(double) * nn);
    memcpy(m->X, X, sizeof(double) * nn);
    memcpy(m->Y, Y, sizeof(double) * nn);
    m->conn = zalloc(sizeof(int) * 4 * ne);
    return m;
}

/* Structured nx x ny Q4 grid with the given node coordinates (node (i,j) has
 * id j*(nx+1)+i; element (i,j) id j*nx+i with CCW nodes (i,j),(i+1,j),
 * (i+1,j+1),(i,j+1)).  Tables are then built generically from conn. */
orc_model_t *orc_create(int nx, int ny, const double *X, const double *Y) {
    if (nx < 2 || ny < 2) return NULL;
    orc_model_t *m = new_model(4, (nx + 1) * (ny + 1), nx * ny, X, Y);
    m->nx = nx;
    m->ny = ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int e = j * nx + i;
            m->conn[4 * e + 0] = j * (nx + 1) + i;
            m->conn[4 * e + 1] = j * (nx + 1) + i + 1;
            m->conn[4 * e + 2] = (j + 1) * (nx + 1) + i + 1;
            m->conn[4 * e + 3] = (j + 1) * (nx + 1) + i;
        }
    build_tables(m);
    return m;
}

/* Unstructured CST mesh: nn nodes, ne triangles with counter-clockwise node
 * triples conn[3 e + 0..2].  Returns NULL for an index out of range, a
 * repeated node in one triangle, or a mesh build_tables rejects.  Positive
 * areas are checked at finalize. */
orc_model_t *orc_create_tri(int nn, const double *X, const double *Y, int ne, const int *conn) {
    if (nn < 3 || ne < 1) return NULL;
    for (int e = 0; e < ne; ++e) {
        const int *c = &conn[3 * e];
        for (int n = 0; n < 3; ++n)
            if (c[n] < 0 || c[n] >= nn) return NULL;
        if (c[0] == c[1] || c[1] == c[2] || c[0] == c[2]) return NULL;
    }
    orc_model_t *m = new_model(3, nn, ne, X, Y);
    for (int e = 0; e < ne; ++e) {
        for (int n = 0; n < 3; ++n) m->conn[4 * e + n] = conn[3 * e + n];
        m->conn[4 * e + 3] = -1;
    }
    if (build_tables(m) != ORC_OK) {
        orc_destroy(m);
        return NULL;
    }
    return m;
}

/* Unstructured Q4 mesh: nn nodes, ne quadrilaterals with counter-clockwise
 * node quadruples conn[4 e + 0..3] (local edge k joins local nodes k and
 * k+1 mod 4, as on the structured grid).  Returns NULL for an index out of
 * range, a repeated node in one element, or a mesh build_tables rejects.
 * Positive areas are checked at finalize. */
orc_model_t *orc_create_q4(int nn, const double *X, const double *Y, int ne, const int *conn) {
    if (nn < 4 || ne < 1) return NULL;
    for (int e = 0; e < ne; ++e) {
        const int *c = &conn[4 * e];
        for (int n = 0; n < 4; ++n) {
            if (c[n] < 0 || c[n] >= nn) return NULL;
            for (int q = 0; q < n; ++q)
                if (c[q] == c[n]) return NULL;
        }
    }
    orc_model_t *m = new_model(4, nn, ne, X, Y);
    memcpy(m->conn, conn, sizeof(int) * 4 * (size_t)ne);
    if (build_tables(m) != ORC_OK) {
        orc_destroy(m);
        return NULL;
    }
    return m;
}

int orc_set_material(orc_model_t *m, double E, double nu, double rho, const double *Gc,
                     double Gc_uniform, double gamma) {
    if (!(E > 0.0) || !(nu > -1.0 && nu < 0.5) || !(rho > 0.0) || !(gamma > 0.0)) return ORC_EINVAL;
    m->E = E;
    m->nu = nu;
    m->rho = rho;
    m->gamma = gamma;
    m->D11 = E / (1.0 - nu * nu);
    m->D12 = nu * m->D11;
    m->D33 = E / (2.0 * (1.0 + nu));
    for (int e = 0; e < m->ne; ++e) m->Gc[e] = Gc ? Gc[e] : Gc_uniform;
    return ORC_OK;
}

static int find_edge(const orc_model_t *m, int a, int b) {
    int lo = a < b ? a : b, hi = a < b ? b : a;
    int l = 0, h = m->ns - 1;
    while (l <= h) {
        int mid = (l + h) / 2;
        int ml = m->edge_node[2 * mid], mh = m->edge_node[2 * mid + 1];
        if (ml == lo && mh == hi) return mid;
        if (ml < lo || (ml == lo && mh < hi))
            l = mid + 1;
        else
            h = mid - 1;
    }
    return -1;
}

/* Constant traction t (Pa, 2 per edge) on boundary edges given by node pairs. */
int orc_set_traction(orc_model_t *m, int n, const int *edge_nodes, const double *t) {
    for (int i = 0; i < n; ++i) {
        int s = find_edge(m, edge_nodes[2 * i], edge_nodes[2 * i + 1]);
        if (s < 0 || m->edge_elem[2 * s + 1] >= 0 || m->edge_loaded[s]) return ORC_EINVAL;
        m->edge_loaded[s] = 1;
        m->edge_trac[2 * s] = t[2 * i];
        m->edge_trac[2 * s + 1] = t[2 * i + 1];
    }
    return ORC_OK;
}

int orc_set_velocity_bc(orc_model_t *m, int n, const int *node, const unsigned char *mask,
                        const double *v0, double t_ramp) {
    for (int i = 0; i < n; ++i) {
        if (node[i] < 0 || node[i] >= m->nn || (mask[i] & ~3u)) return ORC_EINVAL;
        m->vmask[node[i]] = mask[i];
        m->v0[2 * node[i]] = v0[2 * i];
        m->v0[2 * node[i] + 1] = v0[2 * i + 1];
    }
    m->t_ramp = t_ramp;
    return ORC_OK;
}

int orc_set_notch(orc_model_t *m, int n, const int *elem, const unsigned char *entry,
                  const unsigned char *exitp) {
    for (int i = 0; i < n; ++i) {
        if (elem[i] < 0 || elem[i] >= m->ne || entry[i] >= m->nv || exitp[i] >= m->nv ||
            entry[i] == exitp[i])
            return ORC_EINVAL;
        m->split[elem[i]] = (unsigned char)(SPLIT_FLAG | (unsigned)(entry[i] << 2) | exitp[i]);
    }
    return ORC_OK;
}

int orc_set_time(orc_model_t *m, double dt, double cfl) {
    m->dt_in = dt;
    m->cfl = cfl;
    return ORC_OK;
}

int orc_finalize(orc_model_t *m) {
    if (!(m->E > 0.0)) return ORC_ESTATE;
    /* lumped mass, element-id order */
    for (int i = 0; i < m->nn; ++i) m->mass[i] = 0.0;
    for (int e = 0; e < m->ne; ++e) {
        if (!(m->area[e] > 0.0)) return ORC_EINVAL;
        double me = m->rho * m->area[e] / (double)m->nv;
        for (int n = 0; n < m->nv; ++n) m->mass[m->conn[4 * e + n]] += me;
    }
    for (int i = 0; i < m->nn; ++i) {
        if (!(m->mass[i] > 0.0)) return ORC_EINVAL; /* a node in no element */
        m->minv[i] = 1.0 / m->mass[i];
    }
    /* consistent nodal forces of the edge tractions, edge-id order */
    for (int i = 0; i < 2 * m->nn; ++i) m->fext[i] = 0.0;
    for (int s = 0; s < m->ns; ++s) {
        if (!m->edge_loaded[s]) continue;
        int a = m->edge_node[2 * s], b = m->edge_node[2 * s + 1];
        double dx = m->X[b] - m->X[a], dy = m->Y[b] - m->Y[a];
        double L = sqrt(dx * dx + dy * dy);
        double fx = m->edge_trac[2 * s] * L * 0.5, fy = m->edge_trac[2 * s + 1] * L * 0.5;
        m->fext[2 * a] += fx;
        m->fext[2 * a + 1] += fy;
        m->fext[2 * b] += fx;
        m->fext[2 * b + 1] += fy;
    }
    /* time step: fraction of (shortest edge) / dilatational wave speed */
    if (m->dt_in > 0.0) {
        m->dt = m->dt_in;
    } else {
        double hmin = INFINITY;
        for (int s = 0; s < m->ns; ++s) {
            int a = m->edge_node[2 * s], b = m->edge_node[2 * s + 1];
            double dx = m->X[b] - m->X[a], dy = m->Y[b] - m->Y[a];
            double L = sqrt(dx * dx + dy * dy);
            if (L < hmin) hmin = L;
        }
        double cd = sqrt(m->E / (m->rho * (1.0 - m->nu * m->nu)));
        m->dt = m->cfl * hmin / cd;
    }
    if (m->sct && m->tip == -2) {
        /* the start tip: the one path end of the pre-notch (an entry or exit
         * edge of a split element whose neighbour is intact) */
        int found = -1, count = 0;
        for (int e = 0; e < m->ne; ++e) {
            if (!m->split[e]) continue;
            int ks[2] = {(m->split[e] >> 2) & 3, m->split[e] & 3};
            for (int q = 0; q < 2; ++q) {
                int t = tip_after(m, e, ks[q]);
                if (t >= 0) {
                    found = t;
                    count++;
                }
            }
        }
        if (count != 1) return ORC_EINVAL;
        m->tip = found;
    }
    m->finalized = 1;
    return ORC_OK;
}

/* Tracking mode: 0 multiple crack tips (default), 1 single crack tip with
 * start tip (element, local edge), or elem < 0 to take the pre-notch's one
 * path end at finalize. */
int orc_set_tracking(orc_model_t *m, int mode, int elem, int edge) {
    if (mode != 0 && mode != 1) return ORC_EINVAL;
    if (mode == 1 && elem >= 0 && (elem >= m->ne || edge < 0 || edge >= m->nv)) return ORC_EINVAL;
    m->sct = mode;
    m->tip = mode == 1 ? (elem >= 0 ? 4 * elem + edge : -2) : -1;
    return ORC_OK;
}

int orc_get_tip(const orc_model_t *m) { return m->tip; }

/* Q4 edge smoothing: 0 the point rule (default), 1 sub-cells. */
int orc_set_smoothing(orc_model_t *m, int mode) {
    if (mode != 0 && mode != 1) return ORC_EINVAL;
    m->subcell = mode;
    return ORC_OK;
}

/* Per-front pick with competition radius rho (> 0; infinity = the global
 * pick); rho = 0 restores the global pick.  Not with single-tip tracking. */
int orc_set_front_pick(orc_model_t *m, double rho) {
    if (!(rho >= 0.0)) return ORC_EINVAL;
    m->front_r2 = rho * rho;
    return ORC_OK;
}

/* Near-threshold decision log with relative tolerance tol (> 0; 0 = off);
 * clears the records. */
int orc_set_near_log(orc_model_t *m, double tol) {
    if (!(tol >= 0.0)) return ORC_EINVAL;
    m->near_tol = tol;
    m->nnear = 0;
    return ORC_OK;
}

int orc_near_count(const orc_model_t *m) { return m->nnear; }

/* Test hooks: the records one candidate (n path values, gate open) or one
 * pick over n accepted candidates (best c) adds at the model's current step
 * (values rounded to real). */
int orc_near_candidate(orc_model_t *m, int f, int a, int n, const double *G, double Gc) {
    real g[3] = {0, 0, 0};
    if (n < 1 || n > 3) return ORC_EINVAL;
    for (int j = 0; j < n; ++j) g[j] = (real)G[j];
    near_candidate(m, f, a, n, g, (real)Gc);
    return ORC_OK;
}

int orc_near_pick(orc_model_t *m, int n, const double *G, const int *elem, const int *a, const int *k, int c) {
    if (n < 1 || c < 0 || c >= n) return ORC_EINVAL;
    real *g = malloc(sizeof(real) * (size_t)n);
    for (int i = 0; i < n; ++i) g[i] = (real)G[i];
    near_pick(m, n, g, elem, a, k, c);
    free(g);
    return ORC_OK;
}

/* The records in the order they were made (steps ascending; in a step the
 * candidates' records in edge-id order, then the pick's). */
void orc_get_near(const orc_model_t *m, int *step, int *elem, int *a, int *kind, int *k, double *G, double *ref) {
    for (int i = 0; i < m->nnear; ++i) {
        const orc_near_t *r = &m->near[i];
        step[i] = r->step;
        elem[i] = r->elem;
        a[i] = r->a;
        kind[i] = r->kind;
        k[i] = r->k;
        G[i] = r->G;
        ref[i] = r->ref;
    }
}

/* Traction load curve (n >= 2 points, t strictly increasing), n = 0 clears. */
int orc_set_load_curve(orc_model_t *m, int n, const double *t, const double *phi) {
    if (n != 0 && n < 2) return ORC_EINVAL;
    for (int i = 0; i + 1 < n; ++i)
        if (!(t[i + 1] > t[i])) return ORC_EINVAL;
    free(m->curve_t);
    free(m->curve_phi);
    m->curve_t = m->curve_phi = NULL;
    m->ncurve = n;
    if (n) {
        m->curve_t = malloc(sizeof(double) * (size_t)n);
        m->curve_phi = malloc(sizeof(double) * (size_t)n);
        memcpy(m->curve_t, t, sizeof(double) * (size_t)n);
        memcpy(m->curve_phi, phi, sizeof(double) * (size_t)n);
    }
    return ORC_OK;
}

int orc_step(orc_model_t *m, long n) {
    if (!m->finalized) return ORC_ESTATE;
    for (long i = 0; i < n; ++i) one_step(m);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* queries and test hooks                                               */
/* ------------------------------------------------------------------ */

void orc_info(const orc_model_t *m, int *ints /*nn,ne,ns,ncolor,nlog,nv*/,
              double *dbls /*dt,Ud*/, long *step) {
    ints[0] = m->nn;
    ints[1] = m->ne;
    ints[2] = m->ns;
    ints[3] = m->ncolor;
    ints[4] = m->nlog;
    ints[5] = m->nv;
    dbls[0] = m->dt;
    dbls[1] = m->Ud;
    *step = m->step;
}

/* binary32 build: the state and the step's results are exact in binary64;
 * inputs given in binary64 are rounded */
static void to_double(int n, const real *a, double *out) {
    for (int i = 0; i < n; ++i) out[i] = (double)a[i];
}

static void to_real(int n, const double *a, real *out) {
    for (int i = 0; i < n; ++i) out[i] = (real)a[i];
}

int orc_precision(void) { return (int)(8 * sizeof(real)); }

void orc_get_state(const orc_model_t *m, double *ux, double *uy, double *vx, double *vy,
                   unsigned char *split) {
    to_double(m->nn, m->ux, ux);
    to_double(m->nn, m->uy, uy);
    to_double(m->nn, m->vx, vx);
    to_double(m->nn, m->vy, vy);
    memcpy(split, m->split, m->ne);
}

void orc_set_state(orc_model_t *m, const double *ux, const double *uy, const double *vx,
                   const double *vy) {
    to_real(m->nn, ux, m->ux);
    to_real(m->nn, uy, m->uy);
    to_real(m->nn, vx, m->vx);
    to_real(m->nn, vy, m->vy);
}

void orc_get_log(const orc_model_t *m, int *step, int *elem, int *entry, int *exitp, double *G) {
    for (int i = 0; i < m->nlog; ++i) {
        step[i] = m->log[i].step;
        elem[i] = m->log[i].elem;
        entry[i] = m->log[i].entry;
        exitp[i] = m->log[i].exit;
        G[i] = m->log[i].G;
    }
}

void orc_get_tables(const orc_model_t *m, int *edge_node, int *edge_elem, int *edge_loc,
                    int *color, double *area, double *mass, double *fext) {
    memcpy(edge_node, m->edge_node, sizeof(int) * 2 * m->ns);
    memcpy(edge_elem, m->edge_elem, sizeof(int) * 2 * m->ns);
    memcpy(edge_loc, m->edge_loc, sizeof(int) * 2 * m->ns);
    memcpy(color, m->color, sizeof(int) * m->ne);
    memcpy(area, m->area, sizeof(double) * m->ne);
    memcpy(mass, m->mass, sizeof(double) * m->nn);
    memcpy(fext, m->fext, sizeof(double) * 2 * m->nn);
}

/* internal force and edge stresses of an arbitrary displacement field
 * (the stored state is restored afterwards) */
void orc_internal_force(orc_model_t *m, const double *ux, const double *uy, double *fx,
                        double *fy, double *sig, unsigned char *sig_ok) {
    real *sx = m->ux, *sy = m->uy;
    real *tx = malloc(sizeof(real) * (size_t)m->nn), *ty = malloc(sizeof(real) * (size_t)m->nn);
    to_real(m->nn, ux, tx);
    to_real(m->nn, uy, ty);
    m->ux = tx;
    m->uy = ty;
    internal_forces(m);
    m->ux = sx;
    m->uy = sy;
    free(tx);
    free(ty);
    to_double(m->nn, m->fx, fx);
    to_double(m->nn, m->fy, fy);
    if (sig) to_double(3 * m->ns, m->sig, sig);
    if (sig_ok) memcpy(sig_ok, m->sig_ok, m->ns);
}

/* Every free-surface candidate of the current state: tip edge, element,
 * local edge a, the three G values, the element decision j (-1 = none).
 * Returns the count (or ORC_ECAPACITY with *count set). */
int orc_candidates(orc_model_t *m, int cap, int *edge, int *elem, int *a, double *G3, int *dec,
                   int *count) {
    edge_stresses(m);
    int nc = 0;
    for (int s = 0; s < m->ns; ++s) {
        int f, la;
        if (!edge_candidate(m, s, &f, &la)) continue;
        if (nc < cap) {
            real g[3];
            edge[nc] = s;
            elem[nc] = f;
            a[nc] = la;
            candidate_G(m, f, la, g);
            to_double(3, g, &G3[3 * nc]);
            dec[nc] = element_rule(m->nv - 1, g, r_gc(m, f), (real)m->gamma);
        }
        nc++;
    }
    *count = nc;
    return nc <= cap ? ORC_OK : ORC_ECAPACITY;
}

/* Crack-surface tips: edges with exactly one intact neighbour whose other
 * neighbour is a split element (the uncracked domain boundary excluded),
 * ascending edge id; xy = reference midpoint. */
int orc_tips(const orc_model_t *m, int cap, int *edge, double *xy, int *count) {
    int nt = 0;
    for (int s = 0; s < m->ns; ++s) {
        int e0 = m->edge_elem[2 * s], e1 = m->edge_elem[2 * s + 1];
        if (e0 < 0 || e1 < 0) continue;
        if (is_intact(m, e0) + is_intact(m, e1) != 1) continue;
        if (nt < cap) {
            int a = m->edge_node[2 * s], b = m->edge_node[2 * s + 1];
            edge[nt] = s;
            xy[2 * nt] = 0.5 * (m->X[a] + m->X[b]);
            xy[2 * nt + 1] = 0.5 * (m->Y[a] + m->Y[b]);
        }
        nt++;
    }
    *count = nt;
    return nt <= cap ? ORC_OK : ORC_ECAPACITY;
}

/* Energies at t_k: kinetic (v^k = v^{k-1/2} + dt/2 a^k; v^0 at k = 0),
 * strain (edge smoothing domains A_s = sum of intact A_j/4, plus split
 * pieces), external work f_ext(t_k) . u (load curve times the constant
 * tractions), dissipated Ud. */
/* (binary32 build: the sums run in binary64 over the binary32 forces,
 * stresses and state) */
void orc_energies(orc_model_t *m, double out[4]) {
    internal_forces(m);
    double ekin = 0.0, estr = 0.0, wext = 0.0;
    double phi = orc_load_factor(m, (double)m->step * m->dt);
    for (int i = 0; i < m->nn; ++i) {
        double ax = (phi * m->fext[2 * i] - (double)m->fx[i]) * m->minv[i];
        double ay = (phi * m->fext[2 * i + 1] - (double)m->fy[i]) * m->minv[i];
        double vx = m->vx[i], vy = m->vy[i];
        if (m->step > 0) {
            if (!(m->vmask[i] & 1)) vx = vx + 0.5 * m->dt * ax;
            if (!(m->vmask[i] & 2)) vy = vy + 0.5 * m->dt * ay;
        }
        ekin += 0.5 * m->mass[i] * (vx * vx + vy * vy);
        wext += phi * m->fext[2 * i] * (double)m->ux[i] + phi * m->fext[2 * i + 1] * (double)m->uy[i];
    }
    for (int s = 0; s < m->ns; ++s) {
        if (!m->sig_ok[s]) continue;
        double As = 0.0;
        for (int side = 0; side < 2; ++side) {
            int e = m->edge_elem[2 * s + side];
            if (!is_intact(m, e)) continue;
            if (m->nv == 4 && m->subcell) {
                real x[3], y[3];
                As += (double)subcell(m, e, m->edge_loc[2 * s + side], NULL, NULL, x, y, NULL, NULL);
            } else {
                As += m->area[e] / (double)m->nv;
            }
        }
        const real *sg = &m->sig[3 * s], *ep = &m->eps[3 * s];
        estr += 0.5 * As *
                ((double)sg[0] * (double)ep[0] + (double)sg[1] * (double)ep[1] + (double)sg[2] * (double)ep[2]);
    }
    real tmp[8];
    for (int e = 0; e < m->ne; ++e)
        if (m->split[e]) estr += (double)split_force(m, e, tmp);
    out[0] = ekin;
    out[1] = estr;
    out[2] = wext;
    out[3] = m->Ud;
}

/* G of one candidate of the current state (fresh edge stresses). */
int orc_candidate_G(orc_model_t *m, int e, int a, double G[3]) {
    real g[3];
    edge_stresses(m);
    int H = candidate_G(m, e, a, g);
    to_double(3, g, G);
    return H;
}

int orc_path_normal(const orc_model_t *m, int e, int a, int k, double out[3]) {
    real nx, ny, len;
    path_normal(m, e, a, k, &nx, &ny, &len);
    out[0] = (double)nx;
    out[1] = (double)ny;
    out[2] = (double)len;
    return ORC_OK;
}

void orc_split_codes(orc_model_t *m, const unsigned char *codes) { memcpy(m->split, codes, m->ne); }

/* number of OpenMP threads the oracle uses (results do not depend on it) */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }
