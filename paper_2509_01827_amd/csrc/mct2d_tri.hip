// HIP kernels (gfx950) of the CST path: ES-FEM with constant-strain
// triangles on an unstructured mesh (Sec. 2.1, Eq. CST_strain_discretization
// and Eq. CST_fint_discretization), the CST energy release rates and the
// two-path element rule (Sec. 2.2, the list after Fig. 2-2), the MCT pick
// (Sec. 3) and the central-difference update.
//
// One time step is one fused launch or two split launches (the host picks).
// Fused: k_fused, one workgroup per patch of consecutive nodes: the forces of
// the patch's elements go to LDS, each owned node sums its slots in colour
// order and is updated; u is double-buffered by step parity; with the
// global multi-tip pick every workgroup first takes the previous step's pick
// from its candidate set (the commit takes a segment's last).  Split:
//   k_force  one thread per element.  An intact element computes its own
//            strain B u and that of each intact neighbour (recomputed
//            rather than stored: the neighbour's B and nodes are cache
//            hits), smooths the strain of its three edges with
//            w_j = A_j / (A_lo + A_hi) (lower element id first), applies
//            Hooke's law, and writes its nodal forces
//            (A/3) B^T (sigma_0 + sigma_1 + sigma_2).  Free-surface edges of
//            the element are evaluated as crack-tip candidates; accepted
//            ones are appended to a list.  A split element writes the
//            forces of its two pieces (a bar and a free node).
//   k_node   one thread per node: gather of the element forces in element
//            colour order (CSR), acceleration, velocity and displacement
//            update; workgroup 0 first picks the split of the step from the
//            candidate list and applies it (it acts from the next step).
// Every value is computed in one thread in the order of the plain
// definition; results are bitwise reproducible and independent of the
// launch geometry.
#include <cmath>

#include "mct2d_device.h"
#include "mct2d_front.h"
#include "mct2d_tri.h"

namespace mct {
namespace tri {
namespace {

constexpr int kB = 256;
static_assert(kPatchMaxNodes <= kB, "a fused patch has one node per thread");

int nb_of(int64_t n) { return (int)((n + kB - 1) / kB > 0 ? (n + kB - 1) / kB : 1); }

struct Geo {
    double bx[3], by[3], A;
};

// Gradients of the linear shape functions and area of the triangle with
// corners a, b, c (in its local node order); recomputed from the node
// coordinates rather than stored.
__device__ __forceinline__ Geo make_geo(const double2 &a, const double2 &b, const double2 &c) {
    const double twoA = (b.x - a.x) * (c.y - a.y) - (c.x - a.x) * (b.y - a.y);
    const double inv = 1.0 / twoA;
    Geo r;
    r.bx[0] = (b.y - c.y) * inv;
    r.bx[1] = (c.y - a.y) * inv;
    r.bx[2] = (a.y - b.y) * inv;
    r.by[0] = (c.x - b.x) * inv;
    r.by[1] = (a.x - c.x) * inv;
    r.by[2] = (b.x - a.x) * inv;
    r.A = 0.5 * twoA;
    return r;
}

__device__ __forceinline__ int node_of(const int4 &c, int n) { return n == 0 ? c.x : (n == 1 ? c.y : c.z); }

// element n of three values by selects (no indexed private arrays)
template <typename T>
__device__ __forceinline__ T sel3(int n, const T &a, const T &b, const T &c) {
    return n == 0 ? a : (n == 1 ? b : c);
}

struct Sig {
    double s[3];
};

// B u of a triangle: terms of nodes 0, 1, 2 accumulated with fma from zero.
__device__ __forceinline__ void strain(const Geo &g, const double2 u[3], double q[3]) {
    double exx = 0.0, eyy = 0.0, gxy = 0.0;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        exx = fma(g.bx[n], u[n].x, exx);
        eyy = fma(g.by[n], u[n].y, eyy);
        gxy = fma(g.by[n], u[n].x, gxy);
        gxy = fma(g.bx[n], u[n].y, gxy);
    }
    q[0] = exx;
    q[1] = eyy;
    q[2] = gxy;
}

// plane-stress Hooke law, engineering shear strain
__device__ __forceinline__ void hooke(const Params &p, const double e[3], double s[3]) {
    s[0] = fma(p.D12, e[1], p.D11 * e[0]);
    s[1] = fma(p.D12, e[0], p.D11 * e[1]);
    s[2] = p.D33 * e[2];
}

__device__ __forceinline__ void load_u(const double2 *u, const int4 &c, double2 out[3]) {  // or coordinates
    out[0] = u[c.x];
    out[1] = u[c.y];
    out[2] = u[c.z];
}

// Split codes as a step sees them: the array, with one pending split (the
// previous step's pick, not yet visible in the array to every workgroup)
// applied on top.
struct SplitView {
    const uint8_t *split;
    int pe;         // pending element, or -1
    uint8_t pcode;  // its code
    __device__ __forceinline__ uint8_t operator()(int e) const { return e == pe ? pcode : split[e]; }
};

// Smoothed strain of local edge k of intact element e (own strain q, area
// A).  The neighbour nb across k runs the shared edge backwards: its local
// node loc is our node k+1 (xb, ub), loc+1 is our node k (xa, ua) and
// loc+2 is its third node (xo, uo); its strain is recomputed in its own
// node order.  two_out: the neighbour is intact; An: its area.
__device__ __forceinline__ void edge_strain(const Params &p, const SplitView &sv, int e, int nb, int loc,
                                            const double2 &xa,
                                            const double2 &xb, const double2 &xo, const double2 &ua,
                                            const double2 &ub, const double2 &uo, const double q[3], double A,
                                            double eps[3], bool &two_out, double &An) {
    const bool two = nb >= 0 && sv(nb) == 0;
    two_out = two;
    An = 0.0;
    if (!two) {
        eps[0] = q[0];
        eps[1] = q[1];
        eps[2] = q[2];
        return;
    }
    double2 u2[3], x2[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        u2[n] = sel3((n - loc + 3) % 3, ub, ua, uo);
        x2[n] = sel3((n - loc + 3) % 3, xb, xa, xo);
    }
    const Geo g2 = make_geo(x2[0], x2[1], x2[2]);
    double q2[3];
    strain(g2, u2, q2);
    An = g2.A;
    const bool self_lo = e < nb;
    const double Alo = self_lo ? A : g2.A, Ahi = self_lo ? g2.A : A;
    const double sum = Alo + Ahi;
    const double w0 = Alo / sum, w1 = Ahi / sum;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double lo = self_lo ? q[c] : q2[c], hi = self_lo ? q2[c] : q[c];
        eps[c] = fma(w1, hi, w0 * lo);
    }
}

// Unit normal of the crack path from the midpoint of local edge a to the
// midpoint of local edge k, oriented toward node n_{a+1}, and its length.
__device__ __forceinline__ void path_geom(const Params &p, const int4 &c, int a, int k, double &nx, double &ny,
                                          double &len) {
    const double2 P0 = p.xy[node_of(c, a)], P1 = p.xy[node_of(c, (a + 1) % 3)];
    const double2 Q0 = p.xy[node_of(c, k)], Q1 = p.xy[node_of(c, (k + 1) % 3)];
    const double g0x = 0.5 * (P0.x + P1.x), g0y = 0.5 * (P0.y + P1.y);
    const double gkx = 0.5 * (Q0.x + Q1.x), gky = 0.5 * (Q0.y + Q1.y);
    const double dx = gkx - g0x, dy = gky - g0y;
    const double L = sqrt(dx * dx + dy * dy);
    double cx = dy / L, cy = -dx / L;
    if (cx * (P1.x - g0x) + cy * (P1.y - g0y) < 0.0) {
        cx = -cx;
        cy = -cy;
    }
    nx = cx;
    ny = cy;
    len = L;
}

// Crack-tip candidate (intact element e, free-surface local edge a): G of
// the two paths k = a+1, a+2 with the Heaviside edge-stretch gate, then the
// two-path element rule.  Returns the accepted path index j or -1.
__device__ __forceinline__ int candidate(const Params &p, int e, const int4 &c, const double2 &ua, const double2 &ub,
                                         const Sig &s0, const Sig &s1, const Sig &s2, int a, double &Gsel) {
    const int i1 = a, i2 = (a + 1) % 3;
    const double2 X1 = p.xy[node_of(c, i1)], X2 = p.xy[node_of(c, i2)];
    const double dux = ub.x - ua.x, duy = ub.y - ua.y;
    const double x1 = X1.x + ua.x, y1 = X1.y + ua.y;
    const double x2 = X2.x + ub.x, y2 = X2.y + ub.y;
    const double lx = x2 - x1, ly = y2 - y1;
    const double Lx = X2.x - X1.x, Ly = X2.y - X1.y;
    if (!((lx * lx + ly * ly) > (Lx * Lx + Ly * Ly))) return -1;  // H = 0: every G is 0
    double G[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = (a + 1 + j) % 3;
        double nx, ny, len;
        path_geom(p, c, a, k, nx, ny, len);
        const Sig sg = sel3(k, s0, s1, s2);
        const double spx = fma(sg.s[2], ny, sg.s[0] * nx);
        const double spy = fma(sg.s[1], ny, sg.s[2] * nx);
        G[j] = 0.5 * fma(duy, spy, dux * spx);
    }
    const double Gc = p.gc[e];
    int best = -1;
#pragma unroll
    for (int j = 0; j < 2; ++j)
        if (G[j] > Gc && (best < 0 || G[j] > G[best])) best = j;
    if (best < 0) return -1;
    const int other = 1 - best;
    if (G[other] > Gc && !(G[best] > p.gamma * (G[best] - G[other]))) return -1;
    Gsel = G[best];
    return best;
}

// One piece of a split triangle: the local nodes after the entry edge up to
// the exit edge, closed by the two crack midpoints.  Two nodes (l0, l1): a
// bar along them with cross-section A_piece / L, force F on l1 and -F on
// l0; one node: nothing.
struct Piece {
    int l0, l1;  // l1 < 0: one-node piece
    double2 F;
    double w;    // strain energy
};

__device__ __forceinline__ Piece piece(const Params &p, const double2 *u, const int4 &c, int entry, int exit) {
    Piece r;
    r.l0 = (entry + 1) % 3;
    r.l1 = -1;
    r.F = make_double2(0.0, 0.0);
    r.w = 0.0;
    if (r.l0 == exit) return r;
    r.l1 = exit;
    const double2 A0 = p.xy[node_of(c, entry)], A1 = p.xy[node_of(c, (entry + 1) % 3)];
    const double2 B0 = p.xy[node_of(c, exit)], B1 = p.xy[node_of(c, (exit + 1) % 3)];
    const double2 P = p.xy[node_of(c, r.l0)], Q = p.xy[node_of(c, r.l1)];
    // polygon M_entry, P, Q, M_exit; area by a fan from its first vertex
    const double px0 = 0.5 * (A0.x + A1.x), py0 = 0.5 * (A0.y + A1.y);
    const double px3 = 0.5 * (B0.x + B1.x), py3 = 0.5 * (B0.y + B1.y);
    double s = 0.0;
    s += (P.x - px0) * (Q.y - py0) - (Q.x - px0) * (P.y - py0);
    s += (Q.x - px0) * (py3 - py0) - (px3 - px0) * (Q.y - py0);
    const double Ap = 0.5 * s;
    const double dx = Q.x - P.x, dy = Q.y - P.y;
    const double L2 = dx * dx + dy * dy;
    const double2 up = u[node_of(c, r.l0)], uq = u[node_of(c, r.l1)];
    const double dux = uq.x - up.x, duy = uq.y - up.y;
    const double str = (dx * dux + dy * duy) / L2;
    const double stress = p.E * str;
    const double coef = Ap * stress / L2;
    r.F = make_double2(coef * dx, coef * dy);
    r.w = 0.5 * Ap * stress * str;
    return r;
}

__device__ __forceinline__ double2 piece_force_at(const Piece &a, const Piece &b, int n) {
    if (a.l1 >= 0 && n == a.l1) return a.F;
    if (a.l1 >= 0 && n == a.l0) return make_double2(-a.F.x, -a.F.y);
    if (b.l1 >= 0 && n == b.l1) return b.F;
    if (b.l1 >= 0 && n == b.l0) return make_double2(-b.F.x, -b.F.y);
    return make_double2(0.0, 0.0);
}

// ---- bilinear quadrilaterals (nv = 4) -----------------------------------
// The Q4 form of the step on an unstructured mesh (Sec. 2.1,
// Eq. QUAD_strain_discretization, edge quadrature at the midpoints of the
// element's own local edges; the four-edge rule after Fig. 2-3): the same
// arithmetic as the structured grid's step, with the neighbours found
// through tables instead of grid indices.

template <typename T>
__device__ __forceinline__ T sel4(int n, const T &a, const T &b, const T &c, const T &d) {
    return n == 0 ? a : (n == 1 ? b : (n == 2 ? c : d));
}

// Area of a quadrilateral: half the cross product of its diagonals.
__device__ __forceinline__ double quad_area(const double x[4], const double y[4]) {
    return 0.5 * ((x[2] - x[0]) * (y[3] - y[1]) - (x[3] - x[1]) * (y[2] - y[0]));
}

// One piece of a split quadrilateral: the np = 1..3 local nodes after the
// entry edge EN up to the exit edge EX, closed by the two crack midpoints
// (area by a fan from the entry midpoint).  Three nodes: a constant-strain
// triangle over them whose forces are scaled by the piece's area; two: a
// bar along them with cross-section A_piece / L; one: nothing.  Adds the
// forces of its nodes to f (each node lies in one piece) and returns the
// strain energy.  The edges are template arguments, so every node value is
// addressed statically.
template <int EN, int EX>
__device__ __forceinline__ double quad_piece(const Params &p, const double2 ue[4], const double x[4],
                                             const double y[4], double2 f[4]) {
    constexpr int np = (EX - EN) & 3;
    constexpr int l0 = (EN + 1) & 3, l1 = (EN + 2) & 3, l2 = (EN + 3) & 3;
    if constexpr (np == 1) {
        f[l0] = make_double2(0.0, 0.0);
        return 0.0;
    } else {
        const double px0 = 0.5 * (x[EN] + x[(EN + 1) & 3]), py0 = 0.5 * (y[EN] + y[(EN + 1) & 3]);
        const double pxm = 0.5 * (x[EX] + x[(EX + 1) & 3]), pym = 0.5 * (y[EX] + y[(EX + 1) & 3]);
        const double2 P0 = make_double2(x[l0], y[l0]), P1 = make_double2(x[l1], y[l1]);
        // fan terms over the polygon M_entry, P0, .., M_exit
        double s = 0.0;
        s += (P0.x - px0) * (P1.y - py0) - (P1.x - px0) * (P0.y - py0);
        if constexpr (np == 3) {
            const double2 P2 = make_double2(x[l2], y[l2]);
            s += (P1.x - px0) * (P2.y - py0) - (P2.x - px0) * (P1.y - py0);
            s += (P2.x - px0) * (pym - py0) - (pxm - px0) * (P2.y - py0);
            const double Ap = 0.5 * s;
            const double2 u3[3] = {ue[l0], ue[l1], ue[l2]};
            const Geo g = make_geo(P0, P1, P2);
            double q[3], sg[3];
            strain(g, u3, q);
            hooke(p, q, sg);
            f[l0] = make_double2(Ap * fma(g.by[0], sg[2], g.bx[0] * sg[0]), Ap * fma(g.bx[0], sg[2], g.by[0] * sg[1]));
            f[l1] = make_double2(Ap * fma(g.by[1], sg[2], g.bx[1] * sg[0]), Ap * fma(g.bx[1], sg[2], g.by[1] * sg[1]));
            f[l2] = make_double2(Ap * fma(g.by[2], sg[2], g.bx[2] * sg[0]), Ap * fma(g.bx[2], sg[2], g.by[2] * sg[1]));
            return 0.5 * Ap * ((sg[0] * q[0] + sg[1] * q[1]) + sg[2] * q[2]);
        } else {
            s += (P1.x - px0) * (pym - py0) - (pxm - px0) * (P1.y - py0);
            const double Ap = 0.5 * s;
            const double dx = P1.x - P0.x, dy = P1.y - P0.y;
            const double L2 = dx * dx + dy * dy;
            const double dux = ue[l1].x - ue[l0].x, duy = ue[l1].y - ue[l0].y;
            const double str = (dx * dux + dy * duy) / L2;
            const double stress = p.E * str;
            const double coef = Ap * stress / L2;
            f[l1] = make_double2(coef * dx, coef * dy);
            f[l0] = make_double2(-(coef * dx), -(coef * dy));
            return 0.5 * Ap * stress * str;
        }
    }
}

// Forces (into f) and strain energy (returned) of a quadrilateral split
// along the path from local edge EN to local edge EX: the piece after the
// entry edge, then the piece after the exit edge.
template <int EN, int EX>
__device__ __forceinline__ double quad_split(const Params &p, const double2 ue[4], const double x[4],
                                             const double y[4], double2 f[4]) {
    double w = quad_piece<EN, EX>(p, ue, x, y, f);
    w += quad_piece<EX, EN>(p, ue, x, y, f);
    return w;
}

// Crack-tip candidates of an intact quadrilateral with free-surface edges
// (two[a] false): for each such edge a (single-tip tracking: the tip edge
// only) with the stretch gate open, G of the three paths k = a+1, a+2, a+3
// from the smoothed edge stresses (sig(k, s) gives edge k's), then the
// four-edge element rule (Sec. 2.2); an accepted candidate is appended to
// clist.
template <class SigFn>
__device__ __forceinline__ void quad_candidates(const Params &p, int e, const double x[4], const double y[4],
                                                const double ux[4], const double uy[4], SigFn &&sig,
                                                const bool two[4], Cand *clist, int32_t *ccount) {
    const int tip = p.sct ? p.ctl->tip : -1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (two[a]) continue;
        if (p.sct && tip != 4 * e + a) continue;
        const int a1 = (a + 1) & 3;
        const double dux = ux[a1] - ux[a], duy = uy[a1] - uy[a];
        const double x1 = x[a] + ux[a], y1 = y[a] + uy[a];
        const double x2 = x[a1] + ux[a1], y2 = y[a1] + uy[a1];
        const double lx = x2 - x1, ly = y2 - y1;
        const double Lx = x[a1] - x[a], Ly = y[a1] - y[a];
        if (!((lx * lx + ly * ly) > (Lx * Lx + Ly * Ly))) continue;  // H = 0: every G is 0
        double G[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int k = (a + 1 + j) & 3;
            double nx, ny, len, sg[3];
            dev::path_geom(x, y, a, k, nx, ny, len);
            sig(k, sg);
            const double spx = fma(sg[2], ny, sg[0] * nx);
            const double spy = fma(sg[1], ny, sg[2] * nx);
            G[j] = 0.5 * fma(duy, spy, dux * spx);
        }
        const double Gc = p.gc[e];
        int best = -1;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (G[j] > Gc && (best < 0 || G[j] > sel3(best, G[0], G[1], G[2]))) best = j;
        if (best < 0) continue;
        const double Gb = sel3(best, G[0], G[1], G[2]);
        bool ok = true;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (j != best && G[j] > Gc && !(Gb > p.gamma * (Gb - G[j]))) ok = false;
        if (!ok) continue;
        const int slot = atomicAdd(ccount, 1);
        Cand cd;
        cd.G = Gb;
        cd.elem = e;
        cd.ak = (a << 2) | ((a + 1 + best) & 3);
        clist[slot] = cd;
    }
}

// Everything a quadrilateral element contributes to one pass: its four
// nodal forces (force of local node n at fe[n fs]), with `cands` its crack-tip
// candidates, with EVAL the query outputs.  An intact element computes the
// strain of each local edge k at the edge's midpoint from its own nodes and,
// if the neighbour across k is intact, that of the neighbour at the same
// edge (recomputed in the neighbour's own node order: its local nodes loc,
// loc+1 are our k+1, k and loc+2, loc+3 come from the tables), smooths them
// with w = A_lo / (A_lo + A_hi), applies Hooke's law and adds
// B_k^T sigma_k over k = 0..3, scaled by A/4 (Sec. 2.1, the c_{e,k} = A/4
// reading).  A free-surface edge a (no intact neighbour) is a candidate: G
// of the three paths k = a+1, a+2, a+3 with the stretch gate, then the
// four-edge element rule (Sec. 2.2).
template <bool EVAL>
__device__ __forceinline__ void quad_element(const Params &p, const SplitView &sv, const double2 *u, int e,
                                             bool cands, Cand *clist, int32_t *ccount, const Eval &ev,
                                             double2 *fe, int64_t fs) {
    const int4 c = p.conn[e];
    const uint8_t code = sv(e);
    double2 ue[4], xe[4];
    ue[0] = u[c.x];
    ue[1] = u[c.y];
    ue[2] = u[c.z];
    ue[3] = u[c.w];
    xe[0] = p.xy[c.x];
    xe[1] = p.xy[c.y];
    xe[2] = p.xy[c.z];
    xe[3] = p.xy[c.w];
    double x[4], y[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        x[n] = xe[n].x;
        y[n] = xe[n].y;
    }
    if (code) {
        double2 f[4];
        double w = 0.0;
        switch (code & 15) {
#define QSPLIT(EN, EX) \
    case (EN << 2) | EX: w = quad_split<EN, EX>(p, ue, x, y, f); break;
            QSPLIT(0, 1) QSPLIT(0, 2) QSPLIT(0, 3) QSPLIT(1, 0) QSPLIT(1, 2) QSPLIT(1, 3)
            QSPLIT(2, 0) QSPLIT(2, 1) QSPLIT(2, 3) QSPLIT(3, 0) QSPLIT(3, 1) QSPLIT(3, 2)
#undef QSPLIT
            default:  // entry = exit: rejected at set-up and never picked
#pragma unroll
                for (int n = 0; n < 4; ++n) f[n] = make_double2(0.0, 0.0);
                break;
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) fe[n * fs] = f[n];
        if constexpr (EVAL) {
            if (ev.pe) ev.pe[e] = w;
            if (ev.es_ek)
                for (int k = 0; k < 4; ++k) ev.es_ek[4 * (int64_t)e + k] = 0.0;
            if (ev.principal) ev.principal[e] = NAN;
            if (ev.sig_ek)
                for (int k = 0; k < 12; ++k) ev.sig_ek[12 * (int64_t)e + k] = NAN;
        }
        return;
    }
    const double A = quad_area(x, y);
    const int4 nb = p.q_nbr[e];
    const uint32_t lc = p.q_loc[e];
    const int4 oa = p.q_oa[e], ob = p.q_ob[e];
    double ux[4], uy[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        ux[n] = ue[n].x;
        uy[n] = ue[n].y;
    }
    double sig[4][3], eps[4][3], An[4], sx[4], sy[4];
    bool two[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double gx[4], gy[4], q[3];
        dev::q4_grad(x, y, k, gx, gy);
        dev::strain<4>(gx, gy, ux, uy, q);
        const int n = sel4(k, nb.x, nb.y, nb.z, nb.w);
        two[k] = n >= 0 && sv(n) == 0;
        An[k] = 0.0;
        if (!two[k]) {
            eps[k][0] = q[0];
            eps[k][1] = q[1];
            eps[k][2] = q[2];
        } else {
            const int loc = (lc >> (2 * k)) & 3;
            const int ia = sel4(k, oa.x, oa.y, oa.z, oa.w), ib = sel4(k, ob.x, ob.y, ob.z, ob.w);
            const double2 XA = p.xy[ia], XB = p.xy[ib], UA = u[ia], UB = u[ib];
            const int k1 = (k + 1) & 3;
            double x2[4], y2[4], u2x[4], u2y[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int t = (m - loc) & 3;
                x2[m] = sel4(t, x[k1], x[k], XA.x, XB.x);
                y2[m] = sel4(t, y[k1], y[k], XA.y, XB.y);
                u2x[m] = sel4(t, ux[k1], ux[k], UA.x, UB.x);
                u2y[m] = sel4(t, uy[k1], uy[k], UA.y, UB.y);
            }
            const double A2 = quad_area(x2, y2);
            double hx[4], hy[4], q2[3];
            dev::q4_grad_rt(x2, y2, loc, hx, hy);
            dev::strain<4>(hx, hy, u2x, u2y, q2);
            An[k] = A2;
            const bool self_lo = e < n;
            const double Alo = self_lo ? A : A2, Ahi = self_lo ? A2 : A;
            const double sum = Alo + Ahi;
            const double w0 = Alo / sum, w1 = Ahi / sum;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const double lo = self_lo ? q[cc] : q2[cc], hi = self_lo ? q2[cc] : q[cc];
                eps[k][cc] = fma(w1, hi, w0 * lo);
            }
        }
        hooke(p, eps[k], sig[k]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double tx = fma(gy[m], sig[k][2], gx[m] * sig[k][0]);
            const double ty = fma(gx[m], sig[k][2], gy[m] * sig[k][1]);
            sx[m] = k == 0 ? tx : sx[m] + tx;
            sy[m] = k == 0 ? ty : sy[m] + ty;
        }
    }
    const double cA = 0.25 * A;
#pragma unroll
    for (int m = 0; m < 4; ++m) fe[m * fs] = make_double2(cA * sx[m], cA * sy[m]);
    if constexpr (EVAL) {
        if (ev.pe) ev.pe[e] = 0.0;
        if (ev.sig_ek)
            for (int k = 0; k < 4; ++k)
                for (int cc = 0; cc < 3; ++cc) ev.sig_ek[12 * (int64_t)e + 3 * k + cc] = sig[k][cc];
        if (ev.es_ek) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int n = sel4(k, nb.x, nb.y, nb.z, nb.w);
                double term = 0.0;
                if (!two[k] || e < n) {
                    // smoothing domain: a quarter of each intact neighbour,
                    // lower element id first
                    double As = 0.0;
                    As += A / 4.0;
                    if (two[k]) As += An[k] / 4.0;
                    term = 0.5 * As * (sig[k][0] * eps[k][0] + sig[k][1] * eps[k][1] + sig[k][2] * eps[k][2]);
                }
                ev.es_ek[4 * (int64_t)e + k] = term;
            }
        }
        if (ev.principal) {
            double m[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) m[cc] = (((sig[0][cc] + sig[1][cc]) + sig[2][cc]) + sig[3][cc]) / 4.0;
            const double cc = 0.5 * (m[0] + m[1]), hd = 0.5 * (m[0] - m[1]);
            ev.principal[e] = cc + sqrt(hd * hd + m[2] * m[2]);
        }
        return;
    }
    if (!cands || (two[0] && two[1] && two[2] && two[3])) return;
    quad_candidates(
        p, e, x, y, ux, uy,
        [&](int k, double sg[3]) {
            sg[0] = sig[k][0];
            sg[1] = sig[k][1];
            sg[2] = sig[k][2];
        },
        two, clist, ccount);
}

// Forces of element e on its three local nodes from displacement u (the
// step's element pass).  An intact element computes its own strain and that
// of each intact neighbour (recomputed from u and the coordinates; the
// neighbour's third node comes from the opposite-node table), smooths the
// strain of its three edges with w = A_lo / (A_lo + A_hi) (lower element id
// first), applies Hooke's law and returns (A/3) B^T (sigma_0 + sigma_1 +
// sigma_2); with `cands` its free-surface edges are evaluated as crack-tip
// candidates and accepted ones appended to the list.  A split element
// returns the forces of its two pieces.  Candidates go to clist, counted
// by *ccount.
__device__ __forceinline__ void element_force(const Params &p, const SplitView &sv, const double2 *u, int e,
                                              bool cands, Cand *clist, int32_t *ccount, double2 f[3]) {
    const int4 c = p.conn[e];
    const uint8_t code = sv(e);
    if (code) {
        const Piece pa = piece(p, u, c, (code >> 2) & 3, code & 3);
        const Piece pb = piece(p, u, c, code & 3, (code >> 2) & 3);
        f[0] = piece_force_at(pa, pb, 0);
        f[1] = piece_force_at(pa, pb, 1);
        f[2] = piece_force_at(pa, pb, 2);
        return;
    }
    const int4 nb = p.nbr[e];
    const int2 op = p.opp[e];  // the far nodes of edges 1, 2 (that of edge 0 is c.w)
    double2 ue[3], uo[3], xe[3], xo[3];
    load_u(u, c, ue);
    load_u(p.xy, c, xe);
    const double2 z2 = make_double2(0.0, 0.0);
    uo[0] = c.w >= 0 ? u[c.w] : z2;
    uo[1] = op.x >= 0 ? u[op.x] : z2;
    uo[2] = op.y >= 0 ? u[op.y] : z2;
    xo[0] = c.w >= 0 ? p.xy[c.w] : z2;
    xo[1] = op.x >= 0 ? p.xy[op.x] : z2;
    xo[2] = op.y >= 0 ? p.xy[op.y] : z2;
    const Geo g = make_geo(xe[0], xe[1], xe[2]);
    double q[3];
    strain(g, ue, q);
    double sig[3][3];
    bool two[3];
    double eps[3][3], An[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        edge_strain(p, sv, e, k == 0 ? nb.x : (k == 1 ? nb.y : nb.z), (nb.w >> (2 * k)) & 3, xe[k], xe[(k + 1) % 3],
                    xo[k], ue[k], ue[(k + 1) % 3], uo[k], q, g.A, eps[k], two[k], An[k]);
        hooke(p, eps[k], sig[k]);
    }
    double S[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) S[cc] = (sig[0][cc] + sig[1][cc]) + sig[2][cc];
    const double coef = g.A / 3.0;
#pragma unroll
    for (int n = 0; n < 3; ++n)
        f[n] = make_double2(coef * fma(g.by[n], S[2], g.bx[n] * S[0]), coef * fma(g.bx[n], S[2], g.by[n] * S[1]));
    if (!cands || (two[0] && two[1] && two[2])) return;
    const int tip = p.sct ? p.ctl->tip : -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (two[a]) continue;
        if (p.sct && tip != 4 * e + a) continue;
        double G;
        const Sig s0 = {{sig[0][0], sig[0][1], sig[0][2]}}, s1 = {{sig[1][0], sig[1][1], sig[1][2]}},
                  s2 = {{sig[2][0], sig[2][1], sig[2][2]}};
        const int j = candidate(p, e, c, sel3(a, ue[0], ue[1], ue[2]), sel3((a + 1) % 3, ue[0], ue[1], ue[2]), s0,
                                s1, s2, a, G);
        if (j < 0) continue;
        const int k = (a + 1 + j) % 3;
        const int slot = atomicAdd(ccount, 1);
        Cand cd;
        cd.G = G;
        cd.elem = e;
        cd.ak = (a << 2) | k;
        clist[slot] = cd;
    }
}

// element_force of an intact triangle whose neighbours' strains and areas
// sit in LDS (s_q[c][slot], s_A[slot]; area 0: a split or absent element),
// slots and lower-id flags in nbs (the fused step's patch tables).  The
// element's own geometry g, strain q and values ue come from the caller;
// its node record is read only for candidates.
// Arithmetic as edge_strain's: a neighbour's strain there is recomputed in
// the neighbour's own node order, so it equals the one the neighbour
// computed for itself, which is what the LDS holds.
__device__ __forceinline__ void element_force_shared(const Params &p, int e, const double2 ue[3],
                                                     const Geo &g, const double q[3], uint2 nbs,
                                                     const double (*s_q)[2 * kB], const double *s_A, bool cands,
                                                     Cand *clist, int32_t *ccount, double2 f[3]) {
    double sig[3][3];
    bool two[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint32_t sl = (nbs.x >> (10 * k)) & kNoSlot;
        const double A2 = sl != kNoSlot ? s_A[sl] : 0.0;
        two[k] = A2 != 0.0;
        double eps[3];
        if (!two[k]) {
            eps[0] = q[0];
            eps[1] = q[1];
            eps[2] = q[2];
        } else {
            const double q2[3] = {s_q[0][sl], s_q[1][sl], s_q[2][sl]};
            const bool self_lo = ((nbs.y >> (10 + k)) & 1u) != 0;
            const double Alo = self_lo ? g.A : A2, Ahi = self_lo ? A2 : g.A;
            const double sum = Alo + Ahi;
            const double w0 = Alo / sum, w1 = Ahi / sum;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const double lo = self_lo ? q[cc] : q2[cc], hi = self_lo ? q2[cc] : q[cc];
                eps[cc] = fma(w1, hi, w0 * lo);
            }
        }
        hooke(p, eps, sig[k]);
    }
    double S[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) S[cc] = (sig[0][cc] + sig[1][cc]) + sig[2][cc];
    const double coef = g.A / 3.0;
#pragma unroll
    for (int n = 0; n < 3; ++n)
        f[n] = make_double2(coef * fma(g.by[n], S[2], g.bx[n] * S[0]), coef * fma(g.bx[n], S[2], g.by[n] * S[1]));
    if (!cands || (two[0] && two[1] && two[2])) return;
    const int4 c = p.conn[e];  // a free-surface element: its nodes, for the path geometry
    const int tip = p.sct ? p.ctl->tip : -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (two[a]) continue;
        if (p.sct && tip != 4 * e + a) continue;
        double G;
        const Sig s0 = {{sig[0][0], sig[0][1], sig[0][2]}}, s1 = {{sig[1][0], sig[1][1], sig[1][2]}},
                  s2 = {{sig[2][0], sig[2][1], sig[2][2]}};
        const int j = candidate(p, e, c, sel3(a, ue[0], ue[1], ue[2]), sel3((a + 1) % 3, ue[0], ue[1], ue[2]), s0,
                                s1, s2, a, G);
        if (j < 0) continue;
        const int k = (a + 1 + j) % 3;
        const int slot = atomicAdd(ccount, 1);
        Cand cd;
        cd.G = G;
        cd.elem = e;
        cd.ak = (a << 2) | k;
        clist[slot] = cd;
    }
}

// Element pass.  eval: query mode (u given, outputs in ev, no candidates).
template <bool EVAL>
__global__ __launch_bounds__(kB) void k_force(Params p, const double2 *u, Eval ev, int j) {
    const int e = dev::xcd_tile(blockIdx.x, gridDim.x) * kB + threadIdx.x;
    if (e >= p.ne) return;
    if constexpr (!EVAL) {
        if (((p.ctl->base + j) & 1) != 0) u = p.u1;  // u^k
        double2 f[3];
        element_force(p, SplitView{p.split, -1, 0}, u, e, true, p.cand, &p.ctl->nacc, f);
        p.fe[e] = f[0];
        p.fe[p.ne + e] = f[1];
        p.fe[2 * (int64_t)p.ne + e] = f[2];
        return;
    }
    const int4 c = p.conn[e];
    const uint8_t code = p.split[e];
    // slot-major element forces: node slot n of element e at fe[n ne + e]
    double2 *fe = p.fe + e;
    const int64_t fs = p.ne;
    if (code) {
        const Piece pa = piece(p, u, c, (code >> 2) & 3, code & 3);
        const Piece pb = piece(p, u, c, code & 3, (code >> 2) & 3);
        double w = pa.w;
        w += pb.w;
        fe[0] = piece_force_at(pa, pb, 0);
        fe[fs] = piece_force_at(pa, pb, 1);
        fe[2 * fs] = piece_force_at(pa, pb, 2);
        if constexpr (EVAL) {
            if (ev.pe) ev.pe[e] = w;
            if (ev.es_ek)
                for (int k = 0; k < 3; ++k) ev.es_ek[3 * (int64_t)e + k] = 0.0;
            if (ev.principal) ev.principal[e] = NAN;
            // stresses of the edges seen from a split element: the intact
            // neighbour (if any) writes them; mark this side absent
            if (ev.sig_ek)
                for (int k = 0; k < 9; ++k) ev.sig_ek[9 * (int64_t)e + k] = NAN;
        }
        return;
    }
    const int4 nb = p.nbr[e];
    const int2 op = p.opp[e];  // the far nodes of edges 1, 2 (that of edge 0 is c.w)
    double2 ue[3], uo[3], xe[3], xo[3];
    load_u(u, c, ue);
    load_u(p.xy, c, xe);
    const double2 z2 = make_double2(0.0, 0.0);
    uo[0] = c.w >= 0 ? u[c.w] : z2;
    uo[1] = op.x >= 0 ? u[op.x] : z2;
    uo[2] = op.y >= 0 ? u[op.y] : z2;
    xo[0] = c.w >= 0 ? p.xy[c.w] : z2;
    xo[1] = op.x >= 0 ? p.xy[op.x] : z2;
    xo[2] = op.y >= 0 ? p.xy[op.y] : z2;
    const Geo g = make_geo(xe[0], xe[1], xe[2]);
    double q[3];
    strain(g, ue, q);
    double sig[3][3];
    bool two[3];
    double eps[3][3], An[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        edge_strain(p, SplitView{p.split, -1, 0}, e, k == 0 ? nb.x : (k == 1 ? nb.y : nb.z), (nb.w >> (2 * k)) & 3, xe[k], xe[(k + 1) % 3],
                    xo[k], ue[k], ue[(k + 1) % 3], uo[k], q, g.A, eps[k], two[k], An[k]);
        hooke(p, eps[k], sig[k]);
    }
    double S[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) S[cc] = (sig[0][cc] + sig[1][cc]) + sig[2][cc];
    const double coef = g.A / 3.0;
#pragma unroll
    for (int n = 0; n < 3; ++n)
        fe[n * fs] = make_double2(coef * fma(g.by[n], S[2], g.bx[n] * S[0]), coef * fma(g.bx[n], S[2], g.by[n] * S[1]));
    if constexpr (EVAL) {
        if (ev.pe) ev.pe[e] = 0.0;
        if (ev.sig_ek)
            for (int k = 0; k < 3; ++k)
                for (int cc = 0; cc < 3; ++cc) ev.sig_ek[9 * (int64_t)e + 3 * k + cc] = sig[k][cc];
        if (ev.es_ek) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int n = k == 0 ? nb.x : (k == 1 ? nb.y : nb.z);
                double term = 0.0;
                if (!two[k] || e < n) {
                    // smoothing domain: one third of each intact neighbour,
                    // lower element id first
                    double As = 0.0;
                    if (two[k]) {
                        As += g.A / 3.0;
                        As += An[k] / 3.0;
                    } else {
                        As += g.A / 3.0;
                    }
                    term = 0.5 * As * (sig[k][0] * eps[k][0] + sig[k][1] * eps[k][1] + sig[k][2] * eps[k][2]);
                }
                ev.es_ek[3 * (int64_t)e + k] = term;
            }
        }
        if (ev.principal) {
            const double m0 = S[0] / 3.0, m1 = S[1] / 3.0, m2 = S[2] / 3.0;
            const double cc = 0.5 * (m0 + m1);
            const double hd = 0.5 * (m0 - m1);
            ev.principal[e] = cc + sqrt(hd * hd + m2 * m2);
        }
        return;
    }
}

// Element pass of a quadrilateral mesh (as k_force).
template <bool EVAL>
__global__ __launch_bounds__(kB) void k_qforce(Params p, const double2 *u, Eval ev, int j) {
    const int e = dev::xcd_tile(blockIdx.x, gridDim.x) * kB + threadIdx.x;
    if (e >= p.ne) return;
    if constexpr (!EVAL) {
        if (((p.ctl->base + j) & 1) != 0) u = p.u1;  // u^k
    }
    // slot-major element forces: node slot n of element e at fe[n ne + e]
    quad_element<EVAL>(p, SplitView{p.split, -1, 0}, u, e, !EVAL, p.cand, &p.ctl->nacc, ev, p.fe + e, p.ne);
}

__device__ __forceinline__ double load_factor(const Params &p, double t) {
    if (p.ncurve == 0) return 1.0;
    if (t <= p.curve_t[0]) return p.curve_phi[0];
    const int n = p.ncurve;
    if (t >= p.curve_t[n - 1]) return p.curve_phi[n - 1];
    // largest i with curve_t[i] <= t
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (p.curve_t[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    const int i = lo;
    const double slope = (p.curve_phi[i + 1] - p.curve_phi[i]) / (p.curve_t[i + 1] - p.curve_t[i]);
    return p.curve_phi[i] + (t - p.curve_t[i]) * slope;
}

// better(a, b): larger G, ties to the lower element id, then the lower tip edge
__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
    if (a.G != b.G) return a.G > b.G;
    if (a.elem != b.elem) return a.elem < b.elem;
    return (a.ak >> 2) < (b.ak >> 2);
}

// Best of n accepted candidates (largest G, then lower element, then lower
// tip edge) and the smallest G, by the whole workgroup; valid in thread 0.
// n is uniform over the workgroup.  Each thread scans its share of the
// list, each wave holding an entry reduces by shuffles (the order is total,
// so the result does not depend on the grouping), and thread 0 merges the
// waves' results.
__device__ __forceinline__ void best_of(const Cand *list, int n, Cand &best_out, double &gmin_out) {
    __shared__ Cand s_best[kB / 64];
    __shared__ double s_min[kB / 64];
    Cand best;
    best.G = -1.0;
    best.elem = 0x7fffffff;
    best.ak = 0;
    double gmin = INFINITY;
    for (int t = threadIdx.x; t < n; t += kB) {
        const Cand cd = list[t];
        if (better(cd, best)) best = cd;
        gmin = fmin(gmin, cd.G);
    }
    if (__ballot(best.G >= 0.0) != 0ull) {  // uniform over the wave
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            Cand o;
            o.G = __shfl_xor(best.G, off, 64);
            o.elem = __shfl_xor(best.elem, off, 64);
            o.ak = __shfl_xor(best.ak, off, 64);
            const double gm = __shfl_xor(gmin, off, 64);
            if (better(o, best)) best = o;
            gmin = fmin(gmin, gm);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_best[wave] = best;
        s_min[wave] = gmin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kB / 64; ++w) {
            if (better(s_best[w], best)) best = s_best[w];
            gmin = fmin(gmin, s_min[w]);
        }
    }
    best_out = best;
    gmin_out = gmin;
}

// Record the split of step k picked from candidate b: its code, the log,
// U_d (Gc * crack-path length) and, in single-tip tracking, the next tip.
// One thread.
__device__ void apply_pick(const Params &p, const Cand &b, int64_t k) {
    Ctl *ctl = p.ctl;
    const int e = b.elem, a = b.ak >> 2, kx = b.ak & 3;
    p.split[e] = (uint8_t)(kSplitFlag | b.ak);
    const int64_t ns = ctl->nsplit;
    if (ns < p.log_cap) {
        LogRec r;
        r.step = (int32_t)k;
        r.elem = e;
        r.entry = (uint8_t)a;
        r.exit = (uint8_t)kx;
        r.pad0 = r.pad1 = 0;
        r.pad2 = 0;
        r.G = b.G;
        p.log[ns] = r;
    } else {
        ctl->overflow = 1;
    }
    ctl->nsplit = ns + 1;
    const int4 c = p.conn[e];
    double nx, ny, len;
    if (p.nv == 4) {
        const double2 P0 = p.xy[sel4(a, c.x, c.y, c.z, c.w)], P1 = p.xy[sel4((a + 1) & 3, c.x, c.y, c.z, c.w)];
        const double2 Q0 = p.xy[sel4(kx, c.x, c.y, c.z, c.w)], Q1 = p.xy[sel4((kx + 1) & 3, c.x, c.y, c.z, c.w)];
        dev::path_geom_pts(P0.x, P0.y, P1.x, P1.y, Q0.x, Q0.y, Q1.x, Q1.y, nx, ny, len);
    } else {
        path_geom(p, c, a, kx, nx, ny, len);
    }
    ctl->Ud = ctl->Ud + p.gc[e] * len;
    if (p.sct) {
        int m, loc;
        if (p.nv == 4) {
            const int4 nb = p.q_nbr[e];
            m = sel4(kx, nb.x, nb.y, nb.z, nb.w);
            loc = (p.q_loc[e] >> (2 * kx)) & 3;
        } else {
            const int4 nb = p.nbr[e];
            m = kx == 0 ? nb.x : (kx == 1 ? nb.y : nb.z);
            loc = (nb.w >> (2 * kx)) & 3;
        }
        ctl->tip = (m < 0 || p.split[m] != 0) ? -1 : 4 * m + loc;
    }
}

// The global pick of step k over the accepted candidates list[0..*count):
// the best one splits if it passes the split-ratio test against every
// other (the smallest G is the hardest one to pass); *count is reset.
__device__ void pick_from(const Params &p, const Cand *list, int32_t *count, int64_t k) {
    const int n = *count;
    if (n == 0) return;  // uniform over the workgroup
    Cand b;
    double Gmin;
    best_of(list, n, b, Gmin);
    if (threadIdx.x == 0) {
        *count = 0;
        if (b.G > p.gamma * (b.G - Gmin)) apply_pick(p, b, k);
    }
}

__device__ __forceinline__ void pick(const Params &p, int64_t k) { pick_from(p, p.cand, &p.ctl->nacc, k); }

__device__ __forceinline__ double prescribed(const Params &p, double v0, double t) {
    if (p.t_ramp > 0.0 && t < p.t_ramp) return v0 * (t / p.t_ramp);
    return v0;
}

// Sum of the element forces on node i in colour order.  W > 0: padded
// slot-major lists of width W (all loads issued before the adds); W = 0:
// the CSR lists.
template <int W>
__device__ __forceinline__ double2 gather(const Params &p, int i) {
    double fx = 0.0, fy = 0.0;
    if constexpr (W > 0) {
        int ent[W];
        double2 f[W];
#pragma unroll
        for (int d = 0; d < W; ++d) ent[d] = p.nlist[(int64_t)i * W + d];
#pragma unroll
        for (int d = 0; d < W; ++d) f[d] = ent[d] >= 0 ? p.fe[ent[d]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int d = 0; d < W; ++d)
            if (ent[d] >= 0) {
                fx = fx + f[d].x;
                fy = fy + f[d].y;
            }
    } else {
        const int t1 = p.csr_off[i + 1];
        for (int t = p.csr_off[i]; t < t1; ++t) {
            const double2 f = p.fe[p.csr_ent[t]];
            fx = fx + f.x;
            fy = fy + f.y;
        }
    }
    return make_double2(fx, fy);
}

template <int W>
__global__ __launch_bounds__(kB) void k_node(Params p, int j) {
    __shared__ double s_phi;
    const int64_t k = p.ctl->base + j;
    if (blockIdx.x == 0) pick(p, k);
    if (threadIdx.x == 0) s_phi = load_factor(p, (double)k * p.dt);
    __syncthreads();
    const int i = dev::xcd_tile(blockIdx.x, gridDim.x) * kB + threadIdx.x;
    if (i >= p.nn) return;
    const double2 f = gather<W>(p, i);
    const uint8_t fl = p.nflag[i];
    const double2 fx = (fl & kLoaded) ? p.fext[i] : make_double2(0.0, 0.0);
    const double phi = s_phi, mi = p.minv[i];
    double ax = (phi * fx.x - f.x) * mi;
    double ay = (phi * fx.y - f.y) * mi;
    if (fl & kFixX) ax = 0.0;
    if (fl & kFixY) ay = 0.0;
    const double dtv = (k == 0) ? 0.5 * p.dt : p.dt;
    const double th = ((double)k + 0.5) * p.dt;
    double2 v = p.v[i];
    double vx = v.x + dtv * ax;
    double vy = v.y + dtv * ay;
    if (fl & (kFixX | kFixY)) {
        const double2 v0 = p.v0[i];
        if (fl & kFixX) vx = prescribed(p, v0.x, th);
        if (fl & kFixY) vy = prescribed(p, v0.y, th);
    }
    p.v[i] = make_double2(vx, vy);
    const bool odd = (k & 1) != 0;
    const double2 u = (odd ? p.u1 : p.u0)[i];
    (odd ? p.u0 : p.u1)[i] = make_double2(u.x + p.dt * vx, u.y + p.dt * vy);
}

// LDS slots of the quadrilateral fused step: 256 patch elements and 128 ring
// elements, each with its four edge-midpoint strains and its area.
constexpr int kQuadSlots = kB + kB / 2;

// Coordinates and displacements of the four nodes of quadrilateral e.
__device__ __forceinline__ void quad_nodes(const Params &p, const double2 *u, int e, double x[4], double y[4],
                                           double ux[4], double uy[4]) {
    const int4 c = p.conn[e];
    const double2 u0 = u[c.x], u1 = u[c.y], u2 = u[c.z], u3 = u[c.w];
    const double2 x0 = p.xy[c.x], x1 = p.xy[c.y], x2 = p.xy[c.z], x3 = p.xy[c.w];
    x[0] = x0.x, x[1] = x1.x, x[2] = x2.x, x[3] = x3.x;
    y[0] = x0.y, y[1] = x1.y, y[2] = x2.y, y[3] = x3.y;
    ux[0] = u0.x, ux[1] = u1.x, ux[2] = u2.x, ux[3] = u3.x;
    uy[0] = u0.y, uy[1] = u1.y, uy[2] = u2.y, uy[3] = u3.y;
}

// An intact quadrilateral's strains at its four edge midpoints (row 3k + c
// of s_qd) and its area (row 12) into LDS slot l.
__device__ __forceinline__ void quad_store_strains(const double x[4], const double y[4], const double ux[4],
                                                   const double uy[4], double *s_qd, int l) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double gx[4], gy[4], q[3];
        dev::q4_grad(x, y, k, gx, gy);
        dev::strain<4>(gx, gy, ux, uy, q);
#pragma unroll
        for (int c = 0; c < 3; ++c) s_qd[(3 * k + c) * kQuadSlots + l] = q[c];
    }
    s_qd[12 * kQuadSlots + l] = quad_area(x, y);
}

// Smoothed stress of local edge k of an intact quadrilateral (area A, nodes
// x, y, ux, uy) whose neighbours' edge strains sit in LDS, and its gradients
// at that edge's midpoint.  Arithmetic as quad_element's: the neighbour's
// strain there, recomputed in the neighbour's own node order, equals the one
// the neighbour stored for itself.
__device__ __forceinline__ void quad_edge_sigma_shared(const Params &p, int k, const double x[4], const double y[4],
                                                       const double ux[4], const double uy[4], double A,
                                                       uint2 nbs, const double *s_qd, double gx[4], double gy[4],
                                                       double sg[3], bool &two) {
    double q[3], eps[3];
    dev::q4_grad(x, y, k, gx, gy);
    dev::strain<4>(gx, gy, ux, uy, q);
    const uint32_t sl = k < 3 ? (nbs.x >> (10 * k)) & kNoSlot : nbs.y & kNoSlot;
    const double A2 = sl != kNoSlot ? s_qd[12 * kQuadSlots + sl] : 0.0;
    two = A2 != 0.0;
    if (!two) {
        eps[0] = q[0];
        eps[1] = q[1];
        eps[2] = q[2];
    } else {
        const int loc = (nbs.y >> (16 + 2 * k)) & 3;
        const bool self_lo = ((nbs.y >> (10 + k)) & 1u) != 0;
        const double Alo = self_lo ? A : A2, Ahi = self_lo ? A2 : A;
        const double sum = Alo + Ahi;
        const double w0 = Alo / sum, w1 = Ahi / sum;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double q2 = s_qd[(3 * loc + c) * kQuadSlots + sl];
            const double lo = self_lo ? q[c] : q2, hi = self_lo ? q2 : q[c];
            eps[c] = fma(w1, hi, w0 * lo);
        }
    }
    hooke(p, eps, sg);
}

// Fused step of one patch of patch_nodes consecutive nodes (NV nodes per
// element: 3 triangles, 4 quadrilaterals): the forces of every
// element touching the patch (elements on patch borders are computed by
// each patch they touch; only the owning patch evaluates their candidates)
// go to LDS, then every owned node sums its slots in colour order and is
// updated.  u^k is read from buffer k & 1 and u^{k+1} written to the other,
// so neighbouring workgroups never see a half-updated displacement.
template <int NV, int W, int EMAX>
__global__ __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(NV == 3 && EMAX == kB ? 5 : 1)))
void k_fused(Params p, int j) {
    // triangles in patches of at most 256 elements and 256 ring elements
    // share their strains through LDS (one element and one ring element per
    // thread); the other forms recompute each neighbour's strain
    constexpr bool SHARED3 = NV == 3 && EMAX == kB;
    // quadrilaterals likewise with 128 ring elements; their forces reuse the
    // strains' LDS once every element has read its neighbours' strains
    constexpr bool SHARED4 = NV == 4 && EMAX == kB;
    __shared__ double2 s_fa[SHARED4 ? 1 : NV * EMAX];
    __shared__ double s_q[SHARED3 ? 3 : 1][SHARED3 ? 2 * kB : 1];
    __shared__ double s_A[SHARED3 ? 2 * kB : 1];
    __shared__ __align__(16) double s_qd[SHARED4 ? 13 * kQuadSlots : 1];
    double2 *const s_f = SHARED4 ? reinterpret_cast<double2 *>(s_qd) : s_fa;
    static_assert(!SHARED3 || NV * EMAX >= 2 * kPatchLocalNodes, "the staged nodes fit the forces' LDS");
    __shared__ double s_phi;
    __shared__ int s_pe;
    __shared__ uint8_t s_pcode;
    const int64_t k = p.ctl->base + j;
    const bool odd = (k & 1) != 0;
    const double2 *u = odd ? p.u1 : p.u0;
    const int b = dev::xcd_tile(blockIdx.x, gridDim.x), tid = threadIdx.x;
    Cand *clist = p.cand;
    int32_t *ccount = &p.ctl->nacc;
    const int s0 = p.patch_off[b], s1 = p.patch_off[b + 1];
    // shared-strain triangles: this thread's staged nodes (slots tid and
    // tid + kB of the patch's node list) and its element records, loaded
    // here, before the folded pick, which they do not depend on
    static_assert(kPatchLocalNodes <= 2 * kB, "at most two staged nodes per thread");
    double2 st_u0, st_x0, st_u1, st_x1;
    bool st0 = false, st1 = false;
    int32_t rec = 0, er = -1;
    uint2 lc = make_uint2(0, 0), rlc = make_uint2(0, 0);
    if constexpr (SHARED3) {
        const int nown = min(p.patch_nodes, p.nn - b * p.patch_nodes);
        const int h0 = p.patch_halo_off[b], nloc = nown + p.patch_halo_off[b + 1] - h0;
        const int la = tid, lb = tid + kB;
        st0 = la < nloc;
        st1 = lb < nloc;
        if (st0) {
            const int g = la < nown ? b * p.patch_nodes + la : p.patch_halo[h0 + la - nown];
            st_u0 = u[g];
            st_x0 = p.xy[g];
        }
        if (st1) {
            const int g = lb < nown ? b * p.patch_nodes + lb : p.patch_halo[h0 + lb - nown];
            st_u1 = u[g];
            st_x1 = p.xy[g];
        }
        if (s0 + tid < s1) {
            rec = p.patch_elem[s0 + tid];
            lc = p.patch_lconn[s0 + tid];
        }
        const int r = p.patch_ring_off[b] + tid;
        if (r < p.patch_ring_off[b + 1]) {
            er = p.patch_ring[r];
            rlc = p.patch_ring_lconn[r];
        }
    }
    if (p.fold) {
        // the pick of the segment's previous step, from its candidates (set
        // (j - 1) mod 3), taken alike by every workgroup; workgroup 0 records
        // it, the others see it through the split view
        const int prev = (j + 2) % 3;
        const int n = j > 0 ? p.fold_n[prev] : 0;  // uniform
        if (tid == 0) s_pe = -1;
        if (n > 0) {
            Cand bst;
            double gmin;
            best_of(p.fold_cand + (int64_t)prev * NV * p.ne, n, bst, gmin);
            if (tid == 0 && bst.G > p.gamma * (bst.G - gmin)) {
                s_pe = bst.elem;
                s_pcode = (uint8_t)(kSplitFlag | bst.ak);
                if (b == 0) apply_pick(p, bst, k - 1);
            }
        }
        // set (j + 1) mod 3 was last read by step j - 1: clear it for step j + 1
        if (b == 0 && tid == 0) p.fold_n[(j + 1) % 3] = 0;
        __syncthreads();
        clist = p.fold_cand + (int64_t)(j % 3) * NV * p.ne;
        ccount = p.fold_n + j % 3;
    }
    const SplitView sv{p.split, p.fold ? s_pe : -1, p.fold ? s_pcode : (uint8_t)0};
    if constexpr (SHARED3) {
        // the patch's node values into LDS (its own nodes, contiguous, then
        // its halo), in the space the forces take over later; then the own
        // strain and area of this thread's patch element and ring element
        // from there into the LDS slots tid and (s1 - s0) + tid
        double2 *const s_nu = s_f, *const s_nx = s_f + kPatchLocalNodes;
        if (st0) s_nu[tid] = st_u0, s_nx[tid] = st_x0;
        if (st1) s_nu[tid + kB] = st_u1, s_nx[tid + kB] = st_x1;
        const int s = s0 + tid;
        const bool mine = s < s1;
        const int e = rec & (kOwned - 1);
        const bool owned = (rec & kOwned) != 0;
        const uint8_t code = mine ? sv(e) : 0;
        const bool ringel = er >= 0;
        const uint8_t rcode = ringel ? sv(er) : 1;
        __syncthreads();
        double2 ue[3];
        Geo g;
        double q[3];
        if (mine) {
            if (code == 0) {
                double2 xe[3];
                const int l0 = lc.x & 0xffff, l1 = lc.x >> 16, l2 = lc.y;
                ue[0] = s_nu[l0], ue[1] = s_nu[l1], ue[2] = s_nu[l2];
                xe[0] = s_nx[l0], xe[1] = s_nx[l1], xe[2] = s_nx[l2];
                g = make_geo(xe[0], xe[1], xe[2]);
                strain(g, ue, q);
                s_q[0][tid] = q[0];
                s_q[1][tid] = q[1];
                s_q[2][tid] = q[2];
                s_A[tid] = g.A;
            } else {
                s_A[tid] = 0.0;
            }
        }
        if (ringel) {
            const int l = s1 - s0 + tid;
            if (rcode == 0) {
                const int l0 = rlc.x & 0xffff, l1 = rlc.x >> 16, l2 = rlc.y;
                const double2 ur[3] = {s_nu[l0], s_nu[l1], s_nu[l2]};
                const Geo gr = make_geo(s_nx[l0], s_nx[l1], s_nx[l2]);
                double qr[3];
                strain(gr, ur, qr);
                s_q[0][l] = qr[0];
                s_q[1][l] = qr[1];
                s_q[2][l] = qr[2];
                s_A[l] = gr.A;
            } else {
                s_A[l] = 0.0;
            }
        }
        __syncthreads();  // strains stored, node values read: the forces take the node space over
        if (mine) {
            double2 f[3];
            if (code) {
                const int4 c = p.conn[e];
                const Piece pa = piece(p, u, c, (code >> 2) & 3, code & 3);
                const Piece pb = piece(p, u, c, code & 3, (code >> 2) & 3);
                f[0] = piece_force_at(pa, pb, 0);
                f[1] = piece_force_at(pa, pb, 1);
                f[2] = piece_force_at(pa, pb, 2);
            } else {
                element_force_shared(p, e, ue, g, q, p.patch_nbr[s], s_q, s_A, owned, clist, ccount, f);
            }
            s_f[3 * tid] = f[0];
            s_f[3 * tid + 1] = f[1];
            s_f[3 * tid + 2] = f[2];
        }
    } else if constexpr (SHARED4) {
        const int s = s0 + tid;
        const bool mine = s < s1;
        int e = 0;
        bool owned = false;
        uint8_t code = 0;
        double x[4], y[4], ux[4], uy[4];
        if (mine) {
            const int32_t rec = p.patch_elem[s];
            e = rec & (kOwned - 1);
            owned = (rec & kOwned) != 0;
            code = sv(e);
            quad_nodes(p, u, e, x, y, ux, uy);
            if (code == 0)
                quad_store_strains(x, y, ux, uy, s_qd, tid);
            else
                s_qd[12 * kQuadSlots + tid] = 0.0;
        }
        const int r = p.patch_ring_off[b] + tid;
        if (r < p.patch_ring_off[b + 1]) {
            const int er = p.patch_ring[r];
            const int l = s1 - s0 + tid;
            if (sv(er) == 0) {
                double xr[4], yr[4], uxr[4], uyr[4];
                quad_nodes(p, u, er, xr, yr, uxr, uyr);
                quad_store_strains(xr, yr, uxr, uyr, s_qd, l);
            } else {
                s_qd[12 * kQuadSlots + l] = 0.0;
            }
        }
        __syncthreads();
        double2 f[4];
        if (mine) {
            if (code) {
                const double2 ue[4] = {make_double2(ux[0], uy[0]), make_double2(ux[1], uy[1]),
                                       make_double2(ux[2], uy[2]), make_double2(ux[3], uy[3])};
                switch (code & 15) {
#define QSPLIT(EN, EX) \
    case (EN << 2) | EX: (void)quad_split<EN, EX>(p, ue, x, y, f); break;
                    QSPLIT(0, 1) QSPLIT(0, 2) QSPLIT(0, 3) QSPLIT(1, 0) QSPLIT(1, 2) QSPLIT(1, 3)
                    QSPLIT(2, 0) QSPLIT(2, 1) QSPLIT(2, 3) QSPLIT(3, 0) QSPLIT(3, 1) QSPLIT(3, 2)
#undef QSPLIT
                    default:
#pragma unroll
                        for (int n = 0; n < 4; ++n) f[n] = make_double2(0.0, 0.0);
                        break;
                }
            } else {
                const uint2 nbs = p.patch_nbr[s];
                const double A = s_qd[12 * kQuadSlots + tid];
                bool two[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t sl = k < 3 ? (nbs.x >> (10 * k)) & kNoSlot : nbs.y & kNoSlot;
                    two[k] = sl != kNoSlot && s_qd[12 * kQuadSlots + sl] != 0.0;
                }
                if (owned && !(two[0] && two[1] && two[2] && two[3])) {
                    // a free-surface element: the edge stresses its candidates
                    // need, each computed where it is used
                    quad_candidates(
                        p, e, x, y, ux, uy,
                        [&](int k, double sg[3]) {
                            // an opaque copy of the area keeps the compiler from
                            // merging these calls into four stresses held at once
                            double Ak = A;
                            asm volatile("" : "+v"(Ak));
                            double gx[4], gy[4];
                            bool t;
                            quad_edge_sigma_shared(p, k, x, y, ux, uy, Ak, nbs, s_qd, gx, gy, sg, t);
                        },
                        two, clist, ccount);
                }
                double sx[4], sy[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    double gx[4], gy[4], sg[3];
                    bool t;
                    quad_edge_sigma_shared(p, k, x, y, ux, uy, A, nbs, s_qd, gx, gy, sg, t);
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const double tx = fma(gy[m], sg[2], gx[m] * sg[0]);
                        const double ty = fma(gx[m], sg[2], gy[m] * sg[1]);
                        sx[m] = k == 0 ? tx : sx[m] + tx;
                        sy[m] = k == 0 ? ty : sy[m] + ty;
                    }
                }
                const double cA = 0.25 * A;
#pragma unroll
                for (int m = 0; m < 4; ++m) f[m] = make_double2(cA * sx[m], cA * sy[m]);
            }
        }
        __syncthreads();  // every strain read: the forces take the LDS over
        if (mine) {
#pragma unroll
            for (int n = 0; n < 4; ++n) s_f[4 * tid + n] = f[n];
        }
    } else {
        // the other forms: each element re-derives its neighbours' strains
        for (int s = s0 + tid; s < s1; s += kB) {
            const int32_t rec = p.patch_elem[s];
            const int l = NV * (s - s0);
            if constexpr (NV == 3) {
                double2 f[3];
                element_force(p, sv, u, rec & (kOwned - 1), (rec & kOwned) != 0, clist, ccount, f);
                s_f[l] = f[0];
                s_f[l + 1] = f[1];
                s_f[l + 2] = f[2];
            } else {
                quad_element<false>(p, sv, u, rec & (kOwned - 1), (rec & kOwned) != 0, clist, ccount, Eval{},
                                    s_f + l, 1);
            }
        }
    }
    if (tid == 0) s_phi = load_factor(p, (double)k * p.dt);
    __syncthreads();
    const int i = b * p.patch_nodes + tid;
    if (tid >= p.patch_nodes || i >= p.nn) return;
    uint16_t sl[W];
#pragma unroll
    for (int d = 0; d < W; ++d) sl[d] = p.patch_slots[(int64_t)i * W + d];
    double fx = 0.0, fy = 0.0;
#pragma unroll
    for (int d = 0; d < W; ++d)
        if (sl[d] != 0xffff) {
            const double2 f = s_f[sl[d]];
            fx = fx + f.x;
            fy = fy + f.y;
        }
    const uint8_t fl = p.nflag[i];
    const double2 fxt = (fl & kLoaded) ? p.fext[i] : make_double2(0.0, 0.0);
    const double phi = s_phi, mi = p.minv[i];
    double ax = (phi * fxt.x - fx) * mi;
    double ay = (phi * fxt.y - fy) * mi;
    if (fl & kFixX) ax = 0.0;
    if (fl & kFixY) ay = 0.0;
    const double dtv = (k == 0) ? 0.5 * p.dt : p.dt;
    const double th = ((double)k + 0.5) * p.dt;
    const double2 v = p.v[i];
    double vx = v.x + dtv * ax;
    double vy = v.y + dtv * ay;
    if (fl & (kFixX | kFixY)) {
        const double2 v0 = p.v0[i];
        if (fl & kFixX) vx = prescribed(p, v0.x, th);
        if (fl & kFixY) vy = prescribed(p, v0.y, th);
    }
    p.v[i] = make_double2(vx, vy);
    const double2 uk = u[i];
    (odd ? p.u0 : p.u1)[i] = make_double2(uk.x + p.dt * vx, uk.y + p.dt * vy);
}

// The global pick of step base + j after a fused step (one workgroup).
__global__ __launch_bounds__(kB) void k_pick(Params p, int j) { pick(p, p.ctl->base + j); }

__global__ void k_commit(Params p, int n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p.ctl->base = p.ctl->base + n;
}

// Segment close with the folded pick: the pick of the segment's last step,
// then every candidate set cleared and the step counter advanced.
__global__ __launch_bounds__(kB) void k_commit_fold(Params p, int n) {
    const int64_t base = p.ctl->base;
    if (n > 0) {
        const int set = (n + 2) % 3;
        pick_from(p, p.fold_cand + (int64_t)set * p.nv * p.ne, p.fold_n + set, base + n - 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        p.fold_n[0] = 0;
        p.fold_n[1] = 0;
        p.fold_n[2] = 0;
        p.ctl->base = base + n;
    }
}

// Query: internal force, acceleration and energy terms per node.
__global__ __launch_bounds__(kB) void k_eval_nodes(Params p, const double2 *u, const double2 *v, int64_t k,
                                                   double phi, const double *mass, Eval ev) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= p.nn) return;
    const double2 f = gather<0>(p, i);
    if (ev.fint) {
        ev.fint[i] = f.x;
        ev.fint[p.nn + i] = f.y;
    }
    const uint8_t fl = p.nflag[i];
    const double2 fx = (fl & kLoaded) ? p.fext[i] : make_double2(0.0, 0.0);
    const double mi = p.minv[i];
    double ax = (phi * fx.x - f.x) * mi;
    double ay = (phi * fx.y - f.y) * mi;
    if (fl & kFixX) ax = 0.0;
    if (fl & kFixY) ay = 0.0;
    if (ev.acc) {
        ev.acc[i] = ax;
        ev.acc[p.nn + i] = ay;
    }
    if (ev.node_e && v) {
        double2 vv = v[i];
        double vx = vv.x, vy = vv.y;
        if (k > 0) {
            if (!(fl & kFixX)) vx = vx + 0.5 * p.dt * ax;
            if (!(fl & kFixY)) vy = vy + 0.5 * p.dt * ay;
        }
        const double2 uu = u[i];
        ev.node_e[2 * (int64_t)i] = 0.5 * mass[i] * (vx * vx + vy * vy);
        ev.node_e[2 * (int64_t)i + 1] = phi * fx.x * uu.x + phi * fx.y * uu.y;
    }
}

__global__ __launch_bounds__(kB) void k_tip_flags(Params p, const int32_t *edge_elem, int64_t ns, uint8_t *flag) {
    const int64_t s = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (s >= ns) return;
    const int e0 = edge_elem[2 * s], e1 = edge_elem[2 * s + 1];
    uint8_t r = 0;
    if (e0 >= 0 && e1 >= 0) {
        const int i0 = p.split[e0] == 0, i1 = p.split[e1] == 0;
        r = (i0 + i1 == 1) ? 1 : 0;
    }
    flag[s] = r;
}

// Power iteration on M^-1/2 K M^-1/2 over the free components.
__global__ __launch_bounds__(kB) void k_scale_in(Params p, const double *y, double2 *u) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= p.nn) return;
    const uint8_t fl = p.nflag[i];
    const double r = sqrt(p.minv[i]);
    u[i] = make_double2((fl & kFixX) ? 0.0 : y[i] * r, (fl & kFixY) ? 0.0 : y[p.nn + i] * r);
}

__global__ __launch_bounds__(kB) void k_scale_out(Params p, const double *fint, const double *y, double *z,
                                                  double *yz_zz) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= p.nn) return;
    const uint8_t fl = p.nflag[i];
    const double r = sqrt(p.minv[i]);
    const double zx = (fl & kFixX) ? 0.0 : fint[i] * r;
    const double zy = (fl & kFixY) ? 0.0 : fint[p.nn + i] * r;
    z[i] = zx;
    z[p.nn + i] = zy;
    yz_zz[2 * (int64_t)i] = y[i] * zx + y[p.nn + i] * zy;
    yz_zz[2 * (int64_t)i + 1] = zx * zx + zy * zy;
}

__global__ __launch_bounds__(kB) void k_normalize(int64_t n, const double *z, const double *zz, double *y) {
    const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (t >= n) return;
    const double s = sqrt(*zz);
    y[t] = s > 0.0 ? z[t] / s : 0.0;
}

// Per-front pick (variant of the Sec. 3 pick) over the step's candidate
// list, one workgroup, between k_force and k_node (whose own pick then sees
// an empty list).
constexpr int kFrontThreads = 1024;

struct TriGeom {
    const int4 *conn;
    const double2 *xy;
    int nv;
    __device__ int node(const int4 &c, int n) const { return sel4(n % nv, c.x, c.y, c.z, c.w); }
    __device__ double2 tip(int e, int a) const {
        const int4 c = conn[e];
        const double2 P = xy[node(c, a)], Q = xy[node(c, a + 1)];
        return make_double2(0.5 * (P.x + Q.x), 0.5 * (P.y + Q.y));
    }
    __device__ double path_len(int e, int a, int k) const {
        const int4 c = conn[e];
        const double2 P0 = xy[node(c, a)], P1 = xy[node(c, a + 1)];
        const double2 Q0 = xy[node(c, k)], Q1 = xy[node(c, k + 1)];
        const double g0x = 0.5 * (P0.x + P1.x), g0y = 0.5 * (P0.y + P1.y);
        const double gkx = 0.5 * (Q0.x + Q1.x), gky = 0.5 * (Q0.y + Q1.y);
        const double dx = gkx - g0x, dy = gky - g0y;
        return sqrt(dx * dx + dy * dy);
    }
};

__host__ __device__ inline FrontView tri_front_view(const Params &p) {
    FrontView v;
    v.cand = p.cand;
    v.count = reinterpret_cast<uint32_t *>(&p.ctl->nacc);
    v.mid = p.fmid;
    v.len = p.flen;
    v.order = p.forder;
    v.bucket = p.fbucket;
    v.sorted = p.fsorted;
    v.plist = p.fplist;
    v.cell = p.fcell;
    v.split = p.split;
    v.log = p.log;
    v.log_cap = p.log_cap;
    v.nsplit = &p.ctl->nsplit;
    v.Ud = &p.ctl->Ud;
    v.overflow = &p.ctl->overflow;
    v.base = &p.ctl->base;
    v.gc = p.gc;
    v.gc_uniform = 0.0;
    v.gamma = p.gamma;
    v.rho2 = p.front_r2;
    return v;
}

__host__ __device__ inline TriGeom tri_geom(const Params &p) {
    TriGeom g;
    g.conn = p.conn;
    g.xy = p.xy;
    g.nv = p.nv;
    return g;
}

__global__ __launch_bounds__(kFrontThreads) void k_front(Params p, int j) {
    front_pick_block<kFrontThreads>(tri_front_view(p), tri_geom(p), j);
}

// The per-front pick: over the whole GPU when the mesh has its bucket
// table, else one workgroup.
hipError_t launch_front(const Params &p, int j, hipStream_t st) {
    if (p.fgrid) return launch_front_grid(tri_front_view(p), tri_geom(p), p.fgrid, j, false, st);
    k_front<<<1, kFrontThreads, 0, st>>>(p, j);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(const Params &p, int j, hipStream_t st) {
    if (p.patch_emax > 0) {
        if ((p.nv != 3 && p.nv != 4) || p.patch_nodes < 1 || p.patch_nodes > kPatchMaxNodes ||
            p.patch_emax > 1024)
            return hipErrorInvalidValue;
        const int np = (p.nn + p.patch_nodes - 1) / p.patch_nodes;
        const int key = (p.nv * 32 + p.nlist_w) * 4 + (p.patch_emax <= 256 ? 0 : p.patch_emax <= 512 ? 1 : 2);
        switch (key) {
#define FUSED(NVv, Wv, E, kk) \
    case (NVv * 32 + Wv) * 4 + kk: k_fused<NVv, Wv, E><<<np, kB, 0, st>>>(p, j); break;
#define FUSED_W(NVv, Wv) FUSED(NVv, Wv, 256, 0) FUSED(NVv, Wv, 512, 1) FUSED(NVv, Wv, 1024, 2)
            FUSED_W(3, 4) FUSED_W(3, 8) FUSED_W(3, 12) FUSED_W(3, 16)
            FUSED_W(4, 4) FUSED_W(4, 8) FUSED_W(4, 12) FUSED_W(4, 16)
#undef FUSED_W
#undef FUSED
            default: return hipErrorInvalidValue;
        }
        if (p.fold) return hipGetLastError();  // the next step (or the commit) picks
        if (p.front_r2 > 0.0) return launch_front(p, j, st);
        k_pick<<<1, kB, 0, st>>>(p, j);
        return hipGetLastError();
    }
    if (p.nv == 4)
        k_qforce<false><<<nb_of(p.ne), kB, 0, st>>>(p, p.u0, Eval{}, j);
    else
        k_force<false><<<nb_of(p.ne), kB, 0, st>>>(p, p.u0, Eval{}, j);
    if (p.front_r2 > 0.0) {
        const hipError_t e = launch_front(p, j, st);
        if (e != hipSuccess) return e;
    }
    const int nb = nb_of(p.nn);
    switch (p.nlist ? p.nlist_w : 0) {
        case 4: k_node<4><<<nb, kB, 0, st>>>(p, j); break;
        case 8: k_node<8><<<nb, kB, 0, st>>>(p, j); break;
        case 12: k_node<12><<<nb, kB, 0, st>>>(p, j); break;
        case 16: k_node<16><<<nb, kB, 0, st>>>(p, j); break;
        default: k_node<0><<<nb, kB, 0, st>>>(p, j); break;
    }
    return hipGetLastError();
}

hipError_t launch_commit(const Params &p, int n, hipStream_t st) {
    if (p.fold)
        k_commit_fold<<<1, kB, 0, st>>>(p, n);
    else
        k_commit<<<1, 64, 0, st>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_eval(const Params &p, const double2 *u, const double2 *v, int64_t k, double phi,
                       const double *mass, const Eval &ev, hipStream_t st) {
    (void)hipGetLastError();
    if (p.nv == 4)
        k_qforce<true><<<nb_of(p.ne), kB, 0, st>>>(p, u, ev, 0);
    else
        k_force<true><<<nb_of(p.ne), kB, 0, st>>>(p, u, ev, 0);
    k_eval_nodes<<<nb_of(p.nn), kB, 0, st>>>(p, u, v, k, phi, mass, ev);
    return hipGetLastError();
}

hipError_t launch_tip_flags(const Params &p, const int32_t *edge_elem, int64_t ns, uint8_t *flag, hipStream_t st) {
    (void)hipGetLastError();
    k_tip_flags<<<nb_of(ns), kB, 0, st>>>(p, edge_elem, ns, flag);
    return hipGetLastError();
}

hipError_t launch_power_step(const Params &p, const Eval &ev, double *y, double2 *u, double *z, double *yz_zz,
                             double *part, double *sums, hipStream_t st) {
    (void)hipGetLastError();
    k_scale_in<<<nb_of(p.nn), kB, 0, st>>>(p, y, u);
    Eval e2{};
    e2.fint = ev.fint;
    hipError_t e = launch_eval(p, u, nullptr, 0, 1.0, nullptr, e2, st);
    if (e != hipSuccess) return e;
    k_scale_out<<<nb_of(p.nn), kB, 0, st>>>(p, ev.fint, y, z, yz_zz);
    e = launch_sum(yz_zz, p.nn, 2, 0, part, sums, st);
    if (e == hipSuccess) e = launch_sum(yz_zz, p.nn, 2, 1, part, sums + 1, st);
    if (e != hipSuccess) return e;
    k_normalize<<<nb_of(2 * (int64_t)p.nn), kB, 0, st>>>(2 * (int64_t)p.nn, z, sums + 1, y);
    return hipGetLastError();
}

}  // namespace tri
}  // namespace mct
