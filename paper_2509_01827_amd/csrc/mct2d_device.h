// Element-level device arithmetic shared by the step and screen kernels
// (binary64 or binary32, compiled with -ffp-contract=off; fma only where
// written).
#pragma once

#include "mct2d_impl.h"

namespace mct {
namespace dev {

// natural coordinates of Q4 nodes and of the edge midpoints
__device__ __forceinline__ double xi_n(int n) { return (n == 1 || n == 2) ? 1.0 : -1.0; }
__device__ __forceinline__ double eta_n(int n) { return (n >= 2) ? 1.0 : -1.0; }
__device__ __forceinline__ double xi_m(int k) { return k == 1 ? 1.0 : (k == 3 ? -1.0 : 0.0); }
__device__ __forceinline__ double eta_m(int k) { return k == 0 ? -1.0 : (k == 2 ? 1.0 : 0.0); }

// Map workgroups onto work blocks (tiles, runs of elements or nodes) so that
// consecutive workgroups of one XCD (the hardware deals workgroup ids
// round-robin over the 8 XCDs) own a contiguous band of blocks and share the
// lines at the band's inner borders in their L2.  A bijection of [0, nwg).
__device__ __forceinline__ int xcd_tile(int b, int nwg) {
    const int q = nwg / 8, r = nwg % 8;
    const int x = b % 8, l = b / 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

// Pointer parameters that may receive nullptr take their type from another
// argument.
template <class T>
struct Same {
    using type = T;
};

// The helpers below are templates over the arithmetic type T (double for
// the binary64 step, float for the binary32 step); every constant is a T,
// so an expression never widens to double.

// Fused multiply-add of one rounding in T.  The overloaded fma can resolve
// to the binary64 version for float arguments inside a generic lambda, so
// templated code calls this one.
template <class T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "float or double");
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

// dN/dx, dN/dy of the bilinear element at the midpoint of its local edge k.
//
// The shape-function derivatives in natural coordinates at an edge midpoint
// are 0, +-1/4 or +-1/2, so every product with them is exact.  The sums are
// written over the non-zero terms only: adding a zero product to a running
// sum, or subtracting one, leaves every non-zero value unchanged (at most
// the sign of a zero differs), so the result equals the plain evaluation
//   J = sum_n dN_n/d(xi,eta) * (x_n, y_n)    (fma chain from 0, n = 0..3)
//   dN_n/dx = (J22 dN_n/dxi - J12 dN_n/deta) / det J  (as * (1/det))
//   dN_n/dy = (J11 dN_n/deta - J21 dN_n/dxi) / det J
// bit for bit.  With k a compile-time constant after unrolling, the zero
// tests fold away.
template <class T>
__device__ __forceinline__ T exact_dot4(const T c[4], const T v[4]) {
    T s = T(0);
    bool first = true;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        if (c[n] != T(0)) {
            s = first ? c[n] * v[n] : fmat(c[n], v[n], s);
            first = false;
        }
    }
    return s;
}

template <class T>
__device__ __forceinline__ void q4_grad(const T x[4], const T y[4], int k, T dndx[4], T dndy[4]) {
    T dxi[4], deta[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        dxi[n] = T(0.25) * T(xi_n(n)) * (T(1) + T(eta_m(k)) * T(eta_n(n)));
        deta[n] = T(0.25) * T(eta_n(n)) * (T(1) + T(xi_m(k)) * T(xi_n(n)));
    }
    const T j11 = exact_dot4(dxi, x);
    const T j12 = exact_dot4(dxi, y);
    const T j21 = exact_dot4(deta, x);
    const T j22 = exact_dot4(deta, y);
    const T det = j11 * j22 - j12 * j21;
    const T inv = T(1) / det;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        T a, b;
        if (dxi[n] != T(0) && deta[n] != T(0)) {
            a = fmat(j22, dxi[n], -(j12 * deta[n]));
            b = fmat(j11, deta[n], -(j21 * dxi[n]));
        } else if (dxi[n] != T(0)) {
            a = j22 * dxi[n];
            b = -(j21 * dxi[n]);
        } else {
            a = -(j12 * deta[n]);
            b = j11 * deta[n];
        }
        dndx[n] = a * inv;
        dndy[n] = b * inv;
    }
}

// q4_grad with the edge index as a template argument (for runtime k).
template <class T>
__device__ __forceinline__ void q4_grad_rt(const T x[4], const T y[4], int k, T dndx[4], T dndy[4]) {
    switch (k) {
        case 0: q4_grad(x, y, 0, dndx, dndy); break;
        case 1: q4_grad(x, y, 1, dndx, dndy); break;
        case 2: q4_grad(x, y, 2, dndx, dndy); break;
        default: q4_grad(x, y, 3, dndx, dndy); break;
    }
}

// Sub-cell of a Q4 element at its local edge k: the triangle (n_k, n_k+1,
// c), c the vertex centroid; the displacement at c is the mean of the four
// nodal displacements.  Gradients b (d/dx), c (d/dy) of the triangle's
// linear shape functions in corner order (n_k, n_k+1, c), the strain of
// its corner displacements, and its area (returned).
template <int K, class T>
__device__ __forceinline__ T subcell(const T x[4], const T y[4], const typename Same<T>::type *ux,
                                     const typename Same<T>::type *uy, T b[3], T c[3],
                                     typename Same<T>::type *q) {
    constexpr int K1 = (K + 1) & 3;
    const T xa = x[K], ya = y[K], xb = x[K1], yb = y[K1];
    const T xc = T(0.25) * (((x[0] + x[1]) + x[2]) + x[3]);
    const T yc = T(0.25) * (((y[0] + y[1]) + y[2]) + y[3]);
    const T twoA = (xb - xa) * (yc - ya) - (xc - xa) * (yb - ya);
    const T inv = T(1) / twoA;
    b[0] = (yb - yc) * inv;
    b[1] = (yc - ya) * inv;
    b[2] = (ya - yb) * inv;
    c[0] = (xc - xb) * inv;
    c[1] = (xa - xc) * inv;
    c[2] = (xb - xa) * inv;
    if (ux) {
        const T pu[3] = {ux[K], ux[K1], T(0.25) * (((ux[0] + ux[1]) + ux[2]) + ux[3])};
        const T pv[3] = {uy[K], uy[K1], T(0.25) * (((uy[0] + uy[1]) + uy[2]) + uy[3])};
        T exx = T(0), eyy = T(0), gxy = T(0);
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            exx = fmat(b[n], pu[n], exx);
            eyy = fmat(c[n], pv[n], eyy);
            gxy = fmat(c[n], pu[n], gxy);
            gxy = fmat(b[n], pv[n], gxy);
        }
        q[0] = exx;
        q[1] = eyy;
        q[2] = gxy;
    }
    return T(0.5) * twoA;
}

// subcell with the edge index at run time
template <class T>
__device__ __forceinline__ T subcell_rt(const T x[4], const T y[4], const typename Same<T>::type *ux,
                                        const typename Same<T>::type *uy, int k, T b[3], T c[3],
                                        typename Same<T>::type *q) {
    switch (k) {
        case 0: return subcell<0>(x, y, ux, uy, b, c, q);
        case 1: return subcell<1>(x, y, ux, uy, b, c, q);
        case 2: return subcell<2>(x, y, ux, uy, b, c, q);
        default: return subcell<3>(x, y, ux, uy, b, c, q);
    }
}

// Force of an intact Q4 element with sub-cell smoothing: sum over its edges
// k of A_T B_T^T sigma_k, the centroid corner's share a quarter to each
// node; per node and edge the bracket t_a + t_c/4 (node k), t_b + t_c/4
// (node k+1) or t_c/4, scaled by A_T, summed over k = 0..3 in order.
template <class T>
__device__ __forceinline__ void subcell_force(const T bb[4][3], const T cb[4][3], const T AT[4],
                                              const T sig[4][3], T fe[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T s0 = sig[k][0], s1 = sig[k][1], s2 = sig[k][2];
        T tx[3], ty[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            tx[i] = fmat(cb[k][i], s2, bb[k][i] * s0);
            ty[i] = fmat(bb[k][i], s2, cb[k][i] * s1);
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            T gx = T(0.25) * tx[2], gy = T(0.25) * ty[2];
            if (n == k) {
                gx = tx[0] + T(0.25) * tx[2];
                gy = ty[0] + T(0.25) * ty[2];
            } else if (n == ((k + 1) & 3)) {
                gx = tx[1] + T(0.25) * tx[2];
                gy = ty[1] + T(0.25) * ty[2];
            }
            const T vx = AT[k] * gx, vy = AT[k] * gy;
            if (k == 0) {
                fe[2 * n] = vx;
                fe[2 * n + 1] = vy;
            } else {
                fe[2 * n] = fe[2 * n] + vx;
                fe[2 * n + 1] = fe[2 * n + 1] + vy;
            }
        }
    }
}

template <int NN, class T>
__device__ __forceinline__ void strain(const T *dndx, const T *dndy, const T *ux, const T *uy, T eps[3]) {
    T exx = T(0), eyy = T(0), gxy = T(0);
#pragma unroll
    for (int n = 0; n < NN; ++n) {
        exx = fmat(dndx[n], ux[n], exx);
        eyy = fmat(dndy[n], uy[n], eyy);
        gxy = fmat(dndy[n], ux[n], gxy);
        gxy = fmat(dndx[n], uy[n], gxy);
    }
    eps[0] = exx;
    eps[1] = eyy;
    eps[2] = gxy;
}

template <class T>
__device__ __forceinline__ void hooke(const StepParamsT<T> &p, const T eps[3], T sig[3]) {
    sig[0] = fmat(p.D12, eps[1], p.D11 * eps[0]);
    sig[1] = fmat(p.D12, eps[0], p.D11 * eps[1]);
    sig[2] = p.D33 * eps[2];
}

// Unit normal and length of the crack path from the midpoint of local edge
// a (end nodes (xa0, ya0), (xa1, ya1) = n_a, n_{a+1}) to the midpoint of
// local edge k (end nodes n_k, n_{k+1}), oriented toward node n_{a+1}
// (reference coordinates).  Uses correctly rounded sqrt and division only.
template <class T>
__device__ __forceinline__ void path_geom_pts(T xa0, T ya0, T xa1, T ya1, T xk0, T yk0, T xk1, T yk1, T &nxo,
                                              T &nyo, T &len) {
    const T g0x = T(0.5) * (xa0 + xa1), g0y = T(0.5) * (ya0 + ya1);
    const T gkx = T(0.5) * (xk0 + xk1), gky = T(0.5) * (yk0 + yk1);
    const T dx = gkx - g0x, dy = gky - g0y;
    const T L = sqrt(dx * dx + dy * dy);
    T cx = dy / L, cy = -dx / L;
    if (cx * (xa1 - g0x) + cy * (ya1 - g0y) < T(0)) {
        cx = -cx;
        cy = -cy;
    }
    nxo = cx;
    nyo = cy;
    len = L;
}

template <class T>
__device__ __forceinline__ void path_geom(const T x[4], const T y[4], int a, int k, T &nxo, T &nyo, T &len) {
    const int a1 = (a + 1) & 3, k1 = (k + 1) & 3;
    path_geom_pts(x[a], y[a], x[a1], y[a1], x[k], y[k], x[k1], y[k1], nxo, nyo, len);
}


// Edge s of the structured grid (ids in ascending (smaller node, larger
// node) order): its nodes and its neighbour elements (e0 the lower id, -1
// outside the mesh).
struct EdgeInfo {
    int lo, hi;    // node ids
    int e0, e1;    // neighbour elements (-1 if none)
};

__device__ __forceinline__ EdgeInfo edge_info(int64_t s, int nx, int ny) {
    EdgeInfo r;
    const int64_t row = 2 * (int64_t)nx + 1;
    int i, j;
    bool horiz;
    if (s < (int64_t)ny * row) {
        j = (int)(s / row);
        const int q = (int)(s % row);
        if (q < 2 * nx) {
            i = q >> 1;
            horiz = (q & 1) == 0;
        } else {
            i = nx;
            horiz = false;
        }
    } else {
        j = ny;
        i = (int)(s - (int64_t)ny * row);
        horiz = true;
    }
    r.lo = j * (nx + 1) + i;
    if (horiz) {
        r.hi = r.lo + 1;
        r.e0 = (j > 0) ? (j - 1) * nx + i : -1;
        r.e1 = (j < ny) ? j * nx + i : -1;
    } else {
        r.hi = r.lo + nx + 1;
        r.e0 = (i > 0) ? j * nx + i - 1 : -1;
        r.e1 = (i < nx) ? j * nx + i : -1;
    }
    return r;
}

// Id of the horizontal edge starting at node (i, j) and of the vertical one.
__device__ __forceinline__ int64_t edge_h(int64_t i, int64_t j, int nx, int ny) {
    const int64_t row = 2 * (int64_t)nx + 1;
    return j < ny ? j * row + 2 * i : (int64_t)ny * row + i;
}
__device__ __forceinline__ int64_t edge_v(int64_t i, int64_t j, int nx) {
    const int64_t row = 2 * (int64_t)nx + 1;
    return j * row + (i < nx ? 2 * i + 1 : 2 * (int64_t)nx);
}

// Load factor of the tractions at time t: piecewise linear through the
// curve points, constant beyond its ends, 1 without a curve.
template <class T>
__device__ __forceinline__ double load_factor(const StepParamsT<T> &p, double t) {
    if (p.ncurve == 0) return 1.0;
    if (t <= p.curve_t[0]) return p.curve_phi[0];
    const int n = p.ncurve;
    if (t >= p.curve_t[n - 1]) return p.curve_phi[n - 1];
    int i = 0;
    while (p.curve_t[i + 1] <= t) ++i;
    const double slope = (p.curve_phi[i + 1] - p.curve_phi[i]) / (p.curve_t[i + 1] - p.curve_t[i]);
    return p.curve_phi[i] + (t - p.curve_t[i]) * slope;
}

}  // namespace dev
}  // namespace mct
