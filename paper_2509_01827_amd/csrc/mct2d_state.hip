// HIP kernels (gfx950) for state queries: smoothed edge stresses, element
// and nodal internal forces, accelerations, energies, the largest
// eigenvalue of M^-1 K (stability limit of the explicit step) and a
// finiteness check of the fields.  They use the step's element arithmetic
// (same helpers, same orders) but are not on the step's path.
#include <algorithm>

#include "mct2d_device.h"
#include "mct2d_impl.h"
#include "mct2d_tri.h"

namespace mct {

namespace {
using namespace dev;

constexpr int kB = 256;

__device__ __forceinline__ void elem_nodes(const StepParams &p, int64_t e, int64_t nd[4]) {
    const int64_t i = e % p.nx, j = e / p.nx;
    const int64_t n0 = j * (p.nx + 1) + i;
    nd[0] = n0;
    nd[1] = n0 + 1;
    nd[2] = n0 + p.nx + 2;
    nd[3] = n0 + p.nx + 1;
}

// Smoothed strain and stress of every edge (Sec. 2.1: strain averaged over
// the intact neighbours with w_j = A_j / (A_lo + A_hi), lower id first; one
// intact neighbour: its own strain), plus the edge's strain energy
// 1/2 A_s sigma:eps with smoothing-domain area A_s = sum of intact A_j / 4.
// Edges without an intact neighbour get NaN stresses and zero energy.
__global__ __launch_bounds__(kB) void k_eval_edges(StepParams p, const double *ux, const double *uy, EvalDev d) {
    const int64_t ns = 2 * (int64_t)p.nx * p.ny + p.nx + p.ny;
    const int64_t s = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (s >= ns) return;
    const EdgeInfo ei = edge_info(s, p.nx, p.ny);
    const bool horiz = ei.hi == ei.lo + 1;
    double q[2][3], A[2], As = 0.0;
    int cnt = 0;
    for (int side = 0; side < 2; ++side) {
        const int64_t e = side ? ei.e1 : ei.e0;
        if (e < 0 || p.split[e] != 0) continue;
        const int k = horiz ? (side ? 0 : 2) : (side ? 3 : 1);
        int64_t nd[4];
        elem_nodes(p, e, nd);
        double x[4], y[4], u[4], v[4], gx[4], gy[4];
        for (int n = 0; n < 4; ++n) {
            x[n] = p.X[nd[n]];
            y[n] = p.Y[nd[n]];
            u[n] = ux[nd[n]];
            v[n] = uy[nd[n]];
        }
        if (p.subcell) {
            // sub-cell smoothing: the sub-cell's strain and area
            double b3[3], c3[3];
            A[cnt] = subcell_rt(x, y, u, v, k, b3, c3, q[cnt]);
            As += A[cnt];
        } else {
            q4_grad_rt(x, y, k, gx, gy);
            strain<4>(gx, gy, u, v, q[cnt]);
            A[cnt] = p.area[e];
            As += p.area[e] / 4.0;
        }
        ++cnt;
    }
    double *sg = d.sig + 3 * s;
    if (cnt == 0) {
        sg[0] = sg[1] = sg[2] = __builtin_nan("");
        d.es[s] = 0.0;
        return;
    }
    double eps[3];
    if (cnt == 1) {
        for (int c = 0; c < 3; ++c) eps[c] = q[0][c];
    } else {
        const double sum = A[0] + A[1];
        const double w0 = A[0] / sum, w1 = A[1] / sum;
        for (int c = 0; c < 3; ++c) eps[c] = fma(w1, q[1][c], w0 * q[0][c]);
    }
    double t[3];
    hooke(p, eps, t);
    sg[0] = t[0];
    sg[1] = t[1];
    sg[2] = t[2];
    d.es[s] = 0.5 * As * (t[0] * eps[0] + t[1] * eps[1] + t[2] * eps[2]);
}

// One piece of a split element: nodes entry+1 .. exit (CCW) closed by the
// midpoints of the exit and entry edges; constant-strain triangle (3
// nodes), bar along the uncut edge (2 nodes) or nothing (1 node).  Writes
// the forces of its nodes and returns its strain energy.
__device__ double piece(const StepParams &p, const double x[4], const double y[4], const double u[4],
                        const double v[4], int entry, int exit_, double f[8]) {
    int loc[3];
    int np = 0;
    for (int k = (entry + 1) & 3;; k = (k + 1) & 3) {
        loc[np++] = k;
        if (k == exit_) break;
    }
    double px[5], py[5];
    int nv = 0;
    px[nv] = 0.5 * (x[entry] + x[(entry + 1) & 3]);
    py[nv++] = 0.5 * (y[entry] + y[(entry + 1) & 3]);
    for (int i = 0; i < np; ++i) {
        px[nv] = x[loc[i]];
        py[nv++] = y[loc[i]];
    }
    px[nv] = 0.5 * (x[exit_] + x[(exit_ + 1) & 3]);
    py[nv++] = 0.5 * (y[exit_] + y[(exit_ + 1) & 3]);
    double sa = 0.0;
    for (int i = 1; i + 1 < nv; ++i)
        sa += (px[i] - px[0]) * (py[i + 1] - py[0]) - (px[i + 1] - px[0]) * (py[i] - py[0]);
    const double Ap = 0.5 * sa;
    if (np == 3) {
        const double x1 = px[1], y1 = py[1], x2 = px[2], y2 = py[2], x3 = px[3], y3 = py[3];
        const double twoA = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1);
        const double inv = 1.0 / twoA;
        const double b[3] = {(y2 - y3) * inv, (y3 - y1) * inv, (y1 - y2) * inv};
        const double c[3] = {(x3 - x2) * inv, (x1 - x3) * inv, (x2 - x1) * inv};
        double pu[3], pv[3], eps[3], sg[3];
        for (int i = 0; i < 3; ++i) {
            pu[i] = u[loc[i]];
            pv[i] = v[loc[i]];
        }
        strain<3>(b, c, pu, pv, eps);
        hooke(p, eps, sg);
        for (int i = 0; i < 3; ++i) {
            f[2 * loc[i]] = Ap * fma(c[i], sg[2], b[i] * sg[0]);
            f[2 * loc[i] + 1] = Ap * fma(b[i], sg[2], c[i] * sg[1]);
        }
        return 0.5 * Ap * (sg[0] * eps[0] + sg[1] * eps[1] + sg[2] * eps[2]);
    }
    if (np == 2) {
        const int a0 = loc[0], a1 = loc[1];
        const double dx = x[a1] - x[a0], dy = y[a1] - y[a0];
        const double L2 = dx * dx + dy * dy;
        const double du = u[a1] - u[a0], dv = v[a1] - v[a0];
        const double st = (dx * du + dy * dv) / L2;
        const double stress = p.E * st;
        const double coef = Ap * stress / L2;
        f[2 * a1] = coef * dx;
        f[2 * a1 + 1] = coef * dy;
        f[2 * a0] = -(coef * dx);
        f[2 * a0 + 1] = -(coef * dy);
        return 0.5 * Ap * stress * st;
    }
    f[2 * loc[0]] = 0.0;
    f[2 * loc[0] + 1] = 0.0;
    return 0.0;
}

// Element forces (Eq. QUAD_fint_discretization for intact elements, the
// pieces for split ones) and the split pieces' strain energy.
__global__ __launch_bounds__(kB) void k_eval_elements(StepParams p, const double *ux, const double *uy,
                                                      EvalDev d) {
    const int64_t ne = (int64_t)p.nx * p.ny;
    const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (e >= ne) return;
    int64_t nd[4];
    elem_nodes(p, e, nd);
    double x[4], y[4], u[4], v[4];
    for (int n = 0; n < 4; ++n) {
        x[n] = p.X[nd[n]];
        y[n] = p.Y[nd[n]];
        u[n] = ux[nd[n]];
        v[n] = uy[nd[n]];
    }
    double f[8];
    const uint8_t code = p.split[e];
    if (code == 0 && p.subcell) {
        const int64_t i = e % p.nx, j = e / p.nx;
        const int64_t sid[4] = {edge_h(i, j, p.nx, p.ny), edge_v(i + 1, j, p.nx), edge_h(i, j + 1, p.nx, p.ny),
                                edge_v(i, j, p.nx)};
        double bb[4][3], cb[4][3], at[4], sg[4][3];
        at[0] = subcell<0>(x, y, nullptr, nullptr, bb[0], cb[0], nullptr);
        at[1] = subcell<1>(x, y, nullptr, nullptr, bb[1], cb[1], nullptr);
        at[2] = subcell<2>(x, y, nullptr, nullptr, bb[2], cb[2], nullptr);
        at[3] = subcell<3>(x, y, nullptr, nullptr, bb[3], cb[3], nullptr);
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) sg[k][c] = d.sig[3 * sid[k] + c];
        subcell_force(bb, cb, at, sg, f);
        d.pe[e] = 0.0;
    } else if (code == 0) {
        const int64_t i = e % p.nx, j = e / p.nx;
        const int64_t sid[4] = {edge_h(i, j, p.nx, p.ny), edge_v(i + 1, j, p.nx), edge_h(i, j + 1, p.nx, p.ny),
                                edge_v(i, j, p.nx)};
        double sx[4], sy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double gx[4], gy[4];
            q4_grad(x, y, k, gx, gy);
            const double *sg = d.sig + 3 * sid[k];
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const double tx = fma(gy[n], sg[2], gx[n] * sg[0]);
                const double ty = fma(gx[n], sg[2], gy[n] * sg[1]);
                if (k == 0) {
                    sx[n] = tx;
                    sy[n] = ty;
                } else {
                    sx[n] = sx[n] + tx;
                    sy[n] = sy[n] + ty;
                }
            }
        }
        const double c = 0.25 * p.area[e];
        for (int n = 0; n < 4; ++n) {
            f[2 * n] = c * sx[n];
            f[2 * n + 1] = c * sy[n];
        }
        d.pe[e] = 0.0;
    } else {
        const int a = (code >> 2) & 3, b = code & 3;
        double w = piece(p, x, y, u, v, a, b, f);
        w += piece(p, x, y, u, v, b, a, f);
        d.pe[e] = w;
    }
    for (int c = 0; c < 8; ++c) d.fe[8 * e + c] = f[c];
}

__device__ __forceinline__ int perimeter(int i, int j, int nx, int ny) {
    if (j == 0) return i;
    if (j == ny) return (nx + 1) + i;
    if (i == 0) return 2 * (nx + 1) + (j - 1);
    if (i == nx) return 2 * (nx + 1) + (ny - 1) + (j - 1);
    return -1;
}

// Nodal internal force (sum over the node's elements in colour order,
// colour (i mod 2) + 2 (j mod 2)), acceleration (phi f_ext - f_int) / m with
// prescribed components zero, and per node: kinetic energy at t_k
// (v^k = v^{k-1/2} + dt/2 a^k for free components after the first step)
// and external work f_ext . u.
__global__ __launch_bounds__(kB) void k_eval_nodes(StepParams p, const double *ux, const double *uy,
                                                   const double *vx, const double *vy, int64_t step, double phi,
                                                   EvalDev d) {
    const int64_t nn = (int64_t)(p.nx + 1) * (p.ny + 1);
    const int64_t g = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (g >= nn) return;
    const int i = (int)(g % (p.nx + 1)), j = (int)(g / (p.nx + 1));
    double fx = 0.0, fy = 0.0;
    for (int c = 0; c < 4; ++c) {
        const int ei = (((i - 1) & 1) == (c & 1)) ? i - 1 : i;
        const int ej = (((j - 1) & 1) == (c >> 1)) ? j - 1 : j;
        if (ei < 0 || ei >= p.nx || ej < 0 || ej >= p.ny) continue;
        const int dx = i - ei, dy = j - ej;
        const int n = dy == 0 ? (dx == 0 ? 0 : 1) : (dx == 1 ? 2 : 3);
        const int64_t e = (int64_t)ej * p.nx + ei;
        fx = fx + d.fe[8 * e + 2 * n];
        fy = fy + d.fe[8 * e + 2 * n + 1];
    }
    double fex = 0.0, fey = 0.0;
    unsigned mask = 0;
    const int pidx = perimeter(i, j, p.nx, p.ny);
    if (pidx >= 0) {
        fex = p.fext_p[2 * pidx];
        fey = p.fext_p[2 * pidx + 1];
        mask = p.vmask_p[pidx];
    }
    const double minv = p.minv[g];
    const double ax = (phi * fex - fx) * minv, ay = (phi * fey - fy) * minv;
    d.fint[g] = fx;
    d.fint[nn + g] = fy;
    d.acc[g] = (mask & 1u) ? 0.0 : ax;
    d.acc[nn + g] = (mask & 2u) ? 0.0 : ay;
    double wx = vx ? vx[g] : 0.0, wy = vy ? vy[g] : 0.0;
    if (step > 0) {
        if (!(mask & 1u)) wx = wx + 0.5 * p.dt * ax;
        if (!(mask & 2u)) wy = wy + 0.5 * p.dt * ay;
    }
    d.node_e[2 * g] = 0.5 * (wx * wx + wy * wy) / minv;
    d.node_e[2 * g + 1] = phi * fex * ux[g] + phi * fey * uy[g];
}

// Maximum principal stress of the mean of an intact element's four edge
// stresses; NaN for split elements.
__global__ __launch_bounds__(kB) void k_principal(StepParams p, EvalDev d, double *out) {
    const int64_t ne = (int64_t)p.nx * p.ny;
    const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (e >= ne) return;
    if (p.split[e] != 0) {
        out[e] = __builtin_nan("");
        return;
    }
    const int64_t i = e % p.nx, j = e / p.nx;
    const int64_t sid[4] = {edge_h(i, j, p.nx, p.ny), edge_v(i + 1, j, p.nx), edge_h(i, j + 1, p.nx, p.ny),
                            edge_v(i, j, p.nx)};
    double m[3];
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s = s + d.sig[3 * sid[k] + c];
        m[c] = s / 4.0;
    }
    const double cc = 0.5 * (m[0] + m[1]), hd = 0.5 * (m[0] - m[1]);
    out[e] = cc + sqrt(hd * hd + m[2] * m[2]);
}

// Deterministic sums: per-workgroup partials (tree in LDS), then one
// workgroup adds the partials in order.  Sums x[off + stride * t], t < n.
constexpr int kSumBlocks = 512;

__global__ __launch_bounds__(kB) void k_partial_sum(const double *x, int64_t n, int stride, int off, double *part) {
    __shared__ double s_v[kB];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB)
        acc += x[off + stride * t];
    s_v[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_v[threadIdx.x] += s_v[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s_v[0];
}

// One wave: lane l sums partials l*c .. l*c+c-1 in order (c = nparts / 64,
// nparts a multiple of 64), lane 0 then sums the 64 lane sums in order.
__global__ __launch_bounds__(64) void k_final_sum(const double *part, int nparts, double *out) {
    __shared__ double s_l[64];
    const int c = nparts / 64;
    double s = 0.0;
    for (int b = 0; b < c; ++b) s += part[threadIdx.x * c + b];
    s_l[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int l = 0; l < 64; ++l) t += s_l[l];
        *out = t;
    }
}
static_assert(kSumBlocks % 64 == 0, "final sum splits the partials over one wave");

// Power iteration on M^-1/2 K M^-1/2 over the free components: u = y m^-1/2
// (prescribed components zero), and after f = K u (k_eval_*): z = f m^-1/2.
__global__ __launch_bounds__(kB) void k_scale_in(StepParams p, const double *y, double *u) {
    const int64_t nn = (int64_t)(p.nx + 1) * (p.ny + 1);
    const int64_t g = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (g >= nn) return;
    const int i = (int)(g % (p.nx + 1)), j = (int)(g / (p.nx + 1));
    const int pidx = perimeter(i, j, p.nx, p.ny);
    const unsigned mask = pidx >= 0 ? p.vmask_p[pidx] : 0u;
    const double r = sqrt(p.minv[g]);
    u[g] = (mask & 1u) ? 0.0 : y[g] * r;
    u[nn + g] = (mask & 2u) ? 0.0 : y[nn + g] * r;
}

__global__ __launch_bounds__(kB) void k_scale_out(StepParams p, EvalDev d, const double *y, double *z,
                                                  double *yz_zz) {
    const int64_t nn = (int64_t)(p.nx + 1) * (p.ny + 1);
    const int64_t g = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (g >= nn) return;
    const int i = (int)(g % (p.nx + 1)), j = (int)(g / (p.nx + 1));
    const int pidx = perimeter(i, j, p.nx, p.ny);
    const unsigned mask = pidx >= 0 ? p.vmask_p[pidx] : 0u;
    const double r = sqrt(p.minv[g]);
    const double zx = (mask & 1u) ? 0.0 : d.fint[g] * r;
    const double zy = (mask & 2u) ? 0.0 : d.fint[nn + g] * r;
    z[g] = zx;
    z[nn + g] = zy;
    yz_zz[2 * g] = y[g] * zx + y[nn + g] * zy;
    yz_zz[2 * g + 1] = zx * zx + zy * zy;
}

__global__ __launch_bounds__(kB) void k_normalize(int64_t n, const double *z, const double *zz, double *y) {
    const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (t >= n) return;
    const double s = sqrt(*zz);
    y[t] = s > 0.0 ? z[t] / s : 0.0;
}

__global__ __launch_bounds__(kB) void k_check_finite(const double *a, const double *b, const double *c,
                                                     const double *d4, int64_t n, int32_t *flag) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB) {
        const double s = a[t] + b[t] + c[t] + d4[t];
        if (!isfinite(s)) *flag = 1;  // any writer, same value
    }
}

int nb_of(int64_t n) { return (int)std::max<int64_t>(1, (n + kB - 1) / kB); }

// Up to six arrays of n values converted between binary32 and binary64.
struct Arrays6 {
    const void *src[6];
    void *dst[6];
};

template <class S, class D>
__global__ __launch_bounds__(kB) void k_convert(Arrays6 a, int count, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB)
        for (int q = 0; q < count; ++q)
            static_cast<D *>(a.dst[q])[t] = (D) static_cast<const S *>(a.src[q])[t];
}

hipError_t sum_into(const double *x, int64_t n, int stride, int off, double *part, double *out, hipStream_t st) {
    k_partial_sum<<<kSumBlocks, kB, 0, st>>>(x, n, stride, off, part);
    k_final_sum<<<1, 64, 0, st>>>(part, kSumBlocks, out);
    return hipGetLastError();
}

}  // namespace

int eval_partials() { return kSumBlocks; }
int sum_partials() { return kSumBlocks; }

hipError_t launch_sum(const double *x, int64_t n, int stride, int off, double *part, double *out, hipStream_t st) {
    (void)hipGetLastError();
    return sum_into(x, n, stride, off, part, out, st);
}

hipError_t launch_eval(const StepParams &p, const double *ux, const double *uy, const double *vx,
                       const double *vy, int64_t step, double phi, const EvalDev &d, hipStream_t st) {
    (void)hipGetLastError();
    const int64_t nn = (int64_t)(p.nx + 1) * (p.ny + 1), ne = (int64_t)p.nx * p.ny;
    const int64_t ns = 2 * ne + p.nx + p.ny;
    k_eval_edges<<<nb_of(ns), kB, 0, st>>>(p, ux, uy, d);
    k_eval_elements<<<nb_of(ne), kB, 0, st>>>(p, ux, uy, d);
    k_eval_nodes<<<nb_of(nn), kB, 0, st>>>(p, ux, uy, vx, vy, step, phi, d);
    return hipGetLastError();
}

hipError_t launch_energies(const StepParams &p, const EvalDev &d, double *out3, hipStream_t st) {
    (void)hipGetLastError();
    const int64_t nn = (int64_t)(p.nx + 1) * (p.ny + 1), ne = (int64_t)p.nx * p.ny;
    const int64_t ns = 2 * ne + p.nx + p.ny;
    hipError_t e = sum_into(d.node_e, nn, 2, 0, d.part, out3, st);               // kinetic
    if (e == hipSuccess) e = sum_into(d.es, ns, 1, 0, d.part, out3 + 3, st);     // edges
    if (e == hipSuccess) e = sum_into(d.pe, ne, 1, 0, d.part, out3 + 4, st);     // split pieces
    if (e == hipSuccess) e = sum_into(d.node_e, nn, 2, 1, d.part, out3 + 2, st); // external work
    return e;
}

hipError_t launch_principal(const StepParams &p, const EvalDev &d, double *out, hipStream_t st) {
    (void)hipGetLastError();
    k_principal<<<nb_of((int64_t)p.nx * p.ny), kB, 0, st>>>(p, d, out);
    return hipGetLastError();
}

hipError_t launch_power_step(const StepParams &p, const EvalDev &d, double *y, double *u, double *z,
                             double *scratch2, double *sums, hipStream_t st) {
    (void)hipGetLastError();
    const int64_t nn = (int64_t)(p.nx + 1) * (p.ny + 1);
    k_scale_in<<<nb_of(nn), kB, 0, st>>>(p, y, u);
    hipError_t e = launch_eval(p, u, u + nn, nullptr, nullptr, 0, 1.0, d, st);
    if (e != hipSuccess) return e;
    k_scale_out<<<nb_of(nn), kB, 0, st>>>(p, d, y, z, scratch2);
    e = sum_into(scratch2, nn, 2, 0, d.part, sums, st);      // y . z
    if (e == hipSuccess) e = sum_into(scratch2, nn, 2, 1, d.part, sums + 1, st);  // z . z
    if (e != hipSuccess) return e;
    k_normalize<<<nb_of(2 * nn), kB, 0, st>>>(2 * nn, z, sums + 1, y);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double *a, const double *b, const double *c, const double *d4, int64_t n,
                               int32_t *flag, hipStream_t st) {
    (void)hipGetLastError();
    const int nb = (int)std::min<int64_t>(nb_of(n), 2048);
    k_check_finite<<<nb, kB, 0, st>>>(a, b, c, d4, n, flag);
    return hipGetLastError();
}

hipError_t launch_widen(const float *const src[6], double *const dst[6], int count, int64_t n, hipStream_t st) {
    (void)hipGetLastError();
    if (count < 1 || count > 6) return hipErrorInvalidValue;
    Arrays6 a{};
    for (int q = 0; q < count; ++q) {
        a.src[q] = src[q];
        a.dst[q] = dst[q];
    }
    const int nb = (int)std::min<int64_t>(nb_of(n), 2048);
    k_convert<float, double><<<nb, kB, 0, st>>>(a, count, n);
    return hipGetLastError();
}

hipError_t launch_narrow(const double *const src[6], float *const dst[6], int count, int64_t n, hipStream_t st) {
    (void)hipGetLastError();
    if (count < 1 || count > 6) return hipErrorInvalidValue;
    Arrays6 a{};
    for (int q = 0; q < count; ++q) {
        a.src[q] = src[q];
        a.dst[q] = dst[q];
    }
    const int nb = (int)std::min<int64_t>(nb_of(n), 2048);
    k_convert<double, float><<<nb, kB, 0, st>>>(a, count, n);
    return hipGetLastError();
}

}  // namespace mct
