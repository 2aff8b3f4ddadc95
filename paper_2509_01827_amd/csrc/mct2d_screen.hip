// HIP kernels (gfx950) of the learned split-screen.
//
// The screen is an extension of the method (not in the paper): every
// `period` steps all free-surface candidates of the element-split
// criterion (Sec. 2.2) are evaluated exactly; at that step a small MLP
// (10 -> 64 -> 64 -> 1, GELU, bfloat16 MFMA with FP32 accumulation) scores
// every candidate from 10 features, and during the following steps the step
// kernel evaluates G only for candidates scored above a threshold or created
// since.  The pick of every step stays the MCT pick over the evaluated set.
//
//   k_front        crack-path ends (midpoints)
//   k_features     per element: screen state reset, candidate rows with
//                  their 10 features
//   k_mlp_fwd      logits, 32 rows per wavefront, and the screen state of
//                  each row's candidate
//   k_mlp_train, k_grad_reduce, k_adam    training (gradient + Adam)
#include <algorithm>

#include "mct2d_device.h"
#include "mct2d_impl.h"

namespace mct {

namespace {
using namespace dev;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlk = 256;

// ------------------------------------------------------------ candidates

// Free-surface candidates of element e: bit k set when e is intact and its
// neighbour across local edge k is split or outside the mesh.
__device__ __forceinline__ unsigned cand_mask(const StepParams &p, int64_t e) {
    if (p.split[e] != 0) return 0;
    const int i = (int)(e % p.nx), j = (int)(e / p.nx);
    unsigned m = 0;
    if (j == 0 || p.split[e - p.nx] != 0) m |= 1u;
    if (i == p.nx - 1 || p.split[e + 1] != 0) m |= 2u;
    if (j == p.ny - 1 || p.split[e + p.nx] != 0) m |= 4u;
    if (i == 0 || p.split[e - 1] != 0) m |= 8u;
    return m;
}

// ---------------------------------------------------------------- features

struct ElemData {
    double x[4], y[4], ux[4], uy[4];
};

__device__ __forceinline__ void load_elem(const StepParams &p, const double *ux, const double *uy, int64_t e,
                                          ElemData &d) {
    const int64_t i = e % p.nx, j = e / p.nx;
    const int64_t n0 = j * (p.nx + 1) + i;
    const int64_t nd[4] = {n0, n0 + 1, n0 + p.nx + 2, n0 + p.nx + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        d.x[q] = p.X[nd[q]];
        d.y[q] = p.Y[nd[q]];
        d.ux[q] = ux[nd[q]];
        d.uy[q] = uy[nd[q]];
    }
}

// neighbour of element e across local edge k, -1 outside the mesh
__device__ __forceinline__ int64_t neighbour(const StepParams &p, int64_t e, int k) {
    const int i = (int)(e % p.nx), j = (int)(e / p.nx);
    if (k == 0) return j > 0 ? e - p.nx : -1;
    if (k == 1) return i < p.nx - 1 ? e + 1 : -1;
    if (k == 2) return j < p.ny - 1 ? e + p.nx : -1;
    return i > 0 ? e - 1 : -1;
}

// Smoothed stress of local edge k of intact element e: the edge strain
// eps = w_hi (B u)_hi + w_lo (B u)_lo over the intact neighbours of the edge
// (lower element id first, w_j = A_j / (A_lo + A_hi)), then plane stress.
__device__ __forceinline__ void edge_stress(const StepParams &p, int64_t e, const ElemData &d, int k, int64_t nb,
                                            bool nb_intact, const ElemData &dn, double sg[3]) {
    double gx[4], gy[4], qf[3], eps[3];
    q4_grad(d.x, d.y, k, gx, gy);
    strain<4>(gx, gy, d.ux, d.uy, qf);
    if (nb_intact) {
        double qn[3];
        q4_grad(dn.x, dn.y, (k + 2) & 3, gx, gy);
        strain<4>(gx, gy, dn.ux, dn.uy, qn);
        const double Af = p.area[e], An = p.area[nb];
        if (k == 1 || k == 2) {  // e has the lower id
            const double w0 = Af / (Af + An), w1 = An / (Af + An);
#pragma unroll
            for (int c = 0; c < 3; ++c) eps[c] = fma(w1, qn[c], w0 * qf[c]);
        } else {
            const double w0 = An / (An + Af), w1 = Af / (An + Af);
#pragma unroll
            for (int c = 0; c < 3; ++c) eps[c] = fma(w1, qf[c], w0 * qn[c]);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) eps[c] = qf[c];
    }
    hooke(p, eps, sg);
}

constexpr double kTipCap = 64.0;

// Crack-path ends: entry or exit edge of a split element whose neighbour
// across it is intact; appended in any order (only the nearest matters).
__global__ __launch_bounds__(kBlk) void k_front(StepParams p, ScreenDev s) {
    const int64_t ne = (int64_t)p.nx * p.ny;
    for (int64_t e = (int64_t)blockIdx.x * kBlk + threadIdx.x; e < ne; e += (int64_t)gridDim.x * kBlk) {
        const uint8_t c = p.split[e];
        if (c == 0) continue;
        const int ks[2] = {(c >> 2) & 3, c & 3};
        for (int q = 0; q < 2; ++q) {
            const int k = ks[q];
            const int64_t nb = neighbour(p, e, k);
            if (nb < 0 || p.split[nb] != 0) continue;
            const int64_t i = e % p.nx, j = e / p.nx;
            const int64_t n0 = j * (p.nx + 1) + i;
            const int64_t nd[4] = {n0, n0 + 1, n0 + p.nx + 2, n0 + p.nx + 1};
            const int64_t a0 = nd[k], a1 = nd[(k + 1) & 3];
            const int idx = atomicAdd(s.nfront, 1);
            s.front_xy[2 * idx] = 0.5 * (p.X[a0] + p.X[a1]);
            s.front_xy[2 * idx + 1] = 0.5 * (p.Y[a0] + p.Y[a1]);
        }
    }
}

// One thread per element: clears the element's screen state and, for an
// element with candidates, appends one row per candidate (e, a) with its
// ten features (principal stresses and energy density of the element's mean
// edge stress, G / Gc now and at the previous sweep, distance to the nearest
// crack-path end, neighbour flags; definitions in the C header).
__global__ __launch_bounds__(kBlk) void k_features(StepParams p, ScreenDev s, const double *ux,
                                                   const double *uy) {
    const int64_t ne = (int64_t)p.nx * p.ny;
    const int sweep = *s.sweep;
    const double nu = p.D12 / p.D11;
    for (int64_t e = (int64_t)blockIdx.x * kBlk + threadIdx.x; e < ne; e += (int64_t)gridDim.x * kBlk) {
        const uint32_t w_old = s.screen[e];
        if (w_old) s.screen[e] = 0u;
        const unsigned mask = cand_mask(p, e);
        if (!mask) continue;
        // the element and its four neighbours, all loads issued together
        ElemData d, dn[4];
        int64_t nbs[4];
        bool nbi[4];
        load_elem(p, ux, uy, e, d);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            nbs[k] = neighbour(p, e, k);
            nbi[k] = nbs[k] >= 0 && p.split[nbs[k]] == 0;
            load_elem(p, ux, uy, nbi[k] ? nbs[k] : e, dn[k]);
        }
        double sig[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) edge_stress(p, e, d, k, nbs[k], nbi[k], dn[k], sig[k]);
        double sm[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) sm[q] = ((((0.0 + sig[0][q]) + sig[1][q]) + sig[2][q]) + sig[3][q]) / 4.0;
        const double cc = 0.5 * (sm[0] + sm[1]);
        const double hd = 0.5 * (sm[0] - sm[1]);
        const double rr = sqrt(hd * hd + sm[2] * sm[2]);
        const double exx = (sm[0] - nu * sm[1]) / p.E;
        const double eyy = (sm[1] - nu * sm[0]) / p.E;
        const double gxy = 2.0 * (1.0 + nu) * sm[2] / p.E;
        const double Wd = 0.5 * (sm[0] * exx + sm[1] * eyy + sm[2] * gxy);
        const double gc = p.gc ? p.gc[e] : p.gc_uniform;
        const double h = sqrt(p.area[e]);
        const double sref = sqrt(p.E * gc / h);
        float fl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) fl[k] = nbi[k] ? 0.0f : 1.0f;
        int row = atomicAdd(s.nrows, __popc(mask));
        for (int a = 0; a < 4; ++a) {
            if (!((mask >> a) & 1u)) continue;
            // G of the three paths (zero when edge a is not stretched)
            const int a1 = (a + 1) & 3;
            const double dux = d.ux[a1] - d.ux[a], duy = d.uy[a1] - d.uy[a];
            const double x1 = d.x[a] + d.ux[a], y1 = d.y[a] + d.uy[a];
            const double x2 = d.x[a1] + d.ux[a1], y2 = d.y[a1] + d.uy[a1];
            const double lx = x2 - x1, ly = y2 - y1;
            const double Lx = d.x[a1] - d.x[a], Ly = d.y[a1] - d.y[a];
            const bool H = (lx * lx + ly * ly) > (Lx * Lx + Ly * Ly);
            double gmax = 0.0;
            if (H) {
                for (int j = 0; j < 3; ++j) {
                    const int k = (a + 1 + j) & 3;
                    double cx, cy, len;
                    path_geom(d.x, d.y, a, k, cx, cy, len);
                    const double spx = fma(sig[k][2], cy, sig[k][0] * cx);
                    const double spy = fma(sig[k][1], cy, sig[k][2] * cx);
                    const double G = 0.5 * fma(duy, spy, dux * spx);
                    if (j == 0 || G > gmax) gmax = G;
                }
            }
            const double g_now = gmax / gc;
            const int64_t hk = e * 4 + a;
            const double g_prev = (s.hist_t[hk] == sweep - 1) ? s.hist_g[hk] : 0.0;
            s.hist_g[hk] = g_now;
            s.hist_t[hk] = sweep;
            // feature 5 is filled in by k_front_distance from these
            s.row_geo[3 * (int64_t)row] = 0.5 * (d.x[a] + d.x[a1]);
            s.row_geo[3 * (int64_t)row + 1] = 0.5 * (d.y[a] + d.y[a1]);
            s.row_geo[3 * (int64_t)row + 2] = h;
            s.cand[row] = (int32_t)hk;
            float *f = s.feat + (int64_t)row * kFeat;
            f[0] = (float)((cc + rr) / sref);
            f[1] = (float)((cc - rr) / sref);
            f[2] = (float)(Wd * h / gc);
            f[3] = (float)g_now;
            f[4] = (float)g_prev;
            f[5] = 1.0f;
            f[6] = fl[0];
            f[7] = fl[1];
            f[8] = fl[2];
            f[9] = fl[3];
            ++row;
            // a candidate the previous screen skipped although G > Gc now
            if (((w_old >> (8 * a)) & 0xFFu) == kScreenSkip && g_now > 1.0)
                atomicAdd(&s.stats[kStatMisses], 1ull);
        }
    }
}

// Feature 5 of every row: distance from the row's edge midpoint to the
// nearest crack-path end, over h, capped.  The ends are staged through LDS
// in chunks shared by the workgroup's rows.
constexpr int kFrontChunk = 512;

__global__ __launch_bounds__(kBlk) void k_front_distance(ScreenDev s) {
    __shared__ double s_xy[2 * kFrontChunk];
    const int n = *s.nrows, nfront = *s.nfront;
    if (nfront == 0) return;  // feature stays 1 (uniform over the grid)
    for (int r0 = blockIdx.x * kBlk; r0 < n; r0 += gridDim.x * kBlk) {
        const int r = r0 + threadIdx.x;
        double mx = 0.0, my = 0.0;
        if (r < n) {
            mx = s.row_geo[3 * (int64_t)r];
            my = s.row_geo[3 * (int64_t)r + 1];
        }
        double d2 = __builtin_inf();
        for (int c0 = 0; c0 < nfront; c0 += kFrontChunk) {
            const int cn = min(kFrontChunk, nfront - c0);
            __syncthreads();
            for (int i = threadIdx.x; i < 2 * cn; i += kBlk) s_xy[i] = s.front_xy[2 * (int64_t)c0 + i];
            __syncthreads();
            for (int t = 0; t < cn; ++t) {
                const double dx = s_xy[2 * t] - mx, dy = s_xy[2 * t + 1] - my;
                const double q = dx * dx + dy * dy;
                d2 = (q < d2) ? q : d2;
            }
        }
        if (r < n) {
            const double h = s.row_geo[3 * (int64_t)r + 2];
            s.feat[(int64_t)r * kFeat + 5] = (float)(fmin(sqrt(d2) / h, kTipCap) / kTipCap);
        }
    }
}

// Close an evaluation: count it, keep its row count, reset the counters.
__global__ void k_sweep_advance(ScreenDev s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int n = *s.nrows;
        *s.sweep = *s.sweep + 1;
        s.stats[kStatSweeps] += 1ull;
        s.stats[kStatCands] += (unsigned long long)n;
        *s.nrows_last = n;
        *s.nrows = 0;
        *s.nfront = 0;
    }
}

__global__ __launch_bounds__(kBlk) void k_fill_u32(uint32_t *a, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlk) a[i] = v;
}

// --------------------------------------------------------------------- MLP
//
// One wavefront takes 32 rows at a time as two 16-row halves.  MFMA
// v_mfma_f32_16x16x32_bf16 operand layout (lane l, i = 0..7 / 0..3):
//   A[16][32]: row l & 15, k = 8 (l >> 4) + i
//   B[32][16]: column l & 15, k = 8 (l >> 4) + i
//   D[16][16]: column l & 15, row 4 (l >> 4) + i
// Rounding points (as in the reference): inputs, weights, hidden
// activations and backpropagated pre-activation gradients are bfloat16;
// accumulation, biases, GELU and the loss are FP32.

constexpr int kRows = 32;
constexpr int kIn = 32;  // padded input width

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
    const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float phi = expf(-0.5f * z * z) * 0.39894228040143268f;
    return Phi + z * phi;
}
__device__ __forceinline__ __bf16 to_bf(float v) { return (__bf16)v; }
__device__ __forceinline__ float from_bf(__bf16 v) { return (float)v; }

struct MlpShared {
    alignas(16) __bf16 w1[kIn * kHidden];      // [k][n]
    alignas(16) __bf16 w2[kHidden * kHidden];  // [m][n]
    __bf16 w3[kHidden];
    float b1[kHidden], b2[kHidden];
    float b3;
    __bf16 x[kRows * kIn];         // [row][k]
    __bf16 h1[kRows * kHidden];    // [row][m]
    __bf16 dz[kRows * kHidden];    // dZ2, then dZ1 [row][n]
};

__device__ void load_weights(const MlpDev &m, MlpShared &sh) {
    // 16-byte copies (8 bfloat16 each); the arrays are 256-byte aligned
    const uint4 *w1 = reinterpret_cast<const uint4 *>(m.w1b);
    const uint4 *w2 = reinterpret_cast<const uint4 *>(m.w2b);
    uint4 *s1 = reinterpret_cast<uint4 *>(sh.w1);
    uint4 *s2 = reinterpret_cast<uint4 *>(sh.w2);
    for (int i = threadIdx.x; i < kIn * kHidden / 8; i += blockDim.x) s1[i] = w1[i];
    for (int i = threadIdx.x; i < kHidden * kHidden / 8; i += blockDim.x) s2[i] = w2[i];
    const __bf16 *w3 = reinterpret_cast<const __bf16 *>(m.w3b);
    for (int i = threadIdx.x; i < kHidden; i += blockDim.x) {
        sh.w3[i] = w3[i];
        sh.b1[i] = m.master[kOffB1 + i];
        sh.b2[i] = m.master[kOffB2 + i];
    }
    if (threadIdx.x == 0) sh.b3 = m.master[kOffB3];
}

__device__ void load_rows(const float *X, int64_t r0, int64_t n, MlpShared &sh) {
    for (int i = threadIdx.x; i < kRows * kIn; i += blockDim.x) {
        const int r = i / kIn, k = i % kIn;
        float v = 0.0f;
        if (k < kFeat && r0 + r < n) v = X[(r0 + r) * kFeat + k];
        sh.x[i] = to_bf(v);
    }
}

// Forward pass of one 32-row tile.  Leaves h1 in LDS and returns in
// registers z1, z2 (D layout) and the logit of this lane's rows (all 16
// lanes of a row group hold the sum).
struct Fwd {
    float z1[2][4][4], z2[2][4][4], h2[2][4][4];
    float z3[2][4];
};

__device__ void forward_tile(MlpShared &sh, Fwd &f) {
    const int l = threadIdx.x & 63, r16 = l & 15, kq = 8 * (l >> 4), rq = 4 * (l >> 4);
    // layer 1
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        bf16x8 a;
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = sh.x[(16 * h + r16) * kIn + kq + i];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            bf16x8 b;
#pragma unroll
            for (int i = 0; i < 8; ++i) b[i] = sh.w1[(kq + i) * kHidden + 16 * t + r16];
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[i] + sh.b1[16 * t + r16];
                f.z1[h][t][i] = z;
                sh.h1[(16 * h + rq + i) * kHidden + 16 * t + r16] = to_bf(gelu_f(z));
            }
        }
    }
    __syncthreads();
    // layer 2 and the output layer
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                bf16x8 a, b;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    a[i] = sh.h1[(16 * h + r16) * kHidden + 32 * kc + kq + i];
                    b[i] = sh.w2[(32 * kc + kq + i) * kHidden + 16 * t + r16];
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[i] + sh.b2[16 * t + r16];
                f.z2[h][t][i] = z;
                const float hv = from_bf(to_bf(gelu_f(z)));
                f.h2[h][t][i] = hv;
                part[i] += hv * from_bf(sh.w3[16 * t + r16]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = part[i];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
            f.z3[h][i] = v + sh.b3;
        }
    }
}

__global__ __launch_bounds__(64) void k_mlp_fwd(MlpDev m, const float *X, const int32_t *n_dev, int64_t n_host,
                                                float *logits, const int32_t *cand, uint32_t *screen, float tau,
                                                unsigned long long *stats) {
    __shared__ MlpShared sh;
    const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
    load_weights(m, sh);
    const int l = threadIdx.x, r16 = l & 15, rq = 4 * (l >> 4);
    uint8_t *bytes = reinterpret_cast<uint8_t *>(screen);
    for (int64_t r0 = (int64_t)blockIdx.x * kRows; r0 < n; r0 += (int64_t)gridDim.x * kRows) {
        __syncthreads();  // weights loaded / previous tile consumed
        load_rows(X, r0, n, sh);
        __syncthreads();
        Fwd f;
        forward_tile(sh, f);
        int flagged = 0;
        if (r16 == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t r = r0 + 16 * h + rq + i;
                    if (r >= n) continue;
                    const float z = f.z3[h][i];
                    logits[r] = z;
                    if (screen) {
                        const bool flag = z > tau;
                        bytes[cand[r]] = flag ? kScreenFlagged : kScreenSkip;
                        flagged += flag;
                    }
                }
        }
        if (screen) {
#pragma unroll
            for (int off = 16; off < 64; off <<= 1) flagged += __shfl_xor(flagged, off, 64);
            if (l == 0 && flagged) atomicAdd(&stats[kStatFlagged], (unsigned long long)flagged);
        }
    }
}

// Gradient of the mean weighted logistic loss, one partial per workgroup:
// partials[b * (kParams + 1) + q], q = kParams is the loss.
__global__ __launch_bounds__(64) void k_mlp_train(MlpDev m, const float *X, const float *Y, int64_t n,
                                                  float pos_weight, float *partials) {
    __shared__ MlpShared sh;
    load_weights(m, sh);
    const int l = threadIdx.x, r16 = l & 15, kq = 8 * (l >> 4), rq = 4 * (l >> 4);
    const float inv_n = 1.0f / (float)n;
    f32x4 gW2[4][4], gW1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0};
    float gb3 = 0.0f, loss = 0.0f;
    for (int64_t r0 = (int64_t)blockIdx.x * kRows; r0 < n; r0 += (int64_t)gridDim.x * kRows) {
        __syncthreads();
        load_rows(X, r0, n, sh);
        __syncthreads();
        Fwd f;
        forward_tile(sh, f);
        // output layer and dZ2
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t r = r0 + 16 * h + rq + i;
                float dz3 = 0.0f;
                if (r < n) {
                    const float y = Y[r];
                    const float w = (y > 0.5f) ? pos_weight : 1.0f;
                    const float z = f.z3[h][i];
                    const float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));  // softplus
                    if (r16 == 0) loss += w * (sp - y * z) * inv_n;
                    dz3 = w * (1.0f / (1.0f + expf(-z)) - y) * inv_n;
                }
                if (r16 == 0) gb3 += dz3;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int col = 16 * t + r16;
                    gw3[t] += f.h2[h][t][i] * dz3;
                    const float dh2 = dz3 * from_bf(sh.w3[col]);
                    const __bf16 dz2 = to_bf(dh2 * gelu_d(f.z2[h][t][i]));
                    gb2[t] += from_bf(dz2);
                    sh.dz[(16 * h + rq + i) * kHidden + col] = dz2;
                }
            }
        __syncthreads();
        // gW2 += H1^T dZ2 (K = the 32 rows of the tile)
#pragma unroll
        for (int tm = 0; tm < 4; ++tm) {
            bf16x8 a;
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = sh.h1[(kq + i) * kHidden + 16 * tm + r16];
#pragma unroll
            for (int tn = 0; tn < 4; ++tn) {
                bf16x8 b;
#pragma unroll
                for (int i = 0; i < 8; ++i) b[i] = sh.dz[(kq + i) * kHidden + 16 * tn + r16];
                gW2[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, gW2[tm][tn], 0, 0, 0);
            }
        }
        // dH1 = dZ2 W2^T, then dZ1 (held until the dZ2 tile is no longer read)
        __bf16 dz1v[2][4][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int tm = 0; tm < 4; ++tm) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kc = 0; kc < 2; ++kc) {
                    bf16x8 a, b;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        a[i] = sh.dz[(16 * h + r16) * kHidden + 32 * kc + kq + i];
                        b[i] = sh.w2[(16 * tm + r16) * kHidden + 32 * kc + kq + i];
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const __bf16 v = to_bf(acc[i] * gelu_d(f.z1[h][tm][i]));
                    dz1v[h][tm][i] = v;
                    gb1[tm] += from_bf(v);
                }
            }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int i = 0; i < 4; ++i) sh.dz[(16 * h + rq + i) * kHidden + 16 * tm + r16] = dz1v[h][tm][i];
        __syncthreads();
        // gW1 += X^T dZ1 (input rows padded to 16)
        {
            bf16x8 a;
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = sh.x[(kq + i) * kIn + r16];
#pragma unroll
            for (int tn = 0; tn < 4; ++tn) {
                bf16x8 b;
#pragma unroll
                for (int i = 0; i < 8; ++i) b[i] = sh.dz[(kq + i) * kHidden + 16 * tn + r16];
                gW1[tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, gW1[tn], 0, 0, 0);
            }
        }
    }
    // column sums over the four row groups of the wavefront
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gb1[t] += __shfl_xor(gb1[t], 16, 64);
        gb1[t] += __shfl_xor(gb1[t], 32, 64);
        gb2[t] += __shfl_xor(gb2[t], 16, 64);
        gb2[t] += __shfl_xor(gb2[t], 32, 64);
        gw3[t] += __shfl_xor(gw3[t], 16, 64);
        gw3[t] += __shfl_xor(gw3[t], 32, 64);
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        gb3 += __shfl_xor(gb3, off, 64);
        loss += __shfl_xor(loss, off, 64);
    }
    float *out = partials + (int64_t)blockIdx.x * (kParams + 1);
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rq + i;
            if (row < kFeat) out[row * kHidden + 16 * tn + r16] = gW1[tn][i];
        }
#pragma unroll
    for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[kOffW2 + (16 * tm + rq + i) * kHidden + 16 * tn + r16] = gW2[tm][tn][i];
    if (l < 16) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            out[kOffB1 + 16 * t + l] = gb1[t];
            out[kOffB2 + 16 * t + l] = gb2[t];
            out[kOffW3 + 16 * t + l] = gw3[t];
        }
    }
    if (l == 0) {
        out[kOffB3] = gb3;
        out[kParams] = loss;
    }
}

// grad[q] = sum over workgroups in index order (deterministic)
__global__ __launch_bounds__(kBlk) void k_grad_reduce(const float *partials, int nblocks, float *grad) {
    const int q = blockIdx.x * kBlk + threadIdx.x;
    if (q > kParams) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * (kParams + 1) + q];
    grad[q] = s;
}

__device__ __forceinline__ void refresh_bf16(const MlpDev &m, int q) {
    __bf16 *w1 = reinterpret_cast<__bf16 *>(m.w1b);
    __bf16 *w2 = reinterpret_cast<__bf16 *>(m.w2b);
    __bf16 *w3 = reinterpret_cast<__bf16 *>(m.w3b);
    const float v = m.master[q];
    if (q < kOffB1) w1[q] = to_bf(v);  // [k][n], rows 0..9
    else if (q >= kOffW2 && q < kOffB2) w2[q - kOffW2] = to_bf(v);
    else if (q >= kOffW3 && q < kOffB3) w3[q - kOffW3] = to_bf(v);
}

__global__ __launch_bounds__(kBlk) void k_mlp_prep(MlpDev m) {
    const int q = blockIdx.x * kBlk + threadIdx.x;
    if (q < kParams) refresh_bf16(m, q);
    // zero padding rows 10..31 of W1
    __bf16 *w1 = reinterpret_cast<__bf16 *>(m.w1b);
    if (q < (kIn - kFeat) * kHidden) w1[kFeat * kHidden + q] = to_bf(0.0f);
}

__global__ __launch_bounds__(kBlk) void k_adam(MlpDev m, const float *grad, float lr, float c1, float c2) {
    const int q = blockIdx.x * kBlk + threadIdx.x;
    if (q >= kParams) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = grad[q];
    const float mm = b1 * m.m[q] + (1.0f - b1) * g;
    const float vv = b2 * m.v[q] + (1.0f - b2) * g * g;
    m.m[q] = mm;
    m.v[q] = vv;
    const float mh = mm / c1, vh = vv / c2;
    m.master[q] = m.master[q] - lr * mh / (sqrtf(vh) + eps);
    refresh_bf16(m, q);
}

}  // namespace

hipError_t launch_screen_evaluate(const StepParams &p, const ScreenDev &s, int par, hipStream_t st) {
    (void)hipGetLastError();
    const int64_t ne = (int64_t)p.nx * p.ny;
    const int nb = (int)std::min<int64_t>((ne + kBlk - 1) / kBlk, 2048);
    const double *ux = par ? p.ux1 : p.ux0;
    const double *uy = par ? p.uy1 : p.uy0;
    k_front<<<nb, kBlk, 0, st>>>(p, s);
    k_features<<<nb, kBlk, 0, st>>>(p, s, ux, uy);
    k_front_distance<<<64, kBlk, 0, st>>>(s);
    return hipGetLastError();
}

hipError_t launch_sweep_advance(const ScreenDev &s, hipStream_t st) {
    (void)hipGetLastError();
    k_sweep_advance<<<1, 64, 0, st>>>(s);
    return hipGetLastError();
}

// Snapshot of a screened window's starting state: u^k (buffer par), v, the
// split codes and the control block, saved to or restored from the screen's
// buffers by one grid-stride copy; saving also clears the trip flag.
__global__ __launch_bounds__(kBlk) void k_snapshot(StepParams p, ScreenDev s, int par, int save) {
    const int64_t nn = (int64_t)(p.nx + 1) * (p.ny + 1), ne = (int64_t)p.nx * p.ny;
    double *ux = par ? p.ux1 : p.ux0, *uy = par ? p.uy1 : p.uy0;
    double *live[4] = {ux, uy, p.vx, p.vy};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 4 * nn + ne + 1; i += stride) {
        if (i < 4 * nn) {
            const int q = (int)(i / nn);
            const int64_t n = i - q * nn;
            if (save)
                s.snap_u[i] = live[q][n];
            else
                live[q][n] = s.snap_u[i];
        } else if (i < 4 * nn + ne) {
            const int64_t e = i - 4 * nn;
            if (save)
                s.snap_split[e] = p.split[e];
            else
                p.split[e] = s.snap_split[e];
        } else {
            if (save) {
                *s.snap_ctl = *p.ctl;
                *s.trip = 0u;
            } else {
                *p.ctl = *s.snap_ctl;
            }
        }
    }
}

hipError_t launch_snapshot(const StepParams &p, const ScreenDev &s, int par, bool save, hipStream_t st) {
    (void)hipGetLastError();
    const int64_t n = 4 * (int64_t)(p.nx + 1) * (p.ny + 1) + (int64_t)p.nx * p.ny + 1;
    const int64_t nb = std::min<int64_t>((n + kBlk - 1) / kBlk, 8192);
    k_snapshot<<<(int)nb, kBlk, 0, st>>>(p, s, par, save ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *a, int64_t n, uint32_t v, hipStream_t st) {
    (void)hipGetLastError();
    const int64_t nb = std::min<int64_t>((n + kBlk - 1) / kBlk, 4096);
    if (nb > 0) k_fill_u32<<<(int)nb, kBlk, 0, st>>>(a, n, v);
    return hipGetLastError();
}

hipError_t launch_mlp_prep(const MlpDev &m, hipStream_t st) {
    (void)hipGetLastError();
    k_mlp_prep<<<(kParams + kBlk - 1) / kBlk, kBlk, 0, st>>>(m);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev &m, const float *x, const int32_t *n_dev, int64_t n, float *logits,
                              const int32_t *cand, uint32_t *screen, float tau, unsigned long long *stats,
                              hipStream_t st) {
    (void)hipGetLastError();
    int grid = 128;  // device-side row count: each workgroup strides over the tiles
    if (!n_dev) grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kRows - 1) / kRows, 1024));
    k_mlp_fwd<<<grid, 64, 0, st>>>(m, x, n_dev, n, logits, cand, screen, tau, stats);
    return hipGetLastError();
}

int mlp_train_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kRows - 1) / kRows, 512)); }

hipError_t launch_mlp_gradient(const MlpDev &m, const float *x, const float *y, int64_t n, float pos_weight,
                               float *partials, float *grad, hipStream_t st) {
    (void)hipGetLastError();
    const int nb = mlp_train_blocks(n);
    k_mlp_train<<<nb, 64, 0, st>>>(m, x, y, n, pos_weight, partials);
    k_grad_reduce<<<(kParams + 1 + kBlk - 1) / kBlk, kBlk, 0, st>>>(partials, nb, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpDev &m, const float *grad, float lr, int t, hipStream_t st) {
    (void)hipGetLastError();
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    k_adam<<<(kParams + kBlk - 1) / kBlk, kBlk, 0, st>>>(m, grad, lr, c1, c2);
    return hipGetLastError();
}

}  // namespace mct
