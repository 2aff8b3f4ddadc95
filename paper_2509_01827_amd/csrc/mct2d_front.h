// Per-front pick (a variant of the Sec. 3 pick), shared by the Q4 and the
// CST step: an accepted candidate splits iff, against every other accepted
// candidate it competes with -- the same element, or a tip point (midpoint
// of the tip edge, reference coordinates) closer than the radius rho -- it
// has the better key (larger G, then lower element id, then lower tip edge)
// and passes the split-ratio test G_c > gamma (G_c - G_c').  The picked
// candidates never compete with each other (distinct elements); all of them
// split in the same step and are logged in key order.  With rho = infinity
// this is the global pick.  Internal header, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mct2d_impl.h"

namespace mct {

// What the pick kernel reads and writes.  Scratch arrays hold one entry per
// candidate of the list's capacity.
struct FrontView {
    const AccCand *cand;
    uint32_t *count;     // accepted candidates of the step; reset to 0 by the pick
    double2 *mid;        // scratch: tip points
    double *len;         // scratch: crack-path lengths
    int32_t *order;      // scratch: candidate index by rank among the picked
    int32_t *bucket;     // scratch: hash bucket of each candidate
    int32_t *sorted;     // scratch: candidates grouped by bucket
    int32_t *plist;      // scratch: the picked candidates
    uint8_t *split;
    LogRec *log;
    int64_t log_cap;
    int64_t *nsplit;
    double *Ud;
    int32_t *overflow;
    const int64_t *base;  // steps before the running segment
    const double *gc;     // per element, or null for gc_uniform
    double gc_uniform, gamma, rho2;
    double cell;          // hash cell size >= max(rho, largest element diameter)
};

__device__ __forceinline__ bool acc_better(const AccCand &x, const AccCand &y) {
    if (x.G != y.G) return x.G > y.G;
    if (x.elem != y.elem) return x.elem < y.elem;
    return (x.ak >> 2) < (y.ak >> 2);
}

constexpr int kFrontBuckets = 4096;

__device__ __forceinline__ int front_bucket(long long cx, long long cy) {
    const unsigned long long h = (unsigned long long)cx * 0x9E3779B97F4A7C15ull ^
                                 (unsigned long long)cy * 0xC2B2AE3D27D4EB4Full;
    return (int)((h >> 40) & (kFrontBuckets - 1));
}

// The pick of step base + k_rel with one workgroup of NT threads.  Geom
// provides tip(elem, a) -> reference midpoint of local edge a and
// path_len(elem, a, k) -> length of the crack path between the midpoints
// of local edges a and k, computed like the step's own geometry.
//
// Competition is local: candidates are hashed by the cell of their tip
// point (cell >= rho and >= the largest element diameter, so every
// competitor of a candidate -- closer than rho, or in the same element --
// lies in one of the 3 x 3 cells around it); each candidate is decided
// against the candidates of those cells' buckets (others in a bucket are
// filtered by the same test).  The decision of a candidate depends only on
// the set of candidates, not on the order inside a bucket.  rho = infinity
// (everything competes) reduces to the global pick: the best key, if it
// passes the split-ratio test against the smallest G.
template <int NT, class Geom>
__device__ void front_pick_block(const FrontView &v, const Geom &geo, int k_rel) {
    __shared__ int s_cnt[kFrontBuckets];
    __shared__ int s_off[kFrontBuckets + 1];
    __shared__ int s_np;
    __shared__ int s_part[NT];
    __shared__ AccCand s_best[NT];
    __shared__ double s_min[NT];
    const uint32_t n = *v.count;  // uniform
    if (n == 0) return;
    const int tid = threadIdx.x;
    const bool global = !(v.rho2 < INFINITY);
    for (int b = tid; b < kFrontBuckets; b += NT) s_cnt[b] = 0;
    if (tid == 0) s_np = 0;
    __syncthreads();
    for (uint32_t c = tid; c < n; c += NT) {
        const AccCand x = v.cand[c];
        const double2 m = geo.tip(x.elem, x.ak >> 2);
        v.mid[c] = m;
        v.len[c] = geo.path_len(x.elem, x.ak >> 2, x.ak & 3);
        if (!global) {
            const int b = front_bucket((long long)floor(m.x / v.cell), (long long)floor(m.y / v.cell));
            v.bucket[c] = b;
            atomicAdd(&s_cnt[b], 1);
        }
    }
    __syncthreads();
    if (global) {
        // every candidate competes with every other one
        AccCand best;
        best.G = -1.0;
        best.elem = 0x7fffffff;
        best.ak = 0;
        double gmin = INFINITY;
        int bi = -1;
        for (uint32_t c = tid; c < n; c += NT) {
            const AccCand x = v.cand[c];
            if (bi < 0 || acc_better(x, best)) {
                best = x;
                bi = (int)c;
            }
            gmin = fmin(gmin, x.G);
        }
        s_best[tid] = best;
        s_part[tid] = bi;
        s_min[tid] = gmin;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (tid < w) {
                if (s_part[tid + w] >= 0 && (s_part[tid] < 0 || acc_better(s_best[tid + w], s_best[tid]))) {
                    s_best[tid] = s_best[tid + w];
                    s_part[tid] = s_part[tid + w];
                }
                s_min[tid] = fmin(s_min[tid], s_min[tid + w]);
            }
            __syncthreads();
        }
        if (tid == 0 && s_best[0].G > v.gamma * (s_best[0].G - s_min[0])) {
            v.plist[0] = s_part[0];
            s_np = 1;
        }
    } else {
        // exclusive scan of the bucket counts, then candidates grouped by bucket
        constexpr int PER = (kFrontBuckets + NT - 1) / NT;
        int loc = 0;
        for (int q = 0; q < PER; ++q) {
            const int b = tid * PER + q;
            if (b < kFrontBuckets) loc += s_cnt[b];
        }
        s_part[tid] = loc;
        __syncthreads();
        for (int w = 1; w < NT; w <<= 1) {
            const int t = tid >= w ? s_part[tid - w] : 0;
            __syncthreads();
            s_part[tid] += t;
            __syncthreads();
        }
        int run = s_part[tid] - loc;
        for (int q = 0; q < PER; ++q) {
            const int b = tid * PER + q;
            if (b < kFrontBuckets) {
                s_off[b] = run;
                run += s_cnt[b];
                s_cnt[b] = 0;
            }
        }
        if (tid == 0) s_off[kFrontBuckets] = (int)n;
        __syncthreads();
        for (uint32_t c = tid; c < n; c += NT) {
            const int b = v.bucket[c];
            v.sorted[s_off[b] + atomicAdd(&s_cnt[b], 1)] = (int32_t)c;
        }
        __syncthreads();
        for (uint32_t c = tid; c < n; c += NT) {
            const AccCand x = v.cand[c];
            const double2 pc = v.mid[c];
            const long long cx = (long long)floor(pc.x / v.cell), cy = (long long)floor(pc.y / v.cell);
            bool ok = true;
            for (int dy = -1; dy <= 1 && ok; ++dy)
                for (int dx = -1; dx <= 1 && ok; ++dx) {
                    const int b = front_bucket(cx + dx, cy + dy);
                    for (int t = s_off[b]; t < s_off[b + 1] && ok; ++t) {
                        const int d = v.sorted[t];
                        if (d == (int)c) continue;
                        const AccCand y = v.cand[d];
                        const double2 pd = v.mid[d];
                        const double ddx = pc.x - pd.x, ddy = pc.y - pd.y;
                        const bool compete = x.elem == y.elem || ddx * ddx + ddy * ddy < v.rho2;
                        if (!compete) continue;
                        if (!acc_better(x, y)) ok = false;
                        if (!(x.G > v.gamma * (x.G - y.G))) ok = false;
                    }
                }
            if (ok) v.plist[atomicAdd(&s_np, 1)] = (int32_t)c;
        }
    }
    __syncthreads();
    const int np = s_np;
    const int64_t k = *v.base + k_rel;
    const int64_t ns0 = *v.nsplit;
    for (int i = tid; i < np; i += NT) {
        const int c = v.plist[i];
        const AccCand x = v.cand[c];
        int rank = 0;
        for (int j = 0; j < np; ++j)
            if (acc_better(v.cand[v.plist[j]], x)) ++rank;
        v.order[rank] = (int32_t)c;
        v.split[x.elem] = (uint8_t)(kSplitFlag | x.ak);
        if (ns0 + rank < v.log_cap) {
            LogRec r;
            r.step = (int32_t)k;
            r.elem = x.elem;
            r.entry = (uint8_t)(x.ak >> 2);
            r.exit = (uint8_t)(x.ak & 3);
            r.pad0 = r.pad1 = 0;
            r.pad2 = 0;
            r.G = x.G;
            v.log[ns0 + rank] = r;
        }
    }
    __syncthreads();
    if (tid == 0) {
        // U_d in log order
        double Ud = *v.Ud;
        for (int r = 0; r < np; ++r) {
            const int c = v.order[r];
            const int e = v.cand[c].elem;
            const double gc = v.gc ? v.gc[e] : v.gc_uniform;
            Ud = Ud + gc * v.len[c];
        }
        *v.Ud = Ud;
        if (ns0 + np > v.log_cap) *v.overflow = 1;
        *v.nsplit = ns0 + np;
        *v.count = 0;
    }
}

}  // namespace mct
