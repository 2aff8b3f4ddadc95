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
    uint8_t *picked;     // scratch
    uint8_t *split;
    LogRec *log;
    int64_t log_cap;
    int64_t *nsplit;
    double *Ud;
    int32_t *overflow;
    const int64_t *base;  // steps before the running segment
    const double *gc;     // per element, or null for gc_uniform
    double gc_uniform, gamma, rho2;
};

__device__ __forceinline__ bool acc_better(const AccCand &x, const AccCand &y) {
    if (x.G != y.G) return x.G > y.G;
    if (x.elem != y.elem) return x.elem < y.elem;
    return (x.ak >> 2) < (y.ak >> 2);
}

// The pick of step base + k_rel with one workgroup of NT threads.  Geom
// provides tip(elem, a) -> reference midpoint of local edge a and
// path_len(elem, a, k) -> length of the crack path between the midpoints
// of local edges a and k, computed like the step's own geometry.
template <int NT, class Geom>
__device__ void front_pick_block(const FrontView &v, const Geom &geo, int k_rel) {
    __shared__ int s_np;
    const uint32_t n = *v.count;  // uniform
    if (n == 0) return;
    const int tid = threadIdx.x;
    for (uint32_t c = tid; c < n; c += NT) {
        const AccCand x = v.cand[c];
        v.mid[c] = geo.tip(x.elem, x.ak >> 2);
        v.len[c] = geo.path_len(x.elem, x.ak >> 2, x.ak & 3);
    }
    if (tid == 0) s_np = 0;
    __syncthreads();
    for (uint32_t c = tid; c < n; c += NT) {
        const AccCand x = v.cand[c];
        const double2 pc = v.mid[c];
        bool ok = true;
        for (uint32_t d = 0; d < n && ok; ++d) {
            if (d == c) continue;
            const AccCand y = v.cand[d];
            const double2 pd = v.mid[d];
            const double dx = pc.x - pd.x, dy = pc.y - pd.y;
            const bool compete = x.elem == y.elem || dx * dx + dy * dy < v.rho2;
            if (!compete) continue;
            if (!acc_better(x, y)) ok = false;
            if (!(x.G > v.gamma * (x.G - y.G))) ok = false;
        }
        v.picked[c] = ok ? 1 : 0;
        if (ok) atomicAdd(&s_np, 1);
    }
    __syncthreads();
    const int64_t k = *v.base + k_rel;
    const int64_t ns0 = *v.nsplit;
    for (uint32_t c = tid; c < n; c += NT) {
        if (!v.picked[c]) continue;
        const AccCand x = v.cand[c];
        int rank = 0;
        for (uint32_t d = 0; d < n; ++d)
            if (v.picked[d] && acc_better(v.cand[d], x)) ++rank;
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
        const int np = s_np;
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
