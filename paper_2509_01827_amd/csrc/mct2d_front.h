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

__device__ __forceinline__ int front_bucket(long long cx, long long cy, int nbuckets = kFrontBuckets) {
    const unsigned long long h = (unsigned long long)cx * 0x9E3779B97F4A7C15ull ^
                                 (unsigned long long)cy * 0xC2B2AE3D27D4EB4Full;
    return (int)((h >> 40) & (unsigned long long)(nbuckets - 1));
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

// ------------------------------------------------------------------------
// The same pick spread over the whole GPU, for models with many candidates
// per step; the tables are described with kFrontGridBuckets.
//   k_fg_prep   (a thread per candidate) tip point and bucket; the
//               candidate's index goes into the bucket's row of
//               kFrontGridCap slots, or onto its overflow list when full
//               (front_grid_insert).  The grid also clears the other table
//               for the next step (front_grid_clear).  A step kernel that
//               does both itself as it lists the candidates skips it.
//   k_fg_decide (a wavefront per candidate) the own cell's row first, then
//               the other eight cells' rows, one slot per lane, and any
//               overflow list (lane q walks cell q's); the candidate is
//               picked when no lane finds a competitor it fails against,
//               and listed with its U_d term (G_c * path length) beside it.
//   k_fg_close  (one workgroup) puts the picked ones in key order (each
//               ranked by counting the better keys in LDS, or for many a
//               bitonic sort), writes split codes and log records in that
//               order and adds U_d in log order (the decision's products
//               G_c * path length, summed by one thread).
// A candidate's decision depends only on the set of candidates, so the
// picks, the log and U_d are those of front_pick_block, bit for bit.
// ------------------------------------------------------------------------
constexpr int kFrontGridBlocks = 1024;
constexpr int kFrontGridThreads = 256;
constexpr int kFrontCloseThreads = 1024;
constexpr int kFrontSortMax = 2048;
constexpr int kFrontCountMax = 256;
static_assert(kFrontGridCap == 64, "one row slot per lane of a wavefront");

static_assert(kFrontGridHead == kFrontGridCnt + kFrontGridBuckets, "heads follow the counts");

// Candidate c with tip point m into the table tb of its step; next holds
// the overflow lists.
__device__ __forceinline__ void front_grid_insert(int32_t *tb, double cell, int32_t *next, int32_t c, double2 m) {
    const int b = front_bucket((long long)floor(m.x / cell), (long long)floor(m.y / cell), kFrontGridBuckets);
    const int slot = atomicAdd(&tb[kFrontGridCnt + b], 1);
    if (slot < kFrontGridCap)
        tb[kFrontGridTab + (int64_t)b * kFrontGridCap + slot] = c;
    else
        next[c] = atomicExch(&tb[kFrontGridHead + b], c);
}

// Entries t = t0, t0 + stride, ... of the counts and heads of the table
// the next step uses (tables: both; par: this step's parity).
__device__ __forceinline__ void front_grid_clear(int32_t *tables, int par, int64_t t0, int64_t stride) {
    int32_t *nx = tables + (par ^ 1) * kFrontGridTable;
    for (int64_t t = t0; t < 2 * (int64_t)kFrontGridBuckets; t += stride)
        nx[kFrontGridCnt + t] = t < kFrontGridBuckets ? 0 : -1;  // counts, then heads
}

namespace {  // kernels local to each translation unit that includes this header

// acc_better(y, x) without branches, as 0 or 1
__device__ __forceinline__ int acc_better_i(const AccCand &y, const AccCand &x) {
    const bool gt = y.G > x.G, eq = y.G == x.G;
    const bool tie = y.elem < x.elem || (y.elem == x.elem && (y.ak >> 2) < (x.ak >> 2));
    return (int)(gt || (eq && tie));
}

// Ud + t[0] + t[1] + ... + t[m-1], added in this order (t in LDS); the
// loads go out sixteen at a time ahead of the dependent additions.
__device__ __forceinline__ double add_in_order(double Ud, const double *t, int m) {
    int r = 0;
    for (; r + 16 <= m; r += 16) {
        double a[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) a[q] = t[r + q];
#pragma unroll
        for (int q = 0; q < 16; ++q) Ud = Ud + a[q];
    }
    for (; r < m; ++r) Ud = Ud + t[r];
    return Ud;
}

// the table of step base + k_rel
__device__ __forceinline__ int32_t *front_table(const FrontView &v, int32_t *tables, int k_rel) {
    return tables + ((*v.base + k_rel) & 1) * kFrontGridTable;
}

template <class Geom>
__global__ __launch_bounds__(kFrontGridThreads) void k_fg_prep(FrontView v, Geom geo, int32_t *tables, int k_rel) {
    const int par = (int)((*v.base + k_rel) & 1);
    int32_t *tb = tables + par * kFrontGridTable;
    const uint32_t stride = gridDim.x * blockDim.x;
    front_grid_clear(tables, par, blockIdx.x * blockDim.x + threadIdx.x, stride);
    const uint32_t n = *v.count;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const AccCand x = v.cand[c];
        const double2 m = geo.tip(x.elem, x.ak >> 2);
        v.mid[c] = m;
        front_grid_insert(tb, v.cell, v.sorted, (int32_t)c, m);
    }
}

// Does candidate x (index c, tip point pc) fail against candidate d?
__device__ __forceinline__ bool front_fails(const FrontView &v, const AccCand &x, double2 pc, int c, int d) {
    if (d == c) return false;
    const AccCand y = v.cand[d];
    const double2 pd = v.mid[d];
    const double ddx = pc.x - pd.x, ddy = pc.y - pd.y;
    const bool compete = x.elem == y.elem || ddx * ddx + ddy * ddy < v.rho2;
    return compete && (!acc_better(x, y) || !(x.G > v.gamma * (x.G - y.G)));
}

// Split code and log record of the picked candidate x at log position pos.
__device__ __forceinline__ void front_record(const FrontView &v, const AccCand &x, int64_t k, int64_t pos) {
    v.split[x.elem] = (uint8_t)(kSplitFlag | x.ak);
    if (pos < v.log_cap) {
        LogRec r;
        r.step = (int32_t)k;
        r.elem = x.elem;
        r.entry = (uint8_t)(x.ak >> 2);
        r.exit = (uint8_t)(x.ak & 3);
        r.pad0 = r.pad1 = 0;
        r.pad2 = 0;
        r.G = x.G;
        v.log[pos] = r;
    }
}

// Puts the np picked candidates in key order, best first (a bitonic sort
// over N = a power of two >= np entries, padded with keys that beat nothing:
// G = -1, while accepted candidates have G > 0), writes their split codes
// and log records in that order and adds their U_d terms to Ud in that
// order.  key, cix and term (N entries each) are LDS or global memory; the
// terms (G_c x path length, stored by the decision beside each picked
// candidate) move with their keys.  One workgroup of NT threads.
template <int NT>
__device__ __forceinline__ void front_sort_close(const FrontView &v, AccCand *key, int32_t *cix, double *term, int np,
                                                 int N, int64_t k, int64_t ns0, double &Ud) {
    const int tid = threadIdx.x;
    for (int j = tid; j < N; j += NT) {
        AccCand y;
        int32_t c = -1;
        double t = 0.0;
        if (j < np) {
            c = v.plist[j];
            y = v.cand[c];
            t = v.len[j];  // the decision's U_d term of picked candidate j
        } else {
            y.G = -1.0;
            y.elem = 0x7fffffff;
            y.ak = 0;
        }
        key[j] = y;
        cix[j] = c;
        term[j] = t;
    }
    __syncthreads();
    for (int kk = 2; kk <= N; kk <<= 1)
        for (int h = kk >> 1; h > 0; h >>= 1) {
            for (int i = tid; i < N; i += NT) {
                const int l = i ^ h;
                if (l > i) {
                    const AccCand a = key[i], b = key[l];
                    // blocks with (i & kk) == 0 run best first
                    if (((i & kk) == 0) ? acc_better(b, a) : acc_better(a, b)) {
                        key[i] = b;
                        key[l] = a;
                        const int32_t c = cix[i];
                        cix[i] = cix[l];
                        cix[l] = c;
                        const double t = term[i];
                        term[i] = term[l];
                        term[l] = t;
                    }
                }
            }
            __syncthreads();
        }
    // the picked candidates are distinct elements, so their keys are
    // distinct and the order is the key order
    for (int r = tid; r < np; r += NT) front_record(v, key[r], k, ns0 + r);
    if (tid == 0) Ud = add_in_order(Ud, term, np);  // U_d in log order
}

// The end of the pick (one workgroup of NT threads, tb the step's table).
// Up to kFrontCountMax picked candidates (and the table's counting limit):
// each thread ranks its own by counting the better keys (staged in LDS).
// More: a sort, in LDS when it fits there (and within the table's sort
// limit), else in the tip-point, order and path-length scratch arrays,
// which the decision no longer reads (N < 2 np <= 2 ne entries, within
// their capacity).
template <int NT>
__device__ void front_grid_close(const FrontView &v, int32_t *tb, int k_rel) {
    static_assert(kFrontCountMax <= NT && kFrontCountMax <= kFrontSortMax, "one picked candidate per thread");
    __shared__ __align__(16) AccCand s_key[kFrontSortMax];
    __shared__ int32_t s_cix[kFrontSortMax];
    __shared__ double s_term[kFrontSortMax];
    const int tid = threadIdx.x;
    int32_t *np_ = tb + kFrontGridNp;
    const int np = *np_;
    const int lds_max = tb[kFrontGridSortMax];
    const int rank_max = tb[kFrontGridRankMax];
    const int64_t k = *v.base + k_rel;
    const int64_t ns0 = *v.nsplit;
    double Ud = *v.Ud;
    __syncthreads();  // every wave has read the counts before thread 0 resets them
    int N = 2;
    while (N < np) N <<= 1;
    if (np <= rank_max && np <= kFrontCountMax) {
        // keys padded to a multiple of 8 as in the sort
        const int np8 = (np + 7) & ~7;
        AccCand x;
        double t = 0.0;
        if (tid < np) {
            x = v.cand[v.plist[tid]];
            t = v.len[tid];
        } else {
            x.G = -1.0;
            x.elem = 0x7fffffff;
            x.ak = 0;
        }
        if (tid < np8) s_key[tid] = x;
        __syncthreads();
        if (tid < np) {
            int rank = 0;
            for (int j = 0; j < np8; j += 8) {
                AccCand y[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) y[q] = s_key[j + q];
#pragma unroll
                for (int q = 0; q < 8; ++q) rank += acc_better_i(y[q], x);
            }
            s_term[rank] = t;
            front_record(v, x, k, ns0 + rank);
        }
        __syncthreads();
        if (tid == 0) Ud = add_in_order(Ud, s_term, np);  // U_d in log order
    } else if (N <= lds_max && N <= kFrontSortMax) {
        front_sort_close<NT>(v, s_key, s_cix, s_term, np, N, k, ns0, Ud);
    } else {
        front_sort_close<NT>(v, reinterpret_cast<AccCand *>(v.mid), v.order, v.len, np, N, k, ns0, Ud);
    }
    if (tid == 0) {
        *v.Ud = Ud;
        if (ns0 + np > v.log_cap) *v.overflow = 1;
        *v.nsplit = ns0 + np;
        *v.count = 0;
        *np_ = 0;
    }
}

template <class Geom>
__global__ __launch_bounds__(kFrontGridThreads) void k_fg_decide(FrontView v, Geom geo, int32_t *tables, int k_rel) {
    int32_t *tb = front_table(v, tables, k_rel);
    const uint32_t n = *v.count;
    const int lane = threadIdx.x & 63;
    const uint32_t nwave = gridDim.x * (blockDim.x >> 6);
    for (uint32_t c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < n; c += nwave) {
        const AccCand x = v.cand[c];
        const double2 pc = v.mid[c];
        const long long cx = (long long)floor(pc.x / v.cell), cy = (long long)floor(pc.y / v.cell);
        // cell q = 0..8 ((dx, dy) = (q % 3 - 1, q / 3 - 1)); q = 4 is the own cell
        int cnt[9];
        int bq[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            bq[q] = front_bucket(cx + q % 3 - 1, cy + q / 3 - 1, kFrontGridBuckets);
            cnt[q] = tb[kFrontGridCnt + bq[q]];
        }
        bool fail = lane < cnt[4] && front_fails(v, x, pc, (int)c,
                                                  tb[kFrontGridTab + (int64_t)bq[4] * kFrontGridCap + lane]);
        if (__ballot(fail) == 0ull) {
            int d[9];
#pragma unroll
            for (int q = 0; q < 9; ++q)
                d[q] = (q != 4 && lane < cnt[q]) ? tb[kFrontGridTab + (int64_t)bq[q] * kFrontGridCap + lane] : -1;
#pragma unroll
            for (int q = 0; q < 9; ++q)
                if (d[q] >= 0 && front_fails(v, x, pc, (int)c, d[q])) fail = true;
            // overflow lists: lane q walks the list of cell q
            int walk = -1;
#pragma unroll
            for (int q = 0; q < 9; ++q)
                if (lane == q && cnt[q] > kFrontGridCap) walk = tb[kFrontGridHead + bq[q]];
            for (; walk >= 0 && !fail; walk = v.sorted[walk])
                if (front_fails(v, x, pc, (int)c, walk)) fail = true;
        }
        if (__ballot(fail) == 0ull && lane == 0) {
            // picked: listed, with its U_d term G_c x path length beside it
            const int i = atomicAdd(&tb[kFrontGridNp], 1);
            v.plist[i] = (int32_t)c;
            const double gc = v.gc ? v.gc[x.elem] : v.gc_uniform;
            v.len[i] = gc * geo.path_len(x.elem, x.ak >> 2, x.ak & 3);
        }
    }
}

__global__ __launch_bounds__(kFrontCloseThreads) void k_fg_close(FrontView v, int32_t *tables, int k_rel) {
    if (*v.count == 0) return;  // uniform; the count is reset by thread 0 after a barrier
    front_grid_close<kFrontCloseThreads>(v, front_table(v, tables, k_rel), k_rel);
}

}  // namespace

// The launches of the pick of step base + k_rel over the two tables
// (2 kFrontGridTable entries, as front_grid_reset leaves them: each pick
// keeps them so for the next step); prepped: the step kernel has filled
// the table, tip points and cleared the other table itself.
template <class Geom>
hipError_t launch_front_grid(const FrontView &v, const Geom &g, int32_t *tables, int k_rel, bool prepped,
                             hipStream_t st) {
    if (!prepped) k_fg_prep<Geom><<<kFrontGridBlocks, kFrontGridThreads, 0, st>>>(v, g, tables, k_rel);
    k_fg_decide<Geom><<<kFrontGridBlocks, kFrontGridThreads, 0, st>>>(v, g, tables, k_rel);
    k_fg_close<<<1, kFrontCloseThreads, 0, st>>>(v, tables, k_rel);
    return hipGetLastError();
}

}  // namespace mct
