// HIP kernels (gfx950) of the MCT-2D-CEM explicit step.
//
// k_step: one launch = one time step.  A workgroup owns a tile of
// (TXE-1) x (TYE-1) nodes and
//   1. stages u^k and X of the tile plus a 2-node halo, and the split codes
//      of every element touching that halo, in LDS;
//   2. forms the ES-FEM smoothed strain and plane stress at every edge of
//      the (TXE x TYE) elements around its nodes (Sec. 2.1, Eqs.
//      disp_ES_FEM / strain_discretization / QUAD_strain_discretization),
//      one thread per edge, in LDS;
//   3. computes the internal force of each of those elements (Eq.
//      QUAD_fint_discretization for intact ones, reduced pieces for split
//      ones), one thread per element, and scatters it to the owned nodes in
//      colour order 0..3 (four LDS passes, no two elements of one colour
//      share a node, so the per-node sum order is fixed);
//   4. advances its nodes by central differences and writes u^{k+1}, v;
//   5. compacts the free-surface candidates of the elements it owns with
//      wavefront ballots, evaluates G of the three split topologies and the
//      Q4 element rule (Sec. 2.2), reduces the best candidate of the
//      workgroup and publishes it;
//   6. at the start of the next step every workgroup reduces the published
//      candidates and applies the MCT pick with the split-ratio test
//      (Sec. 3) to its staged split codes; workgroup 0 records the split.
//      k_commit does the same for the last step of a launch segment.
//
// Arithmetic follows one fixed expression order (binary64, or binary32 for
// the binary32 step: every value of the step in T, times and the load curve
// in binary64; compiled with -ffp-contract=off; fma only where written), so
// the result does not depend on the tile shape or on the schedule.
#include "mct2d_device.h"
#include "mct2d_impl.h"
#include "mct2d_front.h"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <mutex>

namespace mct {

namespace {
using namespace dev;

// Best-candidate order: larger G, then smaller element id, then smaller a.
template <class T>
__device__ __forceinline__ bool better(T g1, int e1, int a1, T g2, int e2, int a2) {
    return g1 > g2 || (g1 == g2 && (e1 < e2 || (e1 == e2 && a1 < a2)));
}

// A reduction value: the best accepted candidate (G, e, a, k) of a set, the
// second largest accepted G (G2, -1 when the set has one) and the smallest
// accepted G.
template <class T>
struct CandT {
    T G, Gmin, G2;
    int e, a, k;
};
using Cand = CandT<double>;

template <class T>
__device__ __forceinline__ void cand_none(CandT<T> &c) {
    c.G = T(-1);
    c.Gmin = T(__builtin_inff());
    c.G2 = T(-1);
    c.e = INT_MAX;
    c.a = 4;
    c.k = 0;
}

// Merge another set's value (a single candidate has G2 = -1): the second
// largest of the union is the larger of the two second largest values and
// the smaller of the two largest.  Kept only with the near-threshold log
// (NEAR); otherwise G2 stays -1.
template <bool NEAR, class T>
__device__ __forceinline__ void cand_merge(CandT<T> &c, T G, T G2, T Gmin, int e, int a, int k) {
    if constexpr (NEAR) {
        const T lo = G < c.G ? G : c.G;
        const T s2 = G2 > c.G2 ? G2 : c.G2;
        c.G2 = lo > s2 ? lo : s2;
    }
    if (better(G, e, a, c.G, c.e, c.a)) {
        c.G = G;
        c.e = e;
        c.a = a;
        c.k = k;
    }
    if (Gmin < c.Gmin) c.Gmin = Gmin;
}

template <bool NEAR, class T>
__device__ __forceinline__ void cand_wave_reduce(CandT<T> &c) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T G = __shfl_xor(c.G, off, 64);
        T G2 = T(-1);
        if constexpr (NEAR) G2 = __shfl_xor(c.G2, off, 64);
        T Gm = __shfl_xor(c.Gmin, off, 64);
        int e = __shfl_xor(c.e, off, 64);
        int a = __shfl_xor(c.a, off, 64);
        int k = __shfl_xor(c.k, off, 64);
        cand_merge<NEAR>(c, G, G2, Gm, e, a, k);
    }
}

// Workgroup-wide reduction; the result is valid in thread 0.  A wave whose
// lanes hold no candidate (G < 0 everywhere: the empty value, which merging
// leaves unchanged) skips the shuffle tree; its lane 0 already holds the
// wave's result.
template <int NT, bool NEAR, class T>
__device__ __forceinline__ void cand_block_reduce(CandT<T> &c, CandT<T> *red) {
    if (__ballot(c.G >= T(0)) != 0ull) cand_wave_reduce<NEAR>(c);  // uniform over the wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NT / 64; ++w)
            cand_merge<NEAR>(c, red[w].G, red[w].G2, red[w].Gmin, red[w].e, red[w].a, red[w].k);
    }
}

// Prescribed velocity at time t: v0 times the ramp factor t / t_ramp
// (evaluated in binary64 and rounded to T) while t < t_ramp.
template <class T>
__device__ __forceinline__ T prescribed(T v0, double t, double t_ramp) {
    if (t_ramp > 0.0 && t < t_ramp) return v0 * T(t / t_ramp);
    return v0;
}

__device__ __forceinline__ int perimeter_index(int i, int j, int nx, int ny) {
    if (j == 0) return i;
    if (j == ny) return (nx + 1) + i;
    if (i == 0) return 2 * (nx + 1) + (j - 1);
    if (i == nx) return 2 * (nx + 1) + (ny - 1) + (j - 1);
    return -1;
}

// Read-only data the whole launch shares (a batch's unit table and views,
// the lattice constants): read through the constant address space, so that
// a workgroup-uniform address becomes a scalar load.
template <class X>
__device__ __forceinline__ const __attribute__((address_space(4))) X *kconst(const X *ptr) {
    return (const __attribute__((address_space(4))) X *)ptr;
}


// A batch view, copied field by field with scalar loads from the constant
// address space.  Pointers loaded from there are known to point to global
// memory, so the step issues global (not flat) loads and stores through them:
// flat accesses also count against the LDS wait counter, so each LDS wait
// would wait for the memory loads in flight too.  (Every field of
// StepParamsT is copied here.)
template <class T>
__device__ __forceinline__ void load_view(StepParamsT<T> &p, const StepParamsT<T> *v) {
    const __attribute__((address_space(4))) StepParamsT<T> *s = kconst(v);
    p.nx = s->nx; p.ny = s->ny; p.ntx = s->ntx; p.nty = s->nty;
    p.nwg = s->nwg; p.log_cap = s->log_cap; p.X = s->X; p.Y = s->Y;
    p.ux0 = s->ux0; p.uy0 = s->uy0; p.ux1 = s->ux1; p.uy1 = s->uy1;
    p.vx = s->vx; p.vy = s->vy; p.minv = s->minv; p.split = s->split;
    p.area = s->area; p.screen = s->screen; p.strip = s->strip; p.sct = s->sct; p.ncurve = s->ncurve;
    p.curve_t = s->curve_t; p.curve_phi = s->curve_phi; p.gc = s->gc; p.gc_uniform = s->gc_uniform;
    p.fext_p = s->fext_p; p.vmask_p = s->vmask_p; p.v0_p = s->v0_p; p.D11 = s->D11;
    p.D12 = s->D12; p.D33 = s->D33; p.E = s->E; p.dt = s->dt;
    p.t_ramp = s->t_ramp; p.dts = s->dts; p.gamma = s->gamma; p.ctl = s->ctl;
    p.slots = s->slots; p.log = s->log; p.subcell = s->subcell; p.pad_sc = s->pad_sc;
    p.front = s->front; p.fcap = s->fcap; p.front_r2 = s->front_r2; p.fcand = s->fcand;
    p.fcount = s->fcount; p.fmid = s->fmid; p.flen = s->flen; p.forder = s->forder;
    p.fbucket = s->fbucket; p.fsorted = s->fsorted; p.fplist = s->fplist; p.fcell = s->fcell;
    p.fgrid = s->fgrid; p.lat = s->lat; p.near = s->near; p.near_count = s->near_count; p.near_cap = s->near_cap;
    p.pad_near = s->pad_near; p.near_tol = s->near_tol;
}

// Non-zero pattern of the Q4 gradients at the midpoint of local edge k of a
// rectangle (axis-parallel edges): dN_n/dx vanishes where dN_n/dxi does
// (edges 0 and 2: the two nodes off the edge), dN_n/dy where dN_n/deta does
// (edges 1 and 3).
__host__ __device__ constexpr bool lat_nzx(int k, int n) {
    return (k == 1 || k == 3) ? true : (k == 0 ? (n == 0 || n == 1) : (n == 2 || n == 3));
}
__host__ __device__ constexpr bool lat_nzy(int k, int n) {
    return (k == 0 || k == 2) ? true : (k == 1 ? (n == 1 || n == 2) : (n == 0 || n == 3));
}

// Strain (B u) at the midpoint of local edge K of a lattice element with
// the shared gradients B: the terms of strain<4> in the same order, the
// vanishing products left out (adding a zero product changes at most the
// sign of a zero).
template <int K>
__device__ __forceinline__ void strain_lat(const LatticeConst *L, const double ux[4], const double uy[4],
                                           double q[3]) {
    double exx = 0.0, eyy = 0.0, gxy = 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const double bx = kconst(L)->B[K][n], by = kconst(L)->B[K][4 + n];
        if (lat_nzx(K, n)) exx = fma(bx, ux[n], exx);
        if (lat_nzy(K, n)) eyy = fma(by, uy[n], eyy);
        if (lat_nzy(K, n)) gxy = fma(by, ux[n], gxy);
        if (lat_nzx(K, n)) gxy = fma(bx, uy[n], gxy);
    }
    q[0] = exx;
    q[1] = eyy;
    q[2] = gxy;
}

__device__ __forceinline__ void strain_lat_rt(const LatticeConst *L, int k, const double ux[4],
                                              const double uy[4], double q[3]) {
    switch (k) {
        case 0: strain_lat<0>(L, ux, uy, q); break;
        case 1: strain_lat<1>(L, ux, uy, q); break;
        case 2: strain_lat<2>(L, ux, uy, q); break;
        default: strain_lat<3>(L, ux, uy, q); break;
    }
}

template <class T>
__device__ __forceinline__ T absT(T x) {
    return x < T(0) ? -x : x;
}

// Near-threshold records (plain models with the log on).
template <class T>
__device__ __forceinline__ void near_push(const StepParamsT<T> &p, int64_t step, int64_t e, int a, int kind, int k,
                                          T G, T ref) {
    const uint32_t i = atomicAdd(p.near_count, 1u);
    if (i < (uint32_t)p.near_cap) {
        NearRec r;
        r.step = (int32_t)step;
        r.elem = (int32_t)e;
        r.a = (uint8_t)a;
        r.kind = (uint8_t)kind;
        r.k = (uint8_t)k;
        r.pad0 = 0;
        r.pad1 = 0;
        r.G = (double)G;
        r.ref = (double)ref;
        p.near[i] = r;
    }
}

// One evaluated candidate (gate open, path values G[0..2] of exit edges
// a+1, a+2, a+3): paths near Gc; with two or more paths above Gc the gap of
// the largest two and every split-ratio margin of the element rule.
template <class T>
__device__ __forceinline__ void near_candidate(const StepParamsT<T> &p, int64_t step, int64_t e, int a,
                                               const T G[3], T gc) {
    const T tol = p.near_tol, gamma = p.gamma;
    int best = -1, nS = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (absT(G[j] - gc) <= tol * gc) near_push(p, step, e, a, 1, (a + 1 + j) & 3, G[j], gc);
        if (G[j] > gc) {
            nS++;
            if (best < 0 || G[j] > G[best]) best = j;
        }
    }
    if (nS < 2) return;
    T gb = T(0), second = T(-1);
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if (j == best) gb = G[j];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if (j != best && G[j] > gc && G[j] > second) second = G[j];
    if (gb - second <= tol * gb) near_push(p, step, e, a, 2, (a + 1 + best) & 3, gb, second);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j == best || !(G[j] > gc)) continue;
        if (absT(gb - gamma * (gb - G[j])) <= tol * gb) near_push(p, step, e, a, 3, (a + 1 + j) & 3, gb, G[j]);
    }
}

}  // namespace

// The pick's records: the gap of the two largest accepted G and the
// split-ratio margin against the smallest (g holds the reduced set).
template <class T>
__device__ __forceinline__ void near_pick(const StepParamsT<T> &p, int64_t step, const CandT<T> &g) {
    if (!p.near || p.sct || !(g.G >= T(0))) return;
    const T tol = p.near_tol;
    if (g.G2 >= T(0) && g.G - g.G2 <= tol * g.G) near_push(p, step, g.e, g.a, 4, g.k, g.G, g.G2);
    if (absT(g.G - p.gamma * (g.G - g.Gmin)) <= tol * g.G) near_push(p, step, g.e, g.a, 5, g.k, g.G, g.Gmin);
}

// Reduce the candidates published in slot set `set` with the whole
// workgroup; thread 0 receives the result.  Every thread must call it.
// Slots hold binary64 values; a binary32 step's values are exact in them.
template <int NT, bool NEAR, class T>
__device__ __forceinline__ CandT<T> reduce_slots(const StepParamsT<T> &p, int set, uint32_t n, CandT<T> *red) {
    const Slot *sl = p.slots + (size_t)set * p.nwg;
    CandT<T> g;
    cand_none(g);
    for (uint32_t s = threadIdx.x; s < n; s += NT) {
        const Slot x = sl[s];
        cand_merge<NEAR>(g, T(x.G), T(x.G2), T(x.Gmin), x.elem, x.a, x.k);
    }
    cand_block_reduce<NT, NEAR>(g, red);
    return g;
}

// MCT pick: the largest G must pass G* > gamma (G* - G_c) against every other
// accepted candidate; (G* - G_c) grows as G_c shrinks and rounding is
// monotone, so the smallest accepted G decides.
template <class T>
__device__ __forceinline__ bool pick_accepted(const StepParamsT<T> &p, const CandT<T> &g) {
    return g.G >= T(0) && g.G > p.gamma * (g.G - g.Gmin);
}

// Split the picked element (acts from the next step), log it and add
// Gc * crack-path length (a T product, accumulated in binary64) to U_d.
// One thread of one workgroup.
template <class T>
__device__ __forceinline__ void apply_split(const StepParamsT<T> &p, const CandT<T> &g, int64_t kdecided) {
    Control *ctl = p.ctl;
    p.split[g.e] = (uint8_t)(kSplitFlag | (g.a << 2) | g.k);
    const int64_t n = ctl->nsplit;
    if (n < p.log_cap) {
        LogRec r;
        r.step = (int32_t)kdecided;
        r.elem = g.e;
        r.entry = (uint8_t)g.a;
        r.exit = (uint8_t)g.k;
        r.pad0 = r.pad1 = 0;
        r.pad2 = 0;
        r.G = (double)g.G;
        p.log[n] = r;
    } else {
        ctl->overflow = 1;
    }
    ctl->nsplit = n + 1;
    const int64_t i = g.e % p.nx, j = g.e / p.nx;
    const int64_t n0 = j * (p.nx + 1) + i;
    const int64_t nd[4] = {n0, n0 + 1, n0 + p.nx + 2, n0 + p.nx + 1};
    T x[4], y[4];
    for (int q = 0; q < 4; ++q) {
        x[q] = p.X[nd[q]];
        y[q] = p.Y[nd[q]];
    }
    T cx, cy, L;
    path_geom(x, y, g.a, g.k, cx, cy, L);
    const T gc = p.gc ? p.gc[g.e] : p.gc_uniform;
    ctl->Ud = ctl->Ud + (double)(gc * L);
}

// Single-tip mode: the tip after element g.e split with exit edge g.k is
// the same edge seen from the element across it, if that element exists
// and is intact (the only split of a step is g.e's own).
template <class T>
__device__ __forceinline__ int32_t tip_after(const StepParamsT<T> &p, const CandT<T> &g) {
    const int i = g.e % p.nx, j = g.e / p.nx;
    const int ni = (g.k == 1) ? i + 1 : (g.k == 3) ? i - 1 : i;
    const int nj = (g.k == 2) ? j + 1 : (g.k == 0) ? j - 1 : j;
    if (ni < 0 || ni >= p.nx || nj < 0 || nj >= p.ny) return -1;
    const int64_t nb = (int64_t)nj * p.nx + ni;
    if (p.split[nb] != 0) return -1;
    return (int32_t)(nb * 4 + ((g.k + 2) & 3));
}

// One time step.  Steps run in segments (a captured graph or a run of direct
// launches) closed by k_commit; k_rel is the index inside the segment and
// par0 the parity of the segment's first step (u^k lives in buffer k & 1).
// The pick of step k-1 is taken at the start of step k from the candidates
// step k-1 published (slot set (k_rel-1) mod 3): every workgroup reduces
// them, applies the split to its staged codes, and workgroup 0 records it.
//
// BATCHED: the launch covers the tiles of many independent specimens; work
// unit b = (specimen, tile) comes from `units` and the specimen's view (its
// sizes, constants and pre-offset pointers) from `views`.  Otherwise the one
// view `p0` is passed by value and workgroups map to tiles XCD-banded.
//
// UNI (binary64 point rule): every specimen of the launch is a uniform
// lattice, whose element gradients, smoothing weight, force factor and
// crack-path geometry are the shared values in p.lat (set-up verified them
// bitwise equal to what each element would compute).  Only u and the split
// codes are staged; coordinates are read from memory for candidates and
// split elements alone.  Same operations in the same order, so the result
// is the general kernel's bit for bit.
//
// NEAR (plain models, 16 x 16 tiles): the near-threshold decision log is on;
// the reductions also carry the second largest accepted G.
//
// FRONT (plain binary64 models): the per-front pick is on; every accepted
// candidate is listed (one atomic per wavefront), and with the bucket table
// of the pick over the whole GPU its tip point goes into the table.  The
// NEAR instances carry the same code (the near log and the per-front pick
// may be on together).
template <class T, int TXE, int TYE, bool BATCHED, bool SC = false, bool UNI = false, bool NEAR = false,
          bool FRONT = false>
__global__ __launch_bounds__(TXE *TYE, UNI ? 6 : 4) void k_step(StepParamsT<T> p0,
                                                               const StepParamsT<T> *__restrict__ views,
                                                               const int2 *__restrict__ units, int k_rel, int par0) {
    static_assert(!UNI || (sizeof(T) == 8 && !SC), "the lattice kernel is binary64 with the point rule");
    static_assert(!NEAR || !BATCHED, "the near-threshold log is for plain models");
    constexpr int NT = TXE * TYE;
    constexpr int TX = TXE - 1, TY = TYE - 1;  // owned nodes
    constexpr int HX = TXE + 3, HY = TYE + 3;  // staged nodes
    constexpr int EX = TXE + 2, EY = TYE + 2;  // staged elements
    constexpr int NH = TXE * (TYE + 1);        // horizontal edges
    constexpr int NV = (TXE + 1) * TYE;        // vertical edges
    static_assert(NT % 64 == 0, "whole wavefronts");
    static_assert(TX * TY <= NT, "one thread per owned node");

    constexpr int NS = NH + NV;  // component stride of the per-edge array
    // SC (sub-cell smoothing): a fourth component holds the lower-id side's
    // sub-cell area
    constexpr int NQ = ((SC ? 4 : 3) * NS > 8 * NT) ? (SC ? 4 : 3) * NS : 8 * NT;
    constexpr int NXY = UNI ? 1 : HX * HY;
    __shared__ T s_ux[HX * HY], s_uy[HX * HY], s_X[NXY], s_Y[NXY];
    // per edge and component (stride NS): first the strain part of the
    // lower-id element, then the smoothed stress; after the force phase the
    // same memory holds the element forces [8][NT]
    __shared__ T s_e[NQ];
    __shared__ T s_area[UNI ? 1 : EX * EY];
    T *const s_fe = s_e;
    __shared__ uint8_t s_split[EX * EY];
    __shared__ uint16_t s_cand_own[UNI ? 1 : 4 * TX * TY];  // candidate list
    __shared__ uint16_t s_splitl[NT];
    __shared__ int s_ncand, s_ncorner, s_nthru;
    __shared__ int32_t s_tip;
    __shared__ T s_phi;
    // per wavefront: list offsets of the compaction, and whether a staged
    // element is split or outside the grid; the reduction of candidates
    __shared__ int s_wb_own[UNI ? 1 : 4 * (NT / 64)];
    __shared__ CandT<T> s_red_own[UNI ? 1 : NT / 64];
    // The lattice kernel keeps the list and these small arrays in the part
    // of s_e that the edge stresses leave free (none of them is live when
    // the forces are stored there).
    constexpr int kTailCand = 4 * TX * TY * (int)sizeof(uint16_t);
    constexpr int kTailRed = (kTailCand + 15) & ~15;
    constexpr int kTailWb = kTailRed + (NT / 64) * (int)sizeof(CandT<T>);
    constexpr int kTailEnd = kTailWb + 4 * (NT / 64) * (int)sizeof(int);
    static_assert(!UNI || kTailEnd <= (NQ - 3 * NS) * (int)sizeof(T), "small arrays in the tail of s_e");
    char *const s_tail = reinterpret_cast<char *>(s_e + 3 * NS);
    uint16_t *const s_cand = UNI ? reinterpret_cast<uint16_t *>(s_tail) : s_cand_own;
    CandT<T> *const s_red = UNI ? reinterpret_cast<CandT<T> *>(s_tail + kTailRed) : s_red_own;
    int *const s_wbase = UNI ? reinterpret_cast<int *>(s_tail + kTailWb) : s_wb_own;
    int *const s_wbase2 = s_wbase + NT / 64, *const s_wbase3 = s_wbase + 2 * (NT / 64);
    int *const s_free = s_wbase + 3 * (NT / 64);

    const int tid = threadIdx.x;
    int tile;
    StepParamsT<T> p;
    const StepParamsT<T> *vsrc = nullptr;  // batch: the specimen's view
    if constexpr (BATCHED) {
        const __attribute__((address_space(4))) int *uu = kconst(reinterpret_cast<const int *>(units));
        const int2 u = make_int2(uu[2 * blockIdx.x], uu[2 * blockIdx.x + 1]);
        vsrc = views + u.x;
        load_view(p, vsrc);
        tile = u.y;
    } else {
        p = p0;
        tile = xcd_tile(blockIdx.x, p.nwg);
    }
    const bool leader = tile == 0;  // records the specimen's previous pick
    const int nx = p.nx, ny = p.ny;
    const int i0 = (tile % p.ntx) * TX, j0 = (tile / p.ntx) * TY;
    const int par = (par0 + k_rel) & 1;
    const T *ux_c = par ? p.ux1 : p.ux0;
    const T *uy_c = par ? p.uy1 : p.uy0;
    T *ux_n = par ? p.ux0 : p.ux1;
    T *uy_n = par ? p.uy0 : p.uy1;
    const int set_w = k_rel % 3, set_r = (k_rel + 2) % 3, set_c = (k_rel + 1) % 3;
    const int64_t base = p.ctl->base;  // needed late (time, first step, log)
    // single-tip mode: the tip at the start of the previous step (slot by parity)
    const int32_t tip_prev = p.sct ? ((((base + k_rel - 1) & 1) != 0) ? p.ctl->tip1 : p.ctl->tip0) : -1;

    // ---- 1. stage nodes and split codes; prefetch owned-node data ------
    // Every global load of the phase is issued before the first LDS write,
    // so the workgroup waits for one memory latency instead of several.
    constexpr int NHALO = HX * HY, RH = (NHALO + NT - 1) / NT;
    constexpr int NE2 = EX * EY, RE = (NE2 + NT - 1) / NT;
    const uint32_t nprev = p.ctl->nslots[set_r];
    T ra[RH], rb[RH], rc[RH], rd[RH];
#pragma unroll
    for (int r = 0; r < RH; ++r) {
        const int idx = tid + r * NT;
        const int gi = i0 - 2 + idx % HX, gj = j0 - 2 + idx / HX;
        ra[r] = rb[r] = rc[r] = rd[r] = T(0);
        if (idx < NHALO && gi >= 0 && gi <= nx && gj >= 0 && gj <= ny) {
            const int64_t n = (int64_t)gj * (nx + 1) + gi;
            ra[r] = ux_c[n];
            rb[r] = uy_c[n];
            if constexpr (!UNI) {
                rc[r] = p.X[n];
                rd[r] = p.Y[n];
            }
        }
    }
    uint8_t rs[RE];
    T rarea[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int idx = tid + r * NT;
        const int gi = i0 - 2 + idx % EX, gj = j0 - 2 + idx / EX;
        rs[r] = kAbsent;
        rarea[r] = T(0);
        if (idx < NE2 && gi >= 0 && gi < nx && gj >= 0 && gj < ny) {
            const int64_t e = (int64_t)gj * nx + gi;
            rs[r] = p.split[e];
            if constexpr (!UNI) rarea[r] = p.area[e];
        }
    }
    // screen state of this thread's ring element (owned elements only)
    uint32_t scr = 0;
    if (p.screen) {
        const int gi = i0 - 1 + tid % TXE, gj = j0 - 1 + tid / TXE;
        if (tid % TXE >= 1 && tid / TXE >= 1 && gi < nx && gj < ny) scr = p.screen[(int64_t)gj * nx + gi];
    }
    // owned node of this thread
    const int on_l = tid % TX, on_m = tid / TX;
    const int on_i = i0 + on_l, on_j = j0 + on_m;
    const bool on_valid = tid < TX * TY && on_i <= nx && on_j <= ny;
    const int64_t on_n = (int64_t)on_j * (nx + 1) + on_i;
    // owned-node data for the update: the lattice kernel issues these loads
    // with the staging loads (one memory round trip per workgroup); the
    // general kernel, short of registers, once the candidates are done
    T n_minv = T(0), n_vx = T(0), n_vy = T(0), n_fex = T(0), n_fey = T(0), n_v0x = T(0), n_v0y = T(0);
    unsigned n_mask = 0;
    auto load_node = [&]() {
        if (on_valid) {
            n_minv = p.minv[on_n];
            n_vx = p.vx[on_n];
            n_vy = p.vy[on_n];
            const int pidx = perimeter_index(on_i, on_j, nx, ny);
            if (pidx >= 0) {
                n_fex = p.fext_p[2 * pidx];
                n_fey = p.fext_p[2 * pidx + 1];
                n_mask = p.vmask_p[pidx];
                n_v0x = p.v0_p[2 * pidx];
                n_v0y = p.v0_p[2 * pidx + 1];
            }
        }
    };
    if constexpr (UNI) load_node();
#pragma unroll
    for (int r = 0; r < RH; ++r) {
        const int idx = tid + r * NT;
        if (idx < NHALO) {
            s_ux[idx] = ra[r];
            s_uy[idx] = rb[r];
            if constexpr (!UNI) {
                s_X[idx] = rc[r];
                s_Y[idx] = rd[r];
            }
        }
    }
    bool free_el = false;
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int idx = tid + r * NT;
        if (idx < NE2) {
            s_split[idx] = rs[r];
            if constexpr (!UNI) s_area[idx] = rarea[r];
            free_el = free_el || rs[r] != 0;
        }
    }
    {
        const uint64_t b = __ballot(free_el);
        if ((tid & 63) == 0) s_free[tid >> 6] = b != 0ull;
    }
    if (tid == 0) {
        s_ncand = 0;
        s_ncorner = 0;
        s_nthru = 0;
        s_tip = tip_prev;
        s_phi = T(load_factor(p, (double)(base + k_rel) * p.dt));  // traction factor at t_k
    }

    // ---- 2. the pick of the previous step -------------------------------
    if (nprev > 0) {  // uniform over the workgroup
        const CandT<T> g = reduce_slots<NT, NEAR>(p, set_r, nprev, s_red);  // contains a barrier
        if (tid == 0 && pick_accepted(p, g)) {
            const int fx = g.e % nx - (i0 - 2), fy = g.e / nx - (j0 - 2);
            if (fx >= 0 && fx < EX && fy >= 0 && fy < EY) {
                s_split[fy * EX + fx] = (uint8_t)(kSplitFlag | (g.a << 2) | g.k);
                s_free[0] = 1;
            }
            if (p.sct) s_tip = tip_after(p, g);
            if (leader) apply_split(p, g, base + k_rel - 1);
        }
        if constexpr (NEAR)
            if (tid == 0 && leader) near_pick(p, base + k_rel - 1, g);
    }
    if (tid == 0 && leader) {
        p.ctl->nslots[set_c] = 0;
        if (p.sct) {
            if (((base + k_rel) & 1) != 0)
                p.ctl->tip1 = s_tip;
            else
                p.ctl->tip0 = s_tip;
        }
    }
    __syncthreads();
    // a tile without split or absent elements has no free-surface
    // candidates and no split pieces: it skips their listing
    bool tile_free = false;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) tile_free = tile_free || s_free[w] != 0;

    // reference coordinates of the staged node at offset o (lattice: read
    // from memory, only for candidates and split elements)
    auto node_xy = [&](int o, T &x, T &y) {
        if constexpr (UNI) {
            const int64_t n = (int64_t)(j0 - 2 + o / HX) * (nx + 1) + (i0 - 2 + o % HX);
            x = p.X[n];
            y = p.Y[n];
        } else {
            x = s_X[o];
            y = s_Y[o];
        }
    };
    auto elem_xy = [&](int ex, int ey, T x[4], T y[4]) {
        const int b = ey * HX + ex;
        x[0] = s_X[b];
        x[1] = s_X[b + 1];
        x[2] = s_X[b + HX + 1];
        x[3] = s_X[b + HX];
        y[0] = s_Y[b];
        y[1] = s_Y[b + 1];
        y[2] = s_Y[b + HX + 1];
        y[3] = s_Y[b + HX];
    };
    auto elem_u = [&](int ex, int ey, T ux[4], T uy[4]) {
        const int b = ey * HX + ex;
        ux[0] = s_ux[b];
        ux[1] = s_ux[b + 1];
        ux[2] = s_ux[b + HX + 1];
        ux[3] = s_ux[b + HX];
        uy[0] = s_uy[b];
        uy[1] = s_uy[b + 1];
        uy[2] = s_uy[b + HX + 1];
        uy[3] = s_uy[b + HX];
    };

    // staged-node offset of local node n of an element, relative to its node 0
    auto corner = [](int n) { return n == 0 ? 0 : n == 1 ? 1 : n == 2 ? HX + 1 : HX; };
    // edge slot of local edge k of ring element (ie, je)
    auto edge_slot = [](int ie, int je, int k) {
        return k == 0 ? je * TXE + ie
             : k == 1 ? NH + je * (TXE + 1) + ie + 1
             : k == 2 ? (je + 1) * TXE + ie
                      : NH + je * (TXE + 1) + ie;
    };

    // ---- 3. element gradients and smoothed edge stresses -------------------
    // Element (ie, je) of the TXE x TYE ring around the owned nodes keeps its
    // gradients at the four edge midpoints in registers for the force phase.
    // Smoothed strain of an edge: eps_s = w_hi (B u)_hi + w_lo (B u)_lo over
    // its intact neighbours (lower element id first, w_j = A_j / (A_lo +
    // A_hi); w = 1 with one intact neighbour).  Stage A: the lower-id element
    // (local edges 1, 2) stores w_lo (B u)_lo, or (B u)_lo alone when the
    // other side is not intact; the higher-id element (edges 0, 3) keeps
    // (B u)_hi in registers.  Stage B: the higher-id element, when intact,
    // combines the two and stores the plane-stress sigma over the part;
    // otherwise the lower-id element turns its part into sigma.  Elements
    // one further out take part through the edge they share with the ring.
    const int ie = tid % TXE, je = tid / TXE;
    const int ex = ie + 1, ey = je + 1;
    const int e2 = ey * EX + ex;
    int sidx[4];  // edges of this element in local order (bottom, right, top, left)
    sidx[0] = je * TXE + ie;
    sidx[1] = NH + je * (TXE + 1) + ie + 1;
    sidx[2] = (je + 1) * TXE + ie;
    sidx[3] = NH + je * (TXE + 1) + ie;
    const uint8_t code = s_split[e2];
    auto nbr = [&](int e, int k) { return (k == 0) ? e - EX : (k == 1) ? e + 1 : (k == 2) ? e + EX : e - 1; };
    // stage A, lower-id element e (area A; SC: sub-cell area) at its edge k = 1 or 2
    auto lo_part = [&](int e, T A, int k, int sid, const T q[3]) {
        const int nb = nbr(e, k);
        if constexpr (SC) {
#pragma unroll
            for (int c = 0; c < 3; ++c) s_e[c * NS + sid] = q[c];
            s_e[3 * NS + sid] = A;
        } else if (s_split[nb] == 0) {
            T w0;
            if constexpr (UNI)
                w0 = kconst(p.lat)->w;
            else
                w0 = A / (A + s_area[nb]);
#pragma unroll
            for (int c = 0; c < 3; ++c) s_e[c * NS + sid] = w0 * q[c];
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) s_e[c * NS + sid] = q[c];
        }
    };
    // stage B, intact higher-id element e (area A; SC: sub-cell area) at its edge k = 0 or 3
    auto hi_sigma = [&](int e, T A, int k, int sid, const T q[3]) {
        const int nb = nbr(e, k);
        T eps[3], sg[3];
        if (s_split[nb] == 0) {
            if constexpr (SC) {
                const T Alo = s_e[3 * NS + sid];
                const T sum = Alo + A;
                const T w0 = Alo / sum, w1 = A / sum;
#pragma unroll
                for (int c = 0; c < 3; ++c) eps[c] = fmat(w1, q[c], w0 * s_e[c * NS + sid]);
            } else {
                T w1;
                if constexpr (UNI)
                    w1 = kconst(p.lat)->w;
                else
                    w1 = A / (s_area[nb] + A);
#pragma unroll
                for (int c = 0; c < 3; ++c) eps[c] = fmat(w1, q[c], s_e[c * NS + sid]);
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) eps[c] = q[c];
        }
        hooke(p, eps, sg);
#pragma unroll
        for (int c = 0; c < 3; ++c) s_e[c * NS + sid] = sg[c];
    };
    // stage B, lower-id element e at its edge k = 1 or 2 when the other side is not intact
    auto lo_sigma = [&](int e, int k, int sid) {
        if (s_split[nbr(e, k)] != 0) {
            T eps[3], sg[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) eps[c] = s_e[c * NS + sid];
            hooke(p, eps, sg);
#pragma unroll
            for (int c = 0; c < 3; ++c) s_e[c * NS + sid] = sg[c];
        }
    };
    // point rule: Q4 gradients at the edge midpoints; SC: sub-cell
    // gradients (gx[k][0..2], gy[k][0..2]) and areas at[k]
    T gx[4][4], gy[4][4], at[4];
    T qh0[3], qh3[3];
    T my_area;
    if constexpr (UNI)
        my_area = T(0);  // unused: the lattice weights and force factor are shared
    else
        my_area = s_area[e2];
    if (UNI && code == 0) {
        T ux[4], uy[4];
        elem_u(ex, ey, ux, uy);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T q[3];
            if constexpr (UNI) strain_lat_rt(p.lat, k, ux, uy, q);
            if (k == 0) {
                qh0[0] = q[0]; qh0[1] = q[1]; qh0[2] = q[2];
            } else if (k == 3) {
                qh3[0] = q[0]; qh3[1] = q[1]; qh3[2] = q[2];
            } else {
                lo_part(e2, my_area, k, sidx[k], q);
            }
        }
    } else if (!UNI && code == 0) {
        T x[4], y[4];
        elem_xy(ex, ey, x, y);
        T ux[4], uy[4];
        elem_u(ex, ey, ux, uy);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T q[3];
            if constexpr (SC) {
                switch (k) {
                    case 0: at[0] = subcell<0>(x, y, ux, uy, gx[0], gy[0], q); break;
                    case 1: at[1] = subcell<1>(x, y, ux, uy, gx[1], gy[1], q); break;
                    case 2: at[2] = subcell<2>(x, y, ux, uy, gx[2], gy[2], q); break;
                    default: at[3] = subcell<3>(x, y, ux, uy, gx[3], gy[3], q); break;
                }
            } else {
                q4_grad(x, y, k, gx[k], gy[k]);
                strain<4>(gx[k], gy[k], ux, uy, q);
            }
            if (k == 0) {
                qh0[0] = q[0]; qh0[1] = q[1]; qh0[2] = q[2];
            } else if (k == 3) {
                qh3[0] = q[0]; qh3[1] = q[1]; qh3[2] = q[2];
            } else {
                lo_part(e2, SC ? at[k] : my_area, k, sidx[k], q);
            }
        }
    }
    // Elements just outside the ring: wavefront g (g = 0..3) takes the row
    // below, the row above, the column left, the column right, so every
    // wavefront evaluates one edge type.  Below and left are the lower-id
    // side of the shared edge, above and right the higher-id side.
    static_assert(NT >= 256 && TXE <= 64 && TYE <= 64, "four wavefronts for the outer ring");
    const int og = tid >> 6, orr = tid & 63;
    int ore = 0, ork = 0, osid = 0;
    bool oin = false;
    T oq[3] = {T(0), T(0), T(0)};
    T oat = T(0);  // SC: the outer element's sub-cell area at the shared edge
    if (og < 4 && orr < ((og < 2) ? TXE : TYE)) {
        int rex, rey;
        if (og == 0) {  // below the ring: its top edge
            rex = orr + 1; rey = 0; ork = 2; osid = orr;
        } else if (og == 1) {  // above: bottom edge
            rex = orr + 1; rey = TYE + 1; ork = 0; osid = TYE * TXE + orr;
        } else if (og == 2) {  // left: right edge
            rex = 0; rey = orr + 1; ork = 1; osid = NH + orr * (TXE + 1);
        } else {  // right: left edge
            rex = TXE + 1; rey = orr + 1; ork = 3; osid = NH + orr * (TXE + 1) + TXE;
        }
        ore = rey * EX + rex;
        if (s_split[ore] == 0) {
            oin = true;
            T ux[4], uy[4];
            elem_u(rex, rey, ux, uy);
            if constexpr (UNI) {
                strain_lat_rt(p.lat, ork, ux, uy, oq);
                if (og == 0 || og == 2) lo_part(ore, T(0), ork, osid, oq);
            } else {
                T x[4], y[4], dx[4], dy[4];
                elem_xy(rex, rey, x, y);
                if constexpr (SC) {
                    oat = subcell_rt(x, y, ux, uy, ork, dx, dy, oq);
                } else {
                    q4_grad_rt(x, y, ork, dx, dy);
                    strain<4>(dx, dy, ux, uy, oq);
                }
                if (og == 0 || og == 2) lo_part(ore, SC ? oat : s_area[ore], ork, osid, oq);
            }
        }
    }
    __syncthreads();
    if (code == 0) {
        hi_sigma(e2, SC ? at[0] : my_area, 0, sidx[0], qh0);
        hi_sigma(e2, SC ? at[3] : my_area, 3, sidx[3], qh3);
        lo_sigma(e2, 1, sidx[1]);
        lo_sigma(e2, 2, sidx[2]);
    }
    if (oin && (og == 1 || og == 3)) {
        if constexpr (UNI)
            hi_sigma(ore, T(0), ork, osid, oq);
        else
            hi_sigma(ore, SC ? oat : s_area[ore], ork, osid, oq);
    }
    __syncthreads();

    // smoothed stress at edge slot sid
    auto edge_sigma = [&](int sid, T sg[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sg[c] = s_e[c * NS + sid];
    };

    // ---- 4. element forces, one thread per element of the tile ring ----
    // The general kernel computes them here, while the gradients are in
    // registers; the lattice kernel after the candidates (its gradients are
    // shared constants, so the forces need not stay live meanwhile).
    T fe[8];
    auto element_forces = [&]() {
#pragma unroll
    for (int c = 0; c < 8; ++c) fe[c] = T(0);
    if (SC && code == 0) {
        T bb[4][3], cb[4][3], sgk[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            edge_sigma(sidx[k], sgk[k]);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                bb[k][i] = gx[k][i];
                cb[k][i] = gy[k][i];
            }
        }
        subcell_force(bb, cb, at, sgk, fe);
    } else if (UNI && code == 0) {
        // the general loop below with the shared gradients; a vanishing
        // gradient leaves one product of each pair
        T sx[4], sy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T sg[3];
            edge_sigma(sidx[k], sg);
            const T s0 = sg[0], s1 = sg[1], s2 = sg[2];
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const T bx = kconst(p.lat)->B[k][n], by = kconst(p.lat)->B[k][4 + n];
                T tx, ty;
                if (lat_nzx(k, n) && lat_nzy(k, n)) {
                    tx = fmat(by, s2, bx * s0);
                    ty = fmat(bx, s2, by * s1);
                } else if (lat_nzx(k, n)) {
                    tx = bx * s0;
                    ty = bx * s2;
                } else {
                    tx = by * s2;
                    ty = by * s1;
                }
                if (k == 0) {
                    sx[n] = tx;
                    sy[n] = ty;
                } else {
                    sx[n] = sx[n] + tx;
                    sy[n] = sy[n] + ty;
                }
            }
        }
        const T c = kconst(p.lat)->c4;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            fe[2 * n] = c * sx[n];
            fe[2 * n + 1] = c * sy[n];
        }
    } else if (code == 0) {
        T sx[4], sy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T sg[3];
            edge_sigma(sidx[k], sg);
            const T s0 = sg[0], s1 = sg[1], s2 = sg[2];
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const T tx = fmat(gy[k][n], s2, gx[k][n] * s0);
                const T ty = fmat(gx[k][n], s2, gy[k][n] * s1);
                if (k == 0) {
                    sx[n] = tx;
                    sy[n] = ty;
                } else {
                    sx[n] = sx[n] + tx;
                    sy[n] = sy[n] + ty;
                }
            }
        }
        const T c = T(0.25) * my_area;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            fe[2 * n] = c * sx[n];
            fe[2 * n + 1] = c * sy[n];
        }
    }
    };
    if constexpr (!UNI) element_forces();

    // free-surface candidates of the elements this tile owns (node n0 owned),
    // compacted with wavefront ballots into s_cand
    // A screened step lists the candidates the screen skips too (smask):
    // they are not evaluated, only bounded (the judge below).
    const bool owned = ie >= 1 && je >= 1 && code == 0;
    unsigned fmask = 0, smask = 0;
    if (owned && tile_free) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (s_split[nbr(e2, k)] != 0) {
                if (((scr >> (8 * k)) & 0xFFu) != kScreenSkip)
                    fmask |= 1u << k;
                else
                    smask |= 1u << k;
            }
        if (p.sct) {  // single-tip mode: the tip is the only candidate
            const int32_t tip = s_tip;
            const int64_t ge = (int64_t)(j0 - 1 + je) * nx + (i0 - 1 + ie);
            fmask = (tip >= 0 && (tip >> 2) == ge) ? (fmask & (1u << (tip & 3))) : 0u;
            smask = 0;
        }
        if (!p.strip) smask = 0;
    }
    const unsigned cmask = fmask | smask;
    // split elements of the ring, listed by kind: a path between adjacent
    // edges leaves a 3-node piece (constant-strain triangle) and a 1-node
    // piece; a path between opposite edges leaves two 2-node pieces (bars).
    // Corner splits fill s_splitl from the front, through splits from the back.
    const bool is_split = (code & kSplitFlag) != 0;
    const bool is_thru = is_split && ((((code & 3) - ((code >> 2) & 3)) & 3) == 2);
    const bool is_corner = is_split && !is_thru;
    if (tile_free) {  // uniform over the workgroup
        const int lane = tid & 63, wave = tid >> 6;
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        uint64_t bal[4];
        int wtotal = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            bal[k] = __ballot((cmask >> k) & 1u);
            wtotal += __popcll(bal[k]);
        }
        const uint64_t bco = __ballot(is_corner), bth = __ballot(is_thru);
        if (lane == 0 && wtotal) s_wbase[wave] = atomicAdd(&s_ncand, wtotal);
        if (lane == 0 && bco) s_wbase2[wave] = atomicAdd(&s_ncorner, __popcll(bco));
        if (lane == 0 && bth) s_wbase3[wave] = atomicAdd(&s_nthru, __popcll(bth));
        __syncthreads();
        if (is_corner) s_splitl[s_wbase2[wave] + __popcll(bco & lt)] = (uint16_t)tid;
        if (is_thru) s_splitl[NT - 1 - (s_wbase3[wave] + __popcll(bth & lt))] = (uint16_t)tid;
        if (cmask) {
            int off = s_wbase[wave];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((cmask >> k) & 1u)
                    s_cand[off + __popcll(bal[k] & lt)] = (uint16_t)((tid << 2) | k | (((smask >> k) & 1u) << 15));
                off += __popcll(bal[k]);
            }
        }
    }
    const int ncand = s_ncand;
    if (ncand > 0) __syncthreads();  // uniform: the list is complete

    // ---- 5. energy release rate and element rule of the candidates ------
    // Four lanes per candidate: lane j < 3 evaluates G of the path to local
    // edge a+1+j, lane 0 of the quad applies the element rule to the three
    // values.  Node data are read from LDS at computed offsets, so no array
    // is indexed by a run-time value.
    if ((FRONT || NEAR) && p.fgrid)  // per-front pick over the whole GPU: the next step's table
        front_grid_clear(p.fgrid, (int)((base + k_rel) & 1), (int64_t)blockIdx.x * NT + tid, (int64_t)gridDim.x * NT);
    CandT<T> best;
    cand_none(best);
    for (int c0 = 0; c0 < ncand; c0 += NT / 4) {  // same trip count in every lane
        const int c = c0 + (tid >> 2), j = tid & 3;
        const bool live = c < ncand;
        T Gj = T(0), gc = T(0);
        bool H = false, skipped = false;
        int a = 0;
        int64_t ge = 0;
        if (live) {
            const unsigned ent = s_cand[c];
            skipped = (ent >> 15) != 0u;
            const int t = (int)(ent & 0x7FFFu) >> 2;
            a = (int)(ent & 3u);
            const int cie = t % TXE, cje = t / TXE;
            ge = (int64_t)(j0 - 1 + cje) * nx + (i0 - 1 + cie);
            gc = p.gc ? p.gc[ge] : p.gc_uniform;
            const int nb0 = (cje + 1) * HX + (cie + 1);
            const int o1 = nb0 + corner(a), o2 = nb0 + corner((a + 1) & 3);
            T X1, Y1, X2, Y2;
            node_xy(o1, X1, Y1);
            node_xy(o2, X2, Y2);
            const T ux1 = s_ux[o1], uy1 = s_uy[o1], ux2 = s_ux[o2], uy2 = s_uy[o2];
            const T dux = ux2 - ux1, duy = uy2 - uy1;
            const T x1 = X1 + ux1, y1 = Y1 + uy1;
            const T x2 = X2 + ux2, y2 = Y2 + uy2;
            const T lx = x2 - x1, ly = y2 - y1;
            const T Lx = X2 - X1, Ly = Y2 - Y1;
            H = (lx * lx + ly * ly) > (Lx * Lx + Ly * Ly);  // else G = 0 on all three paths
            if (skipped && H && j < 3) {
                // |G_k| = |delta . sigma_k n_k| / 2 = |(sigma_k delta) . n_k| / 2
                // <= |sigma_k delta| / 2 (sigma_k symmetric, n_k a unit vector):
                // lane j holds |sigma_k delta|^2 of its path's edge stress
                T sg[3];
                edge_sigma(edge_slot(cie, cje, (a + 1 + j) & 3), sg);
                const T tx = fmat(sg[2], duy, sg[0] * dux), ty = fmat(sg[1], duy, sg[2] * dux);
                Gj = fmat(ty, ty, tx * tx);
            } else if (H && j < 3) {
                const int k = (a + 1 + j) & 3;
                T sg[3], nxv, nyv, len;
                edge_sigma(edge_slot(cie, cje, k), sg);
                if constexpr (UNI) {
                    const int gq = (a * 3 + j) * 3;
                    const T *geo = &p.lat->geo[0][0][0];  // crack-path geometry (a, j, {nx, ny, L})
                    nxv = geo[gq];
                    nyv = geo[gq + 1];
                    len = geo[gq + 2];
                } else {
                    const int q0 = nb0 + corner(k), q1 = nb0 + corner((k + 1) & 3);
                    path_geom_pts(X1, Y1, X2, Y2, s_X[q0], s_Y[q0], s_X[q1], s_Y[q1], nxv, nyv, len);
                }
                const T spx = fmat(sg[2], nyv, sg[0] * nxv);
                const T spy = fmat(sg[1], nyv, sg[2] * nxv);
                Gj = T(0.5) * fmat(duy, spy, dux * spx);
            }
        }
        const int qb = tid & 60;  // lane of j = 0 in this quad
        const T G1 = __shfl(Gj, qb + 1, 64);
        const T G2 = __shfl(Gj, qb + 2, 64);
        if (live && H && j == 0 && skipped) {
            // the judge of a screened window: a skipped candidate whose bound
            // (max_k |sigma_k delta| / 2, compared squared, with a margin of
            // 1e-9 for rounding) reaches Gc might have been accepted, so the
            // window is replayed with the plain step
            const T f2 = G1 > G2 ? (G1 > Gj ? G1 : Gj) : (G2 > Gj ? G2 : Gj);
            if (T(0.25) * f2 > gc * gc * T(1.0 - 1e-9)) atomicOr(p.strip, 1u);
        }
        bool fr_app = false;  // per-front pick: an accepted candidate to append
        double fr_G = 0.0;
        int32_t fr_ak = 0;
        if (live && H && j == 0 && !skipped) {
            const T Gv[3] = {Gj, G1, G2};
            if constexpr (NEAR) near_candidate(p, base + k_rel, ge, a, Gv, gc);
            int jb = -1;
            T gb = T(0);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (Gv[q] > gc && (jb < 0 || Gv[q] > gb)) {
                    jb = q;
                    gb = Gv[q];
                }
            if (jb >= 0) {
                bool ok = true;
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if (q != jb && Gv[q] > gc && !(gb > p.gamma * (gb - Gv[q]))) ok = false;
                if (ok) cand_merge<NEAR>(best, gb, T(-1), gb, (int)ge, a, (a + 1 + jb) & 3);
                if ((FRONT || NEAR) && ok && p.front) {
                    fr_app = true;
                    fr_G = (double)gb;
                    fr_ak = (a << 2) | ((a + 1 + jb) & 3);
                }
            }
        }
        if ((FRONT || NEAR) && p.front) {  // uniform: the wave's accepted candidates, one atomic per wave
            const uint64_t fm = __ballot(fr_app);
            if (fm != 0ull) {
                const int lane = tid & 63, first = __ffsll((unsigned long long)fm) - 1;
                int slot0 = 0;
                if (lane == first) slot0 = (int)atomicAdd(p.fcount, (uint32_t)__popcll(fm));
                slot0 = __shfl(slot0, first, 64);
                if (fr_app) {
                    const uint32_t slot = (uint32_t)slot0 + (uint32_t)__popcll(fm & ((1ull << lane) - 1ull));
                    AccCand ac;
                    ac.G = fr_G;
                    ac.elem = (int32_t)ge;
                    ac.ak = fr_ak;
                    p.fcand[slot] = ac;
                    if ((FRONT || NEAR) && p.fgrid) {
                        // the pick over the whole GPU: tip point (midpoint of
                        // the tip edge) into the step's bucket table
                        const int t = (int)(s_cand[c] & 0x7FFFu) >> 2;
                        const int nb0 = (t / TXE + 1) * HX + (t % TXE + 1);
                        T X1, Y1, X2, Y2;
                        node_xy(nb0 + corner(a), X1, Y1);
                        node_xy(nb0 + corner((a + 1) & 3), X2, Y2);
                        const double2 m = make_double2(0.5 * ((double)X1 + (double)X2), 0.5 * ((double)Y1 + (double)Y2));
                        p.fmid[slot] = m;
                        front_grid_insert(p.fgrid + ((base + k_rel) & 1) * kFrontGridTable, p.fcell, p.fsorted,
                                          (int32_t)slot, m);
                    }
                }
            }
        }
    }
    if (ncand > 0) cand_block_reduce<NT, NEAR>(best, s_red);  // uniform branch
    if constexpr (!UNI) {
        // the general kernel's owned-node loads (inline: a lambda call here
        // costs it registers); the latency hides behind the split pieces
        if (on_valid) {
            n_minv = p.minv[on_n];
            n_vx = p.vx[on_n];
            n_vy = p.vy[on_n];
            const int pidx = perimeter_index(on_i, on_j, nx, ny);
            if (pidx >= 0) {
                n_fex = p.fext_p[2 * pidx];
                n_fey = p.fext_p[2 * pidx + 1];
                n_mask = p.vmask_p[pidx];
                n_v0x = p.v0_p[2 * pidx];
                n_v0y = p.v0_p[2 * pidx + 1];
            }
        }
    }
    if constexpr (UNI) element_forces();
    __syncthreads();  // strain slots are no longer read: reuse them for forces

    // ---- 6. colour-ordered gather to the owned nodes --------------------
    // f_int at a node = sum over its elements in colour order 0..3 (colour of
    // element (i, j) = (i mod 2) + 2 (j mod 2)), as a coloured scatter
    // would add them.
    if (!is_split) {
#pragma unroll
        for (int c = 0; c < 8; ++c) s_fe[c * NT + tid] = fe[c];
    }
    // Split elements of the tile ring.  Work items: one constant-strain
    // triangle per corner split, then one bar per piece of a through split,
    // so that a wavefront mostly runs one kind.  Each piece spans the crack
    // segment between the midpoints of the entry and exit edges and carries
    // its polygon area; the 1-node piece of a corner split has no stiffness.
    const int ncorner = s_ncorner, nitems = ncorner + 2 * s_nthru;
    for (int it = tid; it < nitems; it += NT) {
        const bool cst = it < ncorner;
        const int t = cst ? s_splitl[it] : s_splitl[NT - 1 - ((it - ncorner) >> 1)];
        const int sx_ = t % TXE + 1, sy_ = t / TXE + 1;
        const uint8_t scode = s_split[sy_ * EX + sx_];
        const int ea = (scode >> 2) & 3, eb = scode & 3;
        const int nb0 = sy_ * HX + sx_;
        // piece from edge F (first node F+1) to edge T, counter-clockwise
        const int F = cst ? ((((eb - ea) & 3) == 3) ? ea : eb) : (((it - ncorner) & 1) ? eb : ea);
        const int n0 = F, n1 = (F + 1) & 3, n2 = (F + 2) & 3, n3 = (F + 3) & 3;
        const int o0 = nb0 + corner(n0), o1 = nb0 + corner(n1), o2 = nb0 + corner(n2), o3 = nb0 + corner(n3);
        T x0, x1, x2, x3, y0, y1, y2, y3;
        node_xy(o0, x0, y0);
        node_xy(o1, x1, y1);
        node_xy(o2, x2, y2);
        node_xy(o3, x3, y3);
        const T gx = T(0.5) * (x0 + x1), gy = T(0.5) * (y0 + y1);  // midpoint of edge F
        if (cst) {
            // polygon: mid(F), n1, n2, n3, mid(F+3); shoelace fanned from mid(F)
            const T hx = T(0.5) * (x3 + x0), hy = T(0.5) * (y3 + y0);
            T sa = T(0);
            sa += (x1 - gx) * (y2 - gy) - (x2 - gx) * (y1 - gy);
            sa += (x2 - gx) * (y3 - gy) - (x3 - gx) * (y2 - gy);
            sa += (x3 - gx) * (hy - gy) - (hx - gx) * (y3 - gy);
            const T Ap = T(0.5) * sa;
            const T twoA = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1);
            const T inv = T(1) / twoA;
            const T bb[3] = {(y2 - y3) * inv, (y3 - y1) * inv, (y1 - y2) * inv};
            const T cc[3] = {(x3 - x2) * inv, (x1 - x3) * inv, (x2 - x1) * inv};
            const T pu[3] = {s_ux[o1], s_ux[o2], s_ux[o3]};
            const T pv[3] = {s_uy[o1], s_uy[o2], s_uy[o3]};
            T eps[3], sg[3];
            strain<3>(bb, cc, pu, pv, eps);
            hooke(p, eps, sg);
            const int nn[3] = {n1, n2, n3};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T tx = fmat(cc[i], sg[2], bb[i] * sg[0]);
                const T ty = fmat(bb[i], sg[2], cc[i] * sg[1]);
                s_fe[(2 * nn[i]) * NT + t] = Ap * tx;
                s_fe[(2 * nn[i] + 1) * NT + t] = Ap * ty;
            }
            s_fe[(2 * n0) * NT + t] = T(0);
            s_fe[(2 * n0 + 1) * NT + t] = T(0);
        } else {
            // polygon: mid(F), n1, n2, mid(F+2); bar along the uncut edge n1-n2
            const T hx = T(0.5) * (x2 + x3), hy = T(0.5) * (y2 + y3);
            T sa = T(0);
            sa += (x1 - gx) * (y2 - gy) - (x2 - gx) * (y1 - gy);
            sa += (x2 - gx) * (hy - gy) - (hx - gx) * (y2 - gy);
            const T Ap = T(0.5) * sa;
            const T dx = x2 - x1, dy = y2 - y1;
            const T L2 = dx * dx + dy * dy;
            const T dux = s_ux[o2] - s_ux[o1], duy = s_uy[o2] - s_uy[o1];
            const T st = (dx * dux + dy * duy) / L2;
            const T stress = p.E * st;
            const T coef = Ap * stress / L2;
            s_fe[(2 * n2) * NT + t] = coef * dx;
            s_fe[(2 * n2 + 1) * NT + t] = coef * dy;
            s_fe[(2 * n1) * NT + t] = -(coef * dx);
            s_fe[(2 * n1 + 1) * NT + t] = -(coef * dy);
        }
    }
    __syncthreads();
    if (on_valid) {
        T fx = T(0), fy = T(0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int dx = ((c & 1) - (i0 - 1 + on_l)) & 1;
            const int dy = ((c >> 1) - (j0 - 1 + on_m)) & 1;
            const int eie = on_l + dx, eje = on_m + dy;  // ring element holding colour c
            if (s_split[(eje + 1) * EX + eie + 1] == kAbsent) continue;
            const int ln = (1 - dx) + 2 * (1 - dy);   // (1,0)->1, (0,0)->0, (1,1)->3, (0,1)->2
            const int n = (ln == 0) ? 0 : (ln == 1) ? 1 : (ln == 3) ? 2 : 3;
            const int t = eje * TXE + eie;
            fx = fx + s_fe[(2 * n) * NT + t];
            fy = fy + s_fe[(2 * n + 1) * NT + t];
        }

        // ---- 7. central-difference update of the owned node --------------
        if constexpr (BATCHED) {
            // the output pointers read from the view again (as for the
            // publication below)
            const StepParamsT<T> *v2 = vsrc;
            int par2 = par0 + k_rel;
            asm volatile("" : "+s"(v2), "+s"(par2));
            const __attribute__((address_space(4))) StepParamsT<T> *w = kconst(v2);
            p.vx = w->vx;
            p.vy = w->vy;
            ux_n = (par2 & 1) ? w->ux0 : w->ux1;
            uy_n = (par2 & 1) ? w->uy0 : w->uy1;
        }
        const int64_t kabs = base + k_rel;
        const int hidx = (on_m + 2) * HX + (on_l + 2);
        const T phi = s_phi;
        T ax = (phi * n_fex - fx) * n_minv;
        T ay = (phi * n_fey - fy) * n_minv;
        if (n_mask & 1u) ax = T(0);
        if (n_mask & 2u) ay = T(0);
        const T dtv = (kabs == 0) ? T(0.5) * p.dts : p.dts;
        const double th = ((double)kabs + 0.5) * p.dt;
        T vx = n_vx + dtv * ax;
        T vy = n_vy + dtv * ay;
        if (n_mask & 1u) vx = prescribed(n_v0x, th, p.t_ramp);
        if (n_mask & 2u) vy = prescribed(n_v0y, th, p.t_ramp);
        p.vx[on_n] = vx;
        p.vy[on_n] = vy;
        ux_n[on_n] = s_ux[hidx] + p.dts * vx;
        uy_n[on_n] = s_uy[hidx] + p.dts * vy;
    }

    // ---- 8. publish the workgroup's best candidate -----------------------
    // Read by the next step after the kernel boundary; no fence here (a
    // device-scope release would write back the whole L2 of the XCD).
    if (tid == 0 && best.G >= T(0) && !p.front) {
        if constexpr (BATCHED) {
            // a batch reads these from the view again (the pointer made
            // opaque, so that the loads are not merged with the ones at the
            // start): scalar registers are short, and held across the step
            // these would be spilled
            const StepParamsT<T> *v2 = vsrc;
            asm volatile("" : "+s"(v2));
            const __attribute__((address_space(4))) StepParamsT<T> *w = kconst(v2);
            p.ctl = w->ctl;
            p.slots = w->slots;
            p.nwg = w->nwg;
        }
        const uint32_t slot = atomicAdd(&p.ctl->nslots[set_w], 1u);
        Slot sl;
        sl.G = (double)best.G;
        sl.Gmin = (double)best.Gmin;
        sl.G2 = (double)best.G2;
        sl.elem = best.e;
        sl.a = best.a;
        sl.k = best.k;
        sl.pad = 0;
        p.slots[(size_t)set_w * p.nwg + slot] = sl;
    }
}

// Close a segment of n steps: take the pick of its last step, clear every
// slot set and advance the step counter.
constexpr int kCommitThreads = 256;

// One workgroup per specimen.
template <class T, bool BATCHED>
__global__ __launch_bounds__(kCommitThreads) void k_commit(StepParamsT<T> p0, const StepParamsT<T> *views, int n) {
    __shared__ CandT<T> s_red[kCommitThreads / 64];
    StepParamsT<T> p;
    if constexpr (BATCHED) {
        load_view(p, views + blockIdx.x);
    }
    else
        p = p0;
    const int set = (n + 2) % 3;
    const CandT<T> g = reduce_slots<kCommitThreads, true>(p, set, p.ctl->nslots[set], s_red);
    if (threadIdx.x != 0) return;
    const int64_t base = p.ctl->base;
    const bool acc = n > 0 && pick_accepted(p, g);
    if (n > 0 && p.near) near_pick(p, base + n - 1, g);
    if (p.sct && n > 0) {
        // the tip at the start of step base + n goes where that step reads the
        // previous step's tip
        const bool odd = ((base + n - 1) & 1) != 0;
        const int32_t t = acc ? tip_after(p, g) : (odd ? p.ctl->tip1 : p.ctl->tip0);
        if (odd)
            p.ctl->tip1 = t;
        else
            p.ctl->tip0 = t;
    }
    if (acc) apply_split(p, g, base + n - 1);
    p.ctl->nslots[0] = 0;
    p.ctl->nslots[1] = 0;
    p.ctl->nslots[2] = 0;
    p.ctl->base = base + n;
}

TileShape tile_shape(int tile) {
    switch (tile) {
        case 1: return {16, 16};
        case 2: return {32, 8};
        default: return {32, 16};
    }
}

// Per-front pick of a plain Q4 model (one workgroup), after k_step.
constexpr int kFrontThreads = 1024;

struct Q4Geom {
    int nx;
    const double *X, *Y;
    __device__ void nodes(int e, int64_t nd[4]) const {
        const int64_t i = e % nx, j = e / nx;
        const int64_t n0 = j * (nx + 1) + i;
        nd[0] = n0;
        nd[1] = n0 + 1;
        nd[2] = n0 + nx + 2;
        nd[3] = n0 + nx + 1;
    }
    __device__ double2 tip(int e, int a) const {
        int64_t nd[4];
        nodes(e, nd);
        const int64_t pa = a == 0 ? nd[0] : a == 1 ? nd[1] : a == 2 ? nd[2] : nd[3];
        const int64_t pb = a == 0 ? nd[1] : a == 1 ? nd[2] : a == 2 ? nd[3] : nd[0];
        return make_double2(0.5 * (X[pa] + X[pb]), 0.5 * (Y[pa] + Y[pb]));
    }
    __device__ double path_len(int e, int a, int k) const {
        int64_t nd[4];
        nodes(e, nd);
        double x[4], y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            x[q] = X[nd[q]];
            y[q] = Y[nd[q]];
        }
        double cx, cy, L;
        dev::path_geom(x, y, a, k, cx, cy, L);
        return L;
    }
};

__host__ __device__ inline FrontView q4_front_view(const StepParams &p) {
    FrontView v;
    v.cand = p.fcand;
    v.count = p.fcount;
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
    v.gc_uniform = p.gc_uniform;
    v.gamma = p.gamma;
    v.rho2 = p.front_r2;
    return v;
}

__host__ __device__ inline Q4Geom q4_geom(const StepParams &p) {
    Q4Geom g;
    g.nx = p.nx;
    g.X = p.X;
    g.Y = p.Y;
    return g;
}

__global__ __launch_bounds__(kFrontThreads) void k_front(StepParams p, int k_rel) {
    front_pick_block<kFrontThreads>(q4_front_view(p), q4_geom(p), k_rel);
}

static int32_t env_limit(const char *name, long lo, long hi, long dflt) {
    const char *e = std::getenv(name);
    if (!e || !*e) return (int32_t)dflt;
    return (int32_t)std::min<long>(std::max<long>(std::strtol(e, nullptr, 10), lo), hi);
}

void front_close_limits(int32_t *sort_lds_max, int32_t *rank_max) {
    *sort_lds_max = env_limit("MCT_FRONT_SORT_LDS_MAX", 2, kFrontSortMax, kFrontSortMax);
    *rank_max = env_limit("MCT_FRONT_RANK_MAX", 0, kFrontCountMax, kFrontCountMax);
}

hipError_t front_grid_reset(int32_t *tables, hipStream_t s) {
    int32_t sort_max, rank_max;
    front_close_limits(&sort_max, &rank_max);
    for (int t = 0; t < 2; ++t) {
        int32_t *tb = tables + t * kFrontGridTable;
        hipError_t e = hipMemsetAsync(tb, 0, sizeof(int32_t) * kFrontGridTable, s);
        if (e == hipSuccess) e = hipMemsetAsync(tb + kFrontGridHead, 0xff, sizeof(int32_t) * kFrontGridBuckets, s);
        if (e == hipSuccess) e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(tb + kFrontGridSortMax), sort_max, 1, s);
        if (e == hipSuccess) e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(tb + kFrontGridRankMax), rank_max, 1, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The per-front pick after the step kernel: over the whole GPU when the
// model has its bucket table, else one workgroup.
static hipError_t launch_front(const StepParams &p, int k_rel, hipStream_t s) {
    if (p.fgrid) return launch_front_grid(q4_front_view(p), q4_geom(p), p.fgrid, k_rel, true, s);
    k_front<<<1, kFrontThreads, 0, s>>>(p, k_rel);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Uniform-lattice check: every element's gradients at its four edge
// midpoints, its area and its twelve crack-path normals and lengths, as the
// general step computes them, compared bit for bit with element 0's.
// ------------------------------------------------------------------------
namespace {

__device__ void lattice_of(const StepParams &p, int64_t e, LatticeConst &L) {
    const int64_t i = e % p.nx, j = e / p.nx;
    const int64_t n0 = j * (p.nx + 1) + i;
    const int64_t nd[4] = {n0, n0 + 1, n0 + p.nx + 2, n0 + p.nx + 1};
    double x[4], y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        x[q] = p.X[nd[q]];
        y[q] = p.Y[nd[q]];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) q4_grad(x, y, k, &L.B[k][0], &L.B[k][4]);
    const double A = p.area[e];
    L.w = A / (A + A);
    L.c4 = 0.25 * A;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
            path_geom(x, y, a, (a + 1 + jj) & 3, L.geo[a][jj][0], L.geo[a][jj][1], L.geo[a][jj][2]);
}

__global__ void k_lattice_ref(StepParams p, LatticeConst *ref, uint32_t *flag) {
    LatticeConst L;
    lattice_of(p, 0, L);
    *ref = L;
    uint32_t f = 0;
    for (int k = 0; k < 4; ++k)
        for (int n = 0; n < 4; ++n) {
            if (!lat_nzx(k, n) && L.B[k][n] != 0.0) f |= 2u;
            if (!lat_nzy(k, n) && L.B[k][4 + n] != 0.0) f |= 2u;
        }
    *flag = f;
}

__global__ __launch_bounds__(256) void k_lattice_check(StepParams p, const LatticeConst *ref, uint32_t *flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ne = (int64_t)p.nx * p.ny;
    bool diff = false;
    if (e < ne) {
        LatticeConst L;
        lattice_of(p, e, L);
        const unsigned long long *a = reinterpret_cast<const unsigned long long *>(&L);
        const unsigned long long *b = reinterpret_cast<const unsigned long long *>(ref);
        for (size_t q = 0; q < sizeof(LatticeConst) / 8; ++q) diff = diff || a[q] != b[q];
        diff = diff || __double_as_longlong(p.area[e]) != __double_as_longlong(p.area[0]);
    }
    if (__ballot(diff) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

}  // namespace

hipError_t launch_lattice_check(const StepParams &p, LatticeConst *ref, uint32_t *flag, hipStream_t s) {
    (void)hipGetLastError();
    const int64_t ne = (int64_t)p.nx * p.ny;
    k_lattice_ref<<<1, 1, 0, s>>>(p, ref, flag);
    k_lattice_check<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(p, ref, flag);
    return hipGetLastError();
}

hipError_t launch_step(int tile, const Launch &L, int k_rel, int par0, hipStream_t s) {
    (void)hipGetLastError();  // report only this launch's error below
    if (L.f32 && L.p0f.near) {
        const StepParamsF &p = L.p0f;
        if (p.subcell)
            k_step<float, 16, 16, false, true, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
        else
            k_step<float, 16, 16, false, false, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
        return hipGetLastError();
    }
    if (!L.f32 && !L.batched && L.p0.near) {
        const StepParams &p = L.p0;
        if (L.uni)
            k_step<double, 16, 16, false, false, true, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
        else if (p.subcell)
            k_step<double, 16, 16, false, true, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
        else
            k_step<double, 16, 16, false, false, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
        if (p.front) return launch_front(p, k_rel, s);
        return hipGetLastError();
    }
    if (!L.f32 && !L.batched && L.p0.front) {
        // per-front pick: the step kernels list every accepted candidate (and
        // fill the bucket table of the pick over the whole GPU)
        const StepParams &p = L.p0;
#define KSTEP_FRONT(TX_, TY_, NT_, SC_, UNI_) \
    k_step<double, TX_, TY_, false, SC_, UNI_, false, true><<<p.nwg, NT_, 0, s>>>(p, nullptr, nullptr, k_rel, par0)
        switch (tile) {
            case 1:
                if (L.uni) KSTEP_FRONT(16, 16, 256, false, true);
                else if (p.subcell) KSTEP_FRONT(16, 16, 256, true, false);
                else KSTEP_FRONT(16, 16, 256, false, false);
                break;
            case 2:
                if (L.uni) KSTEP_FRONT(32, 8, 256, false, true);
                else if (p.subcell) KSTEP_FRONT(32, 8, 256, true, false);
                else KSTEP_FRONT(32, 8, 256, false, false);
                break;
            default:
                if (L.uni) KSTEP_FRONT(32, 16, 512, false, true);
                else if (p.subcell) KSTEP_FRONT(32, 16, 512, true, false);
                else KSTEP_FRONT(32, 16, 512, false, false);
                break;
        }
#undef KSTEP_FRONT
        return launch_front(p, k_rel, s);
    }
    if (L.f32) {
        // binary32 step: plain models with the point rule or sub-cell
        // smoothing and the global or single-tip pick
        const StepParamsF &p = L.p0f;
        switch (tile) {
            case 1:
                if (p.subcell)
                    k_step<float, 16, 16, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                else
                    k_step<float, 16, 16, false><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                break;
            case 2:
                if (p.subcell)
                    k_step<float, 32, 8, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                else
                    k_step<float, 32, 8, false><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                break;
            default:
                if (p.subcell)
                    k_step<float, 32, 16, false, true><<<p.nwg, 512, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                else
                    k_step<float, 32, 16, false><<<p.nwg, 512, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                break;
        }
        return hipGetLastError();
    }
    const StepParams &p = L.p0;
    if (L.uni) {
        // uniform lattices: binary64 point rule (batched, or plain without the
        // per-front pick's extra launch below)
        if (L.batched) {
            switch (tile) {
                case 1:
                    k_step<double, 16, 16, true, false, true><<<L.nunits, 256, 0, s>>>(p, L.views, L.units, k_rel, par0);
                    break;
                case 2:
                    k_step<double, 32, 8, true, false, true><<<L.nunits, 256, 0, s>>>(p, L.views, L.units, k_rel, par0);
                    break;
                default:
                    k_step<double, 32, 16, true, false, true><<<L.nunits, 512, 0, s>>>(p, L.views, L.units, k_rel, par0);
                    break;
            }
        } else {
            switch (tile) {
                case 1:
                    k_step<double, 16, 16, false, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                    break;
                case 2:
                    k_step<double, 32, 8, false, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                    break;
                default:
                    k_step<double, 32, 16, false, false, true><<<p.nwg, 512, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                    break;
            }
            if (p.front) return launch_front(p, k_rel, s);
        }
        return hipGetLastError();
    }
    if (L.batched) {
        switch (tile) {
            case 1: k_step<double, 16, 16, true><<<L.nunits, 256, 0, s>>>(p, L.views, L.units, k_rel, par0); break;
            case 2: k_step<double, 32, 8, true><<<L.nunits, 256, 0, s>>>(p, L.views, L.units, k_rel, par0); break;
            default:
                k_step<double, 32, 16, true><<<L.nunits, 512, 0, s>>>(p, L.views, L.units, k_rel, par0);
                break;
        }
    } else {
        switch (tile) {
            case 1:
                if (p.subcell)
                    k_step<double, 16, 16, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                else
                    k_step<double, 16, 16, false><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                break;
            case 2:
                if (p.subcell)
                    k_step<double, 32, 8, false, true><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                else
                    k_step<double, 32, 8, false><<<p.nwg, 256, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                break;
            default:
                if (p.subcell)
                    k_step<double, 32, 16, false, true><<<p.nwg, 512, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                else
                    k_step<double, 32, 16, false><<<p.nwg, 512, 0, s>>>(p, nullptr, nullptr, k_rel, par0);
                break;
        }
        if (p.front) return launch_front(p, k_rel, s);
    }
    return hipGetLastError();
}

hipError_t launch_commit(const Launch &L, int n, hipStream_t s) {
    (void)hipGetLastError();
    if (L.f32)
        k_commit<float, false><<<1, kCommitThreads, 0, s>>>(L.p0f, nullptr, n);
    else if (L.batched)
        k_commit<double, true><<<L.nspec, kCommitThreads, 0, s>>>(L.p0, L.views, n);
    else
        k_commit<double, false><<<1, kCommitThreads, 0, s>>>(L.p0, nullptr, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Crack-surface tips: interior edges with exactly one intact neighbour.
// Three passes give an order-preserving compaction (per-block counts with
// ballots, a scan of the block counts, an in-order write).
// ------------------------------------------------------------------------
namespace {
using namespace dev;
constexpr int kTipBlock = 256;

__device__ __forceinline__ bool is_tip(const EdgeInfo &ei, const uint8_t *split) {
    if (ei.e0 < 0 || ei.e1 < 0) return false;
    return ((split[ei.e0] == 0) + (split[ei.e1] == 0)) == 1;
}

__global__ __launch_bounds__(kTipBlock) void k_tips_count(int nx, int ny, int64_t ns, const uint8_t *split,
                                                          int32_t *counts) {
    __shared__ int s_w[kTipBlock / 64];
    const int64_t s = (int64_t)blockIdx.x * kTipBlock + threadIdx.x;
    bool t = false;
    if (s < ns) t = is_tip(edge_info(s, nx, ny), split);
    const uint64_t b = __ballot(t);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int w = 0; w < kTipBlock / 64; ++w) c += s_w[w];
        counts[blockIdx.x] = c;
    }
}

__global__ __launch_bounds__(1024) void k_tips_scan(int32_t *counts, int nblocks, int32_t *total) {
    // exclusive scan in place, one workgroup, sequential chunks
    __shared__ int s_v[1024];
    __shared__ int s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < nblocks; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = (i < nblocks) ? counts[i] : 0;
        s_v[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = (threadIdx.x >= off) ? s_v[threadIdx.x - off] : 0;
            __syncthreads();
            s_v[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nblocks) counts[i] = s_carry + s_v[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += s_v[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = s_carry;
}

__global__ __launch_bounds__(kTipBlock) void k_tips_write(int nx, int ny, int64_t ns, const double *X,
                                                          const double *Y, const uint8_t *split,
                                                          const int32_t *offsets, int32_t *edge_out,
                                                          double *xy_out, int64_t cap) {
    __shared__ int s_w[kTipBlock / 64];
    const int64_t s = (int64_t)blockIdx.x * kTipBlock + threadIdx.x;
    EdgeInfo ei{0, 0, -1, -1};
    bool t = false;
    if (s < ns) {
        ei = edge_info(s, nx, ny);
        t = is_tip(ei, split);
    }
    const uint64_t b = __ballot(t);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_w[wave] = __popcll(b);
    __syncthreads();
    if (t) {
        int off = offsets[blockIdx.x];
        for (int w = 0; w < wave; ++w) off += s_w[w];
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        off += __popcll(b & lt);
        if (off < cap) {  // the caller's capacity: the count reports the rest
            edge_out[off] = (int32_t)s;
            xy_out[2 * off] = 0.5 * (X[ei.lo] + X[ei.hi]);
            xy_out[2 * off + 1] = 0.5 * (Y[ei.lo] + Y[ei.hi]);
        }
    }
}
}  // namespace

// Crack-path geometry of a list of elements (36 values each: for tip edge a
// and path j (exit edge a+1+j): normal x, normal y, length), evaluated with
// the device function the step uses.
__global__ void k_path_geometry(StepParams p, int n, const int32_t *elem, double *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t e = elem[t];
    const int64_t i = e % p.nx, j = e / p.nx;
    const int64_t n0 = j * (p.nx + 1) + i;
    const int64_t nd[4] = {n0, n0 + 1, n0 + p.nx + 2, n0 + p.nx + 1};
    double x[4], y[4];
    for (int q = 0; q < 4; ++q) {
        x[q] = p.X[nd[q]];
        y[q] = p.Y[nd[q]];
    }
    for (int a = 0; a < 4; ++a)
        for (int jj = 0; jj < 3; ++jj) {
            double cx, cy, L;
            path_geom(x, y, a, (a + 1 + jj) & 3, cx, cy, L);
            double *o = out + (int64_t)t * 36 + a * 9 + 3 * jj;
            o[0] = cx;
            o[1] = cy;
            o[2] = L;
        }
}

hipError_t launch_path_geometry(const StepParams &p, int n, const int32_t *elem, double *out, hipStream_t s) {
    (void)hipGetLastError();
    if (n > 0) k_path_geometry<<<(n + 255) / 256, 256, 0, s>>>(p, n, elem, out);
    return hipGetLastError();
}

int tips_nblocks(int64_t n_edges) { return (int)((n_edges + kTipBlock - 1) / kTipBlock); }

// Scratch of the tip query that allocates nothing (mct_get_tips_noalloc):
// the per-block counts of the compaction, for up to kTipScratchBlocks
// blocks of kTipBlock edges.  Each GPU holds its own copy for the life of
// the process; calls on one GPU share it (and race if they overlap).
__device__ __align__(256) int32_t scratch[kTipScratchBlocks];

hipError_t tips_scratch(int32_t **out) {
    static std::mutex mu;
    static int32_t *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        // the array's address on the current device (the host-side name is
        // not a device address)
        e = hipGetSymbolAddress((void **)&ptr[dev], HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            ptr[dev] = nullptr;
            return e;
        }
    }
    *out = ptr[dev];
    return hipSuccess;
}

hipError_t launch_tips(int32_t nx, int32_t ny, const double *X, const double *Y, const uint8_t *split,
                       int32_t *block_counts, int32_t *nblocks_out, int32_t *edge_out, double *xy_out,
                       int32_t *count_out, int64_t cap, hipStream_t s) {
    const int64_t ns = 2 * (int64_t)nx * ny + nx + ny;
    const int nb = tips_nblocks(ns);
    *nblocks_out = nb;
    (void)hipGetLastError();
    k_tips_count<<<nb, kTipBlock, 0, s>>>(nx, ny, ns, split, block_counts);
    k_tips_scan<<<1, 1024, 0, s>>>(block_counts, nb, count_out);
    if (edge_out)
        k_tips_write<<<nb, kTipBlock, 0, s>>>(nx, ny, ns, X, Y, split, block_counts, edge_out, xy_out, cap);
    return hipGetLastError();
}

}  // namespace mct
