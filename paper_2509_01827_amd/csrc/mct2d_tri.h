// Internal declarations of the CST (unstructured triangle mesh) path of the
// MCT-2D-CEM library: the device view of one mesh, its control block and
// the kernel launchers (mct2d_tri.hip), used by the host side
// (mct2d_tri_host.cpp).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mct2d_impl.h"

namespace mct {
namespace tri {

// One accepted candidate of a step (the layout of the per-front pick's).
using Cand = AccCand;

// Device-resident control block.
struct Ctl {
    int64_t base;      // steps completed before the running segment
    int64_t nsplit;    // splits made by the tracking
    double Ud;         // sum of Gc * crack-path length
    int32_t nacc;      // accepted candidates appended by the running step
    int32_t tip;       // single-tip tracking: element * 4 + local edge, or -1
    int32_t overflow;  // 1 when a split could not be logged
    int32_t pad;
};
static_assert(sizeof(Ctl) == 40, "Ctl layout");

constexpr int kPatchMaxNodes = 256;  // fused step: one node per thread of its workgroup
constexpr uint32_t kNoSlot = 1023;       // patch neighbour slot: none
constexpr int kPatchLocalNodes = 384;    // triangles: nodes of a patch staged in LDS
constexpr int32_t kOwned = 1 << 30;    // patch element flag: evaluate its candidates here

// Node flags (one byte per node).
constexpr uint8_t kFixX = 1, kFixY = 2, kLoaded = 4;

// The kernels' view of one unstructured mesh: constant-strain triangles
// (nv = 3) or bilinear quadrilaterals (nv = 4).  Nodal vectors are
// interleaved (x, y) pairs so that one 16-byte load fetches both components.
struct Params {
    int32_t nn, ne;
    int32_t log_cap;
    int32_t sct;     // 1: single crack-tip tracking
    int32_t ncurve;  // traction load curve points (0: constant tractions)
    int32_t nv;      // nodes (and edges) per element: 3 or 4
    const int4 *conn;    // per element: nodes n0 n1 n2 (n3) (CCW); triangles: .w = the
                         // neighbour's node off the shared edge 0 (-1: none)
    const int4 *nbr;     // per element: neighbour across local edge k = 0, 1, 2 (-1: none);
                         // .w: local index of that edge in the neighbour, 2 bits per k
    const int2 *opp;     // per triangle: the neighbours' nodes off the shared edges 1, 2 (-1: none)
    // quadrilaterals: neighbour across local edge k = 0..3 (-1: none), the
    // local index of that edge in the neighbour (2 bits per k), and the
    // neighbour's two nodes off the shared edge (its local nodes loc + 2 and
    // loc + 3; the shared edge runs backwards in the neighbour)
    const int4 *q_nbr;
    const uint8_t *q_loc;
    const int4 *q_oa, *q_ob;
    const double2 *xy;   // reference coordinates
    double2 *u0, *u1;    // displacement u^k in buffer k & 1 (ping-pong: a step reads one, writes the other)
    double2 *v;          // velocity
    const double *minv;
    const double2 *fext; // read where kLoaded
    const double2 *v0;   // read where kFixX / kFixY
    const uint8_t *nflag;
    uint8_t *split;      // 0 intact, else kSplitFlag | entry << 2 | exit
    const double *gc;    // per element
    double2 *fe;         // 3 ne: force on local node n of element e at [n ne + e]
    const int32_t *csr_off;  // nn + 1
    const int32_t *csr_ent;  // force slot n * ne + e, by element colour per node
    const int32_t *nlist;    // the same lists padded to nlist_w slots (-1), node-major [nn][w];
    int32_t nlist_w;         //   null when a node touches more than 16 elements (CSR is used)
    // fused step (one workgroup per patch of patch_nodes consecutive nodes):
    // the patch's elements (id | kOwned for the one patch that evaluates
    // their candidates) and per owned node its force slots in the patch's LDS
    // (3 slot + local node, 0xffff = none), node-major, nlist_w per node
    int32_t patch_emax;      // largest patch element count (0: fused step off)
    int32_t patch_nodes;     // 64, 128, 256 or the found size (at most kPatchMaxNodes)
    const int32_t *patch_off;
    const int32_t *patch_elem;
    const uint16_t *patch_slots;
    // the ring of each patch (elements outside it next to one of its
    // elements; ids ascending, entries patch_ring_off[b] ..) and per patch
    // element its neighbours' strain slots in the patch's LDS (the patch's
    // elements first, then its ring): .x = slot of the neighbour across
    // local edge k = 0..2 in bits 10k .. 10k + 9, .y bits 0..9 that across
    // edge 3 (kNoSlot: none); .y bit 10 + k set when the element's id is
    // below that neighbour's, .y bits 16 + 2k, 17 + 2k the shared edge's
    // local index in the neighbour
    const int32_t *patch_ring_off;
    const int32_t *patch_ring;
    const uint2 *patch_nbr;
    // triangles: each patch's nodes in LDS (its own nodes b P .. in order,
    // then its halo: the other nodes of its and its ring's triangles,
    // ascending, entries patch_halo_off[b] ..) and every patch and ring
    // triangle's nodes as indices into that list (.x = n0 | n1 << 16, .y = n2)
    const int32_t *patch_halo_off;
    const int32_t *patch_halo;
    const uint2 *patch_lconn;
    const uint2 *patch_ring_lconn;
    Cand *cand;          // 3 ne
    // fused step with the global pick folded in (multi-tip tracking): the
    // accepted candidates of segment step j go to set j mod 3 of fold_cand
    // (3 sets of 3 ne), counted in fold_n[j mod 3]; every workgroup of step
    // j + 1 takes their pick, and the segment's commit takes the last step's
    int32_t fold;
    int32_t pad_fold;
    int32_t *fold_n;     // 3 counters
    Cand *fold_cand;     // 9 ne
    LogRec *log;
    Ctl *ctl;
    const double *curve_t, *curve_phi;
    double D11, D12, D33, E;
    double dt, t_ramp, gamma;
    // per-front pick: front_r2 = rho^2 > 0 replaces the global pick by a
    // separate pick kernel over the candidate list (scratch per candidate)
    double front_r2;
    double2 *fmid;
    double *flen;
    int32_t *forder;
    int32_t *fbucket, *fsorted, *fplist;
    double fcell;  // hash cell of the pick: >= rho and the largest element diameter
    int32_t *fgrid;  // the pick's bucket table over the whole GPU, or null for one workgroup
};

// Evaluation outputs of the query kernels (nullptr = skip).
struct Eval {
    double *sig_ek;     // 3 nv per element: stress at local edge k (NaN where no intact neighbour)
    double *es_ek;      // nv per element: 1/2 A_s sigma:eps of local edge k where this element
                        // owns the edge (lower-id intact neighbour), else 0
    double *pe;         // per element: strain energy of the split pieces
    double *principal;  // per element: largest principal stress of the mean edge stress (NaN split)
    double *fint;       // 2 nn: x block, then y block
    double *acc;        // 2 nn: x block, then y block
    double *node_e;     // 2 per node: 1/2 m v.v, phi f_ext . u
};

// One time step j of the running segment (step index ctl->base + j):
// element forces and candidates, then nodal gather, update and the pick.
hipError_t launch_step(const Params &p, int j, hipStream_t st);
// Close a segment of n steps (ctl->base += n).
hipError_t launch_commit(const Params &p, int n, hipStream_t st);
// Internal force, edge stresses, energy terms and principal stresses of
// displacement u (interleaved) with velocity v (may be null) at step k with
// load factor phi: no candidates, no update.
hipError_t launch_eval(const Params &p, const double2 *u, const double2 *v, int64_t k, double phi,
                       const double *mass, const Eval &ev, hipStream_t st);
// Crack-surface tip flags of the edges (edge_elem: 2 per edge, in edge
// order): 1 where one neighbour is intact and the other split.
hipError_t launch_tip_flags(const Params &p, const int32_t *edge_elem, int64_t ns, uint8_t *flag, hipStream_t st);
// One power-iteration step of M^-1/2 K M^-1/2 over the free components:
// y -> z / |z| with sums[0] = y . z, sums[1] = z . z (y, z: x block then
// y block; u: interleaved scratch of nn pairs).
hipError_t launch_power_step(const Params &p, const Eval &ev, double *y, double2 *u, double *z, double *yz_zz,
                             double *part, double *sums, hipStream_t st);

}  // namespace tri

// Deterministic sum of x[off + stride * i], i < n, into *out (two passes).
hipError_t launch_sum(const double *x, int64_t n, int stride, int off, double *part, double *out, hipStream_t st);
int sum_partials();

}  // namespace mct
