// Host side of the unstructured-mesh path (constant-strain triangles or
// bilinear quadrilaterals): the model a context holds after
// mct_set_mesh_tri or mct_set_mesh_q4, and the functions the C ABI forwards
// to for such a context.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mct2d.h"
#include "mct2d_tri.h"

namespace mct {
namespace tri {

struct Model {
    // mesh (as given) and its tables, built by set_mesh
    int64_t nn = 0, ne = 0, ns = 0;
    int nv = 3;                      // nodes (and edges) per element: 3 or 4
    std::vector<double> X, Y;
    std::vector<int32_t> conn;       // nv per element
    std::vector<int32_t> edge_node;  // 2 per edge (lower node id first), edges sorted by node pair
    std::vector<int32_t> edge_elem;  // 2 per edge (lower element id first, -1 none)
    std::vector<int32_t> elem_edge;  // nv per element
    std::vector<int32_t> nbr;        // nv + 1 per element: neighbours across k = 0..nv-1, packed local edges
    std::vector<double> area;
    // material and loads
    bool have_material = false;
    double E = 0, nu = 0, rho = 0, gamma = 1, gc_uniform = 0;
    std::vector<double> gc;
    std::vector<int64_t> trac_edge;  // sorted edge ids
    std::vector<double> trac;        // 2 per traction edge
    std::vector<int32_t> vbc_node;
    std::vector<uint8_t> vbc_mask;
    std::vector<double> vbc_v0;
    double t_ramp = 0;
    std::vector<int32_t> notch_elem;
    std::vector<uint8_t> notch_code;
    double dt_in = 0, cfl = 0.5;
    std::vector<double> curve_t, curve_phi;
    int sct = 0;
    int32_t sct_elem = -1;
    int sct_edge = 0;
    bool use_graph = true;
    double front_rho = 0;  // per-front pick radius (0: the global pick)
    // derived at finalize
    bool finalized = false;
    double dt = 0, dt_limit = 0;
    std::vector<double> mass;
    Params prm{};
    // device memory
    int4 *dconn = nullptr, *dnbr = nullptr;
    int2 *dopp = nullptr;
    int4 *dq_nbr = nullptr, *dq_oa = nullptr, *dq_ob = nullptr;  // quadrilaterals
    uint8_t *dq_loc = nullptr;
    double *dminv = nullptr, *dgc = nullptr, *dcurve = nullptr, *dmass = nullptr;
    double2 *dxy = nullptr, *du[2] = {nullptr, nullptr}, *dv = nullptr, *dfext = nullptr, *dv0 = nullptr,
            *dfe = nullptr;
    int32_t *dpatch_off = nullptr, *dpatch_elem = nullptr, *dpatch_ring_off = nullptr, *dpatch_ring = nullptr;
    uint2 *dpatch_nbr = nullptr, *dpatch_lconn = nullptr, *dpatch_ring_lconn = nullptr;
    int32_t *dpatch_halo_off = nullptr, *dpatch_halo = nullptr;
    int32_t *dfold_n = nullptr;     // folded pick: 3 candidate counters
    Cand *dfold_cand = nullptr;     //   and 3 candidate sets of 3 ne (triangles only)
    uint16_t *dpatch_slots = nullptr;
    // step kernels: 0 automatic, 1 split, 2/3/4 fused on 64/128/256-node
    // patches, 5 fused on patches of the size sized_patches finds
    int kernels = 0;
    // node -> incident (nv * element + local node) entries in colour order
    std::vector<int32_t> gnoff, gnel;
    uint8_t *dflag = nullptr, *dsplit = nullptr;
    int32_t *dcsr_off = nullptr, *dcsr_ent = nullptr, *dnlist = nullptr, *dedge_elem = nullptr, *dwatch = nullptr;
    Cand *dcand = nullptr;
    double2 *dfmid = nullptr;
    double *dflen = nullptr;
    int32_t *dforder = nullptr, *dfbucket = nullptr, *dfsorted = nullptr, *dfplist = nullptr;
    int32_t *dfgrid = nullptr;  // bucket table of the pick over the whole GPU (large meshes)
    LogRec *dlog = nullptr;
    Ctl *dctl = nullptr;
    // query buffers (allocated on first use)
    Eval ev{};
    double *dpart = nullptr, *dsums = nullptr, *dpow = nullptr;
    uint8_t *dtipflag = nullptr;
    hipGraphExec_t graph = nullptr;
    int64_t steps_enqueued = 0;
};

// Every function returns an mct status and writes a message to err on
// failure.
struct Host {
    std::string &err;
    hipStream_t stream;
};

void release(Model &m);
// nv = 3: triangles (3 nodes per element); nv = 4: convex quadrilaterals.
int set_mesh(Model &m, Host h, int nv, int64_t nn, const double *X, const double *Y, int64_t ne,
             const int32_t *conn);
int set_material(Model &m, Host h, double E, double nu, double rho, const double *Gc, double Gc_uniform,
                 double gamma);
int set_traction(Model &m, Host h, int64_t n, const int32_t *edge_nodes, const double *t);
int set_velocity_bc(Model &m, Host h, int64_t n, const int32_t *node, const uint8_t *mask, const double *v0,
                    double t_ramp);
int set_notch(Model &m, Host h, int64_t n, const int32_t *elem, const uint8_t *entry, const uint8_t *exit);
int set_load_curve(Model &m, Host h, int64_t n, const double *t, const double *phi);
int set_tracking(Model &m, Host h, int mode, int32_t elem, int edge);
int set_time(Model &m, Host h, double dt, double cfl);
int set_front_pick(Model &m, Host h, double rho);
int finalize(Model &m, Host h);
int step(Model &m, Host h, int64_t n);
// Step kernels: 0 automatic, 1 the element kernel plus the node kernel,
// 2/3/4 the fused kernel on patches of 64/128/256 nodes (the split kernels
// where its tables do not fit).  Drops a captured graph (after the stream has
// drained).
int set_kernels(Model &m, Host h, int kind);
int sync(Model &m, Host h);
int get_info(Model &m, Host h, mct_info *out);
int get_crack_set(Model &m, Host h, int64_t cap, int32_t *step, int32_t *elem, uint8_t *entry, uint8_t *exit,
                  double *G, int64_t *count);
int get_tips(Model &m, Host h, int64_t cap, int32_t *edge, double *xy, int64_t *count);
int get_field(Model &m, Host h, int which, int64_t cap, double *out);
int get_energies(Model &m, Host h, double out[4]);
int get_split_codes(Model &m, Host h, int64_t cap, uint8_t *out);
int checkpoint(Model &m, Host h, void *buf, int64_t cap, int64_t *bytes);
// Crack-path normals and lengths of n elements, 36 values each
// (mct_get_path_geometry's layout; NaN where a triangle has no such path).
int get_path_geometry(Model &m, Host h, int64_t n, const int32_t *elem, double *out);
// Device side (mct2d_tri_geom.hip).
hipError_t launch_path_geometry(const Params &p, int n, const int32_t *elem, double *out, hipStream_t st);
int restore(Model &m, Host h, const void *buf, int64_t bytes);

}  // namespace tri
}  // namespace mct
