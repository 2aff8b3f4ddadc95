// Host side of the MCT-2D-CEM library: the C ABI declared in mct2d.h,
// mesh/material/load set-up, device memory, step launching (HIP graphs of
// step kernels), queries, batching of independent specimens and the launch
// autotuner.
//
// A context holds one or more specimens.  A plain context (mct_create) has
// one; a batch (mct_batch_create) has many, which share one launch per time
// step.  Set-up calls and queries act on the selected specimen.
#include "../../include/mct2d.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "mct2d_impl.h"
#include "mct2d_tri_host.h"

using mct::Control;
using mct::LogRec;
using mct::Slot;
using mct::StepParams;

namespace {

constexpr int kGraphSteps = 64;  // steps per captured graph segment
constexpr int kNumOrders = 3;    // work-unit orders of a batch (see build_units)

struct TractionEdge {
    int64_t id;
    int32_t lo, hi;
    double tx, ty;
};

// One specimen: set-up inputs as given, derived sizes and offsets into the
// batch arrays, and the device view the kernels use.
struct Spec {
    int32_t nx = 0, ny = 0;
    std::vector<double> X, Y;
    bool have_material = false;
    double E = 0, nu = 0, rho = 0, gamma = 1, gc_uniform = 0;
    std::vector<double> gc;
    std::vector<TractionEdge> traction;
    std::vector<int32_t> vbc_node;
    std::vector<uint8_t> vbc_mask;
    std::vector<double> vbc_v0;
    double t_ramp = 0;
    std::vector<int32_t> notch_elem;
    std::vector<uint8_t> notch_code;
    double dt_in = 0, cfl = 0.5;
    std::vector<double> curve_t, curve_phi;  // traction load curve (empty: constant)
    int64_t curve_off = 0;
    int sct = 0;             // single crack-tip tracking
    int32_t sct_elem = -1;   // start tip (element, local edge); -1: the pre-notch's path end
    int sct_edge = 0;
    double front_rho = 0;    // per-front pick radius (0: the global pick)
    int subcell = 0;         // Q4 edge smoothing over triangular sub-cells
    // derived
    double dt = 0;
    double dt_limit = 0;  // 2 / omega_max of the set-up mesh (power iteration)
    int64_t nn = 0, ne = 0, ns = 0, np = 0;
    int64_t node_off = 0, elem_off = 0, perim_off = 0, tile_base = 0;
    StepParams prm{};
    mct::StepParamsF prmf{};  // binary32 contexts: the view the step kernels take
};

}  // namespace

struct mct_ctx {
    std::string err;
    int precision = 64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;

    std::vector<Spec> specs;
    int sel = 0;
    bool batch = false;

    bool finalized = false;
    int tile_req = 0, tile = 3;
    int order_req = -1, order = 0;
    bool use_graph = true;

    // device arrays, specimens concatenated
    double *dX = nullptr, *dY = nullptr, *dux[2] = {nullptr, nullptr}, *duy[2] = {nullptr, nullptr};
    double *dvx = nullptr, *dvy = nullptr, *dminv = nullptr, *dgc = nullptr, *darea = nullptr;
    double *dfext = nullptr, *dv0 = nullptr, *dcurve = nullptr;
    // binary32 contexts: the step's arrays (set-up values rounded once, the
    // state); the binary64 arrays above mirror them for the queries
    float *fX = nullptr, *fY = nullptr, *fux[2] = {nullptr, nullptr}, *fuy[2] = {nullptr, nullptr};
    float *fvx = nullptr, *fvy = nullptr, *fminv = nullptr, *fgc = nullptr, *farea = nullptr;
    float *ffext = nullptr, *fv0 = nullptr;
    uint8_t *dvmask = nullptr, *dsplit = nullptr;
    // caller-owned state arrays (mct_bind_device_buffers): used instead of
    // dux, duy, dvx, dvy and never freed by the library
    bool bound = false;
    mct_device_views views{};
    Control *dctl = nullptr;
    Slot *dslots = nullptr;
    LogRec *dlog = nullptr;
    // per-front pick buffers (plain contexts)
    mct::AccCand *dfcand = nullptr;
    uint32_t *dfcount = nullptr;
    double2 *dfmid = nullptr;
    double *dflen = nullptr;
    int32_t *dforder = nullptr, *dfbucket = nullptr, *dfsorted = nullptr, *dfplist = nullptr;
    int32_t *dfgrid = nullptr;  // bucket table of the pick over the whole GPU (large models)
    double front_cell = 0.0;
    StepParams *dviews = nullptr;
    int2 *dunits = nullptr;
    int nunits = 0;
    int32_t *dtip_counts = nullptr, *dtip_total = nullptr;

    // uniform lattices: mode (0 automatic, 1 general kernel always), the
    // shared geometry per specimen, and whether the step runs the lattice
    // kernel (every specimen a lattice)
    int lattice_mode = 0;
    mct::LatticeConst *dlat = nullptr;
    uint32_t *dlat_flag = nullptr;
    bool uni = false;
    // near-threshold decision log (plain contexts): tolerance (0 = off),
    // capacity and device records
    double near_tol = 0.0;
    int64_t near_cap = 0;
    mct::NearRec *dnear = nullptr;
    uint32_t *dnear_count = nullptr;

    hipGraphExec_t graph[2] = {nullptr, nullptr};  // by parity of the first step
    int graph_tile[2] = {0, 0};
    // a shorter segment (fewer than kGraphSteps steps), by parity: its length
    hipGraphExec_t tgraph[2] = {nullptr, nullptr};
    int tgraph_tile[2] = {0, 0}, tgraph_n[2] = {0, 0};
    int64_t steps_enqueued = 0;  // host view of the step counter

    // state queries
    bool ev_alloc = false;
    mct::EvalDev ev{};
    double *dpow = nullptr;    // power iteration: y, u, z, scratch (2 nn_max each)
    int32_t *dflag = nullptr;  // non-finite watchdog

    // unstructured-mesh path (triangles or quadrilaterals): set by
    // mct_set_mesh_tri / mct_set_mesh_q4 (plain binary64 contexts only); the
    // ABI forwards every call of such a context to it
    mct::tri::Model *tri = nullptr;

    // learned split-screen (plain contexts only)
    bool screen_alloc = false, screen_on = false;
    int screen_period = 50;
    float screen_tau = 0.0f;
    mct::ScreenDev sd{};
    mct::MlpDev smlp{};                             // weights in use (no Adam state)
    hipGraphExec_t sgraph[2] = {nullptr, nullptr};  // one screened period, by parity
    int sgraph_tile[2] = {0, 0};
    int64_t screen_windows = 0, screen_replays = 0;  // judged windows, replayed ones
};

struct mct_mlp {
    std::string err;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mct::MlpDev d{};
    float *grad = nullptr;      // kParams + 1 (loss last)
    float *partials = nullptr;  // per-workgroup gradients
    int t = 0;                  // Adam steps taken
};

namespace {

int fail(mct_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                          \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail((ctx), MCT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));               \
    } while (0)

// Forward a call of an unstructured-mesh context to its path.
#define TRI_FWD(c, fn, ...)                                               \
    do {                                                                 \
        if ((c)->tri) return mct::tri::fn(*(c)->tri, mct::tri::Host{(c)->err, (c)->stream}, __VA_ARGS__); \
    } while (0)
#define TRI_FWD0(c, fn)                                                  \
    do {                                                                 \
        if ((c)->tri) return mct::tri::fn(*(c)->tri, mct::tri::Host{(c)->err, (c)->stream}); \
    } while (0)
#define TRI_UNSUPPORTED(c, what)                                                     \
    do {                                                                             \
        if ((c)->tri) return fail((c), MCT_EUNSUPPORTED, "%s: not for an unstructured mesh", what); \
    } while (0)

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void drop_graphs(mct_ctx *c) {
    for (int i = 0; i < 2; ++i) {
        if (c->graph[i]) (void)hipGraphExecDestroy(c->graph[i]);
        c->graph[i] = nullptr;
        if (c->tgraph[i]) (void)hipGraphExecDestroy(c->tgraph[i]);
        c->tgraph[i] = nullptr;
        c->tgraph_n[i] = 0;
        if (c->sgraph[i]) (void)hipGraphExecDestroy(c->sgraph[i]);
        c->sgraph[i] = nullptr;
    }
}

void free_mlp(mct::MlpDev &m) {
    dfree(m.master);
    dfree(m.m);
    dfree(m.v);
    dfree(m.w1b);
    dfree(m.w2b);
    dfree(m.w3b);
}

void free_eval(mct_ctx *c) {
    mct::EvalDev &d = c->ev;
    dfree(d.sig);
    dfree(d.es);
    dfree(d.fe);
    dfree(d.pe);
    dfree(d.fint);
    dfree(d.acc);
    dfree(d.node_e);
    dfree(d.part);
    dfree(d.sums);
    dfree(c->dpow);
    dfree(c->dflag);
    c->ev_alloc = false;
}

void free_screen(mct_ctx *c) {
    mct::ScreenDev &s = c->sd;
    dfree(s.nrows);
    dfree(s.nrows_last);
    dfree(s.cand);
    dfree(s.feat);
    dfree(s.row_geo);
    dfree(s.logits);
    dfree(s.hist_g);
    dfree(s.hist_t);
    dfree(s.sweep);
    dfree(s.screen);
    dfree(s.nfront);
    dfree(s.front_xy);
    dfree(s.stats);
    dfree(s.trip);
    dfree(s.snap_u);
    dfree(s.snap_split);
    dfree(s.snap_ctl);
    free_mlp(c->smlp);
    c->screen_alloc = false;
    c->screen_on = false;
}

void release_device(mct_ctx *c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    dfree(c->dX);
    dfree(c->dY);
    if (c->bound) {  // the caller's arrays
        c->dux[0] = c->dux[1] = c->duy[0] = c->duy[1] = c->dvx = c->dvy = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        dfree(c->dux[i]);
        dfree(c->duy[i]);
        dfree(c->fux[i]);
        dfree(c->fuy[i]);
    }
    dfree(c->dvx);
    dfree(c->dvy);
    dfree(c->fX);
    dfree(c->fY);
    dfree(c->fvx);
    dfree(c->fvy);
    dfree(c->fminv);
    dfree(c->fgc);
    dfree(c->farea);
    dfree(c->ffext);
    dfree(c->fv0);
    dfree(c->dminv);
    dfree(c->dgc);
    dfree(c->darea);
    dfree(c->dfext);
    dfree(c->dcurve);
    dfree(c->dv0);
    dfree(c->dvmask);
    dfree(c->dsplit);
    dfree(c->dctl);
    dfree(c->dslots);
    dfree(c->dlog);
    dfree(c->dfcand);
    dfree(c->dfcount);
    dfree(c->dfmid);
    dfree(c->dflen);
    dfree(c->dforder);
    dfree(c->dfbucket);
    dfree(c->dfsorted);
    dfree(c->dfplist);
    dfree(c->dfgrid);
    dfree(c->dviews);
    dfree(c->dunits);
    dfree(c->dtip_counts);
    dfree(c->dtip_total);
    dfree(c->dlat);
    dfree(c->dlat_flag);
    dfree(c->dnear);
    dfree(c->dnear_count);
    c->uni = false;
    free_screen(c);
    free_eval(c);
    c->finalized = false;
}

Spec &cur(mct_ctx *c) { return c->specs[c->sel]; }

int64_t node_of(const Spec &s, int i, int j) { return (int64_t)j * (s.nx + 1) + i; }

int perimeter_index(int i, int j, int nx, int ny) {
    if (j == 0) return i;
    if (j == ny) return (nx + 1) + i;
    if (i == 0) return 2 * (nx + 1) + (j - 1);
    if (i == nx) return 2 * (nx + 1) + (ny - 1) + (j - 1);
    return -1;
}

// Id of the edge joining nodes a and b of the grid, or -1.  Edges are
// numbered in ascending (smaller node, larger node) order.
int64_t edge_id(const Spec &s, int64_t a, int64_t b) {
    const int64_t lo = std::min(a, b), hi = std::max(a, b);
    const int nx = s.nx, ny = s.ny;
    const int i = (int)(lo % (nx + 1)), j = (int)(lo / (nx + 1));
    const int64_t row = 2 * (int64_t)nx + 1;
    if (hi == lo + 1 && i < nx) return (j < ny) ? j * row + 2 * i : (int64_t)ny * row + i;
    if (hi == lo + nx + 1 && j < ny) return j * row + (i < nx ? 2 * i + 1 : 2 * nx);
    return -1;
}

bool boundary_edge(const Spec &s, int64_t a, int64_t b) {
    const int64_t lo = std::min(a, b), hi = std::max(a, b);
    const int i = (int)(lo % (s.nx + 1)), j = (int)(lo / (s.nx + 1));
    if (hi == lo + 1) return j == 0 || j == s.ny;
    return i == 0 || i == s.nx;
}

double elem_area(const Spec &s, int64_t e) {
    const int i = (int)(e % s.nx), j = (int)(e / s.nx);
    const int64_t n[4] = {node_of(s, i, j), node_of(s, i + 1, j), node_of(s, i + 1, j + 1), node_of(s, i, j + 1)};
    const double *X = s.X.data(), *Y = s.Y.data();
    return 0.5 * ((X[n[2]] - X[n[0]]) * (Y[n[3]] - Y[n[1]]) - (X[n[3]] - X[n[1]]) * (Y[n[2]] - Y[n[0]]));
}

void tiles_of(const Spec &s, int tile, int &ntx, int &nty) {
    const mct::TileShape t = mct::tile_shape(tile);
    ntx = (s.nx + 1 + t.txe - 2) / (t.txe - 1);
    nty = (s.ny + 1 + t.tye - 2) / (t.tye - 1);
}

int pick_tile(const mct_ctx *c) {
    if (c->tile_req >= 1 && c->tile_req <= mct::kNumTiles) return c->tile_req;
    // 16 x 16: four workgroups fit on a CU (LDS and registers), and its
    // halo overhead is the smallest of the 256-thread shapes
    return 1;
}

// Work-unit order of a batch: which (specimen, tile) each workgroup takes.
// Workgroup ids are dealt round-robin over the 8 XCDs, so "banded" orders
// give each XCD a contiguous run of the list (neighbouring tiles share an L2).
//   0: specimens in id order, banded;
//   1: specimens in id order, consecutive workgroups on different XCDs;
//   2: largest specimens first, banded.
std::vector<int2> build_units(const mct_ctx *c, int order) {
    std::vector<int> ord(c->specs.size());
    std::iota(ord.begin(), ord.end(), 0);
    if (order == 2)
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b) { return c->specs[a].prm.nwg > c->specs[b].prm.nwg; });
    std::vector<int2> list;
    for (int s : ord)
        for (int t = 0; t < c->specs[s].prm.nwg; ++t) list.push_back(make_int2(s, t));
    if (order == 1) return list;
    const int n = (int)list.size(), q = n / 8, r = n % 8;
    std::vector<int2> out(n);
    for (int b = 0; b < n; ++b) {
        const int x = b % 8, l = b / 8;
        out[b] = list[(x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l];
    }
    return out;
}

void refresh_f32(mct_ctx *c);

// (Re)build tile geometry, slot sets, views and work units for the chosen
// tile shape and order.  Device state is untouched.
int set_launch_geometry(mct_ctx *c) {
    c->tile = pick_tile(c);
    c->order = (c->order_req >= 0 && c->order_req < kNumOrders) ? c->order_req : 0;
    int64_t base = 0;
    for (Spec &s : c->specs) {
        tiles_of(s, c->tile, s.prm.ntx, s.prm.nty);
        s.prm.nwg = s.prm.ntx * s.prm.nty;
        s.tile_base = base;
        base += s.prm.nwg;
    }
    drop_graphs(c);
    if (!c->finalized) return MCT_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c->dslots);
    HIP_TRY(c, hipMalloc((void **)&c->dslots, 3 * sizeof(Slot) * (size_t)std::max<int64_t>(base, 1)));
    for (Spec &s : c->specs) s.prm.slots = c->dslots + 3 * s.tile_base;
    refresh_f32(c);
    if (c->batch) {
        std::vector<StepParams> views;
        for (const Spec &s : c->specs) views.push_back(s.prm);
        dfree(c->dviews);
        dfree(c->dunits);
        HIP_TRY(c, hipMalloc((void **)&c->dviews, sizeof(StepParams) * views.size()));
        HIP_TRY(c, hipMemcpy(c->dviews, views.data(), sizeof(StepParams) * views.size(), hipMemcpyHostToDevice));
        const std::vector<int2> units = build_units(c, c->order);
        c->nunits = (int)units.size();
        HIP_TRY(c, hipMalloc((void **)&c->dunits, sizeof(int2) * units.size()));
        HIP_TRY(c, hipMemcpy(c->dunits, units.data(), sizeof(int2) * units.size(), hipMemcpyHostToDevice));
    }
    return MCT_OK;
}

// The binary32 view of a plain context: the binary64 view's sizes, tables
// and control pointers with the binary32 arrays and constants (the binary64
// set-up values rounded once).
void refresh_f32(mct_ctx *c) {
    if (c->precision != 32 || !c->finalized) return;
    Spec &s = c->specs[0];
    const StepParams &p = s.prm;
    mct::StepParamsF &f = s.prmf;
    f = mct::StepParamsF{};
    f.nx = p.nx;
    f.ny = p.ny;
    f.ntx = p.ntx;
    f.nty = p.nty;
    f.nwg = p.nwg;
    f.log_cap = p.log_cap;
    f.X = c->fX;
    f.Y = c->fY;
    f.ux0 = c->fux[0];
    f.uy0 = c->fuy[0];
    f.ux1 = c->fux[1];
    f.uy1 = c->fuy[1];
    f.vx = c->fvx;
    f.vy = c->fvy;
    f.minv = c->fminv;
    f.split = p.split;
    f.area = c->farea;
    f.screen = nullptr;
    f.sct = p.sct;
    f.subcell = p.subcell;
    f.ncurve = p.ncurve;
    f.curve_t = p.curve_t;
    f.curve_phi = p.curve_phi;
    f.gc = p.gc ? c->fgc : nullptr;
    f.gc_uniform = (float)p.gc_uniform;
    f.fext_p = c->ffext;
    f.vmask_p = p.vmask_p;
    f.v0_p = c->fv0;
    f.D11 = (float)p.D11;
    f.D12 = (float)p.D12;
    f.D33 = (float)p.D33;
    f.E = (float)p.E;
    f.dt = p.dt;
    f.t_ramp = p.t_ramp;
    f.dts = (float)p.dt;
    f.gamma = (float)p.gamma;
    f.ctl = p.ctl;
    f.slots = p.slots;
    f.log = p.log;
    f.lat = nullptr;
    f.near = p.near;
    f.near_count = p.near_count;
    f.near_cap = p.near_cap;
    f.near_tol = (float)p.near_tol;
}

// Binary32 contexts: copy the state into its binary64 mirror (exact) before
// a query reads it, and back after a restore wrote the mirror.
int widen_state(mct_ctx *c) {
    if (c->precision != 32 || !c->finalized) return MCT_OK;
    const int64_t nn = c->specs[0].nn;
    const float *src[6] = {c->fux[0], c->fuy[0], c->fux[1], c->fuy[1], c->fvx, c->fvy};
    double *dst[6] = {c->dux[0], c->duy[0], c->dux[1], c->duy[1], c->dvx, c->dvy};
    HIP_TRY(c, mct::launch_widen(src, dst, 6, nn, c->stream));
    return MCT_OK;
}

int narrow_state(mct_ctx *c) {
    if (c->precision != 32 || !c->finalized) return MCT_OK;
    const int64_t nn = c->specs[0].nn;
    const double *src[6] = {c->dux[0], c->duy[0], c->dux[1], c->duy[1], c->dvx, c->dvy};
    float *dst[6] = {c->fux[0], c->fuy[0], c->fux[1], c->fuy[1], c->fvx, c->fvy};
    HIP_TRY(c, mct::launch_narrow(src, dst, 6, nn, c->stream));
    return MCT_OK;
}

mct::Launch launch_of(const mct_ctx *c) {
    mct::Launch L;
    L.batched = c->batch;
    L.uni = c->uni;
    L.p0 = c->specs[0].prm;
    L.f32 = c->precision == 32;
    L.p0f = c->specs[0].prmf;
    L.views = c->dviews;
    L.units = c->dunits;
    L.nunits = c->nunits;
    L.nspec = (int)c->specs.size();
    return L;
}

// Where the pick of a step is taken.  A launch of few workgroups folds it
// into the next step: every workgroup reduces the published candidates
// itself (no extra launch; such a launch is one latency-bound wave of
// workgroups).  A batch, or a model of many workgroups (several rounds per
// step), commits every step instead: one small launch (a workgroup per
// specimen) reduces them, splits and logs, so the next step's workgroups
// read the new split codes from memory and skip the reduction and its
// memory round trip.
constexpr int64_t kFoldMaxWorkgroups = 4096;
bool commit_each_step(const mct_ctx *c) {
    if (c->batch) return true;
    const mct::StepParams &p = c->specs[0].prm;
    return p.front == 0 && (int64_t)p.nwg > kFoldMaxWorkgroups;
}

// n steps of a segment starting at parity par0, closed by the commit.
hipError_t enqueue_segment(const mct_ctx *c, const mct::Launch &L, int n, int par0, hipStream_t st) {
    hipError_t e = hipSuccess;
    if (commit_each_step(c)) {
        for (int i = 0; e == hipSuccess && i < n; ++i) {
            e = mct::launch_step(c->tile, L, 0, (par0 + i) & 1, st);
            if (e == hipSuccess) e = mct::launch_commit(L, 1, st);
        }
        return e;
    }
    for (int i = 0; e == hipSuccess && i < n; ++i) e = mct::launch_step(c->tile, L, i, par0, st);
    if (e == hipSuccess) e = mct::launch_commit(L, n, st);
    return e;
}

// A segment of n steps followed by its commit, captured once per parity of
// the segment's first step: n = kGraphSteps in graph[], shorter ones (the
// tail of a request) in tgraph[].
int build_graph(mct_ctx *c, int par0, int n = kGraphSteps) {
    hipGraphExec_t &slot = n == kGraphSteps ? c->graph[par0] : c->tgraph[par0];
    if (slot) (void)hipGraphExecDestroy(slot);
    slot = nullptr;
    hipStream_t cap;
    HIP_TRY(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    const mct::Launch L = launch_of(c);
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) e = enqueue_segment(c, L, n, par0, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&slot, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(c, MCT_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    if (n == kGraphSteps) {
        c->graph_tile[par0] = c->tile;
    } else {
        c->tgraph_tile[par0] = c->tile;
        c->tgraph_n[par0] = n;
    }
    return MCT_OK;
}

// ---------------------------------------------------------------------
// Learned split-screen: device buffers, the sweep pipeline and screened
// stepping.

int alloc_mlp(mct_ctx *c, mct::MlpDev &m, bool with_adam) {
    HIP_TRY(c, hipMalloc((void **)&m.master, sizeof(float) * mct::kParams));
    if (with_adam) {
        HIP_TRY(c, hipMalloc((void **)&m.m, sizeof(float) * mct::kParams));
        HIP_TRY(c, hipMalloc((void **)&m.v, sizeof(float) * mct::kParams));
    }
    HIP_TRY(c, hipMalloc((void **)&m.w1b, sizeof(uint16_t) * 32 * mct::kHidden));
    HIP_TRY(c, hipMalloc((void **)&m.w2b, sizeof(uint16_t) * mct::kHidden * mct::kHidden));
    HIP_TRY(c, hipMalloc((void **)&m.w3b, sizeof(uint16_t) * mct::kHidden));
    return MCT_OK;
}

int ensure_screen(mct_ctx *c) {
    if (c->batch) return fail(c, MCT_EUNSUPPORTED, "the split-screen runs on plain (single specimen) contexts");
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (c->screen_alloc) return MCT_OK;
    const Spec &sp = c->specs[0];
    const int64_t ne = sp.ne, nc = 4 * ne;
    mct::ScreenDev &s = c->sd;
    HIP_TRY(c, hipMalloc((void **)&s.nrows, sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&s.nrows_last, sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&s.cand, sizeof(int32_t) * nc));
    HIP_TRY(c, hipMalloc((void **)&s.feat, sizeof(float) * mct::kFeat * nc));
    HIP_TRY(c, hipMalloc((void **)&s.row_geo, sizeof(double) * 3 * nc));
    HIP_TRY(c, hipMalloc((void **)&s.logits, sizeof(float) * nc));
    HIP_TRY(c, hipMalloc((void **)&s.hist_g, sizeof(double) * nc));
    HIP_TRY(c, hipMalloc((void **)&s.hist_t, sizeof(int32_t) * nc));
    HIP_TRY(c, hipMalloc((void **)&s.sweep, sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&s.screen, sizeof(uint32_t) * ne));
    HIP_TRY(c, hipMalloc((void **)&s.nfront, sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&s.front_xy, sizeof(double) * 4 * ne));
    HIP_TRY(c, hipMalloc((void **)&s.stats, sizeof(unsigned long long) * mct::kNumScreenStats));
    HIP_TRY(c, hipMalloc((void **)&s.trip, sizeof(uint32_t)));
    HIP_TRY(c, hipMalloc((void **)&s.snap_u, sizeof(double) * 4 * (size_t)sp.nn));
    HIP_TRY(c, hipMalloc((void **)&s.snap_split, (size_t)std::max<int64_t>(ne, 1)));
    HIP_TRY(c, hipMalloc((void **)&s.snap_ctl, sizeof(Control)));
    // no evaluation yet: history stamps never match, every candidate unseen
    HIP_TRY(c, mct::launch_fill_u32(reinterpret_cast<uint32_t *>(s.hist_t), nc, 0xFFFFFFFEu, c->stream));
    HIP_TRY(c, hipMemsetAsync(s.sweep, 0, sizeof(int32_t), c->stream));
    HIP_TRY(c, hipMemsetAsync(s.nrows, 0, sizeof(int32_t), c->stream));
    HIP_TRY(c, hipMemsetAsync(s.nrows_last, 0, sizeof(int32_t), c->stream));
    HIP_TRY(c, hipMemsetAsync(s.nfront, 0, sizeof(int32_t), c->stream));
    HIP_TRY(c, hipMemsetAsync(s.screen, 0, sizeof(uint32_t) * ne, c->stream));
    HIP_TRY(c, hipMemsetAsync(s.stats, 0, sizeof(unsigned long long) * mct::kNumScreenStats, c->stream));
    HIP_TRY(c, hipMemsetAsync(s.trip, 0, sizeof(uint32_t), c->stream));
    c->screen_windows = c->screen_replays = 0;
    int rc = alloc_mlp(c, c->smlp, false);
    if (rc) return rc;
    c->screen_alloc = true;
    return MCT_OK;
}

// Crack-path ends, candidate rows and features of the state in u buffer
// `par` (every screen state cleared); with the screen on, logits and the
// new screen states too.  Kernels only (capturable).
hipError_t screen_pipeline(mct_ctx *c, int par, hipStream_t st) {
    const StepParams &p = c->specs[0].prm;
    const mct::ScreenDev &s = c->sd;
    hipError_t e = mct::launch_screen_evaluate(p, s, par, st);
    if (c->screen_on && e == hipSuccess)
        e = mct::launch_mlp_forward(c->smlp, s.feat, s.nrows, 0, s.logits, s.cand, s.screen, c->screen_tau,
                                    s.stats, st);
    if (e == hipSuccess) e = mct::launch_sweep_advance(s, st);
    return e;
}

// Steps k_rel = first .. first + count - 1 of a segment starting at parity
// par0 and global step k0: sweep steps (k % period == 0) run plain and are
// followed by the screen pipeline, the others run screened.
hipError_t screened_steps(mct_ctx *c, int64_t k0, int first, int count, int par0, hipStream_t st) {
    mct::Launch Lp = launch_of(c), Ls = launch_of(c);
    Ls.p0.screen = c->sd.screen;
    Ls.p0.strip = c->sd.trip;
    hipError_t e = hipSuccess;
    for (int i = first; e == hipSuccess && i < first + count; ++i) {
        if ((k0 + i) % c->screen_period == 0) {
            e = mct::launch_step(c->tile, Lp, i, par0, st);
            if (e == hipSuccess) e = screen_pipeline(c, (par0 + i + 1) & 1, st);
        } else {
            e = mct::launch_step(c->tile, Ls, i, par0, st);
        }
    }
    return e;
}

int build_screen_graph(mct_ctx *c, int par0) {
    if (c->sgraph[par0]) (void)hipGraphExecDestroy(c->sgraph[par0]);
    c->sgraph[par0] = nullptr;
    hipStream_t cap;
    HIP_TRY(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) e = screened_steps(c, 0, 0, c->screen_period, par0, cap);
    if (e == hipSuccess) e = mct::launch_commit(launch_of(c), c->screen_period, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->sgraph[par0], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(c, MCT_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    c->sgraph_tile[par0] = c->tile;
    return MCT_OK;
}

// Screened stepping, one window at a time (a period from its exact step,
// or the part of one up to the next exact step).  Each window starts from a
// snapshot of the state; its screened steps bound every candidate the screen
// skips, and when a bound reaches Gc (the skipped candidate might have been
// accepted: the window might differ from the plain step) the window is
// restored and replayed with the plain step.  Otherwise no skipped candidate
// could pass the element rule, so the accepted sets, the picks and the whole
// window equal the plain step's.  Either way the run equals the plain run.
// (The screen evaluation after a window's exact step is kept on a replay: it
// ran on the state after that step, which the replay reproduces.)
int step_screened(mct_ctx *c, int64_t n) {
    const int P = c->screen_period;
    const mct::StepParams &p = c->specs[0].prm;
    int64_t left = n;
    while (left > 0) {
        const int64_t k0 = c->steps_enqueued;
        const int par0 = (int)(k0 & 1);
        const int q = (int)(k0 % P);
        const int seg = (q == 0 && left >= P) ? P : (int)std::min<int64_t>(left, P - q);
        HIP_TRY(c, mct::launch_snapshot(p, c->sd, par0, true, c->stream));
        if (q == 0 && seg == P && c->use_graph) {
            if (!c->sgraph[par0] || c->sgraph_tile[par0] != c->tile) {
                int rc = build_screen_graph(c, par0);
                if (rc) return rc;
            }
            HIP_TRY(c, hipGraphLaunch(c->sgraph[par0], c->stream));
        } else {
            HIP_TRY(c, screened_steps(c, k0, 0, seg, par0, c->stream));
            HIP_TRY(c, mct::launch_commit(launch_of(c), seg, c->stream));
        }
        uint32_t trip = 0;
        HIP_TRY(c, hipMemcpyAsync(&trip, c->sd.trip, sizeof trip, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->screen_windows++;
        if (trip) {
            HIP_TRY(c, mct::launch_snapshot(p, c->sd, par0, false, c->stream));
            HIP_TRY(c, enqueue_segment(c, launch_of(c), seg, par0, c->stream));
            c->screen_replays++;
        }
        left -= seg;
        c->steps_enqueued += seg;
    }
    return MCT_OK;
}

// ---------------------------------------------------------------------
// State queries: evaluation buffers, the stability limit.

int ensure_eval(mct_ctx *c) {
    if (c->ev_alloc) return MCT_OK;
    int64_t nn = 0, ne = 0, ns = 0;
    for (const Spec &s : c->specs) {
        nn = std::max(nn, s.nn);
        ne = std::max(ne, s.ne);
        ns = std::max(ns, s.ns);
    }
    mct::EvalDev &d = c->ev;
    HIP_TRY(c, hipMalloc((void **)&d.sig, sizeof(double) * 3 * ns));
    HIP_TRY(c, hipMalloc((void **)&d.es, sizeof(double) * ns));
    HIP_TRY(c, hipMalloc((void **)&d.fe, sizeof(double) * 8 * ne));
    HIP_TRY(c, hipMalloc((void **)&d.pe, sizeof(double) * ne));
    HIP_TRY(c, hipMalloc((void **)&d.fint, sizeof(double) * 2 * nn));
    HIP_TRY(c, hipMalloc((void **)&d.acc, sizeof(double) * 2 * nn));
    HIP_TRY(c, hipMalloc((void **)&d.node_e, sizeof(double) * 2 * nn));
    HIP_TRY(c, hipMalloc((void **)&d.part, sizeof(double) * mct::eval_partials()));
    HIP_TRY(c, hipMalloc((void **)&d.sums, sizeof(double) * 8));
    HIP_TRY(c, hipMalloc((void **)&c->dpow, sizeof(double) * 8 * nn));
    HIP_TRY(c, hipMalloc((void **)&c->dflag, sizeof(int32_t)));
    c->ev_alloc = true;
    return MCT_OK;
}

// Largest eigenvalue of M^-1 K over the free components by power iteration
// on M^-1/2 K M^-1/2 (K u = internal force of u, split elements as set up),
// started from the alternating pattern that the highest mode of a grid
// resembles plus a small deterministic perturbation.  The Rayleigh quotient
// approaches lambda_max from below, so 2 / sqrt(lambda) is an upper estimate
// of the stability limit of central differences.
int stability_limit(mct_ctx *c, Spec &s) {
    int rc = ensure_eval(c);
    if (rc) return rc;
    const int64_t nn = s.nn;
    std::vector<double> y(2 * nn);
    double norm = 0.0;
    uint64_t h = 0x9E3779B97F4A7C15ull;
    for (int j = 0; j <= s.ny; ++j)
        for (int i = 0; i <= s.nx; ++i) {
            const int64_t g = node_of(s, i, j);
            h ^= h >> 33;
            h *= 0xFF51AFD7ED558CCDull;
            const double r = (double)(h >> 11) * 0x1.0p-53;
            const double sgn = ((i + j) & 1) ? -1.0 : 1.0;
            y[g] = sgn * (1.0 + 0.05 * r);
            y[nn + g] = -sgn * (1.0 + 0.05 * (1.0 - r));
            norm += y[g] * y[g] + y[nn + g] * y[nn + g];
        }
    norm = std::sqrt(norm);
    for (double &v : y) v /= norm;
    double *dy = c->dpow, *du = c->dpow + 2 * nn, *dz = c->dpow + 4 * nn, *dw = c->dpow + 6 * nn;
    HIP_TRY(c, hipMemcpyAsync(dy, y.data(), sizeof(double) * 2 * nn, hipMemcpyHostToDevice, c->stream));
    double lam = 0.0, prev = 0.0;
    for (int it = 1; it <= 2000; ++it) {
        HIP_TRY(c, mct::launch_power_step(s.prm, c->ev, dy, du, dz, dw, c->ev.sums, c->stream));
        if (it % 20 == 0) {
            HIP_TRY(c, hipMemcpyAsync(&lam, c->ev.sums, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (!(lam > 0.0) || !std::isfinite(lam))
                return fail(c, MCT_ENUMERIC, "stability estimate failed (Rayleigh quotient %g)", lam);
            if (std::fabs(lam - prev) <= 1e-7 * lam) break;
            prev = lam;
        }
    }
    s.dt_limit = 2.0 / std::sqrt(lam);
    return MCT_OK;
}

// Traction load factor at t, evaluated like the device helper.
double load_factor_host(const Spec &s, double t) {
    const size_t n = s.curve_t.size();
    if (n == 0) return 1.0;
    if (t <= s.curve_t[0]) return s.curve_phi[0];
    if (t >= s.curve_t[n - 1]) return s.curve_phi[n - 1];
    size_t i = 0;
    while (s.curve_t[i + 1] <= t) ++i;
    const double slope = (s.curve_phi[i + 1] - s.curve_phi[i]) / (s.curve_t[i + 1] - s.curve_t[i]);
    return s.curve_phi[i] + (t - s.curve_t[i]) * slope;
}

// Start tip of single-tip tracking: the given one, or the one path end of
// the pre-notch (an entry or exit edge of a notch element whose neighbour
// across it is intact), as element * 4 + local edge.
int start_tip(mct_ctx *c, size_t q, int32_t *tip) {
    const Spec &s = c->specs[q];
    if (s.sct_elem >= 0) {
        *tip = s.sct_elem * 4 + s.sct_edge;
        return MCT_OK;
    }
    std::vector<uint8_t> split(s.ne, 0);
    for (size_t i = 0; i < s.notch_elem.size(); ++i) split[s.notch_elem[i]] = s.notch_code[i];
    int found = 0;
    for (size_t i = 0; i < s.notch_elem.size(); ++i) {
        const int32_t e = s.notch_elem[i];
        const int ks[2] = {(s.notch_code[i] >> 2) & 3, s.notch_code[i] & 3};
        for (int k : ks) {
            const int ei = e % s.nx, ej = e / s.nx;
            const int ni = k == 1 ? ei + 1 : k == 3 ? ei - 1 : ei, nj = k == 2 ? ej + 1 : k == 0 ? ej - 1 : ej;
            if (ni < 0 || ni >= s.nx || nj < 0 || nj >= s.ny) continue;
            const int32_t nb = nj * s.nx + ni;
            if (split[nb] != 0) continue;
            *tip = nb * 4 + ((k + 2) & 3);
            ++found;
        }
    }
    if (found != 1)
        return fail(c, MCT_EINVAL, "specimen %zu: single-tip tracking needs a start tip (the pre-notch has %d path ends)",
                    q, found);
    return MCT_OK;
}

int create_ctx(mct_ctx **out, int nspec, bool batch, int precision, void *hip_stream) {
    if (!out) return MCT_EINVAL;
    *out = nullptr;
    // binary32: plain contexts only
    if (precision != 64 && !(precision == 32 && !batch)) return MCT_EUNSUPPORTED;
    if (nspec < 1 || nspec > (1 << 20)) return MCT_EINVAL;
    mct_ctx *c = new (std::nothrow) mct_ctx;
    if (!c) return MCT_ENOMEM;
    c->precision = precision;
    c->batch = batch;
    c->specs.resize(nspec);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MCT_EDEVICE;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return MCT_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return MCT_OK;
}

template <typename T>
int upload(mct_ctx *c, T *&dst, const std::vector<T> &src) {
    HIP_TRY(c, hipMalloc((void **)&dst, std::max<size_t>(src.size(), 1) * sizeof(T)));
    if (!src.empty())
        HIP_TRY(c, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return MCT_OK;
}

int read_control(mct_ctx *c, int s, Control *h) {
    HIP_TRY(c, hipMemcpyAsync(h, c->dctl + s, sizeof(Control), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

}  // namespace

extern "C" {

int mct_create(mct_ctx **out, int precision, void *hip_stream) {
    return create_ctx(out, 1, false, precision, hip_stream);
}

int mct_batch_create(mct_ctx **out, int64_t n_specimens, int precision, void *hip_stream) {
    if (n_specimens < 1 || n_specimens > (1 << 20)) return MCT_EINVAL;
    return create_ctx(out, (int)n_specimens, true, precision, hip_stream);
}

int mct_batch_select(mct_ctx *c, int64_t s) {
    if (!c) return MCT_EINVAL;
    if (s < 0 || s >= (int64_t)c->specs.size()) return fail(c, MCT_EINVAL, "specimen %lld out of range", (long long)s);
    c->sel = (int)s;
    return MCT_OK;
}

int mct_destroy(mct_ctx *c) {
    if (!c) return MCT_OK;
    if (c->tri) {
        mct::tri::release(*c->tri);
        delete c->tri;
        c->tri = nullptr;
    }
    release_device(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MCT_OK;
}

const char *mct_last_error(const mct_ctx *c) { return c ? c->err.c_str() : "null context"; }

// Both unstructured element kinds run on the unstructured-mesh path.
static int set_mesh_unstructured(mct_ctx *c, int nv, int64_t n_nodes, const double *X, const double *Y,
                                 int64_t n_elems, const int32_t *conn) {
    if (!c) return MCT_EINVAL;
    const char *what = nv == 4 ? "unstructured quadrilateral" : "triangle";
    if (c->batch) return fail(c, MCT_EUNSUPPORTED, "%s meshes need a plain context", what);
    if (c->precision == 32) return fail(c, MCT_EUNSUPPORTED, "%s meshes need a binary64 context", what);
    release_device(c);
    c->bound = false;
    c->views = mct_device_views{};
    c->specs.assign(1, Spec{});
    c->finalized = false;
    if (!c->tri) c->tri = new (std::nothrow) mct::tri::Model;
    if (!c->tri) return MCT_ENOMEM;
    const int rc =
        mct::tri::set_mesh(*c->tri, mct::tri::Host{c->err, c->stream}, nv, n_nodes, X, Y, n_elems, conn);
    if (rc) {
        mct::tri::release(*c->tri);
        delete c->tri;
        c->tri = nullptr;
    }
    return rc;
}

int mct_set_mesh_tri(mct_ctx *c, int64_t n_nodes, const double *X, const double *Y, int64_t n_elems,
                     const int32_t *conn) {
    return set_mesh_unstructured(c, 3, n_nodes, X, Y, n_elems, conn);
}

int mct_set_mesh_q4(mct_ctx *c, int64_t n_nodes, const double *X, const double *Y, int64_t n_elems,
                    const int32_t *conn) {
    return set_mesh_unstructured(c, 4, n_nodes, X, Y, n_elems, conn);
}

int mct_set_mesh_grid(mct_ctx *c, int32_t nx, int32_t ny, const double *X, const double *Y) {
    if (!c) return MCT_EINVAL;
    if (c->tri) {
        mct::tri::release(*c->tri);
        delete c->tri;
        c->tri = nullptr;
    }
    if (nx < 2 || ny < 2 || !X || !Y) return fail(c, MCT_EINVAL, "grid needs nx, ny >= 2 and coordinates");
    // element ids, and element * 4 + local edge keys, stay in int32
    if ((int64_t)nx * ny > (int64_t)1 << 29) return fail(c, MCT_EINVAL, "grid too large (more than 2^29 elements)");
    release_device(c);
    // a new mesh unbinds caller-owned state arrays (they were sized for the old one)
    c->bound = false;
    c->views = mct_device_views{};
    Spec s;
    s.nx = nx;
    s.ny = ny;
    s.nn = (int64_t)(nx + 1) * (ny + 1);
    s.ne = (int64_t)nx * ny;
    s.ns = 2 * (int64_t)nx * ny + nx + ny;
    s.np = 2 * (int64_t)(nx + 1) + 2 * (int64_t)(ny - 1);
    s.X.assign(X, X + s.nn);
    s.Y.assign(Y, Y + s.nn);
    for (int64_t e = 0; e < s.ne; ++e)
        if (!(elem_area(s, e) > 0.0))
            return fail(c, MCT_EINVAL, "element %lld has non-positive area (clockwise or degenerate)", (long long)e);
    cur(c) = std::move(s);
    return MCT_OK;
}

int mct_set_material(mct_ctx *c, double E, double nu, double rho, const double *Gc, double Gc_uniform,
                     double gamma) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_material, E, nu, rho, Gc, Gc_uniform, gamma);
    Spec &s = cur(c);
    if (!s.nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (!(E > 0) || !(nu > -1.0 && nu < 0.5) || !(rho > 0) || !(gamma > 0))
        return fail(c, MCT_EINVAL, "material out of range");
    if (Gc) {
        for (int64_t e = 0; e < s.ne; ++e)
            if (!(Gc[e] > 0)) return fail(c, MCT_EINVAL, "Gc[%lld] <= 0", (long long)e);
        s.gc.assign(Gc, Gc + s.ne);
    } else {
        if (!(Gc_uniform > 0)) return fail(c, MCT_EINVAL, "Gc_uniform <= 0");
        s.gc.clear();
    }
    s.E = E;
    s.nu = nu;
    s.rho = rho;
    s.gamma = gamma;
    s.gc_uniform = Gc_uniform;
    s.have_material = true;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_traction(mct_ctx *c, int64_t n, const int32_t *edge_nodes, const double *t) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_traction, n, edge_nodes, t);
    Spec &s = cur(c);
    if (!s.nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!edge_nodes || !t))) return fail(c, MCT_EINVAL, "bad traction arrays");
    std::vector<TractionEdge> v;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a = edge_nodes[2 * i], b = edge_nodes[2 * i + 1];
        if (a < 0 || b < 0 || a >= s.nn || b >= s.nn)
            return fail(c, MCT_EINVAL, "traction edge %lld: node out of range", (long long)i);
        const int64_t id = edge_id(s, a, b);
        if (id < 0 || !boundary_edge(s, a, b))
            return fail(c, MCT_EINVAL, "traction edge %lld is not a boundary edge", (long long)i);
        v.push_back({id, (int32_t)std::min(a, b), (int32_t)std::max(a, b), t[2 * i], t[2 * i + 1]});
    }
    std::sort(v.begin(), v.end(), [](const TractionEdge &x, const TractionEdge &y) { return x.id < y.id; });
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i].id == v[i - 1].id) return fail(c, MCT_EINVAL, "repeated traction edge");
    s.traction.swap(v);
    c->finalized = false;
    return MCT_OK;
}

int mct_set_velocity_bc(mct_ctx *c, int64_t n, const int32_t *node, const uint8_t *dof_mask, const double *v0,
                        double t_ramp) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_velocity_bc, n, node, dof_mask, v0, t_ramp);
    Spec &s = cur(c);
    if (!s.nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!node || !dof_mask || !v0)) || !(t_ramp >= 0))
        return fail(c, MCT_EINVAL, "bad velocity arrays");
    for (int64_t i = 0; i < n; ++i) {
        if (node[i] < 0 || node[i] >= s.nn || (dof_mask[i] & ~3u))
            return fail(c, MCT_EINVAL, "velocity bc %lld out of range", (long long)i);
        const int ii = (int)(node[i] % (s.nx + 1)), jj = (int)(node[i] / (s.nx + 1));
        if (perimeter_index(ii, jj, s.nx, s.ny) < 0)
            return fail(c, MCT_EINVAL, "velocity bc on interior node %d is not supported", node[i]);
    }
    s.vbc_node.assign(node, node + n);
    s.vbc_mask.assign(dof_mask, dof_mask + n);
    s.vbc_v0.assign(v0, v0 + 2 * n);
    s.t_ramp = t_ramp;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_notch(mct_ctx *c, int64_t n, const int32_t *elem, const uint8_t *entry, const uint8_t *exit) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_notch, n, elem, entry, exit);
    Spec &s = cur(c);
    if (!s.nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!elem || !entry || !exit))) return fail(c, MCT_EINVAL, "bad notch arrays");
    std::vector<int32_t> el;
    std::vector<uint8_t> code;
    for (int64_t i = 0; i < n; ++i) {
        if (elem[i] < 0 || elem[i] >= s.ne || entry[i] > 3 || exit[i] > 3 || entry[i] == exit[i])
            return fail(c, MCT_EINVAL, "notch element %lld invalid", (long long)i);
        el.push_back(elem[i]);
        code.push_back((uint8_t)(mct::kSplitFlag | (entry[i] << 2) | exit[i]));
    }
    s.notch_elem.swap(el);
    s.notch_code.swap(code);
    c->finalized = false;
    return MCT_OK;
}

int mct_set_load_curve(mct_ctx *c, int64_t n, const double *t, const double *phi) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_load_curve, n, t, phi);
    Spec &s = cur(c);
    if (n != 0 && (n < 2 || n > (1 << 20) || !t || !phi)) return fail(c, MCT_EINVAL, "load curve needs 2..2^20 points");
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(t[i]) || !std::isfinite(phi[i])) return fail(c, MCT_EINVAL, "non-finite load curve");
        if (i > 0 && !(t[i] > t[i - 1])) return fail(c, MCT_EINVAL, "load curve times must increase");
    }
    s.curve_t.assign(t, t + n);
    s.curve_phi.assign(phi, phi + n);
    c->finalized = false;
    return MCT_OK;
}

int mct_set_tracking(mct_ctx *c, int mode, int32_t tip_elem, int tip_edge) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_tracking, mode, tip_elem, tip_edge);
    Spec &s = cur(c);
    if (!s.nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (mode != MCT_TRACK_MCT && mode != MCT_TRACK_SCT) return fail(c, MCT_EINVAL, "unknown tracking mode %d", mode);
    if (mode == MCT_TRACK_SCT && tip_elem >= 0 && (tip_elem >= s.ne || tip_edge < 0 || tip_edge > 3))
        return fail(c, MCT_EINVAL, "start tip out of range");
    s.sct = mode == MCT_TRACK_SCT;
    s.sct_elem = tip_elem;
    s.sct_edge = tip_edge;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_front_pick(mct_ctx *c, double rho) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_front_pick, rho);
    if (!(rho >= 0)) return fail(c, MCT_EINVAL, "front radius must be >= 0 (0: the global pick)");
    if (c->batch && rho > 0) return fail(c, MCT_EUNSUPPORTED, "the per-front pick needs a plain context");
    if (c->precision == 32 && rho > 0) return fail(c, MCT_EUNSUPPORTED, "the per-front pick needs binary64");
    Spec &s = cur(c);
    if (!s.nx) return fail(c, MCT_ESTATE, "set the mesh first");
    s.front_rho = rho;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_smoothing(mct_ctx *c, int mode) {
    if (!c) return MCT_EINVAL;
    if (mode != MCT_SMOOTH_POINT && mode != MCT_SMOOTH_SUBCELL) return fail(c, MCT_EINVAL, "unknown smoothing %d", mode);
    if (c->tri) {
        if (mode == MCT_SMOOTH_SUBCELL)
            return fail(c, MCT_EUNSUPPORTED, "sub-cell smoothing is for structured Q4 grids");
        return MCT_OK;
    }
    if (c->batch && mode == MCT_SMOOTH_SUBCELL)
        return fail(c, MCT_EUNSUPPORTED, "sub-cell smoothing needs a plain context");
    Spec &s = cur(c);
    if (!s.nx) return fail(c, MCT_ESTATE, "set the mesh first");
    s.subcell = mode == MCT_SMOOTH_SUBCELL;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_time(mct_ctx *c, double dt, double cfl_fraction) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, set_time, dt, cfl_fraction);
    if (!(dt > 0) && !(cfl_fraction > 0)) return fail(c, MCT_EINVAL, "need dt > 0 or cfl_fraction > 0");
    Spec &s = cur(c);
    s.dt_in = dt;
    s.cfl = cfl_fraction;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_launch(mct_ctx *c, int tile, int use_graph) {
    if (!c) return MCT_EINVAL;
    if (c->tri) {
        // tile = step kernels: 0 automatic, 1 split, 2..4 fused on 64..256-node
        // patches, 5 fused on patches of the size it finds
        if (tile < 0 || tile > 5) return fail(c, MCT_EINVAL, "an unstructured mesh takes tile 0..5 (step kernels)");
        c->tri->use_graph = use_graph != 0;
        return mct::tri::set_kernels(*c->tri, mct::tri::Host{c->err, c->stream}, tile);
    }
    if (tile < 0 || tile > mct::kNumTiles) return fail(c, MCT_EINVAL, "tile index out of range");
    c->tile_req = tile;
    c->use_graph = use_graph != 0;
    return set_launch_geometry(c);
}

int mct_set_order(mct_ctx *c, int order) {
    if (!c) return MCT_EINVAL;
    if (c->tri) return order == -1 || order == 0 ? MCT_OK : fail(c, MCT_EINVAL, "order out of range");
    if (order < -1 || order >= kNumOrders) return fail(c, MCT_EINVAL, "order out of range");
    c->order_req = order;
    return set_launch_geometry(c);
}

int mct_set_lattice(mct_ctx *c, int mode) {
    if (!c) return MCT_EINVAL;
    if (mode != MCT_LATTICE_AUTO && mode != MCT_LATTICE_GENERAL) return fail(c, MCT_EINVAL, "lattice mode %d", mode);
    if (c->tri) return fail(c, MCT_EUNSUPPORTED, "the lattice kernel is for structured grids");
    c->lattice_mode = mode;
    if (c->finalized) release_device(c);  // takes effect at the next finalize
    return MCT_OK;
}

int mct_get_lattice(mct_ctx *c, int *uniform) {
    if (!c || !uniform) return MCT_EINVAL;
    *uniform = (!c->tri && c->finalized && c->uni) ? 1 : 0;
    return MCT_OK;
}

int mct_set_near_log(mct_ctx *c, double tol, int64_t cap) {
    if (!c) return MCT_EINVAL;
    if (c->tri) return fail(c, MCT_EUNSUPPORTED, "the near-threshold log is for structured grids");
    if (c->batch) return fail(c, MCT_EUNSUPPORTED, "the near-threshold log needs a plain context");
    if (!(tol >= 0.0) || !(tol < 1.0)) return fail(c, MCT_EINVAL, "tolerance %g outside [0, 1)", tol);
    if (tol > 0.0 && (cap < 1 || cap > (int64_t)1 << 30)) return fail(c, MCT_EINVAL, "capacity %lld", (long long)cap);
    if (tol > 0.0 && c->screen_on)
        return fail(c, MCT_EUNSUPPORTED, "the near-threshold log with the split-screen");
    c->near_tol = tol;
    c->near_cap = tol > 0.0 ? cap : 0;
    if (c->finalized) release_device(c);  // takes effect at the next finalize
    return MCT_OK;
}

int mct_get_near_log(mct_ctx *c, int64_t cap, int32_t *step, int32_t *elem, uint8_t *a, uint8_t *kind,
                     uint8_t *k, double *G, double *ref, int64_t *count) {
    if (!c || !count) return MCT_EINVAL;
    *count = 0;
    if (c->tri || c->batch) return fail(c, MCT_EUNSUPPORTED, "no near-threshold log on this context");
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (!c->dnear) return MCT_OK;
    uint32_t n = 0;
    HIP_TRY(c, hipMemcpyAsync(&n, c->dnear_count, sizeof n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *count = (int64_t)n;
    if ((int64_t)n > c->near_cap) return fail(c, MCT_ECAPACITY, "near-threshold log overflow: %u records, capacity %lld",
                                             n, (long long)c->near_cap);
    if (cap < (int64_t)n) return fail(c, MCT_ECAPACITY, "capacity %lld < %u records", (long long)cap, n);
    std::vector<mct::NearRec> r(n);
    if (n) HIP_TRY(c, hipMemcpy(r.data(), c->dnear, sizeof(mct::NearRec) * n, hipMemcpyDeviceToHost));
    // canonical order: the device appends in completion order
    std::sort(r.begin(), r.end(), [](const mct::NearRec &x, const mct::NearRec &y) {
        if (x.step != y.step) return x.step < y.step;
        if (x.kind != y.kind) return x.kind < y.kind;
        if (x.elem != y.elem) return x.elem < y.elem;
        if (x.a != y.a) return x.a < y.a;
        return x.k < y.k;
    });
    for (uint32_t i = 0; i < n; ++i) {
        if (step) step[i] = r[i].step;
        if (elem) elem[i] = r[i].elem;
        if (a) a[i] = r[i].a;
        if (kind) kind[i] = r[i].kind;
        if (k) k[i] = r[i].k;
        if (G) G[i] = r[i].G;
        if (ref) ref[i] = r[i].ref;
    }
    return MCT_OK;
}

int mct_bind_device_buffers(mct_ctx *c, const mct_device_views *v) {
    if (!c) return MCT_EINVAL;
    if (c->tri) return fail(c, MCT_EUNSUPPORTED, "device buffers bind the state of a Q4 grid");
    if (c->batch) return fail(c, MCT_EUNSUPPORTED, "device buffers need a plain context");
    if (c->precision != 64) return fail(c, MCT_EUNSUPPORTED, "device buffers hold binary64 state");
    if (v && (!v->ux[0] || !v->ux[1] || !v->uy[0] || !v->uy[1] || !v->vx || !v->vy))
        return fail(c, MCT_EINVAL, "null device array");
    if (v) {
        const double *a[6] = {v->ux[0], v->ux[1], v->uy[0], v->uy[1], v->vx, v->vy};
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j)
                if (a[i] == a[j]) return fail(c, MCT_EINVAL, "device arrays %d and %d are the same", i, j);
        if (v->n < 1) return fail(c, MCT_EINVAL, "device array length %lld", (long long)v->n);
    }
    release_device(c);  // the state arrays change: finalize again
    c->bound = v != nullptr;
    c->views = v ? *v : mct_device_views{};
    return MCT_OK;
}

int mct_finalize(mct_ctx *c) {
    if (!c) return MCT_EINVAL;
    TRI_FWD0(c, finalize);
    for (size_t q = 0; q < c->specs.size(); ++q)
        if (!c->specs[q].nx || !c->specs[q].have_material)
            return fail(c, MCT_ESTATE, "specimen %zu: mesh and material are required", q);
    release_device(c);

    int64_t nn = 0, ne = 0, np = 0, ncv = 0;
    bool any_gc = false;
    for (Spec &s : c->specs) {
        s.curve_off = ncv;
        ncv += (int64_t)s.curve_t.size();
        s.node_off = nn;
        s.elem_off = ne;
        s.perim_off = np;
        nn += s.nn;
        ne += s.ne;
        np += s.np;
        any_gc = any_gc || !s.gc.empty();
    }
    std::vector<double> X(nn), Y(nn), minv(nn), fext(2 * np, 0.0), v0(2 * np, 0.0), gc, area_all(ne);
    std::vector<uint8_t> vmask(np, 0), split(ne, 0);
    if (any_gc) gc.resize(ne);

    for (Spec &s : c->specs) {
        const int nx = s.nx, ny = s.ny;
        const double *sX = s.X.data(), *sY = s.Y.data();
        std::copy(s.X.begin(), s.X.end(), X.begin() + s.node_off);
        std::copy(s.Y.begin(), s.Y.end(), Y.begin() + s.node_off);
        // lumped mass: rho A_e / 4 from each element, element-id order per node
        double *area = area_all.data() + s.elem_off;
        for (int64_t e = 0; e < s.ne; ++e) area[e] = elem_area(s, e);
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double m = 0.0;
                const int ei[4] = {i - 1, i, i - 1, i}, ej[4] = {j - 1, j - 1, j, j};
                for (int q = 0; q < 4; ++q) {
                    if (ei[q] < 0 || ei[q] >= nx || ej[q] < 0 || ej[q] >= ny) continue;
                    m += s.rho * area[(int64_t)ej[q] * nx + ei[q]] / 4.0;
                }
                minv[s.node_off + node_of(s, i, j)] = 1.0 / m;
            }
        // equivalent nodal forces of the tractions (edge-id order) and
        // prescribed velocities, on perimeter-indexed arrays
        double *fe = fext.data() + 2 * s.perim_off;
        for (const TractionEdge &t : s.traction) {
            const double dx = sX[t.hi] - sX[t.lo], dy = sY[t.hi] - sY[t.lo];
            const double L = std::sqrt(dx * dx + dy * dy);
            const double fx = t.tx * L * 0.5, fy = t.ty * L * 0.5;
            for (int32_t nd : {t.lo, t.hi}) {
                const int pi = perimeter_index(nd % (nx + 1), nd / (nx + 1), nx, ny);
                fe[2 * pi] += fx;
                fe[2 * pi + 1] += fy;
            }
        }
        for (size_t q = 0; q < s.vbc_node.size(); ++q) {
            const int nd = s.vbc_node[q];
            const int pi = perimeter_index(nd % (nx + 1), nd / (nx + 1), nx, ny);
            vmask[s.perim_off + pi] = s.vbc_mask[q];
            v0[2 * (s.perim_off + pi)] = s.vbc_v0[2 * q];
            v0[2 * (s.perim_off + pi) + 1] = s.vbc_v0[2 * q + 1];
        }
        // time step
        if (s.dt_in > 0) {
            s.dt = s.dt_in;
        } else {
            double hmin = INFINITY;
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    const int64_t a = node_of(s, i, j);
                    if (i < nx) {
                        const double dx = sX[a + 1] - sX[a], dy = sY[a + 1] - sY[a];
                        hmin = std::min(hmin, std::sqrt(dx * dx + dy * dy));
                    }
                    if (j < ny) {
                        const int64_t b = a + nx + 1;
                        const double dx = sX[b] - sX[a], dy = sY[b] - sY[a];
                        hmin = std::min(hmin, std::sqrt(dx * dx + dy * dy));
                    }
                }
            const double cd = std::sqrt(s.E / (s.rho * (1.0 - s.nu * s.nu)));
            s.dt = s.cfl * hmin / cd;
        }
        for (size_t q = 0; q < s.notch_elem.size(); ++q) split[s.elem_off + s.notch_elem[q]] = s.notch_code[q];
        if (any_gc && !s.gc.empty()) std::copy(s.gc.begin(), s.gc.end(), gc.begin() + s.elem_off);
    }

    int rc;
    if ((rc = upload(c, c->dX, X))) return rc;
    if ((rc = upload(c, c->dY, Y))) return rc;
    if ((rc = upload(c, c->dminv, minv))) return rc;
    if ((rc = upload(c, c->dfext, fext))) return rc;
    if ((rc = upload(c, c->dv0, v0))) return rc;
    if ((rc = upload(c, c->dvmask, vmask))) return rc;
    if ((rc = upload(c, c->dsplit, split))) return rc;
    if ((rc = upload(c, c->darea, area_all))) return rc;
    if (ncv) {
        std::vector<double> curves(2 * ncv);
        for (const Spec &s : c->specs) {
            std::copy(s.curve_t.begin(), s.curve_t.end(), curves.begin() + s.curve_off);
            std::copy(s.curve_phi.begin(), s.curve_phi.end(), curves.begin() + ncv + s.curve_off);
        }
        if ((rc = upload(c, c->dcurve, curves))) return rc;
    }
    if (any_gc && (rc = upload(c, c->dgc, gc))) return rc;
    if (c->bound && c->views.n < nn)
        return fail(c, MCT_EINVAL, "bound device arrays hold %lld values, the mesh has %lld nodes",
                    (long long)c->views.n, (long long)nn);
    for (int i = 0; i < 2; ++i) {
        if (c->bound) {
            c->dux[i] = c->views.ux[i];
            c->duy[i] = c->views.uy[i];
        } else {
            HIP_TRY(c, hipMalloc((void **)&c->dux[i], sizeof(double) * nn));
            HIP_TRY(c, hipMalloc((void **)&c->duy[i], sizeof(double) * nn));
        }
        HIP_TRY(c, hipMemsetAsync(c->dux[i], 0, sizeof(double) * nn, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->duy[i], 0, sizeof(double) * nn, c->stream));
    }
    if (c->bound) {
        c->dvx = c->views.vx;
        c->dvy = c->views.vy;
    } else {
        HIP_TRY(c, hipMalloc((void **)&c->dvx, sizeof(double) * nn));
        HIP_TRY(c, hipMalloc((void **)&c->dvy, sizeof(double) * nn));
    }
    HIP_TRY(c, hipMemsetAsync(c->dvx, 0, sizeof(double) * nn, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->dvy, 0, sizeof(double) * nn, c->stream));
    if (c->precision == 32) {
        // the binary32 step's arrays: the binary64 set-up values rounded once
        auto to_f32 = [](const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); };
        const std::vector<float> fX = to_f32(X), fY = to_f32(Y), fminv = to_f32(minv), ffext = to_f32(fext),
                                 fv0 = to_f32(v0), farea = to_f32(area_all), fgc = to_f32(gc);
        if ((rc = upload(c, c->fX, fX))) return rc;
        if ((rc = upload(c, c->fY, fY))) return rc;
        if ((rc = upload(c, c->fminv, fminv))) return rc;
        if ((rc = upload(c, c->ffext, ffext))) return rc;
        if ((rc = upload(c, c->fv0, fv0))) return rc;
        if ((rc = upload(c, c->farea, farea))) return rc;
        if (any_gc && (rc = upload(c, c->fgc, fgc))) return rc;
        float **zs[6] = {&c->fux[0], &c->fuy[0], &c->fux[1], &c->fuy[1], &c->fvx, &c->fvy};
        for (float **z : zs) {
            HIP_TRY(c, hipMalloc((void **)z, sizeof(float) * nn));
            HIP_TRY(c, hipMemsetAsync(*z, 0, sizeof(float) * nn, c->stream));
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));  // before the host vectors go
    }
    HIP_TRY(c, hipMalloc((void **)&c->dctl, sizeof(Control) * c->specs.size()));
    {
        std::vector<Control> h0(c->specs.size());
        std::memset(h0.data(), 0, sizeof(Control) * h0.size());
        for (size_t q = 0; q < c->specs.size(); ++q) {
            int32_t tip = -1;
            if (c->specs[q].sct && (rc = start_tip(c, q, &tip))) return rc;
            h0[q].tip0 = h0[q].tip1 = tip;
        }
        HIP_TRY(c, hipMemcpy(c->dctl, h0.data(), sizeof(Control) * h0.size(), hipMemcpyHostToDevice));
    }
    // the log of a specimen holds up to one split per element
    HIP_TRY(c, hipMalloc((void **)&c->dlog, sizeof(LogRec) * (size_t)std::max<int64_t>(ne, 1)));
    const bool front = !c->batch && c->specs[0].front_rho > 0;
    if (front) {
        if (c->specs[0].sct) return fail(c, MCT_EINVAL, "per-front pick and single-tip tracking exclude each other");
        if (c->screen_on) return fail(c, MCT_EUNSUPPORTED, "per-front pick with the split-screen");
        const size_t cap = 4 * (size_t)std::max<int64_t>(ne, 1);  // up to four candidates per element
        HIP_TRY(c, hipMalloc((void **)&c->dfcand, sizeof(mct::AccCand) * cap));
        HIP_TRY(c, hipMalloc((void **)&c->dfcount, sizeof(uint32_t)));
        HIP_TRY(c, hipMemsetAsync(c->dfcount, 0, sizeof(uint32_t), c->stream));
        HIP_TRY(c, hipMalloc((void **)&c->dfmid, sizeof(double2) * cap));
        HIP_TRY(c, hipMalloc((void **)&c->dflen, sizeof(double) * cap));
        HIP_TRY(c, hipMalloc((void **)&c->dforder, sizeof(int32_t) * cap));
        HIP_TRY(c, hipMalloc((void **)&c->dfbucket, sizeof(int32_t) * cap));
        HIP_TRY(c, hipMalloc((void **)&c->dfsorted, sizeof(int32_t) * cap));
        HIP_TRY(c, hipMalloc((void **)&c->dfplist, sizeof(int32_t) * cap));
        if (ne >= mct::kFrontGridMinElements && std::isfinite(c->specs[0].front_rho)) {
            // the pick over the whole GPU: its two bucket tables
            HIP_TRY(c, hipMalloc((void **)&c->dfgrid, sizeof(int32_t) * 2 * mct::kFrontGridTable));
            HIP_TRY(c, mct::front_grid_reset(c->dfgrid, c->stream));
        }
        // hash cell: at least rho and the largest distance between two nodes
        // of an element (so same-element candidates are neighbours too)
        const Spec &s0 = c->specs[0];
        double dmax = 0.0;
        for (int j = 0; j < s0.ny; ++j)
            for (int i = 0; i < s0.nx; ++i) {
                const int64_t nd[4] = {node_of(s0, i, j), node_of(s0, i + 1, j), node_of(s0, i + 1, j + 1),
                                       node_of(s0, i, j + 1)};
                for (int a = 0; a < 4; ++a)
                    for (int b = a + 1; b < 4; ++b)
                        dmax = std::max(dmax, std::hypot(s0.X[nd[a]] - s0.X[nd[b]], s0.Y[nd[a]] - s0.Y[nd[b]]));
            }
        c->front_cell = std::max(s0.front_rho, dmax) * (1.0 + 1e-9);
    }
    int64_t max_ns = 0;
    for (const Spec &s : c->specs) max_ns = std::max(max_ns, s.ns);
    HIP_TRY(c, hipMalloc((void **)&c->dtip_counts, sizeof(int32_t) * (size_t)mct::tips_nblocks(max_ns)));
    HIP_TRY(c, hipMalloc((void **)&c->dtip_total, sizeof(int32_t)));

    for (size_t q = 0; q < c->specs.size(); ++q) {
        Spec &s = c->specs[q];
        StepParams &p = s.prm;
        p.nx = s.nx;
        p.ny = s.ny;
        p.log_cap = (int32_t)std::min<int64_t>(s.ne, INT32_MAX);
        p.X = c->dX + s.node_off;
        p.Y = c->dY + s.node_off;
        p.ux0 = c->dux[0] + s.node_off;
        p.uy0 = c->duy[0] + s.node_off;
        p.ux1 = c->dux[1] + s.node_off;
        p.uy1 = c->duy[1] + s.node_off;
        p.vx = c->dvx + s.node_off;
        p.vy = c->dvy + s.node_off;
        p.minv = c->dminv + s.node_off;
        p.split = c->dsplit + s.elem_off;
        p.area = c->darea + s.elem_off;
        p.gc = s.gc.empty() ? nullptr : c->dgc + s.elem_off;
        p.gc_uniform = s.gc_uniform;
        p.fext_p = c->dfext + 2 * s.perim_off;
        p.vmask_p = c->dvmask + s.perim_off;
        p.v0_p = c->dv0 + 2 * s.perim_off;
        p.D11 = s.E / (1.0 - s.nu * s.nu);
        p.D12 = s.nu * p.D11;
        p.D33 = s.E / (2.0 * (1.0 + s.nu));
        p.E = s.E;
        p.dt = s.dt;
        p.dts = s.dt;
        p.t_ramp = s.t_ramp;
        p.gamma = s.gamma;
        p.sct = s.sct;
        p.ncurve = (int32_t)s.curve_t.size();
        p.curve_t = p.ncurve ? c->dcurve + s.curve_off : nullptr;
        p.curve_phi = p.ncurve ? c->dcurve + ncv + s.curve_off : nullptr;
        p.ctl = c->dctl + q;
        p.log = c->dlog + s.elem_off;
        p.subcell = s.subcell;
        p.front = front ? 1 : 0;
        p.fcap = front ? (int32_t)(4 * s.ne) : 0;
        p.front_r2 = front ? s.front_rho * s.front_rho : 0.0;
        p.fcand = c->dfcand;
        p.fcount = c->dfcount;
        p.fmid = c->dfmid;
        p.flen = c->dflen;
        p.forder = c->dforder;
        p.fbucket = c->dfbucket;
        p.fsorted = c->dfsorted;
        p.fplist = c->dfplist;
        p.fcell = c->front_cell;
        p.fgrid = c->dfgrid;
        p.lat = nullptr;
        p.near = nullptr;
        p.near_count = nullptr;
        p.near_cap = 0;
        p.near_tol = 0.0;
    }
    // near-threshold decision log (plain contexts)
    if (c->near_tol > 0.0 && !c->batch) {
        HIP_TRY(c, hipMalloc((void **)&c->dnear, sizeof(mct::NearRec) * (size_t)c->near_cap));
        HIP_TRY(c, hipMalloc((void **)&c->dnear_count, sizeof(uint32_t)));
        HIP_TRY(c, hipMemsetAsync(c->dnear_count, 0, sizeof(uint32_t), c->stream));
        StepParams &p = c->specs[0].prm;
        p.near = c->dnear;
        p.near_count = c->dnear_count;
        p.near_cap = (int32_t)c->near_cap;
        p.near_tol = c->near_tol;
    }
    // uniform lattices: binary64 point rule, every element's geometry equal
    // bit for bit to element 0's (checked on the device with the step's own
    // arithmetic); the step then takes the shared values
    if (c->precision == 64 && c->lattice_mode == 0) {
        const size_t nsp = c->specs.size();
        HIP_TRY(c, hipMalloc((void **)&c->dlat, sizeof(mct::LatticeConst) * nsp));
        HIP_TRY(c, hipMalloc((void **)&c->dlat_flag, sizeof(uint32_t) * nsp));
        bool all = true;
        for (size_t q = 0; q < nsp; ++q) {
            const Spec &sq = c->specs[q];
            if (sq.subcell) {
                all = false;
                continue;
            }
            HIP_TRY(c, mct::launch_lattice_check(sq.prm, c->dlat + q, c->dlat_flag + q, c->stream));
        }
        std::vector<uint32_t> flags(nsp, 1u);
        HIP_TRY(c, hipMemcpyAsync(flags.data(), c->dlat_flag, sizeof(uint32_t) * nsp, hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (size_t q = 0; q < nsp && all; ++q) all = !c->specs[q].subcell && flags[q] == 0;
        if (all) {
            for (size_t q = 0; q < nsp; ++q) c->specs[q].prm.lat = c->dlat + q;
            c->uni = true;
        }
    }
    c->finalized = true;  // the launch geometry below needs the device arrays
    rc = set_launch_geometry(c);
    if (rc) {
        c->finalized = false;
        return rc;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t q = 0; q < c->specs.size(); ++q) {
        Spec &sp = c->specs[q];
        if ((rc = stability_limit(c, sp))) {
            c->finalized = false;
            return rc;
        }
        if (sp.dt > sp.dt_limit) {
            c->finalized = false;
            return fail(c, MCT_ESTABILITY, "specimen %zu: dt = %g exceeds the stability limit 2/omega_max = %g", q,
                        sp.dt, sp.dt_limit);
        }
    }
    c->steps_enqueued = 0;
    return MCT_OK;
}

int mct_step(mct_ctx *c, int64_t n) {
    if (!c) return MCT_EINVAL;
    TRI_FWD(c, step, n);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (n < 0) return fail(c, MCT_EINVAL, "negative step count");
    if (c->screen_on) return step_screened(c, n);
    int64_t left = n;
    if (c->use_graph) {
        while (left >= kGraphSteps) {
            const int par0 = (int)(c->steps_enqueued & 1);
            if (!c->graph[par0] || c->graph_tile[par0] != c->tile) {
                int rc = build_graph(c, par0);
                if (rc) return rc;
            }
            HIP_TRY(c, hipGraphLaunch(c->graph[par0], c->stream));
            left -= kGraphSteps;
            c->steps_enqueued += kGraphSteps;
        }
        if (left > 0) {  // the tail, as a shorter captured segment
            const int par0 = (int)(c->steps_enqueued & 1);
            const int n_tail = (int)left;
            if (!c->tgraph[par0] || c->tgraph_tile[par0] != c->tile || c->tgraph_n[par0] != n_tail) {
                int rc = build_graph(c, par0, n_tail);
                if (rc) return rc;
            }
            HIP_TRY(c, hipGraphLaunch(c->tgraph[par0], c->stream));
            c->steps_enqueued += n_tail;
            left = 0;
        }
    }
    const mct::Launch L = launch_of(c);
    while (left > 0) {
        // direct segment, closed by its commit
        const int seg = (int)std::min<int64_t>(left, 1 << 20);
        const int par0 = (int)(c->steps_enqueued & 1);
        HIP_TRY(c, enqueue_segment(c, L, seg, par0, c->stream));
        left -= seg;
        c->steps_enqueued += seg;
    }
    return MCT_OK;
}

int mct_profile_step(mct_ctx *c, int64_t n, double out_us[2]) {
    if (!c || !out_us) return MCT_EINVAL;
    if (c->tri) return fail(c, MCT_EUNSUPPORTED, "step timing is for structured grids");
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (c->screen_on) return fail(c, MCT_EUNSUPPORTED, "step timing with the split-screen");
    if (n < 1 || n > 4096) return fail(c, MCT_EINVAL, "step count %lld outside 1..4096", (long long)n);
    const bool each = commit_each_step(c);
    const int nc = each ? (int)n : 1;  // commits timed
    std::vector<hipEvent_t> ev(2 * (size_t)n + 2 * (size_t)nc, nullptr);
    int rc = MCT_OK;
    for (hipEvent_t &e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(c, MCT_EDEVICE, "event create");
    const mct::Launch L = launch_of(c);
    const int par0 = (int)(c->steps_enqueued & 1);
    hipError_t e = hipSuccess;
    for (int64_t i = 0; !rc && e == hipSuccess && i < n; ++i) {
        e = hipEventRecord(ev[2 * i], c->stream);
        if (e == hipSuccess)
            e = each ? mct::launch_step(c->tile, L, 0, (int)((par0 + i) & 1), c->stream)
                     : mct::launch_step(c->tile, L, (int)i, par0, c->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[2 * i + 1], c->stream);
        if (e == hipSuccess && (each || i == n - 1)) {
            const size_t q = 2 * (size_t)n + 2 * (size_t)(each ? i : 0);
            e = hipEventRecord(ev[q], c->stream);
            if (e == hipSuccess) e = mct::launch_commit(L, each ? 1 : (int)n, c->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[q + 1], c->stream);
        }
    }
    if (!rc && e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (!rc && e != hipSuccess) rc = fail(c, MCT_EDEVICE, "step timing: %s", hipGetErrorString(e));
    if (!rc) {
        c->steps_enqueued += n;
        double ts = 0.0, tc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
            ts += ms;
        }
        for (int i = 0; i < nc; ++i) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[2 * n + 2 * i], ev[2 * n + 2 * i + 1]);
            tc += ms;
        }
        out_us[0] = 1e3 * ts / (double)n;
        out_us[1] = 1e3 * tc / (double)n;
    }
    for (hipEvent_t &x : ev)
        if (x) (void)hipEventDestroy(x);
    return rc;
}

int mct_sync(mct_ctx *c) {
    if (!c) return MCT_EINVAL;
    TRI_FWD0(c, sync);
    if (c->finalized) {
        // watchdog: every displacement and velocity of the current step finite
        int rc = ensure_eval(c);
        if (rc) return rc;
        int64_t nn = 0;
        for (const Spec &s : c->specs) nn += s.nn;
        const int par = (int)(c->steps_enqueued & 1);
        int32_t flag = 0;
        if ((rc = widen_state(c))) return rc;
        HIP_TRY(c, hipMemsetAsync(c->dflag, 0, sizeof(int32_t), c->stream));
        HIP_TRY(c, mct::launch_check_finite(c->dux[par], c->duy[par], c->dvx, c->dvy, nn, c->dflag, c->stream));
        HIP_TRY(c, hipMemcpyAsync(&flag, c->dflag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (flag) return fail(c, MCT_ENUMERIC, "non-finite displacement or velocity after step %lld",
                              (long long)c->steps_enqueued);
        return MCT_OK;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

int mct_get_info(mct_ctx *c, mct_info *out) {
    if (!c || !out) return MCT_EINVAL;
    TRI_FWD(c, get_info, out);
    std::memset(out, 0, sizeof *out);
    const Spec &s = cur(c);
    out->n_nodes = s.nn;
    out->n_elems = s.ne;
    out->n_edges = s.ns;
    out->dt = s.dt;
    out->dt_limit = s.dt_limit;
    out->precision = c->precision;
    if (!c->finalized) return MCT_OK;
    Control h;
    int rc = read_control(c, c->sel, &h);
    if (rc) return rc;
    out->step = h.base;
    out->n_splits = h.nsplit;
    out->dissipated = h.Ud;
    out->log_overflow = h.overflow;
    out->tip = s.sct ? ((((h.base - 1) & 1) != 0) ? h.tip1 : h.tip0) : -1;
    return MCT_OK;
}

int mct_get_crack_set(mct_ctx *c, int64_t cap, int32_t *step, int32_t *elem, uint8_t *entry, uint8_t *exit,
                      double *G, int64_t *count) {
    if (!c || !count) return MCT_EINVAL;
    TRI_FWD(c, get_crack_set, cap, step, elem, entry, exit, G, count);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const Spec &s = cur(c);
    Control h;
    int rc = read_control(c, c->sel, &h);
    if (rc) return rc;
    const int64_t n = std::min<int64_t>(h.nsplit, s.prm.log_cap);
    *count = n;
    if (cap < n) return fail(c, MCT_ECAPACITY, "crack set holds %lld splits", (long long)n);
    std::vector<LogRec> v((size_t)n);
    if (n) {
        HIP_TRY(c, hipMemcpyAsync(v.data(), s.prm.log, sizeof(LogRec) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    for (int64_t i = 0; i < n; ++i) {
        if (step) step[i] = v[i].step;
        if (elem) elem[i] = v[i].elem;
        if (entry) entry[i] = v[i].entry;
        if (exit) exit[i] = v[i].exit;
        if (G) G[i] = v[i].G;
    }
    return MCT_OK;
}

int mct_get_tips(mct_ctx *c, int64_t cap, int32_t *edge, double *xy, int64_t *count) {
    if (!c || !count) return MCT_EINVAL;
    TRI_FWD(c, get_tips, cap, edge, xy, count);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const Spec &s = cur(c);
    int32_t nb = 0, total = 0;
    HIP_TRY(c, mct::launch_tips(s.nx, s.ny, s.prm.X, s.prm.Y, s.prm.split, c->dtip_counts, &nb, nullptr, nullptr,
                                c->dtip_total, 0, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&total, c->dtip_total, sizeof total, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *count = total;
    if (cap < total) return fail(c, MCT_ECAPACITY, "%d tips", total);
    if (!total) return MCT_OK;
    int32_t *de = nullptr;
    double *dxy = nullptr;
    HIP_TRY(c, hipMalloc((void **)&de, sizeof(int32_t) * (size_t)total));
    if (hipMalloc((void **)&dxy, sizeof(double) * 2 * (size_t)total) != hipSuccess) {
        (void)hipFree(de);
        return fail(c, MCT_ENOMEM, "tip buffers");
    }
    hipError_t e = mct::launch_tips(s.nx, s.ny, s.prm.X, s.prm.Y, s.prm.split, c->dtip_counts, &nb, de, dxy,
                                    c->dtip_total, total, c->stream);
    if (e == hipSuccess && edge)
        e = hipMemcpyAsync(edge, de, sizeof(int32_t) * (size_t)total, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && xy)
        e = hipMemcpyAsync(xy, dxy, sizeof(double) * 2 * (size_t)total, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(de);
    (void)hipFree(dxy);
    if (e != hipSuccess) return fail(c, MCT_EDEVICE, "tips: %s", hipGetErrorString(e));
    return MCT_OK;
}

int mct_get_tips_noalloc(mct_ctx *c, int64_t cap, int32_t *edge_dev, double *xy_dev, int32_t *count_dev) {
    if (!c) return MCT_EINVAL;
    if (c->tri) return fail(c, MCT_EUNSUPPORTED, "the no-allocation tip query is for structured grids");
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (!count_dev || cap < 0 || (cap > 0 && (!edge_dev || !xy_dev)))
        return fail(c, MCT_EINVAL, "null device output or negative capacity");
    const Spec &s = cur(c);
    if (mct::tips_nblocks(s.ns) > mct::kTipScratchBlocks)
        return fail(c, MCT_EINVAL, "%lld edges: the no-allocation tip query handles at most %lld",
                    (long long)s.ns, (long long)mct::kTipScratchBlocks * 256);
    int dev = -1;
    HIP_TRY(c, hipGetDevice(&dev));
    if (dev != c->device) return fail(c, MCT_EDEVICE, "device %d is current, the context is on device %d", dev, c->device);
    int32_t *scr = nullptr;
    HIP_TRY(c, mct::tips_scratch(&scr));
    int32_t nb = 0;
    // asynchronous on the context's stream: count (block counts in the
    // scratch array, every entry written), scan (the total into *count_dev),
    // write (at most cap tips)
    HIP_TRY(c, mct::launch_tips(s.nx, s.ny, s.prm.X, s.prm.Y, s.prm.split, scr, &nb, cap > 0 ? edge_dev : nullptr,
                                xy_dev, count_dev, cap, c->stream));
    return MCT_OK;
}

int mct_get_field(mct_ctx *c, int which, int64_t cap, double *out) {
    if (!c || !out) return MCT_EINVAL;
    TRI_FWD(c, get_field, which, cap, out);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const Spec &s = cur(c);
    int64_t need;
    switch (which) {
        case MCT_FIELD_U: case MCT_FIELD_V: case MCT_FIELD_A: case MCT_FIELD_FINT: need = 2 * s.nn; break;
        case MCT_FIELD_SIGMA_EDGE: need = 3 * s.ns; break;
        case MCT_FIELD_PRINCIPAL: need = s.ne; break;
        default: return fail(c, MCT_EINVAL, "unknown field %d", which);
    }
    if (cap < need) return fail(c, MCT_ECAPACITY, "field needs %lld values", (long long)need);
    int rc = widen_state(c);
    if (rc) return rc;
    Control h;
    if ((rc = read_control(c, c->sel, &h))) return rc;
    if (which >= MCT_FIELD_A) {
        if ((rc = ensure_eval(c))) return rc;
        const double *ux = (h.base & 1) ? s.prm.ux1 : s.prm.ux0, *uy = (h.base & 1) ? s.prm.uy1 : s.prm.uy0;
        HIP_TRY(c, mct::launch_eval(s.prm, ux, uy, s.prm.vx, s.prm.vy, h.base,
                                    load_factor_host(s, (double)h.base * s.dt), c->ev, c->stream));
        if (which == MCT_FIELD_A || which == MCT_FIELD_FINT) {
            const double *src = which == MCT_FIELD_A ? c->ev.acc : c->ev.fint;
            HIP_TRY(c, hipMemcpyAsync(out, src, sizeof(double) * 2 * s.nn, hipMemcpyDeviceToHost, c->stream));
        } else if (which == MCT_FIELD_SIGMA_EDGE) {
            std::vector<double> sg(3 * s.ns);
            HIP_TRY(c, hipMemcpyAsync(sg.data(), c->ev.sig, sizeof(double) * 3 * s.ns, hipMemcpyDeviceToHost,
                                      c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            for (int64_t e = 0; e < s.ns; ++e)
                for (int q = 0; q < 3; ++q) out[q * s.ns + e] = sg[3 * e + q];
        } else {
            HIP_TRY(c, mct::launch_principal(s.prm, c->ev, c->ev.fe, c->stream));  // fe reused as output
            HIP_TRY(c, hipMemcpyAsync(out, c->ev.fe, sizeof(double) * s.ne, hipMemcpyDeviceToHost, c->stream));
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return MCT_OK;
    }
    const double *sx, *sy;
    if (which == MCT_FIELD_U) {
        sx = (h.base & 1) ? s.prm.ux1 : s.prm.ux0;
        sy = (h.base & 1) ? s.prm.uy1 : s.prm.uy0;
    } else {
        sx = s.prm.vx;
        sy = s.prm.vy;
    }
    HIP_TRY(c, hipMemcpyAsync(out, sx, sizeof(double) * s.nn, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(out + s.nn, sy, sizeof(double) * s.nn, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

int mct_get_energies(mct_ctx *c, double out[4]) {
    if (!c || !out) return MCT_EINVAL;
    TRI_FWD(c, get_energies, out);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    int rc = ensure_eval(c);
    if (rc) return rc;
    const Spec &s = cur(c);
    if ((rc = widen_state(c))) return rc;
    Control h;
    if ((rc = read_control(c, c->sel, &h))) return rc;
    const double *ux = (h.base & 1) ? s.prm.ux1 : s.prm.ux0, *uy = (h.base & 1) ? s.prm.uy1 : s.prm.uy0;
    HIP_TRY(c, mct::launch_eval(s.prm, ux, uy, s.prm.vx, s.prm.vy, h.base,
                                load_factor_host(s, (double)h.base * s.dt), c->ev, c->stream));
    HIP_TRY(c, mct::launch_energies(s.prm, c->ev, c->ev.sums, c->stream));
    double r[8];
    HIP_TRY(c, hipMemcpyAsync(r, c->ev.sums, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out[0] = r[0];
    out[1] = r[3] + r[4];
    out[2] = r[2];
    out[3] = h.Ud;
    return MCT_OK;
}

int mct_get_path_geometry(mct_ctx *c, int64_t n, const int32_t *elem, double *out) {
    if (!c || n < 0 || (n && (!elem || !out))) return MCT_EINVAL;
    TRI_FWD(c, get_path_geometry, n, elem, out);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const Spec &s = cur(c);
    if (n > INT32_MAX / 36) return fail(c, MCT_EINVAL, "too many elements");
    for (int64_t i = 0; i < n; ++i)
        if (elem[i] < 0 || elem[i] >= s.ne) return fail(c, MCT_EINVAL, "element %d out of range", elem[i]);
    if (!n) return MCT_OK;
    int32_t *de = nullptr;
    double *dout = nullptr;
    HIP_TRY(c, hipMalloc((void **)&de, sizeof(int32_t) * (size_t)n));
    if (hipMalloc((void **)&dout, sizeof(double) * 36 * (size_t)n) != hipSuccess) {
        (void)hipFree(de);
        return fail(c, MCT_ENOMEM, "geometry buffer");
    }
    hipError_t e = hipMemcpyAsync(de, elem, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = mct::launch_path_geometry(s.prm, (int)n, de, dout, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dout, sizeof(double) * 36 * (size_t)n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(de);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(c, MCT_EDEVICE, "path geometry: %s", hipGetErrorString(e));
    return MCT_OK;
}

int mct_get_split_codes(mct_ctx *c, int64_t cap, uint8_t *out) {
    if (!c || !out) return MCT_EINVAL;
    TRI_FWD(c, get_split_codes, cap, out);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const Spec &s = cur(c);
    if (cap < s.ne) return fail(c, MCT_ECAPACITY, "need %lld bytes", (long long)s.ne);
    HIP_TRY(c, hipMemcpyAsync(out, s.prm.split, (size_t)s.ne, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

// checkpoint layout: magic, number of specimens, then per specimen: nodes,
// elements, Control, u, v (x then y, binary64; a binary32 context's values
// are exact in them), split codes, log records.  The magic differs by
// precision, so a state moves only between contexts of one precision.
static const uint64_t kMagic = 0x4d43543244434b32ull;    // "MCT2DCK2"
static const uint64_t kMagic32 = 0x4d43543246434b32ull;  // "MCT2FCK2"
static const uint64_t kScreenTag = 0x314e524353544d43ull;  // "MCTSCRN1"

// Optional last section of a plain context's checkpoint: the learned
// split-screen's state (per-element screen states, the per-candidate history
// behind feature 4 and its stamps, the evaluation count, the counters), so
// that a restored screened run continues exactly where it was.
static int64_t screen_section_bytes(const mct_ctx *c) {
    if (c->batch || !c->screen_alloc) return 0;
    const int64_t ne = c->specs[0].ne;
    return 16 + 4 * ne + 8 * 4 * ne + 4 * 4 * ne + 8 + 8 * mct::kNumScreenStats;
}

int mct_checkpoint(mct_ctx *c, void *buf, int64_t cap, int64_t *bytes) {
    if (!c || !bytes) return MCT_EINVAL;
    TRI_FWD(c, checkpoint, buf, cap, bytes);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const int S = (int)c->specs.size();
    int rc = widen_state(c);
    if (rc) return rc;
    std::vector<Control> h(S);
    HIP_TRY(c, hipMemcpyAsync(h.data(), c->dctl, sizeof(Control) * S, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int64_t need = 16;
    for (int q = 0; q < S; ++q) {
        const Spec &s = c->specs[q];
        const int64_t nlog = std::min<int64_t>(h[q].nsplit, s.prm.log_cap);
        need += 16 + (int64_t)sizeof(Control) + 32 * s.nn + s.ne + nlog * (int64_t)sizeof(LogRec);
    }
    need += screen_section_bytes(c);
    *bytes = need;
    if (!buf) return MCT_OK;
    if (cap < need) return fail(c, MCT_ECAPACITY, "checkpoint needs %lld bytes", (long long)need);
    char *p = (char *)buf;
    const uint64_t hdr[2] = {c->precision == 32 ? kMagic32 : kMagic, (uint64_t)S};
    std::memcpy(p, hdr, sizeof hdr);
    p += sizeof hdr;
    for (int q = 0; q < S; ++q) {
        const Spec &s = c->specs[q];
        const uint64_t sh[2] = {(uint64_t)s.nn, (uint64_t)s.ne};
        std::memcpy(p, sh, sizeof sh);
        p += sizeof sh;
        std::memcpy(p, &h[q], sizeof(Control));
        p += sizeof(Control);
        const int par = (int)(h[q].base & 1);
        const double *src[4] = {par ? s.prm.ux1 : s.prm.ux0, par ? s.prm.uy1 : s.prm.uy0, s.prm.vx, s.prm.vy};
        for (int i = 0; i < 4; ++i) {
            HIP_TRY(c, hipMemcpyAsync(p, src[i], 8 * s.nn, hipMemcpyDeviceToHost, c->stream));
            p += 8 * s.nn;
        }
        HIP_TRY(c, hipMemcpyAsync(p, s.prm.split, s.ne, hipMemcpyDeviceToHost, c->stream));
        p += s.ne;
        const int64_t nlog = std::min<int64_t>(h[q].nsplit, s.prm.log_cap);
        if (nlog) HIP_TRY(c, hipMemcpyAsync(p, s.prm.log, sizeof(LogRec) * nlog, hipMemcpyDeviceToHost, c->stream));
        p += sizeof(LogRec) * nlog;
    }
    if (screen_section_bytes(c)) {
        const mct::ScreenDev &sd = c->sd;
        const int64_t ne = c->specs[0].ne;
        const uint64_t sh[2] = {kScreenTag, (uint64_t)ne};
        std::memcpy(p, sh, sizeof sh);
        p += sizeof sh;
        HIP_TRY(c, hipMemcpyAsync(p, sd.screen, 4 * ne, hipMemcpyDeviceToHost, c->stream));
        p += 4 * ne;
        HIP_TRY(c, hipMemcpyAsync(p, sd.hist_g, 8 * 4 * ne, hipMemcpyDeviceToHost, c->stream));
        p += 8 * 4 * ne;
        HIP_TRY(c, hipMemcpyAsync(p, sd.hist_t, 4 * 4 * ne, hipMemcpyDeviceToHost, c->stream));
        p += 4 * 4 * ne;
        HIP_TRY(c, hipMemcpyAsync(p, sd.sweep, 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(p + 4, sd.nrows_last, 4, hipMemcpyDeviceToHost, c->stream));
        p += 8;
        unsigned long long st[4];
        HIP_TRY(c, hipMemcpyAsync(st, sd.stats, sizeof st, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const int64_t all[mct::kNumScreenStats] = {(int64_t)st[0], (int64_t)st[1], (int64_t)st[2], (int64_t)st[3],
                                                  c->screen_windows, c->screen_replays};
        std::memcpy(p, all, sizeof all);
        p += sizeof all;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

int mct_restore(mct_ctx *c, const void *buf, int64_t bytes) {
    if (!c || !buf) return MCT_EINVAL;
    TRI_FWD(c, restore, buf, bytes);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const char *p = (const char *)buf, *end = p + bytes;
    const int S = (int)c->specs.size();
    if (bytes < 16) return fail(c, MCT_EINVAL, "checkpoint too short");
    uint64_t hdr[2];
    std::memcpy(hdr, p, sizeof hdr);
    p += sizeof hdr;
    if (hdr[0] != (c->precision == 32 ? kMagic32 : kMagic) || (int64_t)hdr[1] != S)
        return fail(c, MCT_EINVAL, "checkpoint does not match this context (specimens or precision)");
    // validate the whole buffer before touching the device
    const char *q = p;
    std::vector<Control> hs(S);
    for (int s = 0; s < S; ++s) {
        const Spec &sp = c->specs[s];
        if (end - q < 16 + (int64_t)sizeof(Control)) return fail(c, MCT_EINVAL, "checkpoint truncated");
        uint64_t sh[2];
        std::memcpy(sh, q, sizeof sh);
        if ((int64_t)sh[0] != sp.nn || (int64_t)sh[1] != sp.ne) return fail(c, MCT_EINVAL, "checkpoint mesh mismatch");
        std::memcpy(&hs[s], q + 16, sizeof(Control));
        if (hs[s].base < 0 || hs[s].base != hs[0].base || hs[s].nsplit < 0)
            return fail(c, MCT_EINVAL, "checkpoint step mismatch");
        const int64_t nlog = std::min<int64_t>(hs[s].nsplit, sp.prm.log_cap);
        const int64_t len = 16 + (int64_t)sizeof(Control) + 32 * sp.nn + sp.ne + nlog * (int64_t)sizeof(LogRec);
        if (end - q < len) return fail(c, MCT_EINVAL, "checkpoint truncated");
        q += len;
    }
    // the optional screen section (plain contexts)
    const char *scr = nullptr;
    if (end - q >= 16) {
        uint64_t sh[2];
        std::memcpy(sh, q, sizeof sh);
        const int64_t ne = c->specs[0].ne;
        if (sh[0] != kScreenTag || c->batch || (int64_t)sh[1] != ne)
            return fail(c, MCT_EINVAL, "checkpoint has an unknown trailing section");
        const int64_t len = 16 + 4 * ne + 8 * 4 * ne + 4 * 4 * ne + 8 + 8 * mct::kNumScreenStats;
        if (end - q < len) return fail(c, MCT_EINVAL, "checkpoint truncated (screen state)");
        scr = q + 16;
    }
    if (scr) {
        int rc = ensure_screen(c);
        if (rc) return rc;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < S; ++s) {
        const Spec &sp = c->specs[s];
        p += 16 + sizeof(Control);
        Control h = hs[s];
        h.nslots[0] = h.nslots[1] = h.nslots[2] = 0;
        HIP_TRY(c, hipMemcpyAsync(c->dctl + s, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
        const int par = (int)(h.base & 1);
        double *dst[4] = {par ? sp.prm.ux1 : sp.prm.ux0, par ? sp.prm.uy1 : sp.prm.uy0, sp.prm.vx, sp.prm.vy};
        for (int i = 0; i < 4; ++i) {
            HIP_TRY(c, hipMemcpyAsync(dst[i], p, 8 * sp.nn, hipMemcpyHostToDevice, c->stream));
            p += 8 * sp.nn;
        }
        HIP_TRY(c, hipMemcpyAsync(sp.prm.split, p, sp.ne, hipMemcpyHostToDevice, c->stream));
        p += sp.ne;
        const int64_t nlog = std::min<int64_t>(h.nsplit, sp.prm.log_cap);
        if (nlog) HIP_TRY(c, hipMemcpyAsync(sp.prm.log, p, sizeof(LogRec) * nlog, hipMemcpyHostToDevice, c->stream));
        p += sizeof(LogRec) * nlog;
    }
    if (int rc = narrow_state(c)) return rc;
    if (c->dfgrid) HIP_TRY(c, mct::front_grid_reset(c->dfgrid, c->stream));
    if (scr) {  // the screen continues where the checkpoint was taken
        const mct::ScreenDev &sd = c->sd;
        const int64_t ne = c->specs[0].ne;
        const char *r = scr;
        HIP_TRY(c, hipMemcpyAsync(sd.screen, r, 4 * ne, hipMemcpyHostToDevice, c->stream));
        r += 4 * ne;
        HIP_TRY(c, hipMemcpyAsync(sd.hist_g, r, 8 * 4 * ne, hipMemcpyHostToDevice, c->stream));
        r += 8 * 4 * ne;
        HIP_TRY(c, hipMemcpyAsync(sd.hist_t, r, 4 * 4 * ne, hipMemcpyHostToDevice, c->stream));
        r += 4 * 4 * ne;
        HIP_TRY(c, hipMemcpyAsync(sd.sweep, r, 4, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(sd.nrows_last, r + 4, 4, hipMemcpyHostToDevice, c->stream));
        r += 8;
        int64_t all[mct::kNumScreenStats];
        std::memcpy(all, r, sizeof all);
        unsigned long long st[4] = {(unsigned long long)all[0], (unsigned long long)all[1],
                                    (unsigned long long)all[2], (unsigned long long)all[3]};
        HIP_TRY(c, hipMemcpyAsync(sd.stats, st, sizeof st, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->screen_windows = all[mct::kStatWindows];
        c->screen_replays = all[mct::kStatReplays];
    } else if (c->screen_alloc) {  // no screen state saved: the screen starts afresh
        const mct::ScreenDev &sd = c->sd;
        const int64_t ne = c->specs[0].ne;
        HIP_TRY(c, mct::launch_fill_u32(reinterpret_cast<uint32_t *>(sd.hist_t), 4 * ne, 0xFFFFFFFEu, c->stream));
        HIP_TRY(c, hipMemsetAsync(sd.screen, 0, sizeof(uint32_t) * ne, c->stream));
        HIP_TRY(c, hipMemsetAsync(sd.sweep, 0, sizeof(int32_t), c->stream));
        HIP_TRY(c, hipMemsetAsync(sd.stats, 0, sizeof(unsigned long long) * 4, c->stream));
        c->screen_windows = c->screen_replays = 0;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->steps_enqueued = hs[0].base;
    return MCT_OK;
}

// The step kernels in use on an unstructured mesh as a launch index: 1 split
// (workgroups of the element kernel), 2/3/4 fused on 64/128/256-node
// patches, 5 fused on patches of another size;
// workgroups of the fused kernel = patches.
static int tri_launch_index(const mct::tri::Model &m) {
    const int P = m.prm.patch_emax > 0 ? m.prm.patch_nodes : 0;
    return P == 0 ? 1 : P == 64 ? 2 : P == 128 ? 3 : P == 256 ? 4 : 5;
}

// The autotuner of an unstructured mesh: every step-kernel choice (the
// element plus node kernels, the fused kernel on 64-, 128- and 256-node
// patches and on patches of the size it finds) timed from
// the current state, which is then restored; the fastest choice is kept.
static int autotune_unstructured(mct_ctx *c, int trial_steps, int *tile_out, int *order_out,
                                 double *us_per_step_out) {
    mct::tri::Model &m = *c->tri;
    const mct::tri::Host h{c->err, c->stream};
    if (!m.finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (trial_steps < 1) return fail(c, MCT_EINVAL, "trial_steps must be positive");
    int64_t bytes = 0;
    int rc = mct::tri::checkpoint(m, h, nullptr, 0, &bytes);
    if (rc) return rc;
    std::vector<char> ck((size_t)bytes);
    if ((rc = mct::tri::checkpoint(m, h, ck.data(), bytes, &bytes))) return rc;
    const int saved_kind = m.kernels;
    const bool saved_graph = m.use_graph;
    m.use_graph = false;  // candidates are timed with direct launches
    float best = INFINITY;
    int best_kind = 1;
    const int nkinds = 5;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = MCT_EDEVICE;
    for (int kind = 1; kind <= nkinds && rc == MCT_OK; ++kind) {
        if ((rc = mct::tri::set_kernels(m, h, kind))) break;
        if ((rc = mct::tri::restore(m, h, ck.data(), bytes))) break;
        if ((rc = mct::tri::step(m, h, 2))) break;  // warm
        if (hipEventRecord(e0, c->stream) != hipSuccess) rc = MCT_EDEVICE;
        if (!rc) rc = mct::tri::step(m, h, trial_steps);
        if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = MCT_EDEVICE;
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = MCT_EDEVICE;
        float ms = 0.f;
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MCT_EDEVICE;
        if (!rc && ms < best) {
            best = ms;
            best_kind = kind;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    m.use_graph = saved_graph;
    if (rc) {
        (void)mct::tri::set_kernels(m, h, saved_kind);
        (void)mct::tri::restore(m, h, ck.data(), bytes);
        return rc == MCT_EDEVICE ? fail(c, rc, "autotune timing failed") : rc;
    }
    if ((rc = mct::tri::set_kernels(m, h, best_kind))) return rc;
    if ((rc = mct::tri::restore(m, h, ck.data(), bytes))) return rc;
    if (tile_out) *tile_out = tri_launch_index(m);
    if (order_out) *order_out = 0;
    if (us_per_step_out) *us_per_step_out = 1e3 * (double)best / trial_steps;
    return MCT_OK;
}

int mct_autotune(mct_ctx *c, int trial_steps, int *tile_out, int *order_out, double *us_per_step_out) {
    if (!c) return MCT_EINVAL;
    if (c->tri) return autotune_unstructured(c, trial_steps, tile_out, order_out, us_per_step_out);
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (trial_steps < 1) return fail(c, MCT_EINVAL, "trial_steps must be positive");
    int64_t bytes = 0;
    int rc = mct_checkpoint(c, nullptr, 0, &bytes);
    if (rc) return rc;
    std::vector<char> ck((size_t)bytes);
    if ((rc = mct_checkpoint(c, ck.data(), bytes, &bytes))) return rc;
    const int saved_tile = c->tile_req, saved_order = c->order_req;
    const bool saved_graph = c->use_graph;
    c->use_graph = false;  // candidates are timed with direct launches
    float best = INFINITY;
    int best_tile = 0, best_order = 0;
    const int norders = c->batch ? kNumOrders : 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = MCT_EDEVICE;
    for (int t = 1; t <= mct::kNumTiles && rc == MCT_OK; ++t)
        for (int o = 0; o < norders && rc == MCT_OK; ++o) {
            c->tile_req = t;
            c->order_req = o;
            if ((rc = set_launch_geometry(c))) break;
            if ((rc = mct_restore(c, ck.data(), bytes))) break;
            if ((rc = mct_step(c, 2))) break;  // warm
            if (hipEventRecord(e0, c->stream) != hipSuccess) rc = MCT_EDEVICE;
            if (!rc) rc = mct_step(c, trial_steps);
            if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = MCT_EDEVICE;
            if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = MCT_EDEVICE;
            float ms = 0.f;
            if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MCT_EDEVICE;
            if (!rc && ms < best) {
                best = ms;
                best_tile = t;
                best_order = o;
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->use_graph = saved_graph;
    if (rc) {
        c->tile_req = saved_tile;
        c->order_req = saved_order;
        (void)set_launch_geometry(c);
        (void)mct_restore(c, ck.data(), bytes);
        return rc == MCT_EDEVICE ? fail(c, rc, "autotune timing failed") : rc;
    }
    c->tile_req = best_tile;
    c->order_req = best_order;
    if ((rc = set_launch_geometry(c))) return rc;
    if ((rc = mct_restore(c, ck.data(), bytes))) return rc;
    if (tile_out) *tile_out = best_tile;
    if (order_out) *order_out = best_order;
    if (us_per_step_out) *us_per_step_out = 1e3 * (double)best / trial_steps;
    return MCT_OK;
}

int mct_get_launch(mct_ctx *c, int *tile, int *order, int64_t *workgroups) {
    if (!c) return MCT_EINVAL;
    if (c->tri) {
        const int P = c->tri->prm.patch_emax > 0 ? c->tri->prm.patch_nodes : 0;
        if (tile) *tile = tri_launch_index(*c->tri);
        if (order) *order = 0;
        if (workgroups) *workgroups = P ? (c->tri->nn + P - 1) / P : (c->tri->ne + 255) / 256;
        return MCT_OK;
    }
    if (tile) *tile = c->tile;
    if (order) *order = c->order;
    if (workgroups) *workgroups = c->batch ? c->nunits : c->specs[0].prm.nwg;
    return MCT_OK;
}


// ------------------------------------------------------------- screen

int mct_screen_collect(mct_ctx *c, int64_t cap, float *features, int32_t *elem, uint8_t *entry,
                       int64_t *count) {
    if (!c) return MCT_EINVAL;
    TRI_UNSUPPORTED(c, "the split-screen");
    if (c->precision == 32) return fail(c, MCT_EUNSUPPORTED, "the split-screen needs binary64");
    if (!count || (cap > 0 && (!features || !elem || !entry))) return fail(c, MCT_EINVAL, "null output");
    int rc = ensure_screen(c);
    if (rc) return rc;
    const bool on = c->screen_on;
    c->screen_on = false;  // features only
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    hipError_t e = screen_pipeline(c, (int)(c->steps_enqueued & 1), c->stream);
    c->screen_on = on;
    HIP_TRY(c, e);
    int32_t n = 0;
    HIP_TRY(c, hipMemcpyAsync(&n, c->sd.nrows_last, sizeof n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *count = n;
    if (n > cap) return fail(c, MCT_ECAPACITY, "%d candidates, capacity %lld", n, (long long)cap);
    if (n == 0) return MCT_OK;
    std::vector<int32_t> packed(n);
    std::vector<float> rows((size_t)mct::kFeat * n);
    HIP_TRY(c, hipMemcpyAsync(packed.data(), c->sd.cand, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(rows.data(), c->sd.feat, sizeof(float) * rows.size(), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // rows come in any order: return them by element, then local edge
    std::vector<int32_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return packed[a] < packed[b]; });
    for (int32_t i = 0; i < n; ++i) {
        const int32_t r = ord[i];
        elem[i] = packed[r] >> 2;
        entry[i] = (uint8_t)(packed[r] & 3);
        std::copy(rows.begin() + (size_t)mct::kFeat * r, rows.begin() + (size_t)mct::kFeat * (r + 1),
                  features + (size_t)mct::kFeat * i);
    }
    return MCT_OK;
}

int mct_screen_enable(mct_ctx *c, const mct_mlp *mlp, float tau, int period) {
    if (!c) return MCT_EINVAL;
    TRI_UNSUPPORTED(c, "the split-screen");
    if (c->precision == 32) return fail(c, MCT_EUNSUPPORTED, "the split-screen needs binary64");
    if (!mlp) return fail(c, MCT_EINVAL, "null model");
    if (!c->batch && cur(c).front_rho > 0) return fail(c, MCT_EUNSUPPORTED, "the split-screen with the per-front pick");
    if (!c->batch && cur(c).subcell) return fail(c, MCT_EUNSUPPORTED, "the split-screen with sub-cell smoothing");
    if (period < 2) return fail(c, MCT_EINVAL, "period must be at least 2");
    if (c->near_tol > 0.0) return fail(c, MCT_EUNSUPPORTED, "the split-screen with the near-threshold log");
    int rc = ensure_screen(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(mlp->stream));
    HIP_TRY(c, hipMemcpyAsync(c->smlp.master, mlp->d.master, sizeof(float) * mct::kParams,
                              hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, mct::launch_mlp_prep(c->smlp, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->screen_tau = tau;
    c->screen_period = period;
    c->screen_on = true;
    drop_graphs(c);
    return MCT_OK;
}

int mct_screen_disable(mct_ctx *c) {
    if (!c) return MCT_EINVAL;
    c->screen_on = false;
    drop_graphs(c);
    return MCT_OK;
}

int mct_screen_stats(mct_ctx *c, int64_t out[6]) {
    if (!c || !out) return MCT_EINVAL;
    for (int i = 0; i < mct::kNumScreenStats; ++i) out[i] = 0;
    if (!c->screen_alloc) return MCT_OK;
    unsigned long long h[4];
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(h, c->sd.stats, sizeof h, hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) out[i] = (int64_t)h[i];
    out[mct::kStatWindows] = c->screen_windows;
    out[mct::kStatReplays] = c->screen_replays;
    return MCT_OK;
}

// ------------------------------------------------------------ screen MLP

namespace {
int mfail(mct_mlp *m, int code, const char *what) {
    m->err = what;
    return code;
}
#define MLP_TRY(m, expr)                                                                            \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            (m)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                          \
            return MCT_EDEVICE;                                                                     \
        }                                                                                           \
    } while (0)
}  // namespace

int mct_mlp_create(mct_mlp **out, void *hip_stream) {
    if (!out) return MCT_EINVAL;
    *out = nullptr;
    mct_mlp *m = new (std::nothrow) mct_mlp;
    if (!m) return MCT_ENOMEM;
    bool ok = true;
    if (hip_stream) {
        m->stream = (hipStream_t)hip_stream;
    } else {
        ok = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) == hipSuccess;
        m->own_stream = ok;
    }
    mct::MlpDev &d = m->d;
    ok = ok && hipMalloc((void **)&d.master, sizeof(float) * mct::kParams) == hipSuccess;
    ok = ok && hipMalloc((void **)&d.m, sizeof(float) * mct::kParams) == hipSuccess;
    ok = ok && hipMalloc((void **)&d.v, sizeof(float) * mct::kParams) == hipSuccess;
    ok = ok && hipMalloc((void **)&d.w1b, sizeof(uint16_t) * 32 * mct::kHidden) == hipSuccess;
    ok = ok && hipMalloc((void **)&d.w2b, sizeof(uint16_t) * mct::kHidden * mct::kHidden) == hipSuccess;
    ok = ok && hipMalloc((void **)&d.w3b, sizeof(uint16_t) * mct::kHidden) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->grad, sizeof(float) * (mct::kParams + 1)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->partials,
                         sizeof(float) * (mct::kParams + 1) * (size_t)mct::mlp_train_blocks(INT64_MAX)) == hipSuccess;
    ok = ok && hipMemsetAsync(d.master, 0, sizeof(float) * mct::kParams, m->stream) == hipSuccess;
    ok = ok && hipMemsetAsync(d.m, 0, sizeof(float) * mct::kParams, m->stream) == hipSuccess;
    ok = ok && hipMemsetAsync(d.v, 0, sizeof(float) * mct::kParams, m->stream) == hipSuccess;
    ok = ok && mct::launch_mlp_prep(d, m->stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(m->stream) == hipSuccess;
    if (!ok) {
        mct_mlp_destroy(m);
        return MCT_EDEVICE;
    }
    *out = m;
    return MCT_OK;
}

int mct_mlp_destroy(mct_mlp *m) {
    if (!m) return MCT_OK;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    free_mlp(m->d);
    dfree(m->grad);
    dfree(m->partials);
    if (m->own_stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return MCT_OK;
}

const char *mct_mlp_last_error(const mct_mlp *m) { return m ? m->err.c_str() : "null model"; }

int mct_mlp_set_params(mct_mlp *m, const float *params) {
    if (!m) return MCT_EINVAL;
    if (!params) return mfail(m, MCT_EINVAL, "null parameters");
    for (int i = 0; i < mct::kParams; ++i)
        if (!std::isfinite(params[i])) return mfail(m, MCT_EINVAL, "non-finite parameter");
    MLP_TRY(m, hipMemcpyAsync(m->d.master, params, sizeof(float) * mct::kParams, hipMemcpyHostToDevice, m->stream));
    MLP_TRY(m, hipMemsetAsync(m->d.m, 0, sizeof(float) * mct::kParams, m->stream));
    MLP_TRY(m, hipMemsetAsync(m->d.v, 0, sizeof(float) * mct::kParams, m->stream));
    MLP_TRY(m, mct::launch_mlp_prep(m->d, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
    m->t = 0;
    return MCT_OK;
}

int mct_mlp_get_params(mct_mlp *m, float *params) {
    if (!m) return MCT_EINVAL;
    if (!params) return mfail(m, MCT_EINVAL, "null output");
    MLP_TRY(m, hipMemcpyAsync(params, m->d.master, sizeof(float) * mct::kParams, hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
    return MCT_OK;
}

int mct_mlp_forward(mct_mlp *m, const float *x, int64_t n, float *logits) {
    if (!m) return MCT_EINVAL;
    if (n < 0 || (n > 0 && (!x || !logits))) return mfail(m, MCT_EINVAL, "bad rows or null pointer");
    if (n == 0) return MCT_OK;
    MLP_TRY(m, mct::launch_mlp_forward(m->d, x, nullptr, n, logits, nullptr, nullptr, 0.0f, nullptr, m->stream));
    return MCT_OK;
}

int mct_mlp_gradient(mct_mlp *m, const float *x, const float *y, int64_t n, float pos_weight, float *grad,
                     float *loss) {
    if (!m) return MCT_EINVAL;
    if (n <= 0 || !x || !y || !grad) return mfail(m, MCT_EINVAL, "bad rows or null pointer");
    if (!(pos_weight > 0.0f)) return mfail(m, MCT_EINVAL, "pos_weight must be positive");
    MLP_TRY(m, mct::launch_mlp_gradient(m->d, x, y, n, pos_weight, m->partials, m->grad, m->stream));
    MLP_TRY(m, hipMemcpyAsync(grad, m->grad, sizeof(float) * mct::kParams, hipMemcpyDeviceToHost, m->stream));
    if (loss) MLP_TRY(m, hipMemcpyAsync(loss, m->grad + mct::kParams, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
    return MCT_OK;
}

int mct_mlp_train_step(mct_mlp *m, const float *x, const float *y, int64_t n, float pos_weight, float lr,
                       float *loss) {
    if (!m) return MCT_EINVAL;
    if (n <= 0 || !x || !y) return mfail(m, MCT_EINVAL, "bad rows or null pointer");
    if (!(pos_weight > 0.0f) || !(lr > 0.0f)) return mfail(m, MCT_EINVAL, "pos_weight and lr must be positive");
    MLP_TRY(m, mct::launch_mlp_gradient(m->d, x, y, n, pos_weight, m->partials, m->grad, m->stream));
    m->t += 1;
    MLP_TRY(m, mct::launch_mlp_adam(m->d, m->grad, lr, m->t, m->stream));
    if (loss) {
        MLP_TRY(m, hipMemcpyAsync(loss, m->grad + mct::kParams, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MLP_TRY(m, hipStreamSynchronize(m->stream));
    }
    return MCT_OK;
}

}  // extern "C"
