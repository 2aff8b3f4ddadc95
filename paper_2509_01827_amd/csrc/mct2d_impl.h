// Internal declarations shared by the host side (mct2d_api.cpp) and the
// kernels (mct2d_step.hip) of the MCT-2D-CEM library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mct {

constexpr uint8_t kSplitFlag = 0x80;  // element split code: 0x80 | entry<<2 | exit
constexpr uint8_t kAbsent = 0x40;     // LDS marker for an element outside the grid

// One accepted split made by the tracking.
struct LogRec {
    int32_t step;
    int32_t elem;
    uint8_t entry, exit, pad0, pad1;
    int32_t pad2;
    double G;
};
static_assert(sizeof(LogRec) == 24, "LogRec layout");

// One accepted candidate of a step (per-front pick): G of its chosen path,
// the element, (tip edge a) << 2 | (exit edge k).
struct AccCand {
    double G;
    int32_t elem;
    int32_t ak;
};
static_assert(sizeof(AccCand) == 16, "AccCand layout");

// Per-front pick over the whole GPU, used by models from
// kFrontGridMinElements elements on (with a finite radius; smaller models
// and rho = infinity take one workgroup).  Two int32 tables, one per step
// parity, each: per bucket the number of candidates and the head of its
// overflow list, the picked count, the close's LDS sort and counting-rank
// limits, then kFrontGridCap candidate indices per bucket.  Step k uses table k & 1 and clears the other one (counts 0,
// heads -1) for step k + 1; the picked count returns to 0 at the end of
// each pick.
constexpr int kFrontGridBuckets = 1 << 16;
constexpr int kFrontGridCap = 64;
constexpr int64_t kFrontGridCnt = 0;
constexpr int64_t kFrontGridHead = kFrontGridBuckets;
constexpr int64_t kFrontGridNp = 2 * (int64_t)kFrontGridBuckets;
constexpr int64_t kFrontGridSortMax = kFrontGridNp + 1;  // LDS entries the close may sort in
constexpr int64_t kFrontGridRankMax = kFrontGridNp + 2;  // picked counts the close ranks by counting
constexpr int64_t kFrontGridTab = 2 * (int64_t)kFrontGridBuckets + 64;
constexpr int64_t kFrontGridTable = kFrontGridTab + (int64_t)kFrontGridBuckets * kFrontGridCap;
constexpr int64_t kFrontGridMinElements = 1 << 14;
// both tables as the first pick expects them (after allocation, restore),
// with the close's limits from front_close_limits
hipError_t front_grid_reset(int32_t *tables, hipStream_t s);
// The close's limits (testing knobs from the environment, read here):
// MCT_FRONT_SORT_LDS_MAX (2..2048, default 2048), how many entries its sort
// may hold in LDS before it moves to the scratch arrays, and
// MCT_FRONT_RANK_MAX (0..256, default 256), up to how many picked
// candidates it ranks by counting instead of sorting.
void front_close_limits(int32_t *sort_lds_max, int32_t *rank_max);

// Per-workgroup best candidate of one step (only workgroups with an
// accepted candidate write one).
struct Slot {
    double G;     // largest accepted G of the workgroup
    double Gmin;  // smallest accepted G of the workgroup
    double G2;    // second largest accepted G of the workgroup (-1: none)
    int32_t elem, a, k, pad;
};

// One near-threshold decision: a decision whose margin lies within the
// relative tolerance near_tol (kind 1: a path G against Gc; 2: gap of the
// two largest paths above Gc of an element; 3: the element rule's
// split-ratio margin against one path; 4: gap of the two largest accepted
// candidates of a step; 5: the pick's split-ratio margin against the
// smallest accepted G).  k is the exit edge of the path concerned.
struct NearRec {
    int32_t step, elem;
    uint8_t a, kind, k, pad0;
    int32_t pad1;
    double G, ref;
};
static_assert(sizeof(NearRec) == 32, "NearRec layout");

// Geometry shared by every element of a uniform lattice (a structured grid
// whose element gradients, areas and crack-path geometry set-up found
// bitwise identical for all elements; binary64 point rule): the step takes
// these instead of recomputing them per element.
struct LatticeConst {
    double B[4][8];       // at the midpoint of local edge k: dN_n/dx (n = 0..3), then dN_n/dy
    double w;             // smoothing weight A / (A + A) of two intact neighbours
    double c4;            // 0.25 A, the element force factor
    double geo[4][3][3];  // tip edge a, path j: unit normal x, y and length
};

// Device-resident control block of one model.
struct Control {
    int64_t base;         // steps completed before the running segment
    uint32_t nslots[3];   // slots written by steps k_rel = 0, 1, 2 (mod 3)
    int32_t tip0;         // single-tip mode: tip (e * 4 + a, -1 none) at the start of
    int64_t nsplit;       //   the last even step (tip0) / odd step (tip1)
    double Ud;            // dissipated energy, sum of Gc * path length
    int32_t overflow;     // 1 when a split could not be logged
    int32_t tip1;
};
static_assert(sizeof(Control) == 48, "Control layout");

// One specimen as the kernels see it: sizes, constants and pointers already
// offset to the specimen's part of the batch arrays.  T is the arithmetic
// and storage type of the step (double, or float for the binary32 step,
// whose set-up values are the binary64 ones rounded once); times, the load
// curve, the log, U_d and the pick variant's buffers stay binary64.  (The
// batched step copies a view field by field: load_view in mct2d_step.hip
// lists every field.)
template <class T>
struct StepParamsT {
    int32_t nx, ny;     // elements per direction
    int32_t ntx, nty;   // tiles per direction
    int32_t nwg;        // ntx * nty (also the stride of the three slot sets)
    int32_t log_cap;
    const T *X, *Y;
    T *ux0, *uy0, *ux1, *uy1;  // displacement ping-pong, u^k in (k & 1)
    T *vx, *vy;
    const T *minv;
    uint8_t *split;
    const T *area;  // per element (reference configuration)
    const uint32_t *screen;  // per element, byte a = screen state of candidate (e, a); null = no screen
    uint32_t *strip;         // screened steps: set to 1 when a skipped candidate might pass Gc
    int32_t sct;             // 1: single crack-tip tracking (only the tip is a candidate)
    int32_t ncurve;          // traction load curve points (0: constant tractions)
    const double *curve_t, *curve_phi;
    const T *gc;   // per element, or nullptr for gc_uniform
    T gc_uniform;
    const T *fext_p;          // 2 per perimeter node
    const uint8_t *vmask_p;   // 1 per perimeter node
    const T *v0_p;            // 2 per perimeter node
    T D11, D12, D33, E;
    double dt, t_ramp;  // time step (for times t_k) and velocity ramp
    T dts;              // time step of the update (dt rounded to T)
    T gamma;
    Control *ctl;
    Slot *slots;        // 3 sets of nwg slots
    LogRec *log;
    // Q4 edge smoothing: 0 the point rule, 1 triangular sub-cells (plain models)
    int32_t subcell;
    int32_t pad_sc;
    // per-front pick (plain models): every accepted candidate of a step is
    // appended to fcand and a separate kernel picks; front_r2 = rho^2
    int32_t front;
    int32_t fcap;
    double front_r2;
    AccCand *fcand;
    uint32_t *fcount;
    double2 *fmid;
    double *flen;
    int32_t *forder;
    int32_t *fbucket, *fsorted, *fplist;
    double fcell;  // hash cell of the pick: >= rho and the largest element diameter
    int32_t *fgrid;  // the pick's bucket table over the whole GPU, or null for one workgroup
    // uniform lattice (binary64 point rule): its shared geometry, or null
    const LatticeConst *lat;
    // near-threshold decision log (plain models): null when off
    NearRec *near;
    uint32_t *near_count;
    int32_t near_cap;
    int32_t pad_near;
    T near_tol;
};
using StepParams = StepParamsT<double>;
using StepParamsF = StepParamsT<float>;

// Tile shapes (elements per workgroup in x and y; nodes owned = one less).
struct TileShape {
    int txe, tye;
};
constexpr int kNumTiles = 3;
TileShape tile_shape(int tile);  // tile in 1..kNumTiles

// What one step launch covers: a single specimen (p0, nwg tiles) or a batch
// (nunits work units (specimen, tile) over nspec device-resident views).
// f32: a single binary32 specimen, p0f (p0 holds its binary64 mirror).
struct Launch {
    bool batched;
    bool uni;
    StepParams p0;
    const StepParams *views;
    const int2 *units;
    int nunits, nspec;
    bool f32;
    StepParamsF p0f;
};

// One step of a segment (k_rel = index in the segment, par0 = parity of the
// segment's first step), and the segment close after n steps.  uni: every
// specimen of the launch is a uniform lattice (its views carry lat).
hipError_t launch_step(int tile, const Launch &L, int k_rel, int par0, hipStream_t s);
hipError_t launch_commit(const Launch &L, int n, hipStream_t s);

// Uniform-lattice check of one specimen: ref receives element 0's geometry
// (LatticeConst), flag bit 0 = some element differs bitwise, bit 1 = the
// gradients do not have the zero pattern of a rectangle.
hipError_t launch_lattice_check(const StepParams &p, LatticeConst *ref, uint32_t *flag, hipStream_t s);

// Crack-surface tips: compacted edge ids and reference midpoints (at most
// cap written; count_out receives the total).
hipError_t launch_tips(int32_t nx, int32_t ny, const double *X, const double *Y,
                       const uint8_t *split, int32_t *block_counts, int32_t *nblocks_out,
                       int32_t *edge_out, double *xy_out, int32_t *count_out, int64_t cap, hipStream_t s);
int tips_nblocks(int64_t n_edges);
// The no-allocation tip query's block counts: a static device array, its
// address on the current device (resolved once per device).
constexpr int kTipScratchBlocks = 1 << 16;
constexpr int kMaxDevices = 64;
hipError_t tips_scratch(int32_t **out);

// Crack-path normals and lengths of n elements (36 doubles each).
hipError_t launch_path_geometry(const StepParams &p, int n, const int32_t *elem, double *out, hipStream_t s);

// ---------------------------------------------------------------------
// State queries (fields, energies, stability limit, finiteness).

struct EvalDev {
    double *sig;     // 3 per edge (NaN without an intact neighbour)
    double *es;      // per edge: strain energy of its smoothing domain
    double *fe;      // 8 per element
    double *pe;      // per element: strain energy of split pieces
    double *fint;    // per node, x then y (2 nn)
    double *acc;     // per node, x then y (2 nn)
    double *node_e;  // per node: kinetic energy, external work
    double *part;    // partial sums (eval_partials())
    double *sums;    // 8 results: [0] kinetic, [2] external work, [3] edges, [4] pieces
};

int eval_partials();
hipError_t launch_eval(const StepParams &p, const double *ux, const double *uy, const double *vx,
                       const double *vy, int64_t step, double phi, const EvalDev &d, hipStream_t st);
hipError_t launch_energies(const StepParams &p, const EvalDev &d, double *out, hipStream_t st);
hipError_t launch_principal(const StepParams &p, const EvalDev &d, double *out, hipStream_t st);
hipError_t launch_power_step(const StepParams &p, const EvalDev &d, double *y, double *u, double *z,
                             double *scratch2, double *sums, hipStream_t st);
hipError_t launch_check_finite(const double *a, const double *b, const double *c, const double *d, int64_t n,
                               int32_t *flag, hipStream_t st);
// Binary32 state <-> its binary64 mirror (n values each of up to 6 arrays;
// widening is exact, narrowing rounds to nearest).
hipError_t launch_widen(const float *const src[6], double *const dst[6], int count, int64_t n, hipStream_t st);
hipError_t launch_narrow(const double *const src[6], float *const dst[6], int count, int64_t n, hipStream_t st);

// ---------------------------------------------------------------------
// Learned split-screen.

constexpr int kFeat = 10;                 // features per candidate
constexpr int kHidden = 64;               // hidden width of both layers
constexpr int kParams = kFeat * kHidden + kHidden + kHidden * kHidden + kHidden + kHidden + 1;  // 4929
constexpr int kOffB1 = kFeat * kHidden, kOffW2 = kOffB1 + kHidden, kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden, kOffB3 = kOffW3 + kHidden;
static_assert(kOffB3 + 1 == kParams, "parameter layout");

// screen state byte of a candidate: not seen at the last evaluation
// (evaluated), flagged (evaluated), or screened out (skipped)
constexpr uint8_t kScreenUnseen = 0, kScreenFlagged = 1, kScreenSkip = 2;
enum ScreenStat { kStatSweeps = 0, kStatCands = 1, kStatFlagged = 2, kStatMisses = 3, kStatWindows = 4,
                  kStatReplays = 5 };
constexpr int kNumScreenStats = 6;

// Device MLP: FP32 master parameters, Adam moments, bfloat16 weight copies
// (W1 padded to 32 input rows with zeros).
struct MlpDev {
    float *master, *m, *v;
    uint16_t *w1b;  // [32][64]
    uint16_t *w2b;  // [64][64]
    uint16_t *w3b;  // [64]
};

// Device buffers of a model's screen.
struct ScreenDev {
    int32_t *nrows;         // candidate rows appended by the running evaluation
    int32_t *nrows_last;    // row count of the last completed evaluation
    int32_t *cand;          // packed e * 4 + a per row (capacity 4 ne), any order
    float *feat;            // kFeat per row
    double *row_geo;        // per row: midpoint x, y of edge a and h (for feature 5)
    float *logits;          // one per row
    double *hist_g;         // per (e, a): max path G / Gc at its last evaluation
    int32_t *hist_t;        // per (e, a): sweep index of that evaluation
    int32_t *sweep;         // sweeps done
    uint32_t *screen;       // per element, one state byte per local edge
    int32_t *nfront;        // crack-path ends of the running evaluation
    double *front_xy;       // their midpoints (capacity 2 ne)
    unsigned long long *stats;  // ScreenStat counters
    // the judge of a screened window: its trip flag, and the snapshot of the
    // state at the window's start (u^k, v, split codes, control block)
    uint32_t *trip;
    double *snap_u;      // 4 nn: ux, uy of u^k, then vx, vy
    uint8_t *snap_split; // ne
    Control *snap_ctl;
};

// Copy the state of a model (u^k from buffer par, v, split codes, control
// block) into the screen's snapshot (save) or back (restore), and clear the
// trip flag (save).
hipError_t launch_snapshot(const StepParams &p, const ScreenDev &s, int par, bool save, hipStream_t st);

hipError_t launch_screen_evaluate(const StepParams &p, const ScreenDev &s, int par, hipStream_t st);
hipError_t launch_sweep_advance(const ScreenDev &s, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *a, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_mlp_prep(const MlpDev &m, hipStream_t st);
// logits of n rows (n_dev: device count, else n); with `screen` set, also
// the screen state byte of each row's candidate (flagged when logit > tau)
hipError_t launch_mlp_forward(const MlpDev &m, const float *x, const int32_t *n_dev, int64_t n, float *logits,
                              const int32_t *cand, uint32_t *screen, float tau, unsigned long long *stats,
                              hipStream_t st);
int mlp_train_blocks(int64_t n);
hipError_t launch_mlp_gradient(const MlpDev &m, const float *x, const float *y, int64_t n, float pos_weight,
                               float *partials, float *grad, hipStream_t st);
hipError_t launch_mlp_adam(const MlpDev &m, const float *grad, float lr, int t, hipStream_t st);

}  // namespace mct
