/*
 * mct2d.h - C ABI of the MI355X (gfx950) library for the explicit dynamic
 * step of the two-dimensional Crack Element Model with Multiple Crack-tips
 * Tracking (MCT-2D-CEM, arXiv 2509.01827).
 *
 * One time step (mct_step) runs, entirely on the GPU:
 *   1. ES-FEM smoothed strain and plane stress at every edge quadrature point
 *      (Sec. 2.1, Eqs. disp_ES_FEM, strain_discretization,
 *      QUAD_strain_discretization);
 *   2. Q4 internal force per element, intact (Eq. QUAD_fint_discretization)
 *      or split into pieces, and a deterministic graph-coloured scatter to the
 *      nodes (colour of element (i,j) = (i mod 2) + 2 (j mod 2), summed in
 *      colour order);
 *   3. the central-difference nodal update (the paper's explicit
 *      formulation, Sec. 2) with lumped mass;
 *   4. the energy release rate G of the three split topologies of every
 *      free-surface quadrature point and the Q4 element rule (Sec. 2.2,
 *      Fig. 2-3 and the itemised cases after it);
 *   5. the Multiple Crack-tips Tracking pick over all free-surface
 *      candidates and the split of the chosen element (Sec. 3, Fig. 3-1(b)).
 *
 * Conventions
 *   - Structured Q4 grid of nx x ny elements (nx, ny >= 2).  Node (i,j),
 *     0<=i<=nx, 0<=j<=ny, has id j*(nx+1)+i; element (i,j) has id j*nx+i and
 *     the counter-clockwise nodes (i,j),(i+1,j),(i+1,j+1),(i,j+1).  Local
 *     edge k joins local nodes k and k+1 (0 bottom, 1 right, 2 top, 3 left).
 *     Node coordinates are free (any positive-area, counter-clockwise
 *     elements), so jittered and sheared grids are allowed.
 *   - Edge ids follow the sorted (smaller node, larger node) order.
 *   - Split code of an element: 0 = intact, else 0x80 | (entry << 2) | exit,
 *     entry/exit = local edges whose midpoints the crack joins (pattern I:
 *     adjacent edges, pattern II: opposite edges, Fig. 2-3).
 *   - SI units, unit thickness; energies per unit thickness (J/m).
 *   - All arrays passed in are host pointers; the library copies them during
 *     the call and the caller keeps ownership.  Query outputs are host
 *     pointers with a capacity `cap` (elements of the array); `*count` is
 *     always set and MCT_ECAPACITY is returned when cap < count.
 *   - Every function returns an int status (MCT_OK = 0, negative on error)
 *     and never throws; mct_last_error() gives a message owned by the
 *     context (valid until the next call on it).
 *   - Device work is enqueued on the HIP stream given to mct_create (or on a
 *     stream the library creates when it is NULL).  mct_step returns without
 *     waiting; every query synchronises that stream first.
 *   - Binary64 (and binary32, mct_create): results are bit-reproducible run
 *     to run and independent of the launch shape (fixed summation orders, no
 *     floating-point atomics).
 *   - Triangle meshes (mct_set_mesh_tri) run the same step with
 *     constant-strain triangles (Sec. 2.1, Eqs. CST_strain_discretization,
 *     CST_fint_discretization; the two-path rule after Fig. 2-2), and
 *     quadrilateral meshes of any connectivity (mct_set_mesh_q4) the Q4 step
 *     of the structured grid.
 */
#ifndef MCT2D_H
#define MCT2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MCT_OK = 0,
    MCT_EINVAL = -1,     /* bad argument (null pointer, size, value, mesh) */
    MCT_ESTATE = -2,     /* call out of order (e.g. step before finalize) */
    MCT_ECAPACITY = -3,  /* output capacity too small, *count holds the need */
    MCT_EDEVICE = -4,    /* HIP runtime or kernel launch failure */
    MCT_ENOMEM = -5,     /* device or host allocation failed */
    MCT_EUNSUPPORTED = -6, /* a combination the library does not offer (see the calls) */
    MCT_ESTABILITY = -7, /* dt above the stability limit of the explicit step */
    MCT_ENUMERIC = -8    /* non-finite displacement or velocity */
};

enum {
    MCT_FIELD_U = 0,
    MCT_FIELD_V = 1,
    MCT_FIELD_A = 2,
    MCT_FIELD_FINT = 3,
    MCT_FIELD_SIGMA_EDGE = 4,
    MCT_FIELD_PRINCIPAL = 5
};

typedef struct mct_ctx mct_ctx;

typedef struct {
    int64_t n_nodes, n_elems, n_edges;
    int64_t step;        /* number of completed time steps */
    int64_t n_splits;    /* splits made by the tracking (pre-notch excluded) */
    double dt;           /* time step in use */
    double dissipated;   /* U_d = sum over splits of Gc * crack-path length */
    int32_t log_overflow;/* 1 if more splits happened than the log can hold */
    int32_t precision;
    double dt_limit;     /* stability limit 2 / omega_max of the set-up mesh */
    int64_t tip;         /* single-tip tracking: current tip element * 4 + local
                            edge (-1: none, or multi-tip tracking) */
} mct_info;

/* Create an empty context.  precision: 64 (binary64 state and arithmetic)
 * or 32: the binary32 step on a structured Q4 grid (the set-up -- areas,
 * lumped masses, equivalent nodal forces, D, dt -- is computed in binary64
 * and each value rounded once to binary32; state, strains, stresses,
 * forces, G, the element rule and the pick are binary32; times and the load
 * curve binary64; U_d accumulates the binary32 products Gc * L in binary64).
 * A binary32 context reports u, v, split codes, the crack set (G exact in
 * binary64) and tips as computed; the derived fields and energies are
 * evaluated in binary64 from its state; checkpoints hold that state and
 * restore only into a binary32 context.  Not for binary32: unstructured
 * meshes, batches, the split-screen, the per-front pick (MCT_EUNSUPPORTED
 * from the call that asks for them).  Sub-cell smoothing runs in binary32
 * like the point rule.
 * hip_stream: a hipStream_t to enqueue on, or NULL for a library stream.
 * Errors: MCT_EINVAL (out NULL), MCT_EUNSUPPORTED (precision), MCT_EDEVICE. */
int mct_create(mct_ctx **out, int precision, void *hip_stream);

/* Release every device and host resource of ctx (NULL is a no-op). */
int mct_destroy(mct_ctx *ctx);

/* Message of the last failing call on ctx. */
const char *mct_last_error(const mct_ctx *ctx);

/* Mesh (Sec. 2.1: nodes and element connectivity M^{A_j}): structured grid
 * of nx x ny Q4 elements with reference coordinates X[n], Y[n] of the
 * (nx+1)(ny+1) nodes.  Rejects nx < 2, ny < 2, and non-positive areas.
 * Resets material, loads, notch and time settings. */
int mct_set_mesh_grid(mct_ctx *ctx, int32_t nx, int32_t ny, const double *X, const double *Y);

/* Mesh of constant-strain triangles (CST, the element of the paper's
 * examples; Sec. 2.1, Eqs. CST_strain_discretization and
 * CST_fint_discretization; Sec. 2.2, the two-path rule after Fig. 2-2):
 * n_nodes reference coordinates X, Y and n_elems counter-clockwise node
 * triples conn[3 e + 0..2] of an unstructured mesh (plain contexts only).
 * Local edge k joins local nodes k and (k+1) % 3; split codes and crack
 * records use these local edges (entry/exit in 0..2).  Element ids, edge
 * ids (sorted node pairs) and node ids are the caller's; the library does
 * not renumber, so a locality-preserving element order (e.g. along a
 * space-filling curve) is the caller's choice and pays in cache reuse.
 * After this call the context runs the CST path: every set-up call, step
 * and query below applies to the triangle mesh, except the tile shapes
 * (mct_set_launch and mct_autotune select the step kernels instead) and
 * the split-screen (MCT_EUNSUPPORTED).  Velocity conditions may be
 * prescribed at any node.  Errors: MCT_EINVAL for an index out of range, a
 * repeated node, a non-positive area (clockwise or degenerate), an edge
 * used by more than two triangles or twice in one direction, a node in no
 * triangle; MCT_EUNSUPPORTED on a batch context. */
int mct_set_mesh_tri(mct_ctx *ctx, int64_t n_nodes, const double *X, const double *Y, int64_t n_elems,
                     const int32_t *conn);

/* Mesh of bilinear quadrilaterals with general connectivity (the Q4 element
 * of Sec. 2.1, Eq. QUAD_strain_discretization; Sec. 2.2, the four-edge rule
 * after Fig. 2-3): n_nodes reference coordinates X, Y and n_elems
 * counter-clockwise node quadruples conn[4 e + 0..3] (plain binary64
 * contexts only).  Local edge k joins local nodes k and (k+1) % 4, with the
 * edge midpoints at natural coordinates (0,-1), (1,0), (0,1), (-1,0) as on
 * the structured grid; the step is the grid's, with neighbours taken from
 * the connectivity: B of each element at the midpoint of its own local edge,
 * c_{e,k} = A_e / 4, w_j = A_j / (A_lo + A_hi), lumped mass rho A / 4, the
 * Q4 piece forces of split elements, greedy colouring in element-id order.
 * Split codes and crack records use these local edges (entry/exit in 0..3).
 * Ids are the caller's (no renumbering).  After this call every set-up call,
 * step and query below applies to this mesh as for mct_set_mesh_tri, with
 * the same exceptions (the step kernels are chosen as on a triangle mesh,
 * by mct_set_launch), and sub-cell smoothing is for structured grids
 * only.  Errors: as mct_set_mesh_tri, and
 * MCT_EINVAL for a quadrilateral that is not convex (every corner turning
 * left). */
int mct_set_mesh_q4(mct_ctx *ctx, int64_t n_nodes, const double *X, const double *Y, int64_t n_elems,
                    const int32_t *conn);

/* Linear elastic plane-stress material (Young's modulus E, Poisson ratio
 * nu, density rho) and critical energy release rate: Gc[e] per element
 * (n_elems values) or, if Gc is NULL, Gc_uniform everywhere.  gamma is the
 * split ratio of the element rule and of the MCT pick (Sec. 2.2 and 3; > 0).
 * Errors: MCT_EINVAL for E <= 0, nu outside (-1, 0.5), rho <= 0, gamma <= 0,
 * Gc <= 0; MCT_ESTATE before mct_set_mesh_grid. */
int mct_set_material(mct_ctx *ctx, double E, double nu, double rho, const double *Gc,
                     double Gc_uniform, double gamma);

/* Constant Neumann traction (Pa) on n boundary edges, each given by its two
 * node ids edge_nodes[2i], edge_nodes[2i+1] and the traction vector
 * t[2i], t[2i+1]; each end node receives t * L / 2 (equivalent nodal force),
 * summed in edge-id order.  Rejects interior or repeated edges. */
int mct_set_traction(mct_ctx *ctx, int64_t n, const int32_t *edge_nodes, const double *t);

/* Prescribed velocity on n boundary nodes: dof_mask bit 0 = x, bit 1 = y;
 * v0[2i], v0[2i+1] the target velocity, reached linearly over t_ramp
 * seconds (0 = applied from the first step).  Interior nodes are rejected. */
int mct_set_velocity_bc(mct_ctx *ctx, int64_t n, const int32_t *node, const uint8_t *dof_mask,
                        const double *v0, double t_ramp);

/* Pre-notch: n elements split from the start with the given entry/exit
 * local edges (entry != exit, both 0..3).  Not counted in U_d or the log. */
int mct_set_notch(mct_ctx *ctx, int64_t n, const int32_t *elem, const uint8_t *entry,
                  const uint8_t *exit);

/* Time history of the tractions: they are multiplied by the load factor
 * phi(t), piecewise linear through the n points (t[i], phi[i]) (t strictly
 * increasing), constant beyond the ends, evaluated at t_k = k dt; n = 0
 * restores constant tractions.  The pressure history of Sec. 4.4 (linear
 * rise, exponential decay) is passed as such a sampled curve.  Per
 * specimen; host arrays copied. */
int mct_set_load_curve(mct_ctx *ctx, int64_t n, const double *t, const double *phi);

/* Crack tracking (Sec. 3).  MCT_TRACK_MCT (default): every free-surface
 * candidate is evaluated each step and the pick takes the largest G
 * (Multiple Crack-tips Tracking).  MCT_TRACK_SCT: single crack-tip tracking
 * (Fig. 3-1(a)), only the current tip is evaluated; when its element splits
 * the tip moves to the element across the exit edge (tracking ends at the
 * domain boundary or at a split element).  The start tip is element
 * tip_elem, local edge tip_edge (facing the crack), or with tip_elem < 0 the
 * one path end of the pre-notch (MCT_EINVAL at mct_finalize if it has none
 * or several).  Per specimen. */
enum { MCT_TRACK_MCT = 0, MCT_TRACK_SCT = 1 };
int mct_set_tracking(mct_ctx *ctx, int mode, int32_t tip_elem, int tip_edge);

/* Per-front pick, a variant of the Multiple Crack-tips Tracking pick
 * (Sec. 3): an accepted candidate (one that passed the element rule) splits
 * iff, against every other accepted candidate it competes with -- the same
 * element, or a tip point (reference midpoint of the tip edge) closer than
 * rho -- it has the larger G (ties: lower element id, then lower tip edge)
 * and passes G > gamma (G - G_other).  Fronts farther apart than rho then
 * advance in the same step; picked candidates never compete, so each
 * element splits at most once; the splits of a step are logged in that key
 * order.  rho = +infinity gives the global pick exactly; rho = 0 (default)
 * selects the global pick.  Plain contexts (Q4 grid or CST mesh);
 * MCT_EUNSUPPORTED on a batch or with the split-screen, MCT_EINVAL at
 * finalize together with single-tip tracking.  Models from 16 384 elements
 * on (finite rho) pick over the whole GPU with two bucket tables of 16.5
 * MiB each, allocated at finalize.  Testing knobs (environment, read at
 * finalize and restore; same results): MCT_FRONT_RANK_MAX (0..256) lowers
 * up to how many picked candidates of a step are ranked by counting, and
 * MCT_FRONT_SORT_LDS_MAX (2..2048) how many the sort holds in LDS before it
 * moves to device scratch arrays. */
int mct_set_front_pick(mct_ctx *ctx, double rho);

/* Edge smoothing of Q4 elements.  MCT_SMOOTH_POINT (default): B of a
 * neighbouring element evaluated at the midpoint of the edge in its natural
 * coordinates, weights A_j / (A_lo + A_hi) (Eq. QUAD_strain_discretization
 * with Eq. disp_ES_FEM; the paper leaves the evaluation point open).
 * MCT_SMOOTH_SUBCELL: the edge's smoothing domain is the union of the
 * triangles (edge, vertex centroid of each intact neighbour), the
 * displacement at a centroid the mean of the element's nodal displacements,
 * weights and element forces from those triangles' areas and gradients --
 * edge-based smoothing over triangular sub-cells, which passes the patch
 * test on any quadrilateral mesh (the point rule only on parallelograms,
 * where the two coincide).  Plain Q4 contexts; MCT_EUNSUPPORTED on a batch,
 * with the split-screen, or for a CST mesh (whose smoothing is exact). */
enum { MCT_SMOOTH_POINT = 0, MCT_SMOOTH_SUBCELL = 1 };
int mct_set_smoothing(mct_ctx *ctx, int mode);

/* Time step: dt > 0 is used as given; otherwise dt = cfl_fraction *
 * (shortest edge) / c_d with c_d = sqrt(E / (rho (1 - nu^2))). */
int mct_set_time(mct_ctx *ctx, double dt, double cfl_fraction);

/* Caller-owned device arrays for the state of a plain binary64 Q4 context
 * (e.g. the storage of torch tensors): u^k lives in ux[k & 1], uy[k & 1]
 * (the step reads one pair and writes the other), v in vx, vy; each of the
 * six distinct arrays holds at least n doubles (node-id order; the first
 * n_nodes are used).  Call before mct_finalize, which checks n >= n_nodes
 * (MCT_EINVAL otherwise), zeroes them (on the context's stream: work of
 * other streams on them must be complete) and uses them instead of
 * allocating its own; the caller keeps them alive until mct_destroy (or a
 * later finalize after unbinding) and does not write them while steps are
 * enqueued.  views = NULL unbinds (the next finalize allocates again), and
 * so does a new mesh (mct_set_mesh_grid).  Errors: MCT_EINVAL for a NULL
 * array, two equal arrays or n < 1; MCT_EUNSUPPORTED on a batch, a binary32
 * context or a triangle mesh. */
typedef struct {
    double *ux[2], *uy[2];
    double *vx, *vy;
    int64_t n;  /* doubles each array holds */
} mct_device_views;
int mct_bind_device_buffers(mct_ctx *ctx, const mct_device_views *views);

/* Build the derived arrays (lumped mass, equivalent nodal forces, time
 * step), upload everything and zero the state (u = v = 0, step 0).  Then
 * estimate the stability limit of central differences, 2 / omega_max with
 * omega_max^2 the largest eigenvalue of M^-1 K over the free components
 * (power iteration on the GPU with the set-up split state; the estimate
 * approaches omega_max from below, so the limit is an upper estimate;
 * reported in mct_info.dt_limit).  Errors: MCT_ESTATE if mesh or material is
 * missing, MCT_ESTABILITY if dt exceeds the limit, MCT_ENOMEM /
 * MCT_EDEVICE on device failures. */
int mct_finalize(mct_ctx *ctx);

/* Enqueue n_steps time steps; asynchronous.  Each step splits at most one
 * element with the global pick (several with the per-front pick); a split
 * acts from the next step on. */
int mct_step(mct_ctx *ctx, int64_t n_steps);

/* Step timing (a measurement call, like mct_autotune): enqueues n steps
 * (1..4096) as direct launches with a HIP event pair on the context's stream
 * around every step-kernel launch and every pick/commit launch, waits, and
 * returns the mean duration per step of the step kernel (out_us[0]) and of
 * the pick/commit launches (out_us[1]) in microseconds.  The steps count as
 * ordinary steps (the same results as mct_step).  Structured grids without
 * the split-screen; MCT_EUNSUPPORTED otherwise. */
int mct_profile_step(mct_ctx *ctx, int64_t n, double out_us[2]);

/* Wait for the enqueued work; reports asynchronous device errors, and
 * MCT_ENUMERIC if any displacement or velocity of the current step is not
 * finite. */
int mct_sync(mct_ctx *ctx);

int mct_get_info(mct_ctx *ctx, mct_info *out);

/* Split log in the order the splits were made: step index k (the split was
 * decided on the state at t_k and acts from step k+1), element id, entry
 * and exit local edges, G of the chosen path.  Any output may be NULL. */
int mct_get_crack_set(mct_ctx *ctx, int64_t cap, int32_t *step, int32_t *elem, uint8_t *entry,
                      uint8_t *exit, double *G, int64_t *count);

/* Crack-surface tips (Fig. 3-1(b), free-surface quadrature points on crack
 * faces): interior edges with exactly one intact neighbour, ascending edge
 * id; xy = reference midpoint (2 per tip).  Computed on the GPU. */
int mct_get_tips(mct_ctx *ctx, int64_t cap, int32_t *edge, double *xy, int64_t *count);

/* The tip query for callers that cannot allocate device memory -- code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc -- with device outputs: the same crack-surface tips as
 * mct_get_tips (ascending edge id; reference midpoints), written to the
 * caller's device arrays edge_dev (cap int32) and xy_dev (2 cap doubles),
 * and their number to the device int32 *count_dev (when it exceeds cap only
 * the first cap are written).  Asynchronous on the context's stream: no
 * host synchronisation, no hipMalloc/hipFree.  Its block counts live in a
 * static device array of 2^16 int32 per GPU (256 KiB: meshes of up to
 * 2^24 edges; larger ones give MCT_EINVAL), held until the process ends and
 * shared by every call on that GPU: calls that overlap on one GPU (several
 * streams or threads) race.  The context's device must be current
 * (MCT_EDEVICE otherwise).  Structured grids (MCT_EUNSUPPORTED otherwise);
 * MCT_ESTATE before mct_finalize; MCT_EINVAL for a null count, a negative
 * cap, or null arrays with cap > 0. */
int mct_get_tips_noalloc(mct_ctx *ctx, int64_t cap, int32_t *edge_dev, double *xy_dev, int32_t *count_dev);

/* Field of the current step k (evaluated on the GPU from u^k):
 *   MCT_FIELD_U          u^k, [x of all nodes, y of all nodes] (2 n_nodes);
 *   MCT_FIELD_V          v^{k-1/2} (v^0 at k = 0), same layout;
 *   MCT_FIELD_A          a^k = (phi(t_k) f_ext - f_int(u^k)) / m, prescribed
 *                        components 0, same layout;
 *   MCT_FIELD_FINT       f_int(u^k) (Eqs. QUAD_fint_discretization and the
 *                        split pieces, summed in colour order), same layout;
 *   MCT_FIELD_SIGMA_EDGE smoothed plane stress of every edge (Sec. 2.1),
 *                        [sxx of all edges, syy ..., sxy ...] (3 n_edges),
 *                        NaN where the edge has no intact neighbour;
 *   MCT_FIELD_PRINCIPAL  per element, the maximum principal stress of the
 *                        mean of its four edge stresses (the stress fields
 *                        of Sec. 4), NaN for split elements (n_elems). */
int mct_get_field(mct_ctx *ctx, int which, int64_t cap, double *out);

/* Energies at t_k (J/m): [0] kinetic sum m |v^k|^2 / 2 with
 * v^k = v^{k-1/2} + dt a^k / 2 for free components after the first step;
 * [1] strain: edge smoothing domains (area sum of intact A_j / 4) times
 * sigma:eps / 2 plus the split pieces; [2] phi(t_k) f_ext . u^k (the work of
 * constant tractions; with a load curve, the current load times u^k);
 * [3] dissipated U_d.  Sums are FP64, deterministic
 * run to run. */
int mct_get_energies(mct_ctx *ctx, double out[4]);

/* Crack-path geometry of n elements (Sec. 2.2, Fig. 2-3: the three paths
 * from the midpoint G0 of tip edge a to the midpoints Gk of the other edges)
 * as the step evaluates it on the GPU: 36 doubles per element, for a = 0..3
 * and j = 0..2 (exit edge k = a+1+j mod 4) the unit normal (x, y) of the
 * segment G0-Gk oriented toward node n_{a+1}, and its length (reference
 * coordinates).  On a triangle mesh the paths are a = 0..2, j = 0..1 (exit
 * edge a+1+j mod 3) and the other entries are NaN.  Elements out of range
 * give MCT_EINVAL. */
int mct_get_path_geometry(mct_ctx *ctx, int64_t n, const int32_t *elem, double *out);

/* Split code of every element (n_elems bytes). */
int mct_get_split_codes(mct_ctx *ctx, int64_t cap, uint8_t *out);

/* Copy the full dynamic state (u, v, split codes, step, U_d, log) into a
 * caller buffer; *bytes receives the size (call with host_buf NULL to query).
 * A plain context whose split-screen buffers exist (mct_screen_enable or
 * mct_screen_collect was called) adds the screen's state: per-element
 * screen states of the current window, the history behind feature 4 with
 * its evaluation stamps, the evaluation count and the counters of
 * mct_screen_stats.  mct_restore loads a buffer produced by mct_checkpoint
 * of a context with the same mesh; with a screen section it restores the
 * screen's state too (the window position follows from the step), so a
 * screened run restored and continued with the same screen (mct_screen_enable
 * with the same parameters, tau and period) is the uninterrupted run; without
 * one the screen starts afresh. */
int mct_checkpoint(mct_ctx *ctx, void *host_buf, int64_t cap, int64_t *bytes);
int mct_restore(mct_ctx *ctx, const void *host_buf, int64_t bytes);

/* Launch tuning: tile shape index (0 = automatic, which is 16x16; 1 = 16x16, 2 = 32x8,
 * 3 = 32x16 elements per workgroup) and whether mct_step replays captured
 * HIP graphs (1, default) or launches kernel by kernel (0).  On an
 * unstructured mesh (triangles or quadrilaterals) the tile index selects the
 * step kernels: 1 = an element kernel and a node kernel; 2, 3, 4 = one fused kernel over patches of 64, 128, 256
 * consecutive nodes (element forces summed in LDS; used when its tables fit:
 * at most 16 elements at a node and 1024 in a patch, else the split
 * kernels); 5 = the fused kernel on the largest patches (64 to 256 nodes)
 * that hold at most 256 elements each (shrunk to even out the compute
 * units' shares); 0 = automatic (5).  The environment
 * variable MCT_PATCH_NODES, read when the choice is made, sets the patch
 * size of choice 5 instead (1..256 nodes; a testing and tuning knob).
 * Results do not depend on any of these choices (fixed summation orders).
 * Errors: MCT_EINVAL for a tile index out of range (0..5 on an
 * unstructured mesh). */
int mct_set_launch(mct_ctx *ctx, int tile, int use_graph);

/* Batch of independent specimens (same step, one launch per time step over
 * all their tiles).  Each specimen is set up like a plain model after
 * mct_batch_select(ctx, s); mct_finalize / mct_step act on the whole batch;
 * every query and set-up call acts on the selected specimen.  Specimens may
 * differ in mesh, material, Gc field, loads, notch and time step.  A plain
 * context (mct_create) is a batch of one.  Errors: MCT_EINVAL for
 * n_specimens < 1 or s out of range; MCT_EUNSUPPORTED for a precision other
 * than 64. */
int mct_batch_create(mct_ctx **out, int64_t n_specimens, int precision, void *hip_stream);
int mct_batch_select(mct_ctx *ctx, int64_t s);

/* Order in which the workgroups of a batch take (specimen, tile) units:
 * -1 automatic, 0 specimen order banded per XCD, 1 specimen order
 * interleaved over XCDs, 2 largest specimens first, banded.  Results do not
 * depend on it. */
int mct_set_order(mct_ctx *ctx, int order);

/* Uniform lattices.  A structured grid whose elements all have, bit for
 * bit, the same geometry -- Q4 gradients at the four edge midpoints (Eq.
 * QUAD_strain_discretization), area, and the unit normals and lengths of the
 * twelve crack paths of Sec. 2.2 (Fig. 2-3) -- and the zero pattern of a
 * rectangle (axis-parallel element edges) is a uniform lattice: e.g. a grid
 * of square elements whose node coordinates i h are exact binary fractions.
 * With MCT_LATTICE_AUTO (default) mct_finalize checks this on the device for
 * binary64 contexts with the point rule (every element's values as the step
 * computes them, compared with element 0's), and when every specimen of the
 * context is a lattice the step takes the shared values instead of
 * recomputing them per element (and stages no coordinates): the same
 * operations in the same order, so the results are identical.
 * MCT_LATTICE_GENERAL always runs the general step.  mct_set_lattice acts at
 * the next mct_finalize (a finalized context must be finalized again);
 * mct_get_lattice reports 1 when the finalized context steps with the
 * lattice kernel.  Structured grids only (MCT_EUNSUPPORTED for a triangle
 * or unstructured quadrilateral mesh). */
enum { MCT_LATTICE_AUTO = 0, MCT_LATTICE_GENERAL = 1 };
int mct_set_lattice(mct_ctx *ctx, int mode);
int mct_get_lattice(mct_ctx *ctx, int *uniform);

/* Near-threshold decision log (the floating-point contract of the split
 * decisions: record every decision whose margin is within a relative
 * tolerance, so that a divergence between two runs can be traced).  With
 * tol > 0 every step records, in binary64 or binary32 as the step computes:
 *   kind 1: a path of an evaluated candidate with |G - Gc| <= tol Gc (the
 *           element rule's threshold, Sec. 2.2);
 *   kind 2: a candidate with two or more paths above Gc whose largest two
 *           differ by <= tol times the largest (the rule's argmax);
 *   kind 3: such a candidate's split-ratio margin
 *           |G* - gamma (G* - G_j)| <= tol G* against path j;
 *   kind 4: the step's two largest accepted candidates differ by
 *           <= tol times the largest (the MCT pick of Sec. 3);
 *   kind 5: the pick's split-ratio margin |G* - gamma (G* - G_min)| <=
 *           tol G* against the smallest accepted G.
 * Record fields: step index, element, tip edge a, kind, exit edge k of the
 * path concerned (kinds 1, 3) or chosen (2, 4, 5), the value G and the
 * value it was compared with (ref).  Kinds 4 and 5 come from the global
 * pick only.  cap (>= 1) records are held on the device; mct_set_near_log
 * acts at the next mct_finalize (tol = 0 turns the log off) and the log
 * starts empty there; checkpoints do not hold it.  mct_get_near_log copies
 * the records sorted by (step, kind, element, a, k); MCT_ECAPACITY when
 * more records were made than the device capacity (count reports how many)
 * or than cap.  Plain structured-grid contexts (MCT_EUNSUPPORTED for a
 * batch or an unstructured mesh); outputs may be NULL. */
int mct_set_near_log(mct_ctx *ctx, double tol, int64_t cap);
int mct_get_near_log(mct_ctx *ctx, int64_t cap, int32_t *step, int32_t *elem, uint8_t *a, uint8_t *kind,
                     uint8_t *k, double *G, double *ref, int64_t *count);

/* Launch autotuner: times trial_steps steps for every tile shape (and, for
 * a batch, every unit order) from the current state, restores that state
 * and keeps the fastest choice.  On an unstructured mesh the choices are
 * the step kernels of mct_set_launch (1 the element plus node kernels,
 * 2/3/4 the fused kernel on 64/128/256-node patches, 5 on patches of the
 * size it finds).  Outputs (any may be NULL): the chosen tile (as
 * mct_get_launch reports it), order and its time per step in
 * microseconds. */
int mct_autotune(mct_ctx *ctx, int trial_steps, int *tile, int *order, double *us_per_step);

/* Launch shape in use: tile index, unit order, workgroups per step (on a
 * unstructured mesh: the step kernels in use, 1 split, 2..4 fused on
 * 64..256-node patches or 5 fused on patches of another size, never 0;
 * the workgroups of the fused kernel or of the element kernel). */
int mct_get_launch(mct_ctx *ctx, int *tile, int *order, int64_t *workgroups);

/* ------------------------------------------------------------------------
 * Learned split-screen (an extension; the paper evaluates every candidate
 * each step).  Every `period` steps the step is exact (all free-surface
 * candidates of Sec. 2.2 evaluated) and then a small MLP scores every
 * candidate (f, a); until the next such step, G is evaluated only for the
 * candidates scored above tau and for candidates that appeared since.  The
 * MCT pick (Sec. 3) stays the same over the evaluated set.
 *
 * The exact G is the judge: each window of screened steps (a period, or
 * its part up to the next exact step) starts from a snapshot of the state,
 * and every skipped candidate is bounded at every screened step, by
 * max_k |sigma_k delta| / 2 >= |G_k| (sigma_k the smoothed stress of path k's
 * exit edge, symmetric, and n_k a unit vector; open stretch gate only).  When a bound reaches Gc the
 * skipped candidate might have been accepted, so the window is restored and
 * replayed with the plain step.  Otherwise no skipped candidate can pass the
 * element rule, the accepted sets and picks are the plain step's, and the
 * window equals the plain run.  So a screened run equals the plain run bit
 * for bit whatever the screen flags; a poor screen costs replays.  Each
 * window ends with a synchronisation of the context's stream (the replay
 * decision is taken on the host).
 *
 * Features of a candidate, in order (h = sqrt(A_f), sigma_ref =
 * sqrt(E Gc_f / h), sigma = mean of the four smoothed edge stresses of f):
 *   0, 1 principal stresses of sigma / sigma_ref (larger first);
 *   2    W h / Gc_f, W = sigma:eps / 2 with eps = D^-1 sigma (plane stress);
 *   3    max over the three paths of G / Gc_f (0 when edge a is not
 *        stretched);
 *   4    feature 3 of the same candidate at the previous evaluation (0 if it
 *        was not a candidate then);
 *   5    min(d / h, 64) / 64, d = reference distance from the midpoint of
 *        edge a to the nearest crack-path end, the midpoint of an entry or
 *        exit edge of a split element whose neighbour across it is intact
 *        (1 without such ends);
 *   6-9  1 where the neighbour across local edge 0..3 is split or outside.
 *
 * MLP (4 929 FP32 parameters, one flat host array): W1 [10][64]
 * (input-major), b1 [64], W2 [64][64], b2 [64], w3 [64], b3; GELU (erf form)
 * after both hidden layers; logit = h2 . w3 + b3.  Products run as bfloat16
 * MFMA with FP32 accumulation: inputs, weights, hidden activations and
 * backpropagated pre-activation gradients are rounded to bfloat16 (nearest,
 * ties to even); biases, GELU, the loss and Adam are FP32.
 * ------------------------------------------------------------------------ */
typedef struct mct_mlp mct_mlp;

/* Features of every current candidate (element order, then local edge),
 * computed on the device from the current state; also advances the
 * history behind feature 4 and clears the screen states (also when the capacity is too small, so pass
 * cap >= 4 x elements, the most candidates there can be).  Outputs are host
 * arrays of capacity cap rows (features: 10 floats per row).  Plain contexts
 * only (MCT_EUNSUPPORTED for a batch); MCT_ESTATE before mct_finalize. */
int mct_screen_collect(mct_ctx *ctx, int64_t cap, float *features, int32_t *elem, uint8_t *entry,
                       int64_t *count);

/* Screened stepping with the parameters of `mlp` (copied; mlp may be
 * destroyed afterwards), threshold tau on the logit and the exact-step
 * period (>= 2; steps k with k % period == 0 are exact).  mct_screen_disable
 * returns to plain stepping.  Checkpoints hold the screen's state (see
 * mct_checkpoint).  Not with the near-threshold log (MCT_EUNSUPPORTED). */
int mct_screen_enable(mct_ctx *ctx, const mct_mlp *mlp, float tau, int period);
int mct_screen_disable(mct_ctx *ctx);

/* Counters since the screen buffers were created: [0] exact steps followed
 * by a screen evaluation, [1] candidates at those steps, [2] candidates
 * flagged, [3] misses: candidates skipped by the previous screen whose
 * max G / Gc exceeds 1 at an exact step, [4] windows judged, [5] windows
 * replayed with the plain step (a skipped candidate's bound reached Gc). */
int mct_screen_stats(mct_ctx *ctx, int64_t out[6]);

/* MLP handle with its own HIP stream (NULL = library-created).  Parameters
 * start at zero.  set_params copies 4 929 host floats and resets the Adam
 * state; get_params copies them back. */
int mct_mlp_create(mct_mlp **out, void *hip_stream);
int mct_mlp_destroy(mct_mlp *mlp);
const char *mct_mlp_last_error(const mct_mlp *mlp);
int mct_mlp_set_params(mct_mlp *mlp, const float *params);
int mct_mlp_get_params(mct_mlp *mlp, float *params);

/* Logits of n rows: x and logits are DEVICE pointers (x: 10 floats per
 * row).  Asynchronous on the handle's stream. */
int mct_mlp_forward(mct_mlp *mlp, const float *x, int64_t n, float *logits);

/* Loss L = (1/n) sum_i w_i (softplus(z_i) - y_i z_i), w_i = pos_weight where
 * y_i = 1 else 1, over n rows (x, y DEVICE pointers, y in {0, 1}), and its
 * gradient with respect to the parameters (host output, 4 929 floats;
 * loss may be NULL).  Synchronous. */
int mct_mlp_gradient(mct_mlp *mlp, const float *x, const float *y, int64_t n, float pos_weight, float *grad,
                     float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on that
 * gradient with learning rate lr.  With loss == NULL the call returns
 * without waiting (x and y must stay valid until the stream has run it);
 * otherwise it waits and stores the loss before the update. */
int mct_mlp_train_step(mct_mlp *mlp, const float *x, const float *y, int64_t n, float pos_weight, float lr,
                       float *loss);

#ifdef __cplusplus
}
#endif

#endif /* MCT2D_H */
