// Host side of the MCT-2D-CEM library: the C ABI declared in mct2d.h,
// mesh/material/load set-up, device memory, step launching (HIP graphs of
// step kernels) and queries.
#include "../../include/mct2d.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mct2d_impl.h"

using mct::Control;
using mct::LogRec;
using mct::Slot;
using mct::StepParams;

namespace {

constexpr int kGraphSteps = 64;  // kernels per captured graph

struct TractionEdge {
    int64_t id;
    int32_t lo, hi;
    double tx, ty;
};

}  // namespace

struct mct_ctx {
    std::string err;
    int precision = 64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;

    // mesh and settings (host copies)
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

    // derived
    bool finalized = false;
    double dt = 0;
    int64_t nn = 0, ne = 0, ns = 0, np = 0;
    int tile_req = 0, tile = 3;
    bool use_graph = true;

    // device
    double *dX = nullptr, *dY = nullptr, *dux[2] = {nullptr, nullptr}, *duy[2] = {nullptr, nullptr};
    double *dvx = nullptr, *dvy = nullptr, *dminv = nullptr, *dgc = nullptr, *dgeom = nullptr;
    double *dfext = nullptr, *dv0 = nullptr;
    uint8_t *dvmask = nullptr, *dsplit = nullptr;
    Control *dctl = nullptr;
    Slot *dslots = nullptr;
    LogRec *dlog = nullptr;
    int32_t log_cap = 0;
    int32_t *dtip_counts = nullptr, *dtip_edge = nullptr, *dtip_total = nullptr;
    double *dtip_xy = nullptr;
    StepParams prm{};

    hipGraphExec_t graph[2] = {nullptr, nullptr};  // by parity of the first step
    int graph_tile[2] = {0, 0};
    int64_t steps_enqueued = 0;  // host view of the step counter
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

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void drop_graphs(mct_ctx *c) {
    for (int i = 0; i < 2; ++i) {
        if (c->graph[i]) (void)hipGraphExecDestroy(c->graph[i]);
        c->graph[i] = nullptr;
    }
}

void release_device(mct_ctx *c) {
    drop_graphs(c);
    dfree(c->dX);
    dfree(c->dY);
    for (int i = 0; i < 2; ++i) {
        dfree(c->dux[i]);
        dfree(c->duy[i]);
    }
    dfree(c->dvx);
    dfree(c->dvy);
    dfree(c->dminv);
    dfree(c->dgc);
    dfree(c->dgeom);
    dfree(c->dfext);
    dfree(c->dv0);
    dfree(c->dvmask);
    dfree(c->dsplit);
    dfree(c->dctl);
    dfree(c->dslots);
    dfree(c->dlog);
    dfree(c->dtip_counts);
    dfree(c->dtip_edge);
    dfree(c->dtip_total);
    dfree(c->dtip_xy);
    c->finalized = false;
}

int64_t node_of(const mct_ctx *c, int i, int j) { return (int64_t)j * (c->nx + 1) + i; }

int perimeter_index(int i, int j, int nx, int ny) {
    if (j == 0) return i;
    if (j == ny) return (nx + 1) + i;
    if (i == 0) return 2 * (nx + 1) + (j - 1);
    if (i == nx) return 2 * (nx + 1) + (ny - 1) + (j - 1);
    return -1;
}

// Id of the edge joining nodes a and b of the grid, or -1.  Edges are
// numbered in ascending (smaller node, larger node) order.
int64_t edge_id(const mct_ctx *c, int64_t a, int64_t b) {
    const int64_t lo = std::min(a, b), hi = std::max(a, b);
    const int nx = c->nx, ny = c->ny;
    const int i = (int)(lo % (nx + 1)), j = (int)(lo / (nx + 1));
    const int64_t row = 2 * (int64_t)nx + 1;
    if (hi == lo + 1 && i < nx) return (j < ny) ? j * row + 2 * i : (int64_t)ny * row + i;
    if (hi == lo + nx + 1 && j < ny) return j * row + (i < nx ? 2 * i + 1 : 2 * nx);
    return -1;
}

bool boundary_edge(const mct_ctx *c, int64_t a, int64_t b) {
    const int64_t lo = std::min(a, b), hi = std::max(a, b);
    const int nx = c->nx, ny = c->ny;
    const int i = (int)(lo % (nx + 1)), j = (int)(lo / (nx + 1));
    if (hi == lo + 1) return j == 0 || j == ny;
    return i == 0 || i == nx;
}

void elem_nodes(const mct_ctx *c, int64_t e, int64_t n[4]) {
    const int i = (int)(e % c->nx), j = (int)(e / c->nx);
    n[0] = node_of(c, i, j);
    n[1] = node_of(c, i + 1, j);
    n[2] = node_of(c, i + 1, j + 1);
    n[3] = node_of(c, i, j + 1);
}

double elem_area(const mct_ctx *c, int64_t e) {
    int64_t n[4];
    elem_nodes(c, e, n);
    const double *X = c->X.data(), *Y = c->Y.data();
    return 0.5 * ((X[n[2]] - X[n[0]]) * (Y[n[3]] - Y[n[1]]) - (X[n[3]] - X[n[1]]) * (Y[n[2]] - Y[n[0]]));
}

template <typename T>
int upload(mct_ctx *c, T *&dst, const T *src, size_t n) {
    HIP_TRY(c, hipMalloc((void **)&dst, std::max<size_t>(n, 1) * sizeof(T)));
    if (n) HIP_TRY(c, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return MCT_OK;
}

int pick_tile(const mct_ctx *c) {
    if (c->tile_req >= 1 && c->tile_req <= mct::kNumTiles) return c->tile_req;
    // largest tile that still gives every CU several workgroups
    for (int t : {3, 2, 1}) {
        const mct::TileShape s = mct::tile_shape(t);
        const int64_t nwg = ((c->nx + 1 + s.txe - 2) / (s.txe - 1)) * (int64_t)((c->ny + 1 + s.tye - 2) / (s.tye - 1));
        if (nwg >= 4 * 256) return t;
    }
    return 1;
}

void set_launch_geometry(mct_ctx *c) {
    c->tile = pick_tile(c);
    const mct::TileShape s = mct::tile_shape(c->tile);
    c->prm.ntx = (c->nx + 1 + s.txe - 2) / (s.txe - 1);
    c->prm.nty = (c->ny + 1 + s.tye - 2) / (s.tye - 1);
    c->prm.nwg = c->prm.ntx * c->prm.nty;
}

// A segment of kGraphSteps steps followed by its commit, captured once per
// parity of the segment's first step.
int build_graph(mct_ctx *c, int par0) {
    if (c->graph[par0]) (void)hipGraphExecDestroy(c->graph[par0]);
    c->graph[par0] = nullptr;
    hipStream_t cap;
    HIP_TRY(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    for (int i = 0; e == hipSuccess && i < kGraphSteps; ++i) e = mct::launch_step(c->tile, c->prm, i, par0, cap);
    if (e == hipSuccess) e = mct::launch_commit(c->prm, kGraphSteps, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->graph[par0], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(c, MCT_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    c->graph_tile[par0] = c->tile;
    return MCT_OK;
}

}  // namespace

extern "C" {

int mct_create(mct_ctx **out, int precision, void *hip_stream) {
    if (!out) return MCT_EINVAL;
    *out = nullptr;
    if (precision != 64) return MCT_EUNSUPPORTED;
    mct_ctx *c = new (std::nothrow) mct_ctx;
    if (!c) return MCT_ENOMEM;
    c->precision = precision;
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

int mct_destroy(mct_ctx *c) {
    if (!c) return MCT_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release_device(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MCT_OK;
}

const char *mct_last_error(const mct_ctx *c) { return c ? c->err.c_str() : "null context"; }

int mct_set_mesh_grid(mct_ctx *c, int32_t nx, int32_t ny, const double *X, const double *Y) {
    if (!c) return MCT_EINVAL;
    if (nx < 2 || ny < 2 || !X || !Y) return fail(c, MCT_EINVAL, "grid needs nx, ny >= 2 and coordinates");
    if ((int64_t)nx * ny > (int64_t)1 << 30) return fail(c, MCT_EINVAL, "grid too large");
    release_device(c);
    c->nx = nx;
    c->ny = ny;
    c->nn = (int64_t)(nx + 1) * (ny + 1);
    c->ne = (int64_t)nx * ny;
    c->ns = 2 * (int64_t)nx * ny + nx + ny;
    c->np = 2 * (int64_t)(nx + 1) + 2 * (int64_t)(ny - 1);
    c->X.assign(X, X + c->nn);
    c->Y.assign(Y, Y + c->nn);
    for (int64_t e = 0; e < c->ne; ++e)
        if (!(elem_area(c, e) > 0.0))
            return fail(c, MCT_EINVAL, "element %lld has non-positive area (clockwise or degenerate)", (long long)e);
    c->have_material = false;
    c->gc.clear();
    c->traction.clear();
    c->vbc_node.clear();
    c->vbc_mask.clear();
    c->vbc_v0.clear();
    c->notch_elem.clear();
    c->notch_code.clear();
    c->dt_in = 0;
    c->cfl = 0.5;
    return MCT_OK;
}

int mct_set_material(mct_ctx *c, double E, double nu, double rho, const double *Gc, double Gc_uniform,
                     double gamma) {
    if (!c) return MCT_EINVAL;
    if (!c->nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (!(E > 0) || !(nu > -1.0 && nu < 0.5) || !(rho > 0) || !(gamma > 0))
        return fail(c, MCT_EINVAL, "material out of range");
    if (Gc) {
        for (int64_t e = 0; e < c->ne; ++e)
            if (!(Gc[e] > 0)) return fail(c, MCT_EINVAL, "Gc[%lld] <= 0", (long long)e);
        c->gc.assign(Gc, Gc + c->ne);
    } else {
        if (!(Gc_uniform > 0)) return fail(c, MCT_EINVAL, "Gc_uniform <= 0");
        c->gc.clear();
    }
    c->E = E;
    c->nu = nu;
    c->rho = rho;
    c->gamma = gamma;
    c->gc_uniform = Gc_uniform;
    c->have_material = true;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_traction(mct_ctx *c, int64_t n, const int32_t *edge_nodes, const double *t) {
    if (!c) return MCT_EINVAL;
    if (!c->nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!edge_nodes || !t))) return fail(c, MCT_EINVAL, "bad traction arrays");
    std::vector<TractionEdge> v;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a = edge_nodes[2 * i], b = edge_nodes[2 * i + 1];
        if (a < 0 || b < 0 || a >= c->nn || b >= c->nn) return fail(c, MCT_EINVAL, "traction edge %lld: node out of range", (long long)i);
        const int64_t id = edge_id(c, a, b);
        if (id < 0 || !boundary_edge(c, a, b))
            return fail(c, MCT_EINVAL, "traction edge %lld is not a boundary edge", (long long)i);
        v.push_back({id, (int32_t)std::min(a, b), (int32_t)std::max(a, b), t[2 * i], t[2 * i + 1]});
    }
    std::sort(v.begin(), v.end(), [](const TractionEdge &x, const TractionEdge &y) { return x.id < y.id; });
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i].id == v[i - 1].id) return fail(c, MCT_EINVAL, "repeated traction edge");
    c->traction.swap(v);
    c->finalized = false;
    return MCT_OK;
}

int mct_set_velocity_bc(mct_ctx *c, int64_t n, const int32_t *node, const uint8_t *dof_mask, const double *v0,
                        double t_ramp) {
    if (!c) return MCT_EINVAL;
    if (!c->nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!node || !dof_mask || !v0)) || !(t_ramp >= 0))
        return fail(c, MCT_EINVAL, "bad velocity arrays");
    for (int64_t i = 0; i < n; ++i) {
        if (node[i] < 0 || node[i] >= c->nn || (dof_mask[i] & ~3u))
            return fail(c, MCT_EINVAL, "velocity bc %lld out of range", (long long)i);
        const int ii = (int)(node[i] % (c->nx + 1)), jj = (int)(node[i] / (c->nx + 1));
        if (perimeter_index(ii, jj, c->nx, c->ny) < 0)
            return fail(c, MCT_EINVAL, "velocity bc on interior node %d is not supported", node[i]);
    }
    c->vbc_node.assign(node, node + n);
    c->vbc_mask.assign(dof_mask, dof_mask + n);
    c->vbc_v0.assign(v0, v0 + 2 * n);
    c->t_ramp = t_ramp;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_notch(mct_ctx *c, int64_t n, const int32_t *elem, const uint8_t *entry, const uint8_t *exit) {
    if (!c) return MCT_EINVAL;
    if (!c->nx) return fail(c, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!elem || !entry || !exit))) return fail(c, MCT_EINVAL, "bad notch arrays");
    c->notch_elem.clear();
    c->notch_code.clear();
    for (int64_t i = 0; i < n; ++i) {
        if (elem[i] < 0 || elem[i] >= c->ne || entry[i] > 3 || exit[i] > 3 || entry[i] == exit[i])
            return fail(c, MCT_EINVAL, "notch element %lld invalid", (long long)i);
        c->notch_elem.push_back(elem[i]);
        c->notch_code.push_back((uint8_t)(mct::kSplitFlag | (entry[i] << 2) | exit[i]));
    }
    c->finalized = false;
    return MCT_OK;
}

int mct_set_time(mct_ctx *c, double dt, double cfl_fraction) {
    if (!c) return MCT_EINVAL;
    if (!(dt > 0) && !(cfl_fraction > 0)) return fail(c, MCT_EINVAL, "need dt > 0 or cfl_fraction > 0");
    c->dt_in = dt;
    c->cfl = cfl_fraction;
    c->finalized = false;
    return MCT_OK;
}

int mct_set_launch(mct_ctx *c, int tile, int use_graph) {
    if (!c) return MCT_EINVAL;
    if (tile < 0 || tile > mct::kNumTiles) return fail(c, MCT_EINVAL, "tile index out of range");
    c->tile_req = tile;
    c->use_graph = use_graph != 0;
    if (c->finalized) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        set_launch_geometry(c);
        drop_graphs(c);
        // three slot sets of one entry per workgroup of the chosen shape
        dfree(c->dslots);
        HIP_TRY(c, hipMalloc((void **)&c->dslots, 3 * sizeof(Slot) * (size_t)c->prm.nwg));
        c->prm.slots = c->dslots;
    }
    return MCT_OK;
}

int mct_finalize(mct_ctx *c) {
    if (!c) return MCT_EINVAL;
    if (!c->nx || !c->have_material) return fail(c, MCT_ESTATE, "mesh and material are required");
    release_device(c);
    const int nx = c->nx, ny = c->ny;
    const double *X = c->X.data(), *Y = c->Y.data();

    // lumped mass: rho A_e / 4 from each element, element-id order per node
    std::vector<double> area(c->ne), minv(c->nn);
    for (int64_t e = 0; e < c->ne; ++e) area[e] = elem_area(c, e);
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            double m = 0.0;
            const int ei[4] = {i - 1, i, i - 1, i}, ej[4] = {j - 1, j - 1, j, j};
            for (int q = 0; q < 4; ++q) {
                if (ei[q] < 0 || ei[q] >= nx || ej[q] < 0 || ej[q] >= ny) continue;
                m += c->rho * area[(int64_t)ej[q] * nx + ei[q]] / 4.0;
            }
            minv[node_of(c, i, j)] = 1.0 / m;
        }

    // equivalent nodal forces of the tractions (edge-id order), prescribed
    // velocities, on perimeter-indexed arrays
    std::vector<double> fext(2 * c->np, 0.0), v0(2 * c->np, 0.0);
    std::vector<uint8_t> vmask(c->np, 0);
    for (const TractionEdge &t : c->traction) {
        const double dx = X[t.hi] - X[t.lo], dy = Y[t.hi] - Y[t.lo];
        const double L = std::sqrt(dx * dx + dy * dy);
        const double fx = t.tx * L * 0.5, fy = t.ty * L * 0.5;
        for (int32_t nd : {t.lo, t.hi}) {
            const int pi = perimeter_index(nd % (nx + 1), nd / (nx + 1), nx, ny);
            fext[2 * pi] += fx;
            fext[2 * pi + 1] += fy;
        }
    }
    for (size_t q = 0; q < c->vbc_node.size(); ++q) {
        const int nd = c->vbc_node[q];
        const int pi = perimeter_index(nd % (nx + 1), nd / (nx + 1), nx, ny);
        vmask[pi] = c->vbc_mask[q];
        v0[2 * pi] = c->vbc_v0[2 * q];
        v0[2 * pi + 1] = c->vbc_v0[2 * q + 1];
    }

    // time step
    if (c->dt_in > 0) {
        c->dt = c->dt_in;
    } else {
        double hmin = INFINITY;
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                const int64_t a = node_of(c, i, j);
                if (i < nx) {
                    const double dx = X[a + 1] - X[a], dy = Y[a + 1] - Y[a];
                    hmin = std::min(hmin, std::sqrt(dx * dx + dy * dy));
                }
                if (j < ny) {
                    const int64_t b = a + nx + 1;
                    const double dx = X[b] - X[a], dy = Y[b] - Y[a];
                    hmin = std::min(hmin, std::sqrt(dx * dx + dy * dy));
                }
            }
        const double cd = std::sqrt(c->E / (c->rho * (1.0 - c->nu * c->nu)));
        c->dt = c->cfl * hmin / cd;
    }

    // crack-path geometry per element: for tip edge a and exit edge
    // k = a+1+j, the unit normal of the segment between the two edge
    // midpoints, oriented toward node n_{a+1}, and its length
    std::vector<double> geom((size_t)c->ne * 36);
    for (int64_t e = 0; e < c->ne; ++e) {
        int64_t n[4];
        elem_nodes(c, e, n);
        for (int a = 0; a < 4; ++a) {
            const int64_t p0 = n[a], p1 = n[(a + 1) & 3];
            const double g0x = 0.5 * (X[p0] + X[p1]), g0y = 0.5 * (Y[p0] + Y[p1]);
            for (int j = 0; j < 3; ++j) {
                const int k = (a + 1 + j) & 3;
                const int64_t q0 = n[k], q1 = n[(k + 1) & 3];
                const double gkx = 0.5 * (X[q0] + X[q1]), gky = 0.5 * (Y[q0] + Y[q1]);
                const double dx = gkx - g0x, dy = gky - g0y;
                const double L = std::sqrt(dx * dx + dy * dy);
                double cx = dy / L, cy = -dx / L;
                if (cx * (X[p1] - g0x) + cy * (Y[p1] - g0y) < 0.0) {
                    cx = -cx;
                    cy = -cy;
                }
                double *g = &geom[(size_t)e * 36 + a * 9 + 3 * j];
                g[0] = cx;
                g[1] = cy;
                g[2] = L;
            }
        }
    }

    std::vector<uint8_t> split(c->ne, 0);
    for (size_t q = 0; q < c->notch_elem.size(); ++q) split[c->notch_elem[q]] = c->notch_code[q];

    set_launch_geometry(c);
    c->log_cap = (int32_t)std::min<int64_t>(c->ne, INT32_MAX);

    int rc;
    if ((rc = upload(c, c->dX, X, c->nn))) return rc;
    if ((rc = upload(c, c->dY, Y, c->nn))) return rc;
    if ((rc = upload(c, c->dminv, minv.data(), c->nn))) return rc;
    if ((rc = upload(c, c->dgeom, geom.data(), geom.size()))) return rc;
    if ((rc = upload(c, c->dfext, fext.data(), fext.size()))) return rc;
    if ((rc = upload(c, c->dv0, v0.data(), v0.size()))) return rc;
    if ((rc = upload(c, c->dvmask, vmask.data(), vmask.size()))) return rc;
    if ((rc = upload(c, c->dsplit, split.data(), split.size()))) return rc;
    if (!c->gc.empty() && (rc = upload(c, c->dgc, c->gc.data(), c->gc.size()))) return rc;
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(c, hipMalloc((void **)&c->dux[i], sizeof(double) * c->nn));
        HIP_TRY(c, hipMalloc((void **)&c->duy[i], sizeof(double) * c->nn));
        HIP_TRY(c, hipMemsetAsync(c->dux[i], 0, sizeof(double) * c->nn, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->duy[i], 0, sizeof(double) * c->nn, c->stream));
    }
    HIP_TRY(c, hipMalloc((void **)&c->dvx, sizeof(double) * c->nn));
    HIP_TRY(c, hipMalloc((void **)&c->dvy, sizeof(double) * c->nn));
    HIP_TRY(c, hipMemsetAsync(c->dvx, 0, sizeof(double) * c->nn, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->dvy, 0, sizeof(double) * c->nn, c->stream));
    HIP_TRY(c, hipMalloc((void **)&c->dctl, sizeof(Control)));
    HIP_TRY(c, hipMemsetAsync(c->dctl, 0, sizeof(Control), c->stream));
    HIP_TRY(c, hipMalloc((void **)&c->dslots, 3 * sizeof(Slot) * (size_t)c->prm.nwg));
    HIP_TRY(c, hipMalloc((void **)&c->dlog, sizeof(LogRec) * (size_t)std::max(c->log_cap, 1)));
    const int nb = mct::tips_nblocks(c->ns);
    HIP_TRY(c, hipMalloc((void **)&c->dtip_counts, sizeof(int32_t) * (size_t)nb));
    HIP_TRY(c, hipMalloc((void **)&c->dtip_total, sizeof(int32_t)));

    StepParams &p = c->prm;
    p.nx = nx;
    p.ny = ny;
    p.log_cap = c->log_cap;
    p.X = c->dX;
    p.Y = c->dY;
    p.ux0 = c->dux[0];
    p.uy0 = c->duy[0];
    p.ux1 = c->dux[1];
    p.uy1 = c->duy[1];
    p.vx = c->dvx;
    p.vy = c->dvy;
    p.minv = c->dminv;
    p.split = c->dsplit;
    p.gc = c->dgc;
    p.gc_uniform = c->gc_uniform;
    p.geom = c->dgeom;
    p.fext_p = c->dfext;
    p.vmask_p = c->dvmask;
    p.v0_p = c->dv0;
    p.D11 = c->E / (1.0 - c->nu * c->nu);
    p.D12 = c->nu * p.D11;
    p.D33 = c->E / (2.0 * (1.0 + c->nu));
    p.E = c->E;
    p.dt = c->dt;
    p.t_ramp = c->t_ramp;
    p.gamma = c->gamma;
    p.ctl = c->dctl;
    p.slots = c->dslots;
    p.log = c->dlog;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->steps_enqueued = 0;
    c->finalized = true;
    return MCT_OK;
}

int mct_step(mct_ctx *c, int64_t n) {
    if (!c) return MCT_EINVAL;
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (n < 0) return fail(c, MCT_EINVAL, "negative step count");
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
    }
    while (left > 0) {
        // direct segment, closed by its commit
        const int seg = (int)std::min<int64_t>(left, 1 << 20);
        const int par0 = (int)(c->steps_enqueued & 1);
        for (int i = 0; i < seg; ++i) HIP_TRY(c, mct::launch_step(c->tile, c->prm, i, par0, c->stream));
        HIP_TRY(c, mct::launch_commit(c->prm, seg, c->stream));
        left -= seg;
        c->steps_enqueued += seg;
    }
    return MCT_OK;
}

int mct_sync(mct_ctx *c) {
    if (!c) return MCT_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

static int read_control(mct_ctx *c, Control *h) {
    HIP_TRY(c, hipMemcpyAsync(h, c->dctl, sizeof(Control), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

int mct_get_info(mct_ctx *c, mct_info *out) {
    if (!c || !out) return MCT_EINVAL;
    std::memset(out, 0, sizeof *out);
    out->n_nodes = c->nn;
    out->n_elems = c->ne;
    out->n_edges = c->ns;
    out->dt = c->dt;
    out->precision = c->precision;
    if (!c->finalized) return MCT_OK;
    Control h;
    int rc = read_control(c, &h);
    if (rc) return rc;
    out->step = h.base;
    out->n_splits = h.nsplit;
    out->dissipated = h.Ud;
    out->log_overflow = h.overflow;
    return MCT_OK;
}

int mct_get_crack_set(mct_ctx *c, int64_t cap, int32_t *step, int32_t *elem, uint8_t *entry, uint8_t *exit,
                      double *G, int64_t *count) {
    if (!c || !count) return MCT_EINVAL;
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    Control h;
    int rc = read_control(c, &h);
    if (rc) return rc;
    const int64_t n = std::min<int64_t>(h.nsplit, c->log_cap);
    *count = n;
    if (cap < n) return fail(c, MCT_ECAPACITY, "crack set holds %lld splits", (long long)n);
    std::vector<LogRec> v((size_t)n);
    if (n) {
        HIP_TRY(c, hipMemcpyAsync(v.data(), c->dlog, sizeof(LogRec) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
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
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    int32_t nb = 0, total = 0;
    HIP_TRY(c, mct::launch_tips(c->nx, c->ny, c->dX, c->dY, c->dsplit, c->dtip_counts, &nb, nullptr, nullptr,
                                c->dtip_total, c->stream));
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
    hipError_t e = mct::launch_tips(c->nx, c->ny, c->dX, c->dY, c->dsplit, c->dtip_counts, &nb, de, dxy,
                                    c->dtip_total, c->stream);
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

int mct_get_field(mct_ctx *c, int which, int64_t cap, double *out) {
    if (!c || !out) return MCT_EINVAL;
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (cap < 2 * c->nn) return fail(c, MCT_ECAPACITY, "field needs %lld values", (long long)(2 * c->nn));
    Control h;
    int rc = read_control(c, &h);
    if (rc) return rc;
    const double *sx, *sy;
    if (which == MCT_FIELD_U) {
        sx = c->dux[h.base & 1];
        sy = c->duy[h.base & 1];
    } else if (which == MCT_FIELD_V) {
        sx = c->dvx;
        sy = c->dvy;
    } else {
        return fail(c, MCT_EINVAL, "unknown field %d", which);
    }
    HIP_TRY(c, hipMemcpyAsync(out, sx, sizeof(double) * c->nn, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(out + c->nn, sy, sizeof(double) * c->nn, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

int mct_get_split_codes(mct_ctx *c, int64_t cap, uint8_t *out) {
    if (!c || !out) return MCT_EINVAL;
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    if (cap < c->ne) return fail(c, MCT_ECAPACITY, "need %lld bytes", (long long)c->ne);
    HIP_TRY(c, hipMemcpyAsync(out, c->dsplit, (size_t)c->ne, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

// checkpoint layout: magic, nn, ne, Control, ux, uy, vx, vy, split, log
static const uint64_t kMagic = 0x4d43543244434b31ull;  // "MCT2DCK1"

int mct_checkpoint(mct_ctx *c, void *buf, int64_t cap, int64_t *bytes) {
    if (!c || !bytes) return MCT_EINVAL;
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    Control h;
    int rc = read_control(c, &h);
    if (rc) return rc;
    const int64_t nlog = std::min<int64_t>(h.nsplit, c->log_cap);
    const int64_t need = 3 * 8 + (int64_t)sizeof(Control) + 4 * 8 * c->nn + c->ne + nlog * (int64_t)sizeof(LogRec);
    *bytes = need;
    if (!buf) return MCT_OK;
    if (cap < need) return fail(c, MCT_ECAPACITY, "checkpoint needs %lld bytes", (long long)need);
    char *p = (char *)buf;
    const uint64_t hdr[3] = {kMagic, (uint64_t)c->nn, (uint64_t)c->ne};
    std::memcpy(p, hdr, sizeof hdr);
    p += sizeof hdr;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    const double *src[4] = {c->dux[h.base & 1], c->duy[h.base & 1], c->dvx, c->dvy};
    for (int i = 0; i < 4; ++i) {
        HIP_TRY(c, hipMemcpyAsync(p, src[i], 8 * c->nn, hipMemcpyDeviceToHost, c->stream));
        p += 8 * c->nn;
    }
    HIP_TRY(c, hipMemcpyAsync(p, c->dsplit, c->ne, hipMemcpyDeviceToHost, c->stream));
    p += c->ne;
    if (nlog) HIP_TRY(c, hipMemcpyAsync(p, c->dlog, sizeof(LogRec) * nlog, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCT_OK;
}

int mct_restore(mct_ctx *c, const void *buf, int64_t bytes) {
    if (!c || !buf) return MCT_EINVAL;
    if (!c->finalized) return fail(c, MCT_ESTATE, "finalize first");
    const char *p = (const char *)buf;
    if (bytes < 24 + (int64_t)sizeof(Control)) return fail(c, MCT_EINVAL, "checkpoint too short");
    uint64_t hdr[3];
    std::memcpy(hdr, p, sizeof hdr);
    p += sizeof hdr;
    if (hdr[0] != kMagic || (int64_t)hdr[1] != c->nn || (int64_t)hdr[2] != c->ne)
        return fail(c, MCT_EINVAL, "checkpoint does not match this mesh");
    Control h;
    std::memcpy(&h, p, sizeof h);
    p += sizeof h;
    const int64_t nlog = std::min<int64_t>(h.nsplit, c->log_cap);
    const int64_t need = 24 + (int64_t)sizeof(Control) + 4 * 8 * c->nn + c->ne + nlog * (int64_t)sizeof(LogRec);
    if (bytes < need || h.base < 0) return fail(c, MCT_EINVAL, "checkpoint truncated");
    h.nslots[0] = h.nslots[1] = h.nslots[2] = 0;
    HIP_TRY(c, hipMemcpyAsync(c->dctl, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
    double *dst[4] = {c->dux[h.base & 1], c->duy[h.base & 1], c->dvx, c->dvy};
    for (int i = 0; i < 4; ++i) {
        HIP_TRY(c, hipMemcpyAsync(dst[i], p, 8 * c->nn, hipMemcpyHostToDevice, c->stream));
        p += 8 * c->nn;
    }
    HIP_TRY(c, hipMemcpyAsync(c->dsplit, p, c->ne, hipMemcpyHostToDevice, c->stream));
    p += c->ne;
    if (nlog) HIP_TRY(c, hipMemcpyAsync(c->dlog, p, sizeof(LogRec) * nlog, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->steps_enqueued = h.base;
    return MCT_OK;
}

}  // extern "C"
