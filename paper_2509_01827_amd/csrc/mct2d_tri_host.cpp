// Host side of the unstructured-mesh path (constant-strain triangles or
// bilinear quadrilaterals): mesh tables,
// greedy colouring, lumped mass, equivalent nodal tractions, device memory,
// the time-step loop (HIP graphs of step kernels) and the queries.
//
// The tables follow the plain definitions of the method: edges are the
// sorted (smaller node, larger node) pairs; each edge lists its elements by
// increasing id; element colours come from a greedy colouring in element-id
// order (smallest colour not used by an earlier element sharing a node), and
// the nodal sums of element forces run in colour order.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "mct2d_tri_host.h"

namespace mct {
namespace tri {
namespace {

constexpr int kGraphSteps = 64;

int fail(Host h, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h.err = buf;
    return code;
}

#define TRY(h, expr)                                                                                \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail((h), MCT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

template <typename T>
int upload(Host h, T *&dst, const void *src, size_t n) {
    TRY(h, hipMalloc((void **)&dst, std::max<size_t>(n, 1) * sizeof(T)));
    if (n) TRY(h, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, h.stream));
    return MCT_OK;
}

int64_t find_edge(const Model &m, int64_t a, int64_t b) {
    const int32_t lo = (int32_t)std::min(a, b), hi = (int32_t)std::max(a, b);
    int64_t l = 0, r = m.ns - 1;
    while (l <= r) {
        const int64_t mid = (l + r) / 2;
        const int32_t ml = m.edge_node[2 * mid], mh = m.edge_node[2 * mid + 1];
        if (ml == lo && mh == hi) return mid;
        if (ml < lo || (ml == lo && mh < hi))
            l = mid + 1;
        else
            r = mid - 1;
    }
    return -1;
}

bool need_mesh(const Model &m) { return m.ne == 0; }

void invalidate(Model &m) {
    m.finalized = false;
}

int read_ctl(Model &m, Host h, Ctl *out) {
    TRY(h, hipMemcpyAsync(out, m.dctl, sizeof(Ctl), hipMemcpyDeviceToHost, h.stream));
    TRY(h, hipStreamSynchronize(h.stream));
    return MCT_OK;
}

int ensure_eval(Model &m, Host h) {
    if (m.ev.fint) return MCT_OK;
    const size_t nn = (size_t)m.nn, ne = (size_t)m.ne, ns = (size_t)m.ns;
    TRY(h, hipMalloc((void **)&m.ev.sig_ek, sizeof(double) * 3 * m.nv * ne));
    TRY(h, hipMalloc((void **)&m.ev.es_ek, sizeof(double) * m.nv * ne));
    TRY(h, hipMalloc((void **)&m.ev.pe, sizeof(double) * ne));
    TRY(h, hipMalloc((void **)&m.ev.principal, sizeof(double) * ne));
    TRY(h, hipMalloc((void **)&m.ev.fint, sizeof(double) * 2 * nn));
    TRY(h, hipMalloc((void **)&m.ev.acc, sizeof(double) * 2 * nn));
    TRY(h, hipMalloc((void **)&m.ev.node_e, sizeof(double) * 2 * nn));
    TRY(h, hipMalloc((void **)&m.dpart, sizeof(double) * sum_partials()));
    TRY(h, hipMalloc((void **)&m.dsums, sizeof(double) * 8));
    TRY(h, hipMalloc((void **)&m.dpow, sizeof(double) * 8 * nn));
    TRY(h, hipMalloc((void **)&m.dtipflag, std::max<size_t>(ns, 1)));
    TRY(h, hipMalloc((void **)&m.dwatch, sizeof(int32_t)));
    return MCT_OK;
}

// Largest eigenvalue of M^-1 K over the free components by power iteration
// on M^-1/2 K M^-1/2 (K u = internal force of u with the set-up splits),
// from a deterministic pseudo-random start; the Rayleigh quotient
// approaches lambda_max from below, so 2 / sqrt(lambda) is an upper
// estimate of the stability limit of central differences.
int stability_limit(Model &m, Host h) {
    int rc = ensure_eval(m, h);
    if (rc) return rc;
    const int64_t nn = m.nn;
    std::vector<double> y(2 * nn);
    double norm = 0.0;
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (int64_t i = 0; i < 2 * nn; ++i) {
        s ^= s >> 33;
        s *= 0xFF51AFD7ED558CCDull;
        s ^= s >> 29;
        s += 0x9E3779B97F4A7C15ull;
        const double r = (double)(s >> 11) * 0x1.0p-53;
        y[i] = ((s >> 7) & 1) ? (1.0 + 0.05 * r) : -(1.0 + 0.05 * r);
        norm += y[i] * y[i];
    }
    norm = std::sqrt(norm);
    for (double &v : y) v /= norm;
    double *dy = m.dpow, *dz = m.dpow + 2 * nn, *dyz = m.dpow + 4 * nn;
    double2 *du = reinterpret_cast<double2 *>(m.dpow + 6 * nn);
    TRY(h, hipMemcpyAsync(dy, y.data(), sizeof(double) * 2 * nn, hipMemcpyHostToDevice, h.stream));
    double lam = 0.0, prev = 0.0;
    for (int it = 1; it <= 4000; ++it) {
        TRY(h, launch_power_step(m.prm, m.ev, dy, du, dz, dyz, m.dpart, m.dsums, h.stream));
        if (it % 20 == 0) {
            TRY(h, hipMemcpyAsync(&lam, m.dsums, sizeof(double), hipMemcpyDeviceToHost, h.stream));
            TRY(h, hipStreamSynchronize(h.stream));
            if (!(lam > 0.0) || !std::isfinite(lam))
                return fail(h, MCT_ENUMERIC, "stability estimate failed (Rayleigh quotient %g)", lam);
            if (std::fabs(lam - prev) <= 1e-7 * lam) break;
            prev = lam;
        }
    }
    m.dt_limit = 2.0 / std::sqrt(lam);
    return MCT_OK;
}

int eval_state(Model &m, Host h, Ctl *ctl, bool with_energy) {
    int rc = ensure_eval(m, h);
    if (rc) return rc;
    if ((rc = read_ctl(m, h, ctl))) return rc;
    const int64_t k = ctl->base;
    double phi = 1.0;
    const size_t n = m.curve_t.size();
    if (n) {
        // the step's load factor at t_k (largest i with t_i <= t)
        const double t = (double)k * m.dt;
        if (t <= m.curve_t[0]) {
            phi = m.curve_phi[0];
        } else if (t >= m.curve_t[n - 1]) {
            phi = m.curve_phi[n - 1];
        } else {
            size_t i = 0;
            while (m.curve_t[i + 1] <= t) ++i;
            const double slope = (m.curve_phi[i + 1] - m.curve_phi[i]) / (m.curve_t[i + 1] - m.curve_t[i]);
            phi = m.curve_phi[i] + (t - m.curve_t[i]) * slope;
        }
    }
    TRY(h, launch_eval(m.prm, m.du[k & 1], with_energy ? m.dv : nullptr, k, phi, m.dmass, m.ev, h.stream));
    return MCT_OK;
}

// Fused-step tables for patches of P consecutive nodes (one workgroup each;
// triangles or quadrilaterals, nv nodes per element): the patch's elements
// (every element touching an owned node, ascending id, flagged kOwned in the
// patch of its smallest node, which alone evaluates its candidates) and, per
// owned node, the LDS slots of its element forces in colour order, padded to
// the gather lists' width; each patch's ring (the neighbours of its
// elements outside it, ascending) and per patch element its neighbours'
// strain slots (patch elements first, then the ring), lower-id flags and
// the shared edges' local indices in the neighbours.  Returns the largest
// element count of a patch (257 when it is at most 256 but a ring exceeds
// what the 256-slot kernel holds), 0 if the tables do not fit the kernel
// (more than 16 elements at a node or 1024 in a patch).
int build_patches(Model &m, Host h, int P, int32_t *emax_out, int32_t *rmax_out = nullptr) {
    *emax_out = 0;
    const int64_t nn = m.nn, ne = m.ne;
    const int nv = m.nv;
    const std::vector<int32_t> &noff = m.gnoff, &nel = m.gnel;
    int32_t maxdeg = 0;
    for (int64_t i = 0; i < nn; ++i) maxdeg = std::max(maxdeg, noff[i + 1] - noff[i]);
    const int32_t W = (maxdeg + 3) / 4 * 4;
    if (W > 16) return MCT_OK;
    const int64_t npatch = (nn + P - 1) / P;
    const int st = nv + 1;  // neighbour table stride
    std::vector<int32_t> poff{0}, pelem, slot_of(ne, -1), stamp(ne, -1), els, roff{0}, pring, ring;
    std::vector<uint2> pnbr, plconn, prlconn;
    std::vector<int32_t> hoff{0}, phalo, halo, nstamp(nv == 3 ? nn : 0, -1), nloc(nv == 3 ? nn : 0, 0);
    std::vector<uint16_t> pslots((size_t)npatch * P * W, 0xffff);
    int32_t emax = 0, rmax = 0, lmax = 0;
    for (int64_t b = 0; b < npatch; ++b) {
        const int64_t n0 = b * P, n1 = std::min<int64_t>(nn, n0 + P);
        els.clear();
        for (int64_t i = n0; i < n1; ++i)
            for (int32_t t = noff[i]; t < noff[i + 1]; ++t) {
                const int32_t e = nel[t] / nv;
                if (stamp[e] != (int32_t)b) {
                    stamp[e] = (int32_t)b;
                    els.push_back(e);
                }
            }
        std::sort(els.begin(), els.end());
        if ((int64_t)els.size() > 1024) return MCT_OK;
        emax = std::max<int32_t>(emax, (int32_t)els.size());
        for (size_t q = 0; q < els.size(); ++q) {
            const int32_t e = els[q];
            slot_of[e] = (int32_t)q;
            const int32_t mn = *std::min_element(m.conn.begin() + (int64_t)nv * e, m.conn.begin() + (int64_t)nv * (e + 1));
            pelem.push_back(e | (mn / P == b ? kOwned : 0));
        }
        poff.push_back((int32_t)pelem.size());
        for (int64_t i = n0; i < n1; ++i)
            for (int32_t t = noff[i]; t < noff[i + 1]; ++t)
                pslots[(size_t)i * W + (t - noff[i])] = (uint16_t)(nv * slot_of[nel[t] / nv] + nel[t] % nv);
        // the ring: neighbours outside the patch (stamp marks the patch's own
        // elements with b; the ring's with -2 - b)
        ring.clear();
        for (const int32_t e : els)
            for (int k = 0; k < nv; ++k) {
                const int32_t nb = m.nbr[st * (int64_t)e + k];
                if (nb >= 0 && stamp[nb] != (int32_t)b && stamp[nb] != -2 - (int32_t)b) {
                    stamp[nb] = -2 - (int32_t)b;
                    ring.push_back(nb);
                }
            }
        std::sort(ring.begin(), ring.end());
        rmax = std::max<int32_t>(rmax, (int32_t)ring.size());
        for (size_t q = 0; q < ring.size(); ++q) {
            slot_of[ring[q]] = (int32_t)(els.size() + q);
            pring.push_back(ring[q]);
        }
        roff.push_back((int32_t)pring.size());
        const bool fits = els.size() + ring.size() < kNoSlot;
        for (const int32_t e : els) {
            uint2 r = make_uint2(0, 0);
            const uint32_t locs = (uint32_t)m.nbr[st * (int64_t)e + nv];
            for (int k = 0; k < nv; ++k) {
                const int32_t nb = m.nbr[st * (int64_t)e + k];
                const uint32_t sl = (nb >= 0 && fits) ? (uint32_t)slot_of[nb] : kNoSlot;
                if (k < 3)
                    r.x |= sl << (10 * k);
                else
                    r.y |= sl;
                if (nb >= 0 && e < nb) r.y |= 1u << (10 + k);
                r.y |= ((locs >> (2 * k)) & 3u) << (16 + 2 * k);
            }
            if (nv == 3) r.y |= kNoSlot;
            pnbr.push_back(r);
        }
        if (nv != 3) continue;
        // the patch's nodes: its own (local b P ..), then the halo
        halo.clear();
        for (int64_t i = n0; i < n1; ++i) {
            nstamp[i] = (int32_t)b;
            nloc[i] = (int32_t)(i - n0);
        }
        auto take = [&](int32_t e) {
            for (int n = 0; n < 3; ++n) {
                const int32_t g = m.conn[3 * (int64_t)e + n];
                if (nstamp[g] != (int32_t)b) {
                    nstamp[g] = (int32_t)b;
                    halo.push_back(g);
                }
            }
        };
        for (const int32_t e : els) take(e);
        for (const int32_t e : ring) take(e);
        std::sort(halo.begin(), halo.end());
        for (size_t q = 0; q < halo.size(); ++q) {
            nloc[halo[q]] = (int32_t)(n1 - n0 + q);
            phalo.push_back(halo[q]);
        }
        hoff.push_back((int32_t)phalo.size());
        lmax = std::max<int32_t>(lmax, (int32_t)(n1 - n0 + halo.size()));
        auto lconn = [&](int32_t e) {
            const int32_t *c = &m.conn[3 * (int64_t)e];
            return make_uint2((uint32_t)nloc[c[0]] | ((uint32_t)nloc[c[1]] << 16), (uint32_t)nloc[c[2]]);
        };
        for (const int32_t e : els) plconn.push_back(lconn(e));
        for (const int32_t e : ring) prlconn.push_back(lconn(e));
    }
    dfree(m.dpatch_off);
    dfree(m.dpatch_elem);
    dfree(m.dpatch_slots);
    dfree(m.dpatch_ring_off);
    dfree(m.dpatch_ring);
    dfree(m.dpatch_nbr);
    int rc;
    if ((rc = upload<int32_t>(h, m.dpatch_off, poff.data(), poff.size()))) return rc;
    if ((rc = upload<int32_t>(h, m.dpatch_elem, pelem.data(), pelem.size()))) return rc;
    if ((rc = upload<uint16_t>(h, m.dpatch_slots, pslots.data(), pslots.size()))) return rc;
    if ((rc = upload<int32_t>(h, m.dpatch_ring_off, roff.data(), roff.size()))) return rc;
    if (!pring.empty() && (rc = upload<int32_t>(h, m.dpatch_ring, pring.data(), pring.size()))) return rc;
    if ((rc = upload<uint2>(h, m.dpatch_nbr, pnbr.data(), pnbr.size()))) return rc;
    dfree(m.dpatch_halo_off);
    dfree(m.dpatch_halo);
    dfree(m.dpatch_lconn);
    dfree(m.dpatch_ring_lconn);
    if (nv == 3) {
        if ((rc = upload<int32_t>(h, m.dpatch_halo_off, hoff.data(), hoff.size()))) return rc;
        if (!phalo.empty() && (rc = upload<int32_t>(h, m.dpatch_halo, phalo.data(), phalo.size()))) return rc;
        if ((rc = upload<uint2>(h, m.dpatch_lconn, plconn.data(), plconn.size()))) return rc;
        if (!prlconn.empty() && (rc = upload<uint2>(h, m.dpatch_ring_lconn, prlconn.data(), prlconn.size())))
            return rc;
    }
    TRY(h, hipStreamSynchronize(h.stream));
    // the 256-slot kernel shares strains through LDS and holds 256 ring
    // triangles or 128 ring quadrilaterals (four edge strains each); with a
    // larger ring the patches take the 512-slot kernel, which recomputes
    // the neighbours' strains and reads no ring
    if (emax <= 256 && (rmax > (nv == 3 ? 256 : 128) || lmax > kPatchLocalNodes)) emax = 257;
    *emax_out = emax;
    if (rmax_out) *rmax_out = rmax;
    return MCT_OK;
}

// Patch size of the fused step: the largest patch (64 to kPatchMaxNodes
// nodes) whose patches all hold at most 256 elements and whose rings fit
// the 256-slot kernel (build_patches).  Such patches take that kernel, which
// shares strains through LDS at the smallest LDS and register footprint,
// and compute their elements in one pass of the workgroup; among them the
// largest leave the fewest border elements computed twice and the fewest
// partly idle wavefronts.  Found from kPatchMaxNodes down, each try scaled by
// 256 over the element count of the fullest patch (or the ring limit over
// the largest ring), then shrunk to even out the compute units' shares
// (below); the environment variable
// MCT_PATCH_NODES sets the size instead (a testing and tuning knob).  Leaves
// the tables of the chosen size built; emax 0 when they do not fit.
int sized_patches(Model &m, Host h, int *P_out, int32_t *emax) {
    int64_t P = kPatchMaxNodes;
    if (const char *e = std::getenv("MCT_PATCH_NODES"); e && *e) {
        P = std::min<int64_t>(std::max<long>(std::strtol(e, nullptr, 10), 1), kPatchMaxNodes);
        *P_out = (int)P;
        return build_patches(m, h, (int)P, emax);
    }
    const int32_t rcap = m.nv == 3 ? 256 : 128;  // ring elements the 256-slot kernel holds
    for (;;) {
        int32_t rmax = 0;
        int rc = build_patches(m, h, (int)P, emax, &rmax);
        if (rc) return rc;
        if (*emax <= 256 || P == 64) break;  // fits (or, emax 0, the tables never do)
        const int64_t Pn = (*emax == 257 && rmax > rcap) ? P * rcap / rmax : P * 256 / *emax;
        P = std::max<int64_t>(64, std::min<int64_t>(P - 1, Pn));
    }
    // Then as many patches as fill the next whole number of patches per
    // compute unit: the step lasts as long as the busiest unit's patches, so
    // smaller patches that even the units out cost nothing extra.
    int dev = 0, ncu = 0;
    if (*emax > 0 && *emax <= 256 && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) {
        const int64_t nn = m.nn, per_cu = ((nn + P - 1) / P + ncu - 1) / ncu;
        const int64_t Pe = std::max<int64_t>(64, (nn + per_cu * ncu - 1) / (per_cu * ncu));
        if (Pe < P) {
            int32_t e2 = 0;
            int rc = build_patches(m, h, (int)Pe, &e2);
            if (rc) return rc;
            if (e2 > 0 && e2 <= 256) {
                *emax = e2;
                P = Pe;
            } else if ((rc = build_patches(m, h, (int)P, emax))) {  // keep the larger size
                return rc;
            }
        }
    }
    *P_out = (int)P;
    return MCT_OK;
}

// Step kernels from the requested choice: 1 split kernels; 2, 3, 4 the fused
// kernel on patches of 64, 128, 256 nodes; 5 and 0 (automatic) the fused
// kernel on patches of the size sized_patches finds, and 0 (automatic) the
// same.  A fused choice whose tables do not fit runs the split kernels.
int choose_kernels(Model &m, Host h) {
    Params &p = m.prm;
    p.patch_emax = 0;
    p.patch_nodes = 0;
    p.fold = 0;
    int P = 0;
    if (m.kernels >= 2 && m.kernels <= 4)
        P = 64 << (m.kernels - 2);
    else if (m.kernels == 0 || m.kernels == 5)
        P = -1;
    if (P == 0 || !m.dnlist) return MCT_OK;
    int32_t emax = 0;
    int rc = P > 0 ? build_patches(m, h, P, &emax) : sized_patches(m, h, &P, &emax);
    if (rc) return rc;
    if (emax == 0) return MCT_OK;
    p.patch_emax = emax;
    p.patch_nodes = P;
    p.patch_off = m.dpatch_off;
    p.patch_elem = m.dpatch_elem;
    p.patch_slots = m.dpatch_slots;
    p.patch_ring_off = m.dpatch_ring_off;
    p.patch_ring = m.dpatch_ring;
    p.patch_nbr = m.dpatch_nbr;
    p.patch_halo_off = m.dpatch_halo_off;
    p.patch_halo = m.dpatch_halo;
    p.patch_lconn = m.dpatch_lconn;
    p.patch_ring_lconn = m.dpatch_ring_lconn;
    // the global multi-tip pick folds into the next fused step
    if (!m.sct && !(m.front_rho > 0)) {
        if (!m.dfold_n) {
            TRY(h, hipMalloc((void **)&m.dfold_n, 3 * sizeof(int32_t)));
            TRY(h, hipMemsetAsync(m.dfold_n, 0, 3 * sizeof(int32_t), h.stream));
            // three sets of at most one candidate per element edge
            TRY(h, hipMalloc((void **)&m.dfold_cand, sizeof(Cand) * 3 * m.nv * (size_t)std::max<int64_t>(m.ne, 1)));
            TRY(h, hipStreamSynchronize(h.stream));
        }
        p.fold = 1;
        p.fold_n = m.dfold_n;
        p.fold_cand = m.dfold_cand;
    }
    return MCT_OK;
}

}  // namespace

void release(Model &m) {
    if (m.graph) (void)hipGraphExecDestroy(m.graph);
    m.graph = nullptr;
    dfree(m.dconn);
    dfree(m.dnbr);
    dfree(m.dopp);
    dfree(m.dq_nbr);
    dfree(m.dq_loc);
    dfree(m.dq_oa);
    dfree(m.dq_ob);
    dfree(m.dnlist);
    dfree(m.dminv);
    dfree(m.dgc);
    dfree(m.dcurve);
    dfree(m.dmass);
    dfree(m.dxy);
    dfree(m.du[0]);
    dfree(m.du[1]);
    dfree(m.dpatch_off);
    dfree(m.dpatch_elem);
    dfree(m.dpatch_slots);
    dfree(m.dpatch_ring_off);
    dfree(m.dpatch_ring);
    dfree(m.dpatch_nbr);
    dfree(m.dpatch_halo_off);
    dfree(m.dpatch_halo);
    dfree(m.dpatch_lconn);
    dfree(m.dpatch_ring_lconn);
    dfree(m.dfold_n);
    dfree(m.dfold_cand);
    dfree(m.dv);
    dfree(m.dfext);
    dfree(m.dv0);
    dfree(m.dfe);
    dfree(m.dflag);
    dfree(m.dsplit);
    dfree(m.dcsr_off);
    dfree(m.dcsr_ent);
    dfree(m.dedge_elem);
    dfree(m.dwatch);
    dfree(m.dcand);
    dfree(m.dfmid);
    dfree(m.dflen);
    dfree(m.dforder);
    dfree(m.dfbucket);
    dfree(m.dfsorted);
    dfree(m.dfplist);
    dfree(m.dfgrid);
    dfree(m.dlog);
    dfree(m.dctl);
    dfree(m.ev.sig_ek);
    dfree(m.ev.es_ek);
    dfree(m.ev.pe);
    dfree(m.ev.principal);
    dfree(m.ev.fint);
    dfree(m.ev.acc);
    dfree(m.ev.node_e);
    dfree(m.dpart);
    dfree(m.dsums);
    dfree(m.dpow);
    dfree(m.dtipflag);
    m.finalized = false;
}

int set_mesh(Model &m, Host h, int nv, int64_t nn, const double *X, const double *Y, int64_t ne,
             const int32_t *conn) {
    const char *what = nv == 4 ? "quadrilateral" : "triangle";
    if (nv != 3 && nv != 4) return fail(h, MCT_EINVAL, "elements have 3 or 4 nodes");
    if (nn < nv || ne < 1 || !X || !Y || !conn)
        return fail(h, MCT_EINVAL, "mesh needs >= %d nodes, >= 1 %s", nv, what);
    // element * 4 + edge keys, force slots n * ne + e and list entries
    // nv * e + n stay in int32
    if (ne >= ((int64_t)1 << 29) || nn > ((int64_t)1 << 30)) return fail(h, MCT_EINVAL, "mesh too large");
    release(m);
    Model fresh;
    fresh.nv = nv;
    fresh.nn = nn;
    fresh.ne = ne;
    fresh.X.assign(X, X + nn);
    fresh.Y.assign(Y, Y + nn);
    fresh.conn.assign(conn, conn + nv * ne);
    std::vector<uint8_t> used(nn, 0);
    fresh.area.resize(ne);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *c = &conn[nv * e];
        for (int n = 0; n < nv; ++n) {
            if (c[n] < 0 || c[n] >= nn) return fail(h, MCT_EINVAL, "%s %lld: node out of range", what, (long long)e);
            used[c[n]] = 1;
            for (int q = 0; q < n; ++q)
                if (c[q] == c[n]) return fail(h, MCT_EINVAL, "%s %lld repeats a node", what, (long long)e);
        }
        double A;
        if (nv == 3) {
            const double x0 = X[c[0]], x1 = X[c[1]], x2 = X[c[2]], y0 = Y[c[0]], y1 = Y[c[1]], y2 = Y[c[2]];
            A = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
        } else {
            // half the cross product of the diagonals; every corner must turn
            // left (convex, counter-clockwise), else the bilinear map folds
            A = 0.5 * ((X[c[2]] - X[c[0]]) * (Y[c[3]] - Y[c[1]]) - (X[c[3]] - X[c[1]]) * (Y[c[2]] - Y[c[0]]));
            for (int n = 0; n < 4; ++n) {
                const int32_t a = c[(n + 3) & 3], b = c[n], d = c[(n + 1) & 3];
                const double cr = (X[b] - X[a]) * (Y[d] - Y[b]) - (Y[b] - Y[a]) * (X[d] - X[b]);
                if (!(cr > 0.0))
                    return fail(h, MCT_EINVAL, "quadrilateral %lld is not convex and counter-clockwise", (long long)e);
            }
        }
        if (!(A > 0.0))
            return fail(h, MCT_EINVAL, "%s %lld has non-positive area (clockwise or degenerate)", what, (long long)e);
        fresh.area[e] = A;
    }
    for (int64_t i = 0; i < nn; ++i)
        if (!used[i]) return fail(h, MCT_EINVAL, "node %lld belongs to no element", (long long)i);
    // edges: (lower node, higher node, element, local edge), sorted
    struct Rec {
        int32_t lo, hi, e, k;
    };
    std::vector<Rec> r(nv * ne);
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < nv; ++k) {
            const int32_t a = conn[nv * e + k], b = conn[nv * e + (k + 1) % nv];
            r[nv * e + k] = {std::min(a, b), std::max(a, b), (int32_t)e, k};
        }
    std::sort(r.begin(), r.end(), [](const Rec &p, const Rec &q) {
        if (p.lo != q.lo) return p.lo < q.lo;
        if (p.hi != q.hi) return p.hi < q.hi;
        return p.e < q.e;
    });
    fresh.elem_edge.assign(nv * ne, -1);
    std::vector<int32_t> edge_loc;
    int64_t ns = 0;
    for (size_t i = 0; i < r.size(); ++i) {
        if (i > 0 && r[i].lo == r[i - 1].lo && r[i].hi == r[i - 1].hi) {
            const int64_t s = ns - 1;
            if (fresh.edge_elem[2 * s + 1] >= 0)
                return fail(h, MCT_EINVAL, "edge (%d, %d) belongs to more than two elements", r[i].lo, r[i].hi);
            const int32_t e0 = fresh.edge_elem[2 * s], k0 = edge_loc[2 * s];
            if (conn[nv * e0 + k0] == conn[nv * r[i].e + r[i].k])
                return fail(h, MCT_EINVAL, "elements %d and %d run edge (%d, %d) in the same direction", e0,
                            r[i].e, r[i].lo, r[i].hi);
            fresh.edge_elem[2 * s + 1] = r[i].e;
            edge_loc[2 * s + 1] = r[i].k;
        } else {
            fresh.edge_node.push_back(r[i].lo);
            fresh.edge_node.push_back(r[i].hi);
            fresh.edge_elem.push_back(r[i].e);
            fresh.edge_elem.push_back(-1);
            edge_loc.push_back(r[i].k);
            edge_loc.push_back(-1);
            ++ns;
        }
        fresh.elem_edge[nv * (int64_t)r[i].e + r[i].k] = (int32_t)(ns - 1);
    }
    fresh.ns = ns;
    fresh.nbr.assign((nv + 1) * ne, -1);
    for (int64_t e = 0; e < ne; ++e) {
        int32_t packed = 0;
        for (int k = 0; k < nv; ++k) {
            const int64_t s = fresh.elem_edge[nv * e + k];
            const int side = fresh.edge_elem[2 * s] == e ? 1 : 0;
            fresh.nbr[(nv + 1) * e + k] = fresh.edge_elem[2 * s + side];
            const int32_t loc = fresh.nbr[(nv + 1) * e + k] >= 0 ? edge_loc[2 * s + side] : 0;
            packed |= loc << (2 * k);
        }
        fresh.nbr[(nv + 1) * e + nv] = packed;
    }
    m = std::move(fresh);
    return MCT_OK;
}

int set_material(Model &m, Host h, double E, double nu, double rho, const double *Gc, double Gc_uniform,
                 double gamma) {
    if (need_mesh(m)) return fail(h, MCT_ESTATE, "set the mesh first");
    if (!(E > 0) || !(nu > -1.0 && nu < 0.5) || !(rho > 0) || !(gamma > 0))
        return fail(h, MCT_EINVAL, "material out of range");
    if (Gc) {
        for (int64_t e = 0; e < m.ne; ++e)
            if (!(Gc[e] > 0)) return fail(h, MCT_EINVAL, "Gc[%lld] <= 0", (long long)e);
        m.gc.assign(Gc, Gc + m.ne);
    } else {
        if (!(Gc_uniform > 0)) return fail(h, MCT_EINVAL, "Gc_uniform <= 0");
        m.gc.clear();
    }
    m.E = E;
    m.nu = nu;
    m.rho = rho;
    m.gamma = gamma;
    m.gc_uniform = Gc_uniform;
    m.have_material = true;
    invalidate(m);
    return MCT_OK;
}

int set_traction(Model &m, Host h, int64_t n, const int32_t *edge_nodes, const double *t) {
    if (need_mesh(m)) return fail(h, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!edge_nodes || !t))) return fail(h, MCT_EINVAL, "bad traction arrays");
    std::vector<std::pair<int64_t, int64_t>> v;  // (edge id, input index)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a = edge_nodes[2 * i], b = edge_nodes[2 * i + 1];
        if (a < 0 || b < 0 || a >= m.nn || b >= m.nn)
            return fail(h, MCT_EINVAL, "traction edge %lld: node out of range", (long long)i);
        const int64_t s = find_edge(m, a, b);
        if (s < 0 || m.edge_elem[2 * s + 1] >= 0)
            return fail(h, MCT_EINVAL, "traction edge %lld is not a boundary edge", (long long)i);
        v.push_back({s, i});
    }
    std::sort(v.begin(), v.end());
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i].first == v[i - 1].first) return fail(h, MCT_EINVAL, "repeated traction edge");
    m.trac_edge.clear();
    m.trac.clear();
    for (const auto &q : v) {
        m.trac_edge.push_back(q.first);
        m.trac.push_back(t[2 * q.second]);
        m.trac.push_back(t[2 * q.second + 1]);
    }
    invalidate(m);
    return MCT_OK;
}

int set_velocity_bc(Model &m, Host h, int64_t n, const int32_t *node, const uint8_t *mask, const double *v0,
                    double t_ramp) {
    if (need_mesh(m)) return fail(h, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!node || !mask || !v0)) || !(t_ramp >= 0)) return fail(h, MCT_EINVAL, "bad velocity arrays");
    for (int64_t i = 0; i < n; ++i)
        if (node[i] < 0 || node[i] >= m.nn || (mask[i] & ~3u))
            return fail(h, MCT_EINVAL, "velocity bc %lld out of range", (long long)i);
    m.vbc_node.assign(node, node + n);
    m.vbc_mask.assign(mask, mask + n);
    m.vbc_v0.assign(v0, v0 + 2 * n);
    m.t_ramp = t_ramp;
    invalidate(m);
    return MCT_OK;
}

int set_notch(Model &m, Host h, int64_t n, const int32_t *elem, const uint8_t *entry, const uint8_t *exit) {
    if (need_mesh(m)) return fail(h, MCT_ESTATE, "set the mesh first");
    if (n < 0 || (n && (!elem || !entry || !exit))) return fail(h, MCT_EINVAL, "bad notch arrays");
    std::vector<int32_t> el;
    std::vector<uint8_t> code;
    for (int64_t i = 0; i < n; ++i) {
        if (elem[i] < 0 || elem[i] >= m.ne || entry[i] >= m.nv || exit[i] >= m.nv || entry[i] == exit[i])
            return fail(h, MCT_EINVAL, "notch element %lld invalid", (long long)i);
        el.push_back(elem[i]);
        code.push_back((uint8_t)(kSplitFlag | (entry[i] << 2) | exit[i]));
    }
    m.notch_elem.swap(el);
    m.notch_code.swap(code);
    invalidate(m);
    return MCT_OK;
}

int set_load_curve(Model &m, Host h, int64_t n, const double *t, const double *phi) {
    if (n != 0 && (n < 2 || n > (1 << 20) || !t || !phi)) return fail(h, MCT_EINVAL, "load curve needs 2..2^20 points");
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(t[i]) || !std::isfinite(phi[i])) return fail(h, MCT_EINVAL, "non-finite load curve");
        if (i > 0 && !(t[i] > t[i - 1])) return fail(h, MCT_EINVAL, "load curve times must increase");
    }
    m.curve_t.assign(t, t + n);
    m.curve_phi.assign(phi, phi + n);
    invalidate(m);
    return MCT_OK;
}

int set_tracking(Model &m, Host h, int mode, int32_t elem, int edge) {
    if (need_mesh(m)) return fail(h, MCT_ESTATE, "set the mesh first");
    if (mode != MCT_TRACK_MCT && mode != MCT_TRACK_SCT) return fail(h, MCT_EINVAL, "unknown tracking mode %d", mode);
    if (mode == MCT_TRACK_SCT && elem >= 0 && (elem >= m.ne || edge < 0 || edge >= m.nv))
        return fail(h, MCT_EINVAL, "start tip out of range");
    m.sct = mode == MCT_TRACK_SCT;
    m.sct_elem = elem;
    m.sct_edge = edge;
    invalidate(m);
    return MCT_OK;
}

int set_front_pick(Model &m, Host h, double rho) {
    if (need_mesh(m)) return fail(h, MCT_ESTATE, "set the mesh first");
    if (!(rho >= 0)) return fail(h, MCT_EINVAL, "front radius must be >= 0 (0: the global pick)");
    m.front_rho = rho;
    invalidate(m);
    return MCT_OK;
}

int set_time(Model &m, Host h, double dt, double cfl) {
    if (!(dt > 0) && !(cfl > 0)) return fail(h, MCT_EINVAL, "need dt > 0 or cfl_fraction > 0");
    m.dt_in = dt;
    m.cfl = cfl;
    invalidate(m);
    return MCT_OK;
}

int finalize(Model &m, Host h) {
    if (need_mesh(m) || !m.have_material) return fail(h, MCT_ESTATE, "mesh and material are required");
    const int64_t nn = m.nn, ne = m.ne, ns = m.ns;
    const int nv = m.nv;
    release(m);  // device state only; the host tables stay
    // lumped mass rho A / nv, element-id order per node
    m.mass.assign(nn, 0.0);
    for (int64_t e = 0; e < ne; ++e) {
        const double me = m.rho * m.area[e] / (double)nv;
        for (int n = 0; n < nv; ++n) m.mass[m.conn[nv * e + n]] += me;
    }
    std::vector<double> minv(nn);
    for (int64_t i = 0; i < nn; ++i) minv[i] = 1.0 / m.mass[i];
    // equivalent nodal forces of the tractions, edge-id order
    std::vector<double> fext(2 * nn, 0.0);
    std::vector<uint8_t> flag(nn, 0);
    for (size_t q = 0; q < m.trac_edge.size(); ++q) {
        const int64_t s = m.trac_edge[q];
        const int32_t a = m.edge_node[2 * s], b = m.edge_node[2 * s + 1];
        const double dx = m.X[b] - m.X[a], dy = m.Y[b] - m.Y[a];
        const double L = std::sqrt(dx * dx + dy * dy);
        const double fx = m.trac[2 * q] * L * 0.5, fy = m.trac[2 * q + 1] * L * 0.5;
        fext[2 * a] += fx;
        fext[2 * a + 1] += fy;
        fext[2 * b] += fx;
        fext[2 * b + 1] += fy;
        flag[a] |= kLoaded;
        flag[b] |= kLoaded;
    }
    std::vector<double> v0(2 * nn, 0.0);
    for (size_t q = 0; q < m.vbc_node.size(); ++q) {
        const int32_t nd = m.vbc_node[q];
        flag[nd] = (uint8_t)((flag[nd] & kLoaded) | m.vbc_mask[q]);
        v0[2 * nd] = m.vbc_v0[2 * q];
        v0[2 * nd + 1] = m.vbc_v0[2 * q + 1];
    }
    // time step: fraction of (shortest edge) / dilatational wave speed
    if (m.dt_in > 0) {
        m.dt = m.dt_in;
    } else {
        double hmin = INFINITY;
        for (int64_t s = 0; s < ns; ++s) {
            const int32_t a = m.edge_node[2 * s], b = m.edge_node[2 * s + 1];
            const double dx = m.X[b] - m.X[a], dy = m.Y[b] - m.Y[a];
            hmin = std::min(hmin, std::sqrt(dx * dx + dy * dy));
        }
        const double cd = std::sqrt(m.E / (m.rho * (1.0 - m.nu * m.nu)));
        m.dt = m.cfl * hmin / cd;
    }
    // greedy colouring and the per-node gather lists in colour order
    std::vector<int32_t> noff(nn + 1, 0), nel(nv * ne);
    for (int64_t e = 0; e < ne; ++e)
        for (int n = 0; n < nv; ++n) noff[m.conn[nv * e + n] + 1]++;
    for (int64_t i = 0; i < nn; ++i) noff[i + 1] += noff[i];
    {
        std::vector<int32_t> fill(nn, 0);
        for (int64_t e = 0; e < ne; ++e)
            for (int n = 0; n < nv; ++n) {
                const int32_t g = m.conn[nv * e + n];
                nel[noff[g] + fill[g]++] = (int32_t)(nv * e + n);
            }
    }
    std::vector<int32_t> color(ne, 0);
    for (int64_t e = 0; e < ne; ++e) {
        uint64_t used = 0;
        for (int n = 0; n < nv; ++n) {
            const int32_t g = m.conn[nv * e + n];
            for (int32_t t = noff[g]; t < noff[g + 1]; ++t) {
                const int32_t o = nel[t] / nv;
                if (o < e) used |= 1ull << color[o];
            }
        }
        int c = 0;
        while (c < 64 && (used >> c) & 1ull) ++c;
        if (c == 64) return fail(h, MCT_EINVAL, "element %lld needs more than 64 colours", (long long)e);
        color[e] = c;
    }
    for (int64_t i = 0; i < nn; ++i)
        std::sort(nel.begin() + noff[i], nel.begin() + noff[i + 1],
                  [&](int32_t p, int32_t q) { return color[p / nv] < color[q / nv]; });
    m.gnoff = noff;
    m.gnel = nel;
    // gather entries name force slots n * ne + e (slot-major element forces)
    for (int32_t &v : nel) v = (v % nv) * (int32_t)ne + v / nv;
    // device arrays
    // per element: neighbours, and each neighbour's node off the shared edge
    // (the neighbour runs the edge backwards, so its local node loc + 2); a
    // triangle keeps the one off edge 0 in its node record's free fourth
    // slot (40 B of element records per triangle instead of 48)
    std::vector<int4> c4(ne), n4(ne), qa(nv == 4 ? ne : 0), qb(nv == 4 ? ne : 0);
    std::vector<int2> o2v(nv == 3 ? ne : 0);
    std::vector<uint8_t> ql(nv == 4 ? ne : 0);
    const int st = nv + 1;
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *ce = &m.conn[nv * e];
        c4[e] = make_int4(ce[0], ce[1], ce[2], nv == 4 ? ce[3] : 0);
        int32_t o[4] = {-1, -1, -1, -1}, o2[4] = {-1, -1, -1, -1};
        for (int k = 0; k < nv; ++k) {
            const int32_t nb = m.nbr[st * e + k];
            if (nb < 0) continue;
            const int loc = (m.nbr[st * e + nv] >> (2 * k)) & 3;
            const int32_t *cn = &m.conn[nv * (int64_t)nb];
            if (cn[loc] != ce[(k + 1) % nv] || cn[(loc + 1) % nv] != ce[k])
                return fail(h, MCT_EINVAL, "inconsistent neighbour table at element %lld", (long long)e);
            o[k] = cn[(loc + 2) % nv];
            if (nv == 4) o2[k] = cn[(loc + 3) % nv];
        }
        if (nv == 3) {
            n4[e] = make_int4(m.nbr[st * e], m.nbr[st * e + 1], m.nbr[st * e + 2], m.nbr[st * e + 3]);
            c4[e].w = o[0];
            o2v[e] = make_int2(o[1], o[2]);
        } else {
            n4[e] = make_int4(m.nbr[st * e], m.nbr[st * e + 1], m.nbr[st * e + 2], m.nbr[st * e + 3]);
            ql[e] = (uint8_t)m.nbr[st * e + 4];
            qa[e] = make_int4(o[0], o[1], o[2], o[3]);
            qb[e] = make_int4(o2[0], o2[1], o2[2], o2[3]);
        }
    }
    // padded gather lists (node-major, W slots) when every node touches <= 16 elements
    int32_t maxdeg = 0;
    for (int64_t i = 0; i < nn; ++i) maxdeg = std::max(maxdeg, noff[i + 1] - noff[i]);
    const int32_t W = (maxdeg + 3) / 4 * 4;
    std::vector<int32_t> nlist;
    if (W <= 16) {
        nlist.assign((size_t)W * nn, -1);
        for (int64_t i = 0; i < nn; ++i)
            for (int32_t t = noff[i]; t < noff[i + 1]; ++t) nlist[(size_t)i * W + (t - noff[i])] = nel[t];
    }
    std::vector<double> xy(2 * nn);
    for (int64_t i = 0; i < nn; ++i) {
        xy[2 * i] = m.X[i];
        xy[2 * i + 1] = m.Y[i];
    }
    std::vector<double> gc(ne);
    for (int64_t e = 0; e < ne; ++e) gc[e] = m.gc.empty() ? m.gc_uniform : m.gc[e];
    std::vector<uint8_t> split(ne, 0);
    for (size_t q = 0; q < m.notch_elem.size(); ++q) split[m.notch_elem[q]] = m.notch_code[q];
    int rc;
    if ((rc = upload<int4>(h, m.dconn, c4.data(), ne))) return rc;
    if (nv == 3) {
        if ((rc = upload<int4>(h, m.dnbr, n4.data(), ne))) return rc;
        if ((rc = upload<int2>(h, m.dopp, o2v.data(), ne))) return rc;
    } else {
        if ((rc = upload<int4>(h, m.dq_nbr, n4.data(), ne))) return rc;
        if ((rc = upload<uint8_t>(h, m.dq_loc, ql.data(), ne))) return rc;
        if ((rc = upload<int4>(h, m.dq_oa, qa.data(), ne))) return rc;
        if ((rc = upload<int4>(h, m.dq_ob, qb.data(), ne))) return rc;
    }
    if (!nlist.empty() && (rc = upload<int32_t>(h, m.dnlist, nlist.data(), nlist.size()))) return rc;
    if ((rc = upload<double>(h, m.dminv, minv.data(), nn))) return rc;
    if ((rc = upload<double>(h, m.dmass, m.mass.data(), nn))) return rc;
    if ((rc = upload<double>(h, m.dgc, gc.data(), ne))) return rc;
    if ((rc = upload<double2>(h, m.dxy, xy.data(), nn))) return rc;
    if ((rc = upload<double2>(h, m.dfext, fext.data(), nn))) return rc;
    if ((rc = upload<double2>(h, m.dv0, v0.data(), nn))) return rc;
    if ((rc = upload<uint8_t>(h, m.dflag, flag.data(), nn))) return rc;
    if ((rc = upload<uint8_t>(h, m.dsplit, split.data(), ne))) return rc;
    if ((rc = upload<int32_t>(h, m.dcsr_off, noff.data(), nn + 1))) return rc;
    if ((rc = upload<int32_t>(h, m.dcsr_ent, nel.data(), nv * ne))) return rc;
    if ((rc = upload<int32_t>(h, m.dedge_elem, m.edge_elem.data(), 2 * ns))) return rc;
    const size_t ncv = m.curve_t.size();
    if (ncv) {
        std::vector<double> cv(m.curve_t);
        cv.insert(cv.end(), m.curve_phi.begin(), m.curve_phi.end());
        if ((rc = upload<double>(h, m.dcurve, cv.data(), cv.size()))) return rc;
    }
    TRY(h, hipMalloc((void **)&m.du[0], sizeof(double2) * nn));
    TRY(h, hipMalloc((void **)&m.du[1], sizeof(double2) * nn));
    TRY(h, hipMalloc((void **)&m.dv, sizeof(double2) * nn));
    TRY(h, hipMemsetAsync(m.du[0], 0, sizeof(double2) * nn, h.stream));
    TRY(h, hipMemsetAsync(m.du[1], 0, sizeof(double2) * nn, h.stream));
    TRY(h, hipMemsetAsync(m.dv, 0, sizeof(double2) * nn, h.stream));
    TRY(h, hipMalloc((void **)&m.dfe, sizeof(double2) * nv * ne));
    TRY(h, hipMalloc((void **)&m.dcand, sizeof(Cand) * nv * ne));
    if (m.front_rho > 0) {
        if (m.sct) return fail(h, MCT_EINVAL, "per-front pick and single-tip tracking exclude each other");
        TRY(h, hipMalloc((void **)&m.dfmid, sizeof(double2) * nv * ne));
        TRY(h, hipMalloc((void **)&m.dflen, sizeof(double) * nv * ne));
        TRY(h, hipMalloc((void **)&m.dforder, sizeof(int32_t) * nv * ne));
        TRY(h, hipMalloc((void **)&m.dfbucket, sizeof(int32_t) * nv * ne));
        TRY(h, hipMalloc((void **)&m.dfsorted, sizeof(int32_t) * nv * ne));
        TRY(h, hipMalloc((void **)&m.dfplist, sizeof(int32_t) * nv * ne));
        if (ne >= mct::kFrontGridMinElements && std::isfinite(m.front_rho)) {
            // the pick over the whole GPU: its two bucket tables
            TRY(h, hipMalloc((void **)&m.dfgrid, sizeof(int32_t) * 2 * mct::kFrontGridTable));
            TRY(h, mct::front_grid_reset(m.dfgrid, h.stream));
        }
    }
    TRY(h, hipMalloc((void **)&m.dlog, sizeof(LogRec) * ne));
    TRY(h, hipMalloc((void **)&m.dctl, sizeof(Ctl)));
    // start tip of single-tip tracking: given, or the one path end of the
    // pre-notch (an entry or exit edge of a notch element whose neighbour
    // across it is intact)
    int32_t tip = -1;
    if (m.sct) {
        if (m.sct_elem >= 0) {
            tip = m.sct_elem * 4 + m.sct_edge;
        } else {
            int count = 0;
            for (int64_t e = 0; e < ne; ++e) {
                if (!split[e]) continue;
                const int ks[2] = {(split[e] >> 2) & 3, split[e] & 3};
                for (int k : ks) {
                    const int32_t nb = m.nbr[st * e + k];
                    if (nb < 0 || split[nb]) continue;
                    tip = nb * 4 + ((m.nbr[st * e + nv] >> (2 * k)) & 3);
                    ++count;
                }
            }
            if (count != 1)
                return fail(h, MCT_EINVAL, "single-tip tracking: the pre-notch has %d path ends, need one start tip",
                            count);
        }
    }
    Ctl c0{};
    c0.tip = tip;
    TRY(h, hipMemcpyAsync(m.dctl, &c0, sizeof c0, hipMemcpyHostToDevice, h.stream));
    Params &p = m.prm;
    p = Params{};
    p.nn = (int32_t)nn;
    p.ne = (int32_t)ne;
    p.log_cap = (int32_t)ne;
    p.sct = m.sct;
    p.ncurve = (int32_t)ncv;
    p.nv = nv;
    p.conn = m.dconn;
    p.nbr = m.dnbr;
    p.opp = m.dopp;
    p.q_nbr = m.dq_nbr;
    p.q_loc = m.dq_loc;
    p.q_oa = m.dq_oa;
    p.q_ob = m.dq_ob;
    p.nlist = m.dnlist;
    p.nlist_w = m.dnlist ? W : 0;
    // the fused step's slot lists have the padded lists' width
    if ((rc = choose_kernels(m, h))) return rc;
    p.xy = m.dxy;
    p.u0 = m.du[0];
    p.u1 = m.du[1];
    p.v = m.dv;
    p.minv = m.dminv;
    p.fext = m.dfext;
    p.v0 = m.dv0;
    p.nflag = m.dflag;
    p.split = m.dsplit;
    p.gc = m.dgc;
    p.fe = m.dfe;
    p.csr_off = m.dcsr_off;
    p.csr_ent = m.dcsr_ent;
    p.cand = m.dcand;
    p.log = m.dlog;
    p.ctl = m.dctl;
    p.curve_t = ncv ? m.dcurve : nullptr;
    p.curve_phi = ncv ? m.dcurve + ncv : nullptr;
    p.D11 = m.E / (1.0 - m.nu * m.nu);
    p.D12 = m.nu * p.D11;
    p.D33 = m.E / (2.0 * (1.0 + m.nu));
    p.E = m.E;
    p.dt = m.dt;
    p.t_ramp = m.t_ramp;
    p.gamma = m.gamma;
    p.front_r2 = m.front_rho > 0 ? m.front_rho * m.front_rho : 0.0;
    p.fmid = m.dfmid;
    p.flen = m.dflen;
    p.forder = m.dforder;
    p.fbucket = m.dfbucket;
    p.fsorted = m.dfsorted;
    p.fplist = m.dfplist;
    p.fgrid = m.dfgrid;
    {
        // hash cell: at least rho and the largest distance between two
        // nodes of an element (two tip points of one element are closer)
        double dmax = 0.0;
        for (int64_t e = 0; e < ne; ++e)
            for (int a = 0; a < nv; ++a)
                for (int b = a + 1; b < nv; ++b) {
                    const int32_t i = m.conn[nv * e + a], j = m.conn[nv * e + b];
                    dmax = std::max(dmax, std::hypot(m.X[j] - m.X[i], m.Y[j] - m.Y[i]));
                }
        p.fcell = std::max(m.front_rho, dmax) * (1.0 + 1e-9);
    }
    TRY(h, hipStreamSynchronize(h.stream));
    if ((rc = stability_limit(m, h))) return rc;
    if (m.dt > m.dt_limit)
        return fail(h, MCT_ESTABILITY, "dt = %g exceeds the stability limit 2/omega_max = %g", m.dt, m.dt_limit);
    m.steps_enqueued = 0;
    m.finalized = true;
    return MCT_OK;
}

int step(Model &m, Host h, int64_t n) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    if (n < 0) return fail(h, MCT_EINVAL, "negative step count");
    int64_t left = n;
    if (m.use_graph) {
        while (left >= kGraphSteps) {
            if (!m.graph) {
                hipStream_t cs;
                TRY(h, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
                for (int j = 0; j < kGraphSteps && e == hipSuccess; ++j) e = launch_step(m.prm, j, cs);
                if (e == hipSuccess) e = launch_commit(m.prm, kGraphSteps, cs);
                hipError_t e2 = hipStreamEndCapture(cs, &g);
                if (e == hipSuccess) e = e2;
                if (e == hipSuccess) e = hipGraphInstantiate(&m.graph, g, nullptr, nullptr, 0);
                if (g) (void)hipGraphDestroy(g);
                (void)hipStreamDestroy(cs);
                if (e != hipSuccess) return fail(h, MCT_EDEVICE, "graph capture: %s", hipGetErrorString(e));
            }
            TRY(h, hipGraphLaunch(m.graph, h.stream));
            left -= kGraphSteps;
            m.steps_enqueued += kGraphSteps;
        }
    }
    while (left > 0) {
        const int seg = (int)std::min<int64_t>(left, 1 << 20);
        for (int j = 0; j < seg; ++j) TRY(h, launch_step(m.prm, j, h.stream));
        TRY(h, launch_commit(m.prm, seg, h.stream));
        left -= seg;
        m.steps_enqueued += seg;
    }
    return MCT_OK;
}

int set_kernels(Model &m, Host h, int kind) {
    if (kind < 0 || kind > 5) return fail(h, MCT_EINVAL, "step kernel choice %d out of range (0..5)", kind);
    m.kernels = kind;
    if (!m.finalized) return MCT_OK;
    if (m.graph) {
        TRY(h, hipStreamSynchronize(h.stream));
        (void)hipGraphExecDestroy(m.graph);
        m.graph = nullptr;
    }
    return choose_kernels(m, h);
}

int sync(Model &m, Host h) {
    if (!m.finalized) {
        TRY(h, hipStreamSynchronize(h.stream));
        return MCT_OK;
    }
    int rc = ensure_eval(m, h);
    if (rc) return rc;
    int32_t flag = 0;
    TRY(h, hipMemsetAsync(m.dwatch, 0, sizeof(int32_t), h.stream));
    const double *u = reinterpret_cast<const double *>(m.du[m.steps_enqueued & 1]),
                 *v = reinterpret_cast<const double *>(m.dv);
    TRY(h, launch_check_finite(u, v, u, v, 2 * m.nn, m.dwatch, h.stream));
    TRY(h, hipMemcpyAsync(&flag, m.dwatch, sizeof flag, hipMemcpyDeviceToHost, h.stream));
    TRY(h, hipStreamSynchronize(h.stream));
    if (flag)
        return fail(h, MCT_ENUMERIC, "non-finite displacement or velocity after step %lld", (long long)m.steps_enqueued);
    return MCT_OK;
}

int get_info(Model &m, Host h, mct_info *out) {
    std::memset(out, 0, sizeof *out);
    out->n_nodes = m.nn;
    out->n_elems = m.ne;
    out->n_edges = m.ns;
    out->dt = m.dt;
    out->dt_limit = m.dt_limit;
    out->precision = 64;
    out->tip = -1;
    if (!m.finalized) return MCT_OK;
    Ctl c;
    int rc = read_ctl(m, h, &c);
    if (rc) return rc;
    out->step = c.base;
    out->n_splits = c.nsplit;
    out->dissipated = c.Ud;
    out->log_overflow = c.overflow;
    out->tip = m.sct ? c.tip : -1;
    return MCT_OK;
}

int get_crack_set(Model &m, Host h, int64_t cap, int32_t *step, int32_t *elem, uint8_t *entry, uint8_t *exit,
                  double *G, int64_t *count) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    Ctl c;
    int rc = read_ctl(m, h, &c);
    if (rc) return rc;
    const int64_t n = std::min<int64_t>(c.nsplit, m.prm.log_cap);
    *count = n;
    if (cap < n) return fail(h, MCT_ECAPACITY, "crack set holds %lld splits", (long long)n);
    std::vector<LogRec> lg(n);
    if (n) TRY(h, hipMemcpy(lg.data(), m.dlog, sizeof(LogRec) * n, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) {
        if (step) step[i] = lg[i].step;
        if (elem) elem[i] = lg[i].elem;
        if (entry) entry[i] = lg[i].entry;
        if (exit) exit[i] = lg[i].exit;
        if (G) G[i] = lg[i].G;
    }
    return MCT_OK;
}

int get_tips(Model &m, Host h, int64_t cap, int32_t *edge, double *xy, int64_t *count) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    int rc = ensure_eval(m, h);
    if (rc) return rc;
    TRY(h, launch_tip_flags(m.prm, m.dedge_elem, m.ns, m.dtipflag, h.stream));
    std::vector<uint8_t> fl(m.ns);
    TRY(h, hipMemcpyAsync(fl.data(), m.dtipflag, m.ns, hipMemcpyDeviceToHost, h.stream));
    TRY(h, hipStreamSynchronize(h.stream));
    int64_t n = 0;
    for (int64_t s = 0; s < m.ns; ++s) {
        if (!fl[s]) continue;
        if (n < cap) {
            const int32_t a = m.edge_node[2 * s], b = m.edge_node[2 * s + 1];
            if (edge) edge[n] = (int32_t)s;
            if (xy) {
                xy[2 * n] = 0.5 * (m.X[a] + m.X[b]);
                xy[2 * n + 1] = 0.5 * (m.Y[a] + m.Y[b]);
            }
        }
        ++n;
    }
    *count = n;
    if (cap < n) return fail(h, MCT_ECAPACITY, "%lld tips", (long long)n);
    return MCT_OK;
}

int get_field(Model &m, Host h, int which, int64_t cap, double *out) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    if (!out) return fail(h, MCT_EINVAL, "null output");
    const int64_t nn = m.nn, ne = m.ne, ns = m.ns;
    int64_t need = 2 * nn;
    if (which == MCT_FIELD_SIGMA_EDGE) need = 3 * ns;
    if (which == MCT_FIELD_PRINCIPAL) need = ne;
    if (which < MCT_FIELD_U || which > MCT_FIELD_PRINCIPAL) return fail(h, MCT_EINVAL, "unknown field %d", which);
    if (cap < need) return fail(h, MCT_ECAPACITY, "field needs %lld values", (long long)need);
    if (which == MCT_FIELD_U || which == MCT_FIELD_V) {
        Ctl c0;
        int rc0 = read_ctl(m, h, &c0);
        if (rc0) return rc0;
        std::vector<double> buf(2 * nn);
        TRY(h, hipMemcpyAsync(buf.data(), which == MCT_FIELD_U ? m.du[c0.base & 1] : m.dv, sizeof(double) * 2 * nn,
                              hipMemcpyDeviceToHost, h.stream));
        TRY(h, hipStreamSynchronize(h.stream));
        for (int64_t i = 0; i < nn; ++i) {
            out[i] = buf[2 * i];
            out[nn + i] = buf[2 * i + 1];
        }
        return MCT_OK;
    }
    Ctl c;
    int rc = eval_state(m, h, &c, false);
    if (rc) return rc;
    if (which == MCT_FIELD_A || which == MCT_FIELD_FINT) {
        TRY(h, hipMemcpyAsync(out, which == MCT_FIELD_A ? m.ev.acc : m.ev.fint, sizeof(double) * 2 * nn,
                              hipMemcpyDeviceToHost, h.stream));
        TRY(h, hipStreamSynchronize(h.stream));
        return MCT_OK;
    }
    if (which == MCT_FIELD_PRINCIPAL) {
        TRY(h, hipMemcpyAsync(out, m.ev.principal, sizeof(double) * ne, hipMemcpyDeviceToHost, h.stream));
        TRY(h, hipStreamSynchronize(h.stream));
        return MCT_OK;
    }
    // edge stresses from the element-edge table: the lower-id side if it is
    // intact, else the other side (NaN where neither is)
    const int nv = m.nv;
    std::vector<double> sk(3 * nv * ne);
    TRY(h, hipMemcpyAsync(sk.data(), m.ev.sig_ek, sizeof(double) * 3 * nv * ne, hipMemcpyDeviceToHost, h.stream));
    TRY(h, hipStreamSynchronize(h.stream));
    for (int64_t s = 0; s < ns; ++s) {
        double v[3] = {NAN, NAN, NAN};
        for (int side = 0; side < 2; ++side) {
            const int32_t e = m.edge_elem[2 * s + side];
            if (e < 0) continue;
            int k = 0;
            while (m.elem_edge[nv * (int64_t)e + k] != s) ++k;
            const double *q = &sk[3 * nv * (int64_t)e + 3 * k];
            if (!std::isnan(q[0]) || !std::isnan(q[1]) || !std::isnan(q[2])) {
                v[0] = q[0];
                v[1] = q[1];
                v[2] = q[2];
                break;
            }
        }
        for (int cc = 0; cc < 3; ++cc) out[cc * ns + s] = v[cc];
    }
    return MCT_OK;
}

int get_energies(Model &m, Host h, double out[4]) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    Ctl c;
    int rc = eval_state(m, h, &c, true);
    if (rc) return rc;
    TRY(h, launch_sum(m.ev.node_e, m.nn, 2, 0, m.dpart, m.dsums, h.stream));
    TRY(h, launch_sum(m.ev.node_e, m.nn, 2, 1, m.dpart, m.dsums + 1, h.stream));
    TRY(h, launch_sum(m.ev.es_ek, m.nv * m.ne, 1, 0, m.dpart, m.dsums + 2, h.stream));
    TRY(h, launch_sum(m.ev.pe, m.ne, 1, 0, m.dpart, m.dsums + 3, h.stream));
    double s[4];
    TRY(h, hipMemcpyAsync(s, m.dsums, sizeof s, hipMemcpyDeviceToHost, h.stream));
    TRY(h, hipStreamSynchronize(h.stream));
    out[0] = s[0];
    out[1] = s[2] + s[3];
    out[2] = s[1];
    out[3] = c.Ud;
    return MCT_OK;
}

int get_split_codes(Model &m, Host h, int64_t cap, uint8_t *out) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    if (cap < m.ne) return fail(h, MCT_ECAPACITY, "need %lld bytes", (long long)m.ne);
    TRY(h, hipMemcpyAsync(out, m.dsplit, m.ne, hipMemcpyDeviceToHost, h.stream));
    TRY(h, hipStreamSynchronize(h.stream));
    return MCT_OK;
}

int get_path_geometry(Model &m, Host h, int64_t n, const int32_t *elem, double *out) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    if (n > INT32_MAX / 36) return fail(h, MCT_EINVAL, "too many elements");
    for (int64_t i = 0; i < n; ++i)
        if (elem[i] < 0 || elem[i] >= m.ne) return fail(h, MCT_EINVAL, "element %d out of range", elem[i]);
    if (!n) return MCT_OK;
    int32_t *de = nullptr;
    double *dout = nullptr;
    TRY(h, hipMalloc((void **)&de, sizeof(int32_t) * (size_t)n));
    if (hipMalloc((void **)&dout, sizeof(double) * 36 * (size_t)n) != hipSuccess) {
        (void)hipFree(de);
        return fail(h, MCT_ENOMEM, "geometry buffer");
    }
    hipError_t e = hipMemcpyAsync(de, elem, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, h.stream);
    if (e == hipSuccess) e = launch_path_geometry(m.prm, (int)n, de, dout, h.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dout, sizeof(double) * 36 * (size_t)n, hipMemcpyDeviceToHost, h.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h.stream);
    (void)hipFree(de);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(h, MCT_EDEVICE, "path geometry: %s", hipGetErrorString(e));
    return MCT_OK;
}

// Checkpoint layout: 8-byte magic (one per element kind), n_nodes, n_elems
// (int64), the control block, u and v (interleaved pairs), split codes,
// then the logged splits.
static const uint64_t kMagic = 0x3152544432544d43ull;    // "MCT2DTR1"
static const uint64_t kMagicQ4 = 0x3152554432544d43ull;  // "MCT2DUR1"
static uint64_t magic_of(const Model &m) { return m.nv == 4 ? kMagicQ4 : kMagic; }

int checkpoint(Model &m, Host h, void *buf, int64_t cap, int64_t *bytes) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    Ctl c;
    int rc = read_ctl(m, h, &c);
    if (rc) return rc;
    const int64_t nlog = std::min<int64_t>(c.nsplit, m.prm.log_cap);
    const int64_t need = 24 + (int64_t)sizeof(Ctl) + 32 * m.nn + m.ne + (int64_t)sizeof(LogRec) * nlog;
    *bytes = need;
    if (!buf) return MCT_OK;
    if (cap < need) return fail(h, MCT_ECAPACITY, "checkpoint needs %lld bytes", (long long)need);
    char *p = static_cast<char *>(buf);
    const int64_t hdr[3] = {(int64_t)magic_of(m), m.nn, m.ne};
    std::memcpy(p, hdr, 24);
    p += 24;
    std::memcpy(p, &c, sizeof c);
    p += sizeof c;
    TRY(h, hipMemcpyAsync(p, m.du[c.base & 1], 16 * m.nn, hipMemcpyDeviceToHost, h.stream));
    p += 16 * m.nn;
    TRY(h, hipMemcpyAsync(p, m.dv, 16 * m.nn, hipMemcpyDeviceToHost, h.stream));
    p += 16 * m.nn;
    TRY(h, hipMemcpyAsync(p, m.dsplit, m.ne, hipMemcpyDeviceToHost, h.stream));
    p += m.ne;
    if (nlog) TRY(h, hipMemcpyAsync(p, m.dlog, sizeof(LogRec) * nlog, hipMemcpyDeviceToHost, h.stream));
    TRY(h, hipStreamSynchronize(h.stream));
    return MCT_OK;
}

int restore(Model &m, Host h, const void *buf, int64_t bytes) {
    if (!m.finalized) return fail(h, MCT_ESTATE, "finalize first");
    if (!buf || bytes < 24 + (int64_t)sizeof(Ctl)) return fail(h, MCT_EINVAL, "checkpoint too short");
    const char *p = static_cast<const char *>(buf);
    int64_t hdr[3];
    std::memcpy(hdr, p, 24);
    if ((uint64_t)hdr[0] != magic_of(m) || hdr[1] != m.nn || hdr[2] != m.ne)
        return fail(h, MCT_EINVAL, "checkpoint does not match this mesh");
    Ctl c;
    std::memcpy(&c, p + 24, sizeof c);
    const int64_t nlog = std::min<int64_t>(c.nsplit, m.prm.log_cap);
    if (c.nsplit < 0 || c.base < 0 || c.nacc != 0 ||
        bytes != 24 + (int64_t)sizeof(Ctl) + 32 * m.nn + m.ne + (int64_t)sizeof(LogRec) * nlog)
        return fail(h, MCT_EINVAL, "checkpoint size or control block invalid");
    if (c.tip < -1 || c.tip >= 4 * m.ne || (c.tip >= 0 && (c.tip & 3) >= m.nv))
        return fail(h, MCT_EINVAL, "checkpoint tip invalid");
    p += 24 + sizeof c;
    TRY(h, hipStreamSynchronize(h.stream));
    TRY(h, hipMemcpy(m.dctl, &c, sizeof c, hipMemcpyHostToDevice));
    if (m.dfold_n) TRY(h, hipMemset(m.dfold_n, 0, 3 * sizeof(int32_t)));
    if (m.dfgrid) {
        TRY(h, front_grid_reset(m.dfgrid, h.stream));
        TRY(h, hipStreamSynchronize(h.stream));
    }
    TRY(h, hipMemcpy(m.du[c.base & 1], p, 16 * m.nn, hipMemcpyHostToDevice));
    p += 16 * m.nn;
    TRY(h, hipMemcpy(m.dv, p, 16 * m.nn, hipMemcpyHostToDevice));
    p += 16 * m.nn;
    std::vector<uint8_t> split(p, p + m.ne);
    for (int64_t e = 0; e < m.ne; ++e) {
        const uint8_t s = split[e];
        if (s && (!(s & kSplitFlag) || ((s >> 2) & 3) >= m.nv || (s & 3) >= m.nv || ((s >> 2) & 3) == (s & 3) ||
                  (s & 0x70)))
            return fail(h, MCT_EINVAL, "checkpoint split code of element %lld invalid", (long long)e);
    }
    TRY(h, hipMemcpy(m.dsplit, split.data(), m.ne, hipMemcpyHostToDevice));
    p += m.ne;
    if (nlog) TRY(h, hipMemcpy(m.dlog, p, sizeof(LogRec) * nlog, hipMemcpyHostToDevice));
    m.steps_enqueued = c.base;
    return MCT_OK;
}

}  // namespace tri
}  // namespace mct
