"""Seeded synthetic workloads for the MCT-2D-CEM explicit step.

This module only *describes inputs*: node coordinates of structured Q4
grids, random draws, boundary-condition arrays and pre-notch lists.  It holds
none of the method's arithmetic (no strain, stress, force, mass, time step or
energy release rate), so both the CPU oracle and the HIP library can consume
the same dictionaries.

Grid convention (shared by every consumer):
  * node (i, j), 0 <= i <= nx, 0 <= j <= ny, has id j*(nx+1) + i;
  * element (i, j), 0 <= i < nx, 0 <= j < ny, has id j*nx + i and the
    counter-clockwise nodes (i,j), (i+1,j), (i+1,j+1), (i,j+1);
  * local edge k of an element joins its local nodes k and (k+1) % 4
    (0 = bottom, 1 = right, 2 = top, 3 = left).

Material and loading follow the Neumann crack-branching plate of the paper
(Section 4.2: E = 32 GPa, nu = 0.2, rho = 2450 kg/m^3, Gc = 3 J/m^2, constant
1 MPa traction on the upper and lower edges); the paper's CST meshes are not
available, so structured Q4 stand-ins are generated here.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 250901827

# Material of the Neumann branching plate (Section 4.2).
E_PLATE = 32.0e9
NU_PLATE = 0.2
RHO_PLATE = 2450.0
GC_PLATE = 3.0

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First ``n`` outputs of SplitMix64 (Steele, Lea & Flood, OOPSLA 2014)
    started from state ``seed``: state += golden gamma, then the variant-13
    finaliser (shifts 30/27/31)."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed % (1 << 64)) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """U in [0, 1): the top 53 bits of each SplitMix64 output times 2^-53."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def grid_coords(nx: int, ny: int, lx: float, ly: float,
                jitter: float = 0.0, seed: int | None = None):
    """Node coordinates of an nx x ny grid over [0,lx] x [0,ly].

    With ``jitter`` > 0 every node draws two uniforms (x then y, node-id
    order) and moves by (2U-1)*jitter*h along each axis it is free in:
    boundary nodes slide only along their edge and corners stay put, so the
    plate stays rectangular."""
    hx = lx / nx
    hy = ly / ny
    i = np.arange(nx + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    X = np.tile(i * hx, ny + 1)
    Y = np.repeat(j * hy, nx + 1)
    if jitter > 0.0:
        nn = (nx + 1) * (ny + 1)
        u = uniform01(seed, 2 * nn).reshape(nn, 2)
        ii = np.tile(np.arange(nx + 1), ny + 1)
        jj = np.repeat(np.arange(ny + 1), nx + 1)
        free_x = (ii > 0) & (ii < nx)
        free_y = (jj > 0) & (jj < ny)
        X = X + np.where(free_x, (2.0 * u[:, 0] - 1.0) * jitter * hx, 0.0)
        Y = Y + np.where(free_y, (2.0 * u[:, 1] - 1.0) * jitter * hy, 0.0)
    return np.ascontiguousarray(X), np.ascontiguousarray(Y)


def node_id(nx: int, i, j):
    return np.asarray(j) * (nx + 1) + np.asarray(i)


def elem_id(nx: int, i, j):
    return np.asarray(j) * nx + np.asarray(i)


def edge_traction(nx: int, ny: int, top: float, bottom: float):
    """Boundary edges of the top and bottom rows with a normal traction.

    Returns (edge_nodes[n,2] int32, t[n,2] float64): ``top`` Pa along +y on
    the upper edge, ``bottom`` Pa along -y on the lower edge (both pull the
    plate apart for positive values)."""
    i = np.arange(nx)
    bot = np.stack([node_id(nx, i, 0), node_id(nx, i + 1, 0)], axis=1)
    tp = np.stack([node_id(nx, i, ny), node_id(nx, i + 1, ny)], axis=1)
    nodes = np.concatenate([bot, tp]).astype(np.int32)
    t = np.zeros((2 * nx, 2))
    t[:nx, 1] = -bottom
    t[nx:, 1] = top
    return np.ascontiguousarray(nodes), np.ascontiguousarray(t)


def outward_velocity(nx: int, ny: int, v: float):
    """Outward normal velocity ``v`` on all four edges (corners get both
    components); tangential motion stays free."""
    nodes, masks, vel = [], [], []
    for j in range(ny + 1):
        for i in range(nx + 1):
            m = 0
            vx = vy = 0.0
            if i == 0:
                m |= 1; vx = -v
            if i == nx:
                m |= 1; vx = v
            if j == 0:
                m |= 2; vy = -v
            if j == ny:
                m |= 2; vy = v
            if m:
                nodes.append(j * (nx + 1) + i); masks.append(m); vel.append((vx, vy))
    return (np.asarray(nodes, np.int32), np.asarray(masks, np.uint8),
            np.ascontiguousarray(np.asarray(vel, np.float64)))


def edge_notch(nx: int, ny: int, length: int, row: int | None = None):
    """Pre-notch of ``length`` elements from the left edge: pre-split
    pattern-II elements (entry = left edge 3, exit = right edge 1) in row
    ``row`` (default ny // 2)."""
    if row is None:
        row = ny // 2
    e = elem_id(nx, np.arange(length), row).astype(np.int32)
    return (e, np.full(length, 3, np.uint8), np.full(length, 1, np.uint8))


def weibull_gc(seed: int, n: int, shape: float, scale: float) -> np.ndarray:
    """Per-element Gc = scale * (-ln(1-U))^(1/shape), element-id order."""
    u = uniform01(seed, n)
    return scale * np.power(-np.log1p(-u), 1.0 / shape)


def _empty_bc():
    return (np.zeros(0, np.int32), np.zeros(0, np.uint8), np.zeros((0, 2)))


def _empty_notch():
    return (np.zeros(0, np.int32), np.zeros(0, np.uint8), np.zeros(0, np.uint8))


def plate(nx, ny, lx, ly, *, traction=1.0e6, jitter=0.0, seed=None,
          notch_len=None, notch_row=None, gc=GC_PLATE, gc_field=None,
          gamma=1.0, steps=2000, cfl=0.5, name="plate"):
    """A pre-notched plate pulled by a constant normal traction on its
    upper and lower edges (the Neumann branching set-up)."""
    X, Y = grid_coords(nx, ny, lx, ly, jitter, seed)
    tn, tt = edge_traction(nx, ny, traction, traction)
    if notch_len:
        notch = edge_notch(nx, ny, notch_len, notch_row)
    else:
        notch = _empty_notch()
    return dict(name=name, nx=nx, ny=ny, X=X, Y=Y, E=E_PLATE, nu=NU_PLATE,
                rho=RHO_PLATE, gc_uniform=gc, gc_field=gc_field, gamma=gamma,
                traction_nodes=tn, traction=tt, vbc=_empty_bc(), t_ramp=0.0,
                notch=notch, dt=0.0, cfl=cfl, steps=steps)


def pressure_pulse(t0=1.0e-6, tau=100.0e-6, t_end=400.0e-6, n=401):
    """Load history of the pressured cylinder of Sec. 4.4, normalised to its
    peak: linear rise to 1 at t0, then exp(-(t - t0) / tau) (the printed
    decay constant "100" read as microseconds, like t0), sampled at n
    points on [0, t_end] plus t0 itself.  Returns (t, phi)."""
    t = np.unique(np.concatenate([np.linspace(0.0, t_end, n), [t0]]))
    phi = np.where(t <= t0, t / t0, np.exp(-(t - t0) / tau))
    return np.ascontiguousarray(t), np.ascontiguousarray(phi)


def pulse_plate(nx, ny, lx, ly, *, peak=2.0e6, jitter=0.01, seed=BASE_SEED + 61, notch_len=None, steps=1000,
                t0=1.0e-6, tau=100.0e-6, name="pulse_plate"):
    """The notched plate with its edge tractions following the pressure
    pulse of Sec. 4.4 (peak traction ``peak`` Pa)."""
    c = plate(nx, ny, lx, ly, traction=peak, jitter=jitter, seed=seed,
              notch_len=notch_len if notch_len is not None else nx // 2, steps=steps, name=name)
    c["load_curve"] = pressure_pulse(t0=t0, tau=tau)
    return c


def config1(steps=2000):
    """40x40 Q4 plate, 40x40 mm, notch from the left edge to the centre
    along mid-height, 1 MPa traction, deterministic."""
    return plate(40, 40, 0.04, 0.04, notch_len=20, steps=steps, name="plate40x40")


def config2(steps=20000):
    """400x400 Q4 mesh of the 100x40 mm branching plate (0.25 x 0.1 mm
    elements), half-length edge notch, 1 MPa, +/-1% seeded nodal jitter."""
    return plate(400, 400, 0.1, 0.04, jitter=0.01, seed=BASE_SEED + 2,
                 notch_len=200, steps=steps, name="plate400x400_jitter")


def fragmentation(nx, ny, h, *, v=5.0, seed=BASE_SEED + 3, steps=10000,
                  shape=6.0, scale=GC_PLATE, name="fragment"):
    """Un-notched plate with outward normal velocity on all edges and a
    Weibull Gc field (the Dirichlet fragmentation set-up)."""
    X, Y = grid_coords(nx, ny, nx * h, ny * h)
    nodes, masks, vel = outward_velocity(nx, ny, v)
    gcf = weibull_gc(seed, nx * ny, shape, scale)
    return dict(name=name, nx=nx, ny=ny, X=X, Y=Y, E=E_PLATE, nu=NU_PLATE,
                rho=RHO_PLATE, gc_uniform=0.0, gc_field=gcf, gamma=1.0,
                traction_nodes=np.zeros((0, 2), np.int32), traction=np.zeros((0, 2)),
                vbc=(nodes, masks, vel), t_ramp=0.0, notch=_empty_notch(),
                dt=0.0, cfl=0.5, steps=steps)


# Element side of the workloads whose size the set-up leaves open: binary
# fractions of a metre close to 0.1 mm and 1 mm, so that every node
# coordinate i h is exact and every element of the lattice has bitwise the
# same geometry.
H_FRAGMENT = 2.0 ** -13   # 0.1220703125 mm
H_BATCH = 2.0 ** -10      # 0.9765625 mm


def config3(steps=10000):
    """2000x1000 Q4 mesh (h = 2^-13 m, 0.122 mm: a 244 x 122 mm plate), 5 m/s
    outward on all edges, Weibull(6, 3 N/m) Gc, no notch."""
    return fragmentation(2000, 1000, H_FRAGMENT, steps=steps, name="fragment2000x1000")


# Small cases that the oracle finishes in seconds; they span several GPU
# tiles with ragged tails in both directions.
def small_cases():
    return {
        "plate40x40": config1(),
        "plate70x37_jitter": plate(70, 37, 0.07, 0.037, jitter=0.01,
                                   seed=BASE_SEED + 11, notch_len=30,
                                   steps=1500, name="plate70x37_jitter"),
        "plate64x48_gamma2": plate(64, 48, 0.064, 0.048, notch_len=30,
                                   gamma=2.0, steps=1500, name="plate64x48_gamma2"),
        "fragment97x45": fragmentation(97, 45, 1.0e-3, seed=BASE_SEED + 13,
                                       steps=400, name="fragment97x45"),
    }


def batch_specimens(n=256, *, seed=BASE_SEED + 4, steps=5000, nx_range=(64, 512),
                    ny_range=(64, 256), h=H_BATCH):
    """Independent notched specimens of uneven size (the batched workload).

    Specimen s takes five uniforms u0..u4 from one SplitMix64 stream (seed,
    specimen order): nx = U{nx_range}, ny = U{ny_range}, notch length
    round(U(0.2, 0.6) nx) in row ny // 2, Weibull scale lambda = U(2, 4) N/m,
    traction U(0.5, 1.5) MPa; its Gc field uses the stream seed + 1000 (s+1)
    (Weibull shape 6).  Square elements of side h (2^-10 m by default), so
    all share one time step."""
    u = uniform01(seed, 5 * n).reshape(n, 5)
    out = []
    for s in range(n):
        nx = nx_range[0] + int(u[s, 0] * (nx_range[1] - nx_range[0] + 1))
        ny = ny_range[0] + int(u[s, 1] * (ny_range[1] - ny_range[0] + 1))
        notch = int(round((0.2 + 0.4 * u[s, 2]) * nx))
        lam = 2.0 + 2.0 * u[s, 3]
        trac = (0.5 + u[s, 4]) * 1.0e6
        gcf = weibull_gc(seed + 1000 * (s + 1), nx * ny, 6.0, lam)
        c = plate(nx, ny, nx * h, ny * h, traction=trac, notch_len=notch, gc=0.0,
                  gc_field=gcf, steps=steps, name="specimen%d" % s)
        out.append(c)
    return out


def small_batch(n=12, steps=600):
    """A batch the oracle finishes in seconds (parity tests)."""
    return batch_specimens(n, seed=BASE_SEED + 40, steps=steps, nx_range=(8, 48),
                           ny_range=(6, 40))


# --------------------------------------------------------------------------
# Unstructured triangle (CST) meshes
#
# A CST model is described by the same dictionary with ``conn`` ([ne][3]
# int32, counter-clockwise node triples) in place of ``nx``/``ny``.  Meshes
# are Delaunay triangulations (scipy) of seeded jittered point sets; nodes
# and triangles (by centroid) are numbered along a Morton curve so that
# neighbours have nearby ids (the library keeps the caller's numbering).

E_STEEL = 210.0e9
NU_STEEL = 0.3
RHO_STEEL = 7850.0
GC_STEEL = 2000.0


def _triangulate(X, Y, h):
    """Delaunay triangles of the points, each counter-clockwise and rotated
    to start at its smallest node id, sorted by the Morton code of the
    centroid on a grid of spacing h (ties: lexicographic node triple)."""
    from scipy.spatial import Delaunay
    T = Delaunay(np.stack([X, Y], axis=1)).simplices.astype(np.int64)
    a2 = (X[T[:, 1]] - X[T[:, 0]]) * (Y[T[:, 2]] - Y[T[:, 0]]) - \
         (X[T[:, 2]] - X[T[:, 0]]) * (Y[T[:, 1]] - Y[T[:, 0]])
    T[a2 < 0] = T[a2 < 0][:, [0, 2, 1]]
    r = np.argmin(T, axis=1)
    T = np.stack([T[np.arange(len(T)), (r + q) % 3] for q in range(3)], axis=1)
    return T, _morton_sort(T, X, Y, h)


def _morton_key(x, y, h):
    ix = np.floor((x - x.min()) / h).astype(np.uint64)
    iy = np.floor((y - y.min()) / h).astype(np.uint64)
    key = np.zeros(len(x), np.uint64)
    for b in range(21):
        key |= ((ix >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((iy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def morton_nodes(X, Y, h):
    """Node order along a Morton curve on a grid of spacing h (ties: the
    given order); returns the permutation (new id -> old id)."""
    return np.argsort(_morton_key(X, Y, h), kind="stable")


def _morton_sort(T, X, Y, h):
    cx = (X[T[:, 0]] + X[T[:, 1]] + X[T[:, 2]]) / 3.0
    cy = (Y[T[:, 0]] + Y[T[:, 1]] + Y[T[:, 2]]) / 3.0
    key = _morton_key(cx, cy, h)
    order = np.lexsort((T[:, 2], T[:, 1], T[:, 0], key))
    return np.ascontiguousarray(T[order].astype(np.int32))


def _edge_map(T):
    """{(lo, hi): [(element, local edge), ...]} of a triangle or
    quadrilateral list (local edge k joins local nodes k and k+1)."""
    m = {}
    nv = T.shape[1]
    for t in range(len(T)):
        for k in range(nv):
            a, b = int(T[t, k]), int(T[t, (k + 1) % nv])
            m.setdefault((min(a, b), max(a, b)), []).append((t, k))
    return m


def boundary_edges(T):
    """Edges used by one element, as (a, b) in that element's CCW
    direction (the domain lies to the left of a -> b)."""
    out = []
    nv = T.shape[1]
    for (lo, hi), uses in _edge_map(T).items():
        if len(uses) == 1:
            t, k = uses[0]
            out.append((int(T[t, k]), int(T[t, (k + 1) % nv])))
    out.sort()
    return np.asarray(out, np.int64).reshape(-1, 2)


def strip_notch(X, Y, T, y_c, x_end):
    """Pre-notch along the line y = y_c from the left boundary (x = 0) to
    x_end: the strip of elements (triangles or convex quadrilaterals) the
    line crosses, walked from the boundary edge through each element's other
    crossed edge while that crossing lies at x <= x_end.  Node sides: above
    means Y > y_c.  Returns (elem, entry, exit) with local edge indices."""
    above = Y > y_c
    em = _edge_map(T)
    nv = T.shape[1]

    def crossing_x(a, b):
        return X[a] + (y_c - Y[a]) / (Y[b] - Y[a]) * (X[b] - X[a])

    start = None
    for (lo, hi), uses in em.items():
        if len(uses) == 1 and X[lo] == 0.0 and X[hi] == 0.0 and above[lo] != above[hi]:
            start = uses[0]
    assert start is not None, "no boundary edge crosses the notch line"
    elems, ent, ext = [], [], []
    t, ke = start
    while True:
        ks = [k for k in range(nv) if k != ke and above[T[t, k]] != above[T[t, (k + 1) % nv]]]
        kx = ks[0]
        a, b = int(T[t, kx]), int(T[t, (kx + 1) % nv])
        if crossing_x(a, b) > x_end:
            break
        elems.append(t); ent.append(ke); ext.append(kx)
        uses = em[(min(a, b), max(a, b))]
        if len(uses) == 1:
            break
        t, ke = [u for u in uses if u[0] != t][0]
    return (np.asarray(elems, np.int32), np.asarray(ent, np.uint8), np.asarray(ext, np.uint8))


def tri_plate(nx, ny, lx, ly, *, traction=1.0e6, jitter=0.3, seed=BASE_SEED + 70,
              notch_len=None, gc=GC_PLATE, gc_field=None, gamma=1.0, steps=2000, cfl=0.5,
              name="tri_plate"):
    """The Neumann branching plate on an unstructured CST mesh: Delaunay
    triangulation of an (nx+1) x (ny+1) point grid with +/-``jitter`` h
    seeded moves (boundary points slide along their edge), 1 MPa normal
    traction on the upper and lower edges, pre-notch of length
    ``notch_len`` (m) along mid-height from the left edge."""
    X, Y = grid_coords(nx, ny, lx, ly, jitter, seed)
    h = min(lx / nx, ly / ny)
    perm = morton_nodes(X, Y, h)
    X, Y = np.ascontiguousarray(X[perm]), np.ascontiguousarray(Y[perm])
    T = _triangulate(X, Y, h)[1]
    be = boundary_edges(T)
    top = (Y[be[:, 0]] == ly) & (Y[be[:, 1]] == ly)
    bot = (Y[be[:, 0]] == 0.0) & (Y[be[:, 1]] == 0.0)
    tn = np.concatenate([be[bot], be[top]]).astype(np.int32)
    tt = np.zeros((len(tn), 2))
    tt[:bot.sum(), 1] = -traction
    tt[bot.sum():, 1] = traction
    notch = strip_notch(X, Y, T, 0.5 * ly, notch_len) if notch_len else _empty_notch()
    return dict(name=name, conn=T, X=X, Y=Y, E=E_PLATE, nu=NU_PLATE, rho=RHO_PLATE,
                gc_uniform=gc, gc_field=gc_field, gamma=gamma,
                traction_nodes=np.ascontiguousarray(tn), traction=np.ascontiguousarray(tt),
                vbc=_empty_bc(), t_ramp=0.0, notch=notch, dt=0.0, cfl=cfl, steps=steps)


def ring_points(r_in, r_out, h, *, jitter=0.2, seed=BASE_SEED + 80):
    """Points of an annulus: rings at radii r_in + k dr (dr ~ h sqrt(3)/2),
    ring k with round(2 pi r_k / h) equally spaced points at a random angular
    offset; the inner and outer rings are exact circles, the others move
    radially by +/-``jitter`` dr.  Returns (X, Y, ring index)."""
    nr = max(1, int(round((r_out - r_in) / (h * np.sqrt(3.0) / 2.0))))
    dr = (r_out - r_in) / nr
    u = uniform01(seed, 2 * (nr + 1)).reshape(nr + 1, 2)
    xs, ys, ks = [], [], []
    for k in range(nr + 1):
        r = r_in + k * dr
        n = max(3, int(round(2.0 * np.pi * r / h)))
        th = 2.0 * np.pi * (np.arange(n) + u[k, 0]) / n
        rr = r + (0.0 if k in (0, nr) else (2.0 * u[k, 1] - 1.0) * jitter * dr)
        xs.append(rr * np.cos(th)); ys.append(rr * np.sin(th)); ks.append(np.full(n, k))
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ks)


def tri_cylinder(r_in=0.05, r_out=0.1, h=1.0e-3, *, p0=400.0e6, t0=1.0e-6, tau=100.0e-6, seed=BASE_SEED + 80,
                 gamma=1.0, steps=4000, cfl=0.5, name="tri_cylinder"):
    """The pressure-loaded hollow cylinder of Sec. 4.4 on a CST mesh: steel
    (E 210 GPa, nu 0.3, rho 7850, Gc 2000 N/m), internal pressure p0 times
    the pulse history (rise to 1 at t0, decay exp(-(t - t0)/tau)) as a
    normal traction on the inner boundary edges; no pre-notch.  The default
    size (about 27 000 nodes / 53 000 triangles) is that of the paper's fine
    mesh; its radii are not printed and are a reading."""
    X, Y, ring = ring_points(r_in, r_out, h, seed=seed)
    perm = morton_nodes(X, Y, h)
    X, Y, ring = np.ascontiguousarray(X[perm]), np.ascontiguousarray(Y[perm]), ring[perm]
    T, Ts = _triangulate(X, Y, h)
    cx = (X[Ts[:, 0]] + X[Ts[:, 1]] + X[Ts[:, 2]]) / 3.0
    cy = (Y[Ts[:, 0]] + Y[Ts[:, 1]] + Y[Ts[:, 2]]) / 3.0
    Ts = np.ascontiguousarray(Ts[np.hypot(cx, cy) > r_in])  # drop the hole
    assert len(np.unique(Ts)) == len(X), "a point fell out of the annulus mesh"
    be = boundary_edges(Ts)
    inner = (ring[be[:, 0]] == 0) & (ring[be[:, 1]] == 0)
    tn = be[inner].astype(np.int32)
    dx = X[tn[:, 1]] - X[tn[:, 0]]
    dy = Y[tn[:, 1]] - Y[tn[:, 0]]
    L = np.hypot(dx, dy)
    tt = np.stack([-dy / L, dx / L], axis=1) * p0  # pushes the inner wall outward
    return dict(name=name, conn=Ts, X=X, Y=Y, E=E_STEEL, nu=NU_STEEL, rho=RHO_STEEL,
                gc_uniform=GC_STEEL, gc_field=None, gamma=gamma,
                traction_nodes=np.ascontiguousarray(tn), traction=np.ascontiguousarray(tt),
                vbc=_empty_bc(), t_ramp=0.0, notch=_empty_notch(), dt=0.0, cfl=cfl, steps=steps,
                load_curve=pressure_pulse(t0=t0, tau=tau))


def tri_plate320k(steps=20000):
    """The 100 x 40 mm Neumann branching plate on a Delaunay CST mesh of
    633 x 254 jittered points (h = 0.158 mm, about 320 000 triangles), half-
    length pre-notch: the CST workload at the size of the 400 x 400 Q4
    plate's edge count."""
    return tri_plate(632, 253, 0.1, 0.04, jitter=0.3, seed=BASE_SEED + 72, notch_len=0.05, steps=steps,
                     name="tri_plate320k")


def tri_small_cases():
    """CST cases the oracle finishes in seconds."""
    return {
        "tri_plate40x16": tri_plate(40, 16, 0.1, 0.04, notch_len=0.05, steps=1500, name="tri_plate40x16"),
        "tri_cylinder_coarse": tri_cylinder(h=5.0e-3, steps=1500, name="tri_cylinder_coarse"),
        "tri_fragment": tri_fragment(36, 30, 1.0e-3, steps=600, name="tri_fragment"),
    }


def tri_fragment(nx, ny, h, *, v=5.0, seed=BASE_SEED + 90, steps=2000, name="tri_fragment"):
    """Un-notched CST plate with outward normal velocity on all edges and a
    Weibull(6, 3 N/m) Gc field (the Dirichlet fragmentation set-up)."""
    X, Y = grid_coords(nx, ny, nx * h, ny * h, 0.3, seed)
    perm = morton_nodes(X, Y, h)
    X, Y = np.ascontiguousarray(X[perm]), np.ascontiguousarray(Y[perm])
    T = _triangulate(X, Y, h)[1]
    lx, ly = nx * h, ny * h
    nodes, masks, vel = [], [], []
    for i in range(len(X)):
        m, vx, vy = 0, 0.0, 0.0
        if X[i] == 0.0:
            m |= 1; vx = -v
        if X[i] == lx:
            m |= 1; vx = v
        if Y[i] == 0.0:
            m |= 2; vy = -v
        if Y[i] == ly:
            m |= 2; vy = v
        if m:
            nodes.append(i); masks.append(m); vel.append((vx, vy))
    gcf = weibull_gc(seed + 1, len(T), 6.0, GC_PLATE)
    return dict(name=name, conn=T, X=X, Y=Y, E=E_PLATE, nu=NU_PLATE, rho=RHO_PLATE,
                gc_uniform=0.0, gc_field=gcf, gamma=1.0,
                traction_nodes=np.zeros((0, 2), np.int32), traction=np.zeros((0, 2)),
                vbc=(np.asarray(nodes, np.int32), np.asarray(masks, np.uint8),
                     np.ascontiguousarray(np.asarray(vel, np.float64).reshape(-1, 2))),
                t_ramp=0.0, notch=_empty_notch(), dt=0.0, cfl=0.5, steps=steps)


# ---------------------------------------------------------------------------
# Unstructured Q4 meshes (general connectivity, mct_set_mesh_q4)


def quads_from_triangles(X, Y, T, h):
    """All-quadrilateral mesh from a triangle mesh: every triangle (a, b, c)
    splits into the three convex quadrilaterals (a, m_ab, g, m_ca),
    (b, m_bc, g, m_ab), (c, m_ca, g, m_bc) through its edge midpoints m and
    centroid g, counter-clockwise like the triangle.  Nodes and elements are
    renumbered along a Morton curve (spacing h/2); each quadrilateral starts
    at its smallest node id.  Returns (X, Y, Q)."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    T = np.asarray(T, np.int64)
    nn0 = len(X)
    mid = {}
    xs, ys = list(X), list(Y)

    def midpoint(a, b):
        key = (min(a, b), max(a, b))
        if key not in mid:
            mid[key] = len(xs)
            xs.append(0.5 * (X[a] + X[b]))
            ys.append(0.5 * (Y[a] + Y[b]))
        return mid[key]

    quads = []
    for t in range(len(T)):
        a, b, c = (int(v) for v in T[t])
        mab, mbc, mca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
        g = len(xs)
        xs.append((X[a] + X[b] + X[c]) / 3.0)
        ys.append((Y[a] + Y[b] + Y[c]) / 3.0)
        quads += [(a, mab, g, mca), (b, mbc, g, mab), (c, mca, g, mbc)]
    Xq, Yq = np.asarray(xs), np.asarray(ys)
    Q = np.asarray(quads, np.int64)
    assert len(Xq) == nn0 + len(mid) + len(T)
    perm = morton_nodes(Xq, Yq, 0.5 * h)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    Xq, Yq, Q = Xq[perm], Yq[perm], inv[Q]
    r = np.argmin(Q, axis=1)
    Q = np.stack([Q[np.arange(len(Q)), (r + q) % 4] for q in range(4)], axis=1)
    cx, cy = Xq[Q].mean(axis=1), Yq[Q].mean(axis=1)
    order = np.lexsort((Q[:, 3], Q[:, 2], Q[:, 1], Q[:, 0], _morton_key(cx, cy, 0.5 * h)))
    return np.ascontiguousarray(Xq), np.ascontiguousarray(Yq), np.ascontiguousarray(Q[order].astype(np.int32))


def quad_plate(nx, ny, lx, ly, *, traction=1.0e6, jitter=0.3, seed=BASE_SEED + 100, notch_len=None,
               gc=GC_PLATE, gamma=1.0, steps=2000, cfl=0.5, name="quad_plate"):
    """The Neumann branching plate on an unstructured all-quadrilateral mesh:
    the CST plate's Delaunay triangles (points of an (nx+1) x (ny+1) grid
    moved by +/-``jitter`` h) each split into three quadrilaterals; 1 MPa
    normal traction on the upper and lower edges; pre-notch of length
    ``notch_len`` (m) along a line just above mid-height from the left
    edge."""
    X, Y = grid_coords(nx, ny, lx, ly, jitter, seed)
    h = min(lx / nx, ly / ny)
    T = _triangulate(X, Y, h)[1]
    X, Y, Q = quads_from_triangles(X, Y, T, h)
    be = boundary_edges(Q)
    top = (Y[be[:, 0]] == ly) & (Y[be[:, 1]] == ly)
    bot = (Y[be[:, 0]] == 0.0) & (Y[be[:, 1]] == 0.0)
    tn = np.concatenate([be[bot], be[top]]).astype(np.int32)
    tt = np.zeros((len(tn), 2))
    tt[:bot.sum(), 1] = -traction
    tt[bot.sum():, 1] = traction
    # the notch line avoids the nodes (grid rows, midpoints, centroids)
    notch = strip_notch(X, Y, Q, 0.5 * ly + 0.137 * h, notch_len) if notch_len else _empty_notch()
    return dict(name=name, conn=Q, X=X, Y=Y, E=E_PLATE, nu=NU_PLATE, rho=RHO_PLATE,
                gc_uniform=gc, gc_field=None, gamma=gamma,
                traction_nodes=np.ascontiguousarray(tn), traction=np.ascontiguousarray(tt),
                vbc=_empty_bc(), t_ramp=0.0, notch=notch, dt=0.0, cfl=cfl, steps=steps)


def as_unstructured_q4(cfg, seed=BASE_SEED + 110):
    """A structured-grid workload written as an unstructured Q4 mesh: nodes
    and elements in a seeded random order, each element's node list rotated
    by a seeded offset (local edge k of the grid element becomes local edge
    k - r).  Loads, prescribed velocities, Gc and the notch follow."""
    nx, ny = cfg["nx"], cfg["ny"]
    nn, ne = (nx + 1) * (ny + 1), nx * ny
    u = uniform01(seed, nn + 2 * ne)
    pn = np.argsort(u[:nn], kind="stable")          # new id -> old id
    pe = np.argsort(u[nn:nn + ne], kind="stable")
    rot = np.floor(4.0 * u[nn + ne:]).astype(np.int64) % 4  # per new element
    inv_n = np.empty(nn, np.int64)
    inv_n[pn] = np.arange(nn)
    inv_e = np.empty(ne, np.int64)
    inv_e[pe] = np.arange(ne)
    Q = np.empty((ne, 4), np.int64)
    for e_new in range(ne):
        e = int(pe[e_new])
        i, j = e % nx, e // nx
        nd = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i]
        r = int(rot[e_new])
        Q[e_new] = [inv_n[nd[(q + r) % 4]] for q in range(4)]
    c = dict(cfg)
    c.pop("nx"); c.pop("ny")
    c["name"] = cfg.get("name", "grid") + "_unstructured"
    c["X"] = np.ascontiguousarray(cfg["X"][pn])
    c["Y"] = np.ascontiguousarray(cfg["Y"][pn])
    c["conn"] = np.ascontiguousarray(Q.astype(np.int32))
    tn = np.asarray(cfg["traction_nodes"], np.int64)
    c["traction_nodes"] = np.ascontiguousarray(inv_n[tn].astype(np.int32)) if len(tn) else tn.astype(np.int32)
    vn, vm, vv = cfg["vbc"]
    c["vbc"] = (np.ascontiguousarray(inv_n[np.asarray(vn, np.int64)].astype(np.int32)), vm, vv)
    if cfg.get("gc_field") is not None:
        c["gc_field"] = np.ascontiguousarray(np.asarray(cfg["gc_field"])[pe])
    el, en, ex = cfg["notch"]
    el = np.asarray(el, np.int64)
    rr = rot[inv_e[el]] if len(el) else np.zeros(0, np.int64)
    c["notch"] = (np.ascontiguousarray(inv_e[el].astype(np.int32)),
                  np.ascontiguousarray(((np.asarray(en, np.int64) - rr) % 4).astype(np.uint8)),
                  np.ascontiguousarray(((np.asarray(ex, np.int64) - rr) % 4).astype(np.uint8)))
    c["perm"] = (pn, pe, rot)
    return c


def quad_plate160k(steps=20000):
    """The 100 x 40 mm Neumann branching plate on an unstructured
    all-quadrilateral mesh: the Delaunay triangles of 259 x 104 jittered
    points each split into three quadrilaterals (about 160 000 elements, the
    400 x 400 Q4 plate's element count), half-length pre-notch."""
    return quad_plate(258, 103, 0.1, 0.04, notch_len=0.05, steps=steps, seed=BASE_SEED + 120,
                      name="quad_plate160k")


def quad_small_cases():
    """Unstructured Q4 parity cases: the jittered 70 x 37 plate renumbered,
    and a plate of quadrilaterals split from triangles (irregular valences)."""
    return {
        "grid70x37_unstructured": as_unstructured_q4(small_cases()["plate70x37_jitter"]),
        "quad_plate24x10": quad_plate(24, 10, 0.1, 0.04, notch_len=0.05, steps=1200),
    }
