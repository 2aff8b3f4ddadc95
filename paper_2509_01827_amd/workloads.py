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


def config3(steps=10000):
    """2000x1000 Q4 mesh (h = 0.1 mm), 5 m/s outward on all edges,
    Weibull(6, 3 N/m) Gc, no notch."""
    return fragmentation(2000, 1000, 1.0e-4, steps=steps, name="fragment2000x1000")


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
                    ny_range=(64, 256), h=1.0e-3):
    """Independent notched specimens of uneven size (the batched workload).

    Specimen s takes five uniforms u0..u4 from one SplitMix64 stream (seed,
    specimen order): nx = U{nx_range}, ny = U{ny_range}, notch length
    round(U(0.2, 0.6) nx) in row ny // 2, Weibull scale lambda = U(2, 4) N/m,
    traction U(0.5, 1.5) MPa; its Gc field uses the stream seed + 1000 (s+1)
    (Weibull shape 6).  Square elements of side h, so all share one time
    step."""
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
