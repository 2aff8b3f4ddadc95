"""Thin ctypes binding of libmct2d.so (include/mct2d.h).

Argument marshalling only: every computation of the step runs in the HIP
kernels behind the C ABI.  There is no fallback: if the shared library has
not been built, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libmct2d.so")

MCT_OK = 0
MCT_ECAPACITY = -3
FIELD_U = 0
FIELD_V = 1
FIELD_A = 2
FIELD_FINT = 3
FIELD_SIGMA_EDGE = 4
FIELD_PRINCIPAL = 5
MCT_ESTABILITY = -7
MCT_ENUMERIC = -8


class MctError(RuntimeError):
    pass


class Info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("n_edges", C.c_int64),
                ("step", C.c_int64), ("n_splits", C.c_int64), ("dt", C.c_double),
                ("dissipated", C.c_double), ("log_overflow", C.c_int32), ("precision", C.c_int32),
                ("dt_limit", C.c_double), ("tip", C.c_int64)]


class DeviceViews(C.Structure):
    _fields_ = [("ux", C.c_void_p * 2), ("uy", C.c_void_p * 2), ("vx", C.c_void_p), ("vy", C.c_void_p),
                ("n", C.c_int64)]


EXPORTS = [
    "mct_create", "mct_destroy", "mct_last_error", "mct_set_mesh_grid", "mct_set_material",
    "mct_set_traction", "mct_set_velocity_bc", "mct_set_notch", "mct_set_time", "mct_finalize",
    "mct_step", "mct_sync", "mct_get_info", "mct_get_crack_set", "mct_get_tips", "mct_get_field",
    "mct_get_split_codes", "mct_checkpoint", "mct_restore", "mct_set_launch", "mct_get_path_geometry",
    "mct_batch_create", "mct_batch_select", "mct_set_order", "mct_autotune", "mct_get_launch",
    "mct_screen_collect", "mct_screen_enable", "mct_screen_disable", "mct_screen_stats",
    "mct_mlp_create", "mct_mlp_destroy", "mct_mlp_last_error", "mct_mlp_set_params", "mct_mlp_get_params",
    "mct_mlp_forward", "mct_mlp_gradient", "mct_mlp_train_step", "mct_get_energies", "mct_set_tracking",
    "mct_set_load_curve", "mct_set_mesh_tri", "mct_set_mesh_q4", "mct_set_front_pick",
    "mct_set_smoothing", "mct_bind_device_buffers", "mct_set_lattice", "mct_get_lattice",
    "mct_set_near_log", "mct_get_near_log", "mct_profile_step", "mct_get_tips_noalloc",
]
LATTICE_AUTO = 0
LATTICE_GENERAL = 1
N_FEATURES = 10
N_PARAMS = 4929

_lib = None


def _init_torch_first() -> None:
    """torch brings its own HIP runtime libraries; when this library's HIP
    runtime is loaded and used first, torch later finds no device.  So torch
    initialises its GPU context before the library is loaded."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load() -> C.CDLL:
    """Load the HIP library; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MctError("libmct2d.so is not built (run python -m paper_2509_01827_amd.build)")
    _init_torch_first()
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    dp = np.ctypeslib.ndpointer(np.float64, flags="C")
    ip = np.ctypeslib.ndpointer(np.int32, flags="C")
    bp = np.ctypeslib.ndpointer(np.uint8, flags="C")
    L.mct_create.argtypes = [C.POINTER(P), C.c_int, P]
    L.mct_destroy.argtypes = [P]
    L.mct_last_error.argtypes = [P]
    L.mct_last_error.restype = C.c_char_p
    L.mct_set_mesh_grid.argtypes = [P, C.c_int32, C.c_int32, dp, dp]
    L.mct_set_mesh_tri.argtypes = [P, C.c_int64, dp, dp, C.c_int64, ip]
    L.mct_set_mesh_q4.argtypes = [P, C.c_int64, dp, dp, C.c_int64, ip]
    L.mct_set_material.argtypes = [P, C.c_double, C.c_double, C.c_double, P, C.c_double, C.c_double]
    L.mct_set_traction.argtypes = [P, C.c_int64, ip, dp]
    L.mct_set_velocity_bc.argtypes = [P, C.c_int64, ip, bp, dp, C.c_double]
    L.mct_set_notch.argtypes = [P, C.c_int64, ip, bp, bp]
    L.mct_set_time.argtypes = [P, C.c_double, C.c_double]
    L.mct_set_tracking.argtypes = [P, C.c_int, C.c_int32, C.c_int]
    L.mct_set_load_curve.argtypes = [P, C.c_int64, dp, dp]
    L.mct_set_front_pick.argtypes = [P, C.c_double]
    L.mct_set_smoothing.argtypes = [P, C.c_int]
    L.mct_bind_device_buffers.argtypes = [P, C.POINTER(DeviceViews)]
    L.mct_set_lattice.argtypes = [P, C.c_int]
    L.mct_get_lattice.argtypes = [P, C.POINTER(C.c_int)]
    L.mct_set_near_log.argtypes = [P, C.c_double, C.c_int64]
    L.mct_profile_step.argtypes = [P, C.c_int64, dp]
    L.mct_get_tips_noalloc.argtypes = [P, C.c_int64, P, P, P]
    L.mct_get_near_log.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, C.POINTER(C.c_int64)]
    L.mct_finalize.argtypes = [P]
    L.mct_step.argtypes = [P, C.c_int64]
    L.mct_sync.argtypes = [P]
    L.mct_get_info.argtypes = [P, C.POINTER(Info)]
    L.mct_get_crack_set.argtypes = [P, C.c_int64, P, P, P, P, P, C.POINTER(C.c_int64)]
    L.mct_get_tips.argtypes = [P, C.c_int64, P, P, C.POINTER(C.c_int64)]
    L.mct_get_field.argtypes = [P, C.c_int, C.c_int64, dp]
    L.mct_get_energies.argtypes = [P, dp]
    L.mct_get_split_codes.argtypes = [P, C.c_int64, bp]
    L.mct_checkpoint.argtypes = [P, P, C.c_int64, C.POINTER(C.c_int64)]
    L.mct_restore.argtypes = [P, P, C.c_int64]
    L.mct_set_launch.argtypes = [P, C.c_int, C.c_int]
    L.mct_get_path_geometry.argtypes = [P, C.c_int64, ip, dp]
    L.mct_batch_create.argtypes = [C.POINTER(P), C.c_int64, C.c_int, P]
    L.mct_batch_select.argtypes = [P, C.c_int64]
    L.mct_set_order.argtypes = [P, C.c_int]
    L.mct_autotune.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.mct_get_launch.argtypes = [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int64)]
    L.mct_screen_collect.argtypes = [P, C.c_int64, P, P, P, C.POINTER(C.c_int64)]
    L.mct_screen_enable.argtypes = [P, P, C.c_float, C.c_int]
    L.mct_screen_disable.argtypes = [P]
    L.mct_screen_stats.argtypes = [P, P]
    L.mct_mlp_create.argtypes = [C.POINTER(P), P]
    L.mct_mlp_destroy.argtypes = [P]
    L.mct_mlp_last_error.argtypes = [P]
    L.mct_mlp_last_error.restype = C.c_char_p
    L.mct_mlp_set_params.argtypes = [P, P]
    L.mct_mlp_get_params.argtypes = [P, P]
    L.mct_mlp_forward.argtypes = [P, P, C.c_int64, P]
    L.mct_mlp_gradient.argtypes = [P, P, P, C.c_int64, C.c_float, P, P]
    L.mct_mlp_train_step.argtypes = [P, P, P, C.c_int64, C.c_float, C.c_float, P]
    _lib = L
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def device_views(arrs, n, n_nodes):
    """Checked (addresses, length) of six caller-owned state arrays: distinct
    contiguous float64 torch tensors on one GPU device, or raw device
    addresses with an explicit length n; the length must cover n_nodes."""
    if len(arrs) != 6 or any(a is None for a in arrs):
        raise MctError("bind_device_buffers: all six arrays or none")
    if all(isinstance(a, int) for a in arrs):
        if n is None:
            raise MctError("bind_device_buffers: raw addresses need the length n")
        ptr, length = list(arrs), int(n)
    else:
        import torch
        for a in arrs:
            if not isinstance(a, torch.Tensor):
                raise MctError("bind_device_buffers: torch tensors or raw addresses, not mixed")
            if a.dtype != torch.float64 or not a.is_cuda or not a.is_contiguous():
                raise MctError("bind_device_buffers: contiguous float64 device tensors are required")
            if a.device != arrs[0].device:
                raise MctError("bind_device_buffers: all tensors on one device")
        ptr = [a.data_ptr() for a in arrs]
        length = min(a.numel() for a in arrs)
        if n is not None:
            length = min(length, int(n))
    if len(set(ptr)) != 6 or 0 in ptr:
        raise MctError("bind_device_buffers: six distinct non-null arrays are required")
    if length < max(int(n_nodes), 1):
        raise MctError("bind_device_buffers: %d values per array, the mesh has %d nodes" % (length, n_nodes))
    return ptr, length


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


class Model:
    """One MCT-2D-CEM model on the current HIP device.

    ``stream`` is a raw hipStream_t handle (an int, e.g.
    ``torch.cuda.current_stream().cuda_stream``) or None for a library
    stream."""

    def __init__(self, precision: int = 64, stream: int | None = None, n_specimens: int | None = None):
        L = load()
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream else None
        if n_specimens is None:
            rc = L.mct_create(C.byref(h), int(precision), st)
        else:
            rc = L.mct_batch_create(C.byref(h), int(n_specimens), int(precision), st)
        if rc != MCT_OK:
            raise MctError("create failed: %d" % rc)
        self._h = h
        self._L = L
        self._keep = []

    def _check(self, rc, what=""):
        if rc != MCT_OK:
            msg = self._L.mct_last_error(self._h).decode(errors="replace")
            raise MctError("%s failed (%d): %s" % (what, rc, msg))

    def close(self):
        if getattr(self, "_h", None):
            self._L.mct_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- set-up ---------------------------------------------------------
    def set_mesh_grid(self, nx, ny, X, Y):
        self._check(self._L.mct_set_mesh_grid(self._h, int(nx), int(ny), _f64(X), _f64(Y)), "set_mesh_grid")

    def set_mesh_tri(self, X, Y, conn):
        """Unstructured CST mesh: node coordinates and [ne][3] CCW triangles."""
        conn = _i32(np.asarray(conn).reshape(-1))
        X = _f64(X)
        self._check(self._L.mct_set_mesh_tri(self._h, len(X), X, _f64(Y), len(conn) // 3, conn), "set_mesh_tri")

    def set_mesh_q4(self, X, Y, conn):
        """Unstructured Q4 mesh: node coordinates and [ne][4] CCW convex
        quadrilaterals."""
        conn = _i32(np.asarray(conn).reshape(-1))
        X = _f64(X)
        self._check(self._L.mct_set_mesh_q4(self._h, len(X), X, _f64(Y), len(conn) // 4, conn), "set_mesh_q4")

    def set_material(self, E, nu, rho, gc=None, gc_uniform=0.0, gamma=1.0):
        self._gc = None if gc is None else _f64(gc)
        ptr = None if self._gc is None else self._gc.ctypes.data
        self._check(self._L.mct_set_material(self._h, float(E), float(nu), float(rho), ptr,
                                             float(gc_uniform), float(gamma)), "set_material")

    def set_traction(self, edge_nodes, t):
        en = _i32(np.asarray(edge_nodes).reshape(-1))
        self._check(self._L.mct_set_traction(self._h, len(en) // 2, en, _f64(np.asarray(t).reshape(-1))),
                    "set_traction")

    def set_velocity_bc(self, nodes, mask, v0, t_ramp=0.0):
        nodes = _i32(nodes)
        self._check(self._L.mct_set_velocity_bc(self._h, len(nodes), nodes, _u8(mask),
                                                _f64(np.asarray(v0).reshape(-1)), float(t_ramp)),
                    "set_velocity_bc")

    def set_notch(self, elem, entry, exit_):
        elem = _i32(elem)
        self._check(self._L.mct_set_notch(self._h, len(elem), elem, _u8(entry), _u8(exit_)), "set_notch")

    def set_time(self, dt=0.0, cfl=0.5):
        self._check(self._L.mct_set_time(self._h, float(dt), float(cfl)), "set_time")

    def set_load_curve(self, t, phi):
        t, phi = _f64(t), _f64(phi)
        self._check(self._L.mct_set_load_curve(self._h, len(t), t, phi), "set_load_curve")

    def bind_device_buffers(self, ux0, ux1, uy0, uy1, vx, vy, n=None):
        """Caller-owned state arrays: six distinct contiguous torch float64
        tensors on this context's device (cuda:0 unless the caller's stream
        says otherwise) with at least n_nodes elements each; u^k lives in
        (ux0, uy0) for even k and (ux1, uy1) for odd k.  Call after the mesh
        and before finalize (finalize checks the length against the mesh);
        the tensors are kept referenced by this model.  None for every
        argument unbinds.  Raw device addresses (ints) need the length n."""
        arrs = (ux0, ux1, uy0, uy1, vx, vy)
        if all(a is None for a in arrs):
            self._check(self._L.mct_bind_device_buffers(self._h, None), "bind_device_buffers")
            return
        ptr, length = device_views(arrs, n, self.info()["n_nodes"])
        v = DeviceViews()
        v.ux[0], v.ux[1], v.uy[0], v.uy[1], v.vx, v.vy = ptr
        v.n = length
        self._check(self._L.mct_bind_device_buffers(self._h, C.byref(v)), "bind_device_buffers")
        self._keep.append(arrs)

    def set_smoothing(self, mode="point"):
        """Q4 edge smoothing: "point" (default) or "subcell"."""
        m = {"point": 0, "subcell": 1}[mode]
        self._check(self._L.mct_set_smoothing(self._h, m), "set_smoothing")

    def set_lattice(self, mode=LATTICE_AUTO):
        """Uniform-lattice kernel: LATTICE_AUTO (when set-up finds one) or
        LATTICE_GENERAL (never); acts at the next finalize."""
        self._check(self._L.mct_set_lattice(self._h, int(mode)), "set_lattice")

    def lattice(self) -> bool:
        """True when the finalized context steps with the uniform-lattice kernel."""
        u = C.c_int(0)
        self._check(self._L.mct_get_lattice(self._h, C.byref(u)), "get_lattice")
        return bool(u.value)

    def set_near_log(self, tol, cap=1 << 20):
        """Near-threshold decision log with relative tolerance tol (0: off),
        up to cap records on the device; acts at the next finalize."""
        self._check(self._L.mct_set_near_log(self._h, float(tol), int(cap)), "set_near_log")

    def near_log(self) -> dict:
        """Near-threshold decisions sorted by (step, kind, elem, a, k)."""
        cnt = C.c_int64(0)
        rc = self._L.mct_get_near_log(self._h, 0, None, None, None, None, None, None, None, C.byref(cnt))
        if rc not in (MCT_OK, MCT_ECAPACITY):
            self._check(rc, "get_near_log")
        n = cnt.value
        st, el = np.zeros(n, np.int32), np.zeros(n, np.int32)
        a, kd, k = (np.zeros(n, np.uint8) for _ in range(3))
        G, ref = np.zeros(n), np.zeros(n)
        self._check(self._L.mct_get_near_log(self._h, n, st.ctypes.data, el.ctypes.data, a.ctypes.data,
                                             kd.ctypes.data, k.ctypes.data, G.ctypes.data, ref.ctypes.data,
                                             C.byref(cnt)), "get_near_log")
        return dict(step=st, elem=el, a=a, kind=kd, k=k, G=G, ref=ref)

    def set_front_pick(self, rho):
        """Per-front pick with competition radius rho (m); 0 = the global pick."""
        self._check(self._L.mct_set_front_pick(self._h, float(rho)), "set_front_pick")

    def set_tracking(self, mode="mct", tip_elem=-1, tip_edge=0):
        m = {"mct": 0, "sct": 1}[mode]
        self._check(self._L.mct_set_tracking(self._h, m, int(tip_elem), int(tip_edge)), "set_tracking")

    def tip(self):
        """Single-tip tracking: current tip (element, local edge) or None."""
        t = self.info()["tip"]
        return None if t < 0 else (t >> 2, t & 3)

    def set_launch(self, tile=0, use_graph=True):
        """Tile shape (grids: 0 automatic, 1 16x16, 2 32x8, 3 32x16) or, on
        an unstructured mesh, the step kernels (0 automatic, 1 element plus
        node kernels, 2/3/4 the fused kernel on 64/128/256-node patches, 5
        on patches of the size the library finds); whether steps replay
        captured HIP graphs.  Takes effect at once on a finalized model."""
        self._check(self._L.mct_set_launch(self._h, int(tile), int(bool(use_graph))), "set_launch")

    def select(self, s):
        """Select the specimen of a batch that set-up calls and queries act on."""
        self._check(self._L.mct_batch_select(self._h, int(s)), "batch_select")

    def set_order(self, order=-1):
        self._check(self._L.mct_set_order(self._h, int(order)), "set_order")

    def autotune(self, trial_steps=20):
        t, o, us = C.c_int(0), C.c_int(0), C.c_double(0.0)
        self._check(self._L.mct_autotune(self._h, int(trial_steps), C.byref(t), C.byref(o), C.byref(us)), "autotune")
        return dict(tile=t.value, order=o.value, us_per_step=us.value)

    def launch(self):
        """The launch shape in use: tile (the step kernels on an unstructured
        mesh, never 0), unit order and workgroups per step."""
        t, o, w = C.c_int(0), C.c_int(0), C.c_int64(0)
        self._check(self._L.mct_get_launch(self._h, C.byref(t), C.byref(o), C.byref(w)), "get_launch")
        return dict(tile=t.value, order=o.value, workgroups=w.value)

    def finalize(self):
        self._check(self._L.mct_finalize(self._h), "finalize")

    # -- run ------------------------------------------------------------
    def step(self, n):
        self._check(self._L.mct_step(self._h, int(n)), "step")

    def sync(self):
        self._check(self._L.mct_sync(self._h), "sync")

    def profile_step(self, n):
        """Run n steps as direct launches with HIP events around every
        launch; returns the mean duration per step (microseconds) of the
        step kernel and of the pick/commit launches."""
        out = np.zeros(2)
        self._check(self._L.mct_profile_step(self._h, int(n), out), "profile_step")
        return dict(step_us=float(out[0]), commit_us=float(out[1]))

    # -- queries --------------------------------------------------------
    def info(self) -> dict:
        inf = Info()
        self._check(self._L.mct_get_info(self._h, C.byref(inf)), "get_info")
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    def crack_set(self) -> dict:
        cnt = C.c_int64(0)
        rc = self._L.mct_get_crack_set(self._h, 0, None, None, None, None, None, C.byref(cnt))
        if rc not in (MCT_OK, MCT_ECAPACITY):
            self._check(rc, "get_crack_set")
        n = cnt.value
        st, el = np.zeros(n, np.int32), np.zeros(n, np.int32)
        en, ex = np.zeros(n, np.uint8), np.zeros(n, np.uint8)
        G = np.zeros(n)
        self._check(self._L.mct_get_crack_set(self._h, n, st.ctypes.data, el.ctypes.data, en.ctypes.data,
                                              ex.ctypes.data, G.ctypes.data, C.byref(cnt)), "get_crack_set")
        return dict(step=st, elem=el, entry=en, exit=ex, G=G)

    def tips(self):
        cnt = C.c_int64(0)
        rc = self._L.mct_get_tips(self._h, 0, None, None, C.byref(cnt))
        if rc not in (MCT_OK, MCT_ECAPACITY):
            self._check(rc, "get_tips")
        n = cnt.value
        edge = np.zeros(n, np.int32)
        xy = np.zeros(2 * n)
        self._check(self._L.mct_get_tips(self._h, n, edge.ctypes.data, xy.ctypes.data, C.byref(cnt)), "get_tips")
        return edge, xy.reshape(-1, 2)

    def field(self, which=FIELD_U):
        """Nodal fields (U, V, A, FINT) as (x, y); SIGMA_EDGE as [n_edges][3];
        PRINCIPAL as [n_elems]."""
        inf = self.info()
        nn, ne, ns = inf["n_nodes"], inf["n_elems"], inf["n_edges"]
        n = {FIELD_SIGMA_EDGE: 3 * ns, FIELD_PRINCIPAL: ne}.get(which, 2 * nn)
        out = np.zeros(n)
        self._check(self._L.mct_get_field(self._h, int(which), n, out), "get_field")
        if which == FIELD_SIGMA_EDGE:
            return out.reshape(3, ns).T.copy()
        if which == FIELD_PRINCIPAL:
            return out
        return out[:nn], out[nn:]

    def energies(self) -> dict:
        out = np.zeros(4)
        self._check(self._L.mct_get_energies(self._h, out), "get_energies")
        return dict(kin=out[0], strain=out[1], wext=out[2], Ud=out[3])

    def path_geometry(self, elems):
        """Crack-path normals and lengths as the GPU step computes them:
        array [n, 4 (tip edge a), 3 (path j), 3 (nx, ny, length)]."""
        elems = _i32(elems)
        out = np.zeros(36 * len(elems))
        self._check(self._L.mct_get_path_geometry(self._h, len(elems), elems, out), "get_path_geometry")
        return out.reshape(len(elems), 4, 3, 3)

    def split_codes(self):
        ne = self.info()["n_elems"]
        out = np.zeros(ne, np.uint8)
        self._check(self._L.mct_get_split_codes(self._h, ne, out), "get_split_codes")
        return out

    def checkpoint(self) -> bytes:
        nb = C.c_int64(0)
        self._check(self._L.mct_checkpoint(self._h, None, 0, C.byref(nb)), "checkpoint")
        buf = C.create_string_buffer(nb.value)
        self._check(self._L.mct_checkpoint(self._h, C.cast(buf, C.c_void_p), nb.value, C.byref(nb)), "checkpoint")
        return buf.raw[: nb.value]

    def restore(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(self._L.mct_restore(self._h, C.cast(buf, C.c_void_p), len(data)), "restore")

    # -- learned split-screen --------------------------------------------
    def screen_collect(self):
        """Features of every current candidate: (elem, entry, features [n][10]).
        Each call is one evaluation for the history behind feature 4."""
        cap = 4 * self.info()["n_elems"]  # at most four candidates per element
        cnt = C.c_int64(0)
        F = np.zeros((cap, N_FEATURES), np.float32)
        el = np.zeros(cap, np.int32)
        en = np.zeros(cap, np.uint8)
        self._check(self._L.mct_screen_collect(self._h, cap, F.ctypes.data, el.ctypes.data, en.ctypes.data,
                                               C.byref(cnt)), "screen_collect")
        n = cnt.value
        return el[:n], en[:n], F[:n]

    def screen_enable(self, mlp: "Mlp", tau: float, period: int = 50):
        self._check(self._L.mct_screen_enable(self._h, mlp._h, float(tau), int(period)), "screen_enable")

    def screen_disable(self):
        self._check(self._L.mct_screen_disable(self._h), "screen_disable")

    def screen_stats(self) -> dict:
        out = np.zeros(6, np.int64)
        self._check(self._L.mct_screen_stats(self._h, out.ctypes.data), "screen_stats")
        return dict(sweeps=int(out[0]), candidates=int(out[1]), flagged=int(out[2]), misses=int(out[3]),
                    windows=int(out[4]), replays=int(out[5]))


class Mlp:
    """The split-screen MLP on the device (mct_mlp).  Inputs of forward,
    gradient and train_step are device tensors (torch, float32, contiguous)."""

    def __init__(self, stream: int | None = None):
        L = load()
        h = C.c_void_p()
        rc = L.mct_mlp_create(C.byref(h), C.c_void_p(stream) if stream else None)
        if rc != MCT_OK:
            raise MctError("mlp create failed: %d" % rc)
        self._h, self._L = h, L

    def _check(self, rc, what=""):
        if rc != MCT_OK:
            msg = self._L.mct_mlp_last_error(self._h).decode(errors="replace")
            raise MctError("%s failed (%d): %s" % (what, rc, msg))

    def close(self):
        if getattr(self, "_h", None):
            self._L.mct_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (N_PARAMS,)
        self._check(self._L.mct_mlp_set_params(self._h, p.ctypes.data), "mlp_set_params")

    def params(self):
        p = np.zeros(N_PARAMS, np.float32)
        self._check(self._L.mct_mlp_get_params(self._h, p.ctypes.data), "mlp_get_params")
        return p

    @staticmethod
    def _dev(t, cols=None):
        assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous()
        if cols is not None:
            assert t.dim() == 2 and t.shape[1] == cols
        return t.data_ptr()

    def forward(self, x, out):
        n = x.shape[0]
        self._check(self._L.mct_mlp_forward(self._h, self._dev(x, N_FEATURES), n, self._dev(out)), "mlp_forward")

    def gradient(self, x, y, pos_weight=1.0):
        g = np.zeros(N_PARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        self._check(self._L.mct_mlp_gradient(self._h, self._dev(x, N_FEATURES), self._dev(y), x.shape[0],
                                             float(pos_weight), g.ctypes.data, loss.ctypes.data), "mlp_gradient")
        return float(loss[0]), g

    def train_step(self, x, y, pos_weight=1.0, lr=1e-3, want_loss=False):
        loss = np.zeros(1, np.float32)
        self._check(self._L.mct_mlp_train_step(self._h, self._dev(x, N_FEATURES), self._dev(y), x.shape[0],
                                               float(pos_weight), float(lr),
                                               loss.ctypes.data if want_loss else None), "mlp_train_step")
        return float(loss[0]) if want_loss else None


def _setup(m: Model, cfg: dict):
    if cfg.get("conn") is not None:
        if np.asarray(cfg["conn"]).shape[1] == 4:
            m.set_mesh_q4(cfg["X"], cfg["Y"], cfg["conn"])
        else:
            m.set_mesh_tri(cfg["X"], cfg["Y"], cfg["conn"])
    else:
        m.set_mesh_grid(cfg["nx"], cfg["ny"], cfg["X"], cfg["Y"])
    m.set_material(cfg["E"], cfg["nu"], cfg["rho"], cfg.get("gc_field"), cfg.get("gc_uniform", 0.0),
                   cfg.get("gamma", 1.0))
    m.set_traction(cfg["traction_nodes"], cfg["traction"])
    vn, vm, vv = cfg["vbc"]
    m.set_velocity_bc(vn, vm, vv, cfg.get("t_ramp", 0.0))
    ne_, en_, ex_ = cfg["notch"]
    m.set_notch(ne_, en_, ex_)
    m.set_time(cfg.get("dt", 0.0), cfg.get("cfl", 0.5))
    trk = cfg.get("tracking")
    if trk is not None:  # ("sct", elem or -1, edge)
        m.set_tracking(trk[0], trk[1], trk[2])
    lc = cfg.get("load_curve")
    if lc is not None:  # (t, phi)
        m.set_load_curve(lc[0], lc[1])
    if cfg.get("front_radius"):
        m.set_front_pick(cfg["front_radius"])
    if cfg.get("smoothing"):
        m.set_smoothing(cfg["smoothing"])
    if cfg.get("near_tol"):
        m.set_near_log(cfg["near_tol"], cfg.get("near_cap", 1 << 20))


def from_config(cfg: dict, stream: int | None = None, tile: int = 0, use_graph: bool = True) -> Model:
    """Build and finalize a model from a workload dictionary
    (paper_2509_01827_amd.workloads); cfg key precision 32 selects the
    binary32 step."""
    m = Model(int(cfg.get("precision", 64)), stream)
    _setup(m, cfg)
    if cfg.get("lattice") == "general" and cfg.get("conn") is None:
        m.set_lattice(LATTICE_GENERAL)
    m.set_launch(tile, use_graph)
    m.finalize()
    return m


def batch_from_configs(cfgs, stream: int | None = None, tile: int = 0, order: int = -1,
                       use_graph: bool = True) -> Model:
    """Build and finalize a batch of independent specimens, one per workload
    dictionary."""
    m = Model(64, stream, n_specimens=len(cfgs))
    for s, cfg in enumerate(cfgs):
        m.select(s)
        _setup(m, cfg)
    m.select(0)
    if any(c.get("lattice") == "general" for c in cfgs):
        m.set_lattice(LATTICE_GENERAL)
    m.set_launch(tile, use_graph)
    m.set_order(order)
    m.finalize()
    return m
