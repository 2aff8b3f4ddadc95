"""ctypes wrapper of the plain CPU oracle (mct_oracle.c): the binary64 build
(liboracle.so) and the binary32 build of the same source (liboracle32.so,
the step in binary32 over binary64 set-up values rounded once).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mct_oracle.c")
_LIBS = {64: os.path.join(_HERE, "liboracle.so"), 32: os.path.join(_HERE, "liboracle32.so")}

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]


def build(force: bool = False, precision: int = 64) -> str:
    """Compile liboracle.so (or liboracle32.so) with gcc (plain C, no FMA
    contraction)."""
    path = _LIBS[precision]
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        extra = ["-DORC_FP32"] if precision == 32 else []
        subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def build_all(force: bool = False) -> None:
    for prec in _LIBS:
        build(force, prec)


_libs = {}


def lib(precision: int = 64):
    if precision not in _LIBS:
        raise ValueError("oracle precision is 64 or 32")
    _lib = _libs.get(precision)
    if _lib is None:
        _lib = C.CDLL(build(precision=precision))
        _libs[precision] = _lib
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C")
        bp = np.ctypeslib.ndpointer(np.uint8, flags="C")
        _lib.orc_create.restype = P
        _lib.orc_create.argtypes = [C.c_int, C.c_int, dp, dp]
        _lib.orc_create_tri.restype = P
        _lib.orc_create_tri.argtypes = [C.c_int, dp, dp, C.c_int, ip]
        _lib.orc_create_q4.restype = P
        _lib.orc_create_q4.argtypes = [C.c_int, dp, dp, C.c_int, ip]
        _lib.orc_destroy.argtypes = [P]
        _lib.orc_set_material.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                          C.c_double, C.c_double]
        _lib.orc_set_traction.argtypes = [P, C.c_int, ip, dp]
        _lib.orc_set_velocity_bc.argtypes = [P, C.c_int, ip, bp, dp, C.c_double]
        _lib.orc_set_notch.argtypes = [P, C.c_int, ip, bp, bp]
        _lib.orc_set_time.argtypes = [P, C.c_double, C.c_double]
        _lib.orc_finalize.argtypes = [P]
        _lib.orc_step.argtypes = [P, C.c_long]
        _lib.orc_info.argtypes = [P, ip, dp, C.POINTER(C.c_long)]
        _lib.orc_get_state.argtypes = [P, dp, dp, dp, dp, bp]
        _lib.orc_set_state.argtypes = [P, dp, dp, dp, dp]
        _lib.orc_get_log.argtypes = [P, ip, ip, ip, ip, dp]
        _lib.orc_get_tables.argtypes = [P, ip, ip, ip, ip, dp, dp, dp]
        _lib.orc_internal_force.argtypes = [P, dp, dp, dp, dp, C.c_void_p, C.c_void_p]
        _lib.orc_candidates.argtypes = [P, C.c_int, ip, ip, ip, dp, ip, ip]
        _lib.orc_tips.argtypes = [P, C.c_int, ip, dp, ip]
        _lib.orc_energies.argtypes = [P, dp]
        _lib.orc_candidate_G.argtypes = [P, C.c_int, C.c_int, dp]
        _lib.orc_path_normal.argtypes = [P, C.c_int, C.c_int, C.c_int, dp]
        _lib.orc_split_codes.argtypes = [P, bp]
        _lib.orc_element_rule.argtypes = [dp, C.c_double, C.c_double]
        _lib.orc_element_rule_n.argtypes = [C.c_int, dp, C.c_double, C.c_double]
        _lib.orc_mct_pick.argtypes = [C.c_int, dp, ip, ip, C.c_double]
        _lib.orc_set_tracking.argtypes = [P, C.c_int, C.c_int, C.c_int]
        _lib.orc_set_front_pick.argtypes = [P, C.c_double]
        _lib.orc_set_smoothing.argtypes = [P, C.c_int]
        _lib.orc_front_pick.argtypes = [C.c_int, dp, ip, ip, dp, dp, C.c_double, C.c_double, ip]
        _lib.orc_get_tip.argtypes = [P]
        _lib.orc_get_tip.restype = C.c_int
        _lib.orc_set_load_curve.argtypes = [P, C.c_int, dp, dp]
        _lib.orc_load_factor.argtypes = [P, C.c_double]
        _lib.orc_load_factor.restype = C.c_double
        _lib.orc_set_near_log.argtypes = [P, C.c_double]
        _lib.orc_near_count.argtypes = [P]
        _lib.orc_near_count.restype = C.c_int
        _lib.orc_get_near.argtypes = [P, ip, ip, ip, ip, ip, dp, dp]
        _lib.orc_near_candidate.argtypes = [P, C.c_int, C.c_int, C.c_int, dp, C.c_double]
        _lib.orc_near_pick.argtypes = [P, C.c_int, dp, ip, ip, ip, C.c_int]
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_get_threads.restype = C.c_int
        _lib.orc_precision.restype = C.c_int
        assert _lib.orc_precision() == precision
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def set_threads(n: int) -> None:
    """OpenMP threads used by the oracle (results are thread-count independent)."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def element_rule(G3, Gc, gamma, precision=64):
    return lib(precision).orc_element_rule(_f64(G3), float(Gc), float(gamma))


def element_rule_n(G, Gc, gamma, precision=64):
    """Element decision over len(G) candidate paths (2: CST, 3: Q4)."""
    G = _f64(G)
    return lib(precision).orc_element_rule_n(len(G), G, float(Gc), float(gamma))


def front_pick(G, elem, a, x, y, gamma, rho, precision=64):
    """Indices of the candidates the per-front pick splits, in key order."""
    G = _f64(G)
    out = np.zeros(max(len(G), 1), np.int32)
    n = lib(precision).orc_front_pick(len(G), G, _i32(elem), _i32(a), _f64(x), _f64(y), float(gamma),
                                      float(rho) ** 2, out)
    return out[:n]


def mct_pick(G, elem, a, gamma, precision=64):
    G = _f64(G)
    return lib(precision).orc_mct_pick(len(G), G, _i32(elem), _i32(a), float(gamma))


class Oracle:
    """One model run by the plain CPU oracle: a structured Q4 grid (cfg keys
    nx, ny) or an unstructured mesh (cfg key conn: [ne][3] CST or [ne][4]
    Q4, counter-clockwise); cfg key precision 32 runs the binary32 build."""

    def __init__(self, cfg: dict, *, finalize: bool = True):
        self.precision = int(cfg.get("precision", 64))
        L = self._L = lib(self.precision)
        self.cfg = cfg
        if cfg.get("conn") is not None:
            self.nx = self.ny = 0
            cn = np.asarray(cfg["conn"])
            nv = cn.shape[1]
            conn = _i32(cn.reshape(-1))
            X = _f64(cfg["X"])
            make = L.orc_create_tri if nv == 3 else L.orc_create_q4
            self.h = make(len(X), X, _f64(cfg["Y"]), len(conn) // nv, conn)
        else:
            self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
            self.h = L.orc_create(self.nx, self.ny, _f64(cfg["X"]), _f64(cfg["Y"]))
        if not self.h:
            raise ValueError("oracle: bad mesh")
        gcf = cfg.get("gc_field")
        self._gc = None if gcf is None else _f64(gcf)
        rc = L.orc_set_material(self.h, cfg["E"], cfg["nu"], cfg["rho"],
                                None if self._gc is None else self._gc.ctypes.data,
                                float(cfg.get("gc_uniform", 0.0)), float(cfg.get("gamma", 1.0)))
        self._check(rc)
        tn = _i32(np.asarray(cfg["traction_nodes"]).reshape(-1))
        self._check(L.orc_set_traction(self.h, len(tn) // 2, tn, _f64(np.asarray(cfg["traction"]).reshape(-1))))
        vn, vm, vv = cfg["vbc"]
        self._check(L.orc_set_velocity_bc(self.h, len(vn), _i32(vn), _u8(vm),
                                          _f64(np.asarray(vv).reshape(-1)), float(cfg.get("t_ramp", 0.0))))
        ne_, en_, ex_ = cfg["notch"]
        self._check(L.orc_set_notch(self.h, len(ne_), _i32(ne_), _u8(en_), _u8(ex_)))
        self._check(L.orc_set_time(self.h, float(cfg.get("dt", 0.0)), float(cfg.get("cfl", 0.5))))
        lc = cfg.get("load_curve")
        if lc is not None:  # (t, phi)
            self._lc = (_f64(lc[0]), _f64(lc[1]))
            self._check(L.orc_set_load_curve(self.h, len(self._lc[0]), self._lc[0], self._lc[1]))
        trk = cfg.get("tracking")
        if trk is not None:  # ("sct", elem or -1, edge)
            self._check(L.orc_set_tracking(self.h, 1 if trk[0] == "sct" else 0, int(trk[1]), int(trk[2])))
        if cfg.get("front_radius"):  # per-front pick with this competition radius (m)
            self._check(L.orc_set_front_pick(self.h, float(cfg["front_radius"])))
        if cfg.get("smoothing") == "subcell":  # Q4 edge smoothing over triangular sub-cells
            self._check(L.orc_set_smoothing(self.h, 1))
        if cfg.get("near_tol"):  # near-threshold decision log
            self._check(L.orc_set_near_log(self.h, float(cfg["near_tol"])))
        if finalize:
            self._check(L.orc_finalize(self.h))

    @staticmethod
    def _check(rc):
        if rc != 0:
            raise ValueError("oracle call failed: %d" % rc)

    def __del__(self):
        if getattr(self, "h", None):
            self._L.orc_destroy(self.h)
            self.h = None

    def info(self):
        ints = np.zeros(6, np.int32)
        dbls = np.zeros(2)
        st = C.c_long(0)
        self._L.orc_info(self.h, ints, dbls, C.byref(st))
        return dict(nn=int(ints[0]), ne=int(ints[1]), ns=int(ints[2]), ncolor=int(ints[3]),
                    nlog=int(ints[4]), nv=int(ints[5]), dt=float(dbls[0]), Ud=float(dbls[1]),
                    step=int(st.value))

    def step(self, n):
        self._check(self._L.orc_step(self.h, int(n)))

    def state(self):
        inf = self.info()
        nn, ne = inf["nn"], inf["ne"]
        ux, uy, vx, vy = (np.zeros(nn) for _ in range(4))
        sp = np.zeros(ne, np.uint8)
        self._L.orc_get_state(self.h, ux, uy, vx, vy, sp)
        return dict(ux=ux, uy=uy, vx=vx, vy=vy, split=sp)

    def set_state(self, ux, uy, vx, vy):
        self._L.orc_set_state(self.h, _f64(ux), _f64(uy), _f64(vx), _f64(vy))

    def set_split_codes(self, codes):
        self._L.orc_split_codes(self.h, _u8(codes))

    def log(self):
        n = self.info()["nlog"]
        st, el, en, ex = (np.zeros(n, np.int32) for _ in range(4))
        G = np.zeros(n)
        self._L.orc_get_log(self.h, st, el, en, ex, G)
        return dict(step=st, elem=el, entry=en, exit=ex, G=G)

    def near_log(self):
        """Near-threshold decisions (arrays step, elem, a, kind, k, G, ref)
        in the order they were made."""
        n = self._L.orc_near_count(self.h)
        st, el, a, kd, k = (np.zeros(n, np.int32) for _ in range(5))
        G, ref = np.zeros(n), np.zeros(n)
        self._L.orc_get_near(self.h, st, el, a, kd, k, G, ref)
        return dict(step=st, elem=el, a=a, kind=kd, k=k, G=G, ref=ref)

    def tables(self):
        inf = self.info()
        nn, ne, ns = inf["nn"], inf["ne"], inf["ns"]
        en = np.zeros(2 * ns, np.int32)
        ee = np.zeros(2 * ns, np.int32)
        el = np.zeros(2 * ns, np.int32)
        col = np.zeros(ne, np.int32)
        area = np.zeros(ne)
        mass = np.zeros(nn)
        fext = np.zeros(2 * nn)
        self._L.orc_get_tables(self.h, en, ee, el, col, area, mass, fext)
        return dict(edge_node=en.reshape(-1, 2), edge_elem=ee.reshape(-1, 2),
                    edge_loc=el.reshape(-1, 2), color=col, area=area, mass=mass,
                    fext=fext.reshape(-1, 2))

    def internal_force(self, ux, uy, with_stress=False):
        inf = self.info()
        nn, ns = inf["nn"], inf["ns"]
        fx, fy = np.zeros(nn), np.zeros(nn)
        sig = np.zeros(3 * ns)
        ok = np.zeros(ns, np.uint8)
        self._L.orc_internal_force(self.h, _f64(ux), _f64(uy), fx, fy, sig.ctypes.data, ok.ctypes.data)
        if with_stress:
            return fx, fy, sig.reshape(-1, 3), ok
        return fx, fy

    def candidates(self):
        ns = self.info()["ns"]
        edge, elem, a, dec = (np.zeros(ns, np.int32) for _ in range(4))
        G3 = np.zeros(3 * ns)
        cnt = np.zeros(1, np.int32)
        self._check(self._L.orc_candidates(self.h, ns, edge, elem, a, G3, dec, cnt))
        n = int(cnt[0])
        return dict(edge=edge[:n], elem=elem[:n], a=a[:n], G=G3.reshape(-1, 3)[:n], dec=dec[:n])

    def tips(self):
        ns = self.info()["ns"]
        edge = np.zeros(ns, np.int32)
        xy = np.zeros(2 * ns)
        cnt = np.zeros(1, np.int32)
        self._check(self._L.orc_tips(self.h, ns, edge, xy, cnt))
        n = int(cnt[0])
        return edge[:n], xy.reshape(-1, 2)[:n]

    def energies(self):
        out = np.zeros(4)
        self._L.orc_energies(self.h, out)
        return dict(kin=out[0], strain=out[1], wext=out[2], Ud=out[3])

    def candidate_G(self, e, a):
        G = np.zeros(3)
        H = self._L.orc_candidate_G(self.h, int(e), int(a), G)
        return G, H

    def load_factor(self, t):
        return self._L.orc_load_factor(self.h, float(t))

    def tip(self):
        """Current single-crack tip as (element, local edge), or None."""
        t = self._L.orc_get_tip(self.h)
        return None if t < 0 else (t >> 2, t & 3)

    def path_normal(self, e, a, k):
        out = np.zeros(3)
        self._L.orc_path_normal(self.h, int(e), int(a), int(k), out)
        return out


def run(cfg: dict, steps: int | None = None) -> Oracle:
    o = Oracle(cfg)
    o.step(cfg["steps"] if steps is None else steps)
    return o
