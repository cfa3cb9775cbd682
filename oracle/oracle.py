"""ctypes wrapper of the FP64 oracle library (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

P_ACTIVE, P_STOPPED, P_RETIRED = 0, 1, 2


class _Params(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("lambda0", C.c_double),
                ("h", C.c_double), ("rc", C.c_double), ("a", C.c_double * 2),
                ("b", C.c_double * 2), ("theta", C.c_double), ("branching", C.c_int32),
                ("box_exit", C.c_int32), ("periodic", C.c_int32)]


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dT", C.c_double), ("dT0", C.c_double),
                ("grad", C.c_double * 3), ("rate", C.c_double), ("n", C.c_int32 * 3),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("data", C.POINTER(C.c_float)), ("q", C.c_double), ("U", C.c_double),
                ("alpha", C.c_double), ("x_start", C.c_double), ("x_end", C.c_double),
                ("ys", C.c_double), ("zs", C.c_double), ("r_min", C.c_double),
                ("dT_min", C.c_double), ("T", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("liq_T", C.c_double), ("liq_m", C.c_double)]


_lib = None


def build_oracle():
    from . import build as _b
    return _b.build()


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build_oracle()
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    P = lambda t: np.ctypeslib.ndpointer(dtype=t, flags="C_CONTIGUOUS")  # noqa: E731
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [C.POINTER(_Params)]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_error.argtypes = [vp]
    lib.orc_error.restype = C.c_int32
    lib.orc_set_theta.argtypes = [vp, C.c_double]
    lib.orc_set_kinetics.argtypes = [vp, P(np.float64)]
    lib.orc_set_branching.argtypes = [vp, C.c_int32]
    lib.orc_set_melting.argtypes = [vp, C.c_int32]
    lib.orc_melt_stats.argtypes = [vp, P(np.int64)]
    lib.orc_set_field.argtypes = [vp, C.POINTER(_Field)]
    lib.orc_set_field.restype = C.c_int32
    lib.orc_field_value.argtypes = [vp, C.c_int64, P(np.float64), C.c_double, P(np.float64),
                                    P(np.float64)]
    lib.orc_init_grains.argtypes = [vp, C.c_int32, P(np.float64), P(np.float64), P(np.int32)]
    lib.orc_init_grains.restype = C.c_int32
    lib.orc_nucleate.argtypes = [vp, C.c_int32, P(np.float64), P(np.float64), P(np.float64)]
    lib.orc_nucleate.restype = C.c_int32
    lib.orc_step.argtypes = [vp, C.c_double, C.c_int32]
    lib.orc_step.restype = C.c_int32
    lib.orc_phase.argtypes = [vp, C.c_int32, C.c_double]
    lib.orc_phase.restype = C.c_int32
    lib.orc_contain_decisions.argtypes = [vp, C.c_int32, P(np.uint8)]
    lib.orc_count.argtypes = [vp, C.c_int32]
    lib.orc_count.restype = C.c_int64
    lib.orc_last_stats.argtypes = [vp, P(np.int64), C.POINTER(C.c_double)]
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = C.c_int32
    lib.orc_set_threads.argtypes = [C.c_int32]
    lib.orc_set_threads.restype = None
    lib.orc_time.argtypes = [vp]
    lib.orc_time.restype = C.c_double
    lib.orc_get_particles.argtypes = [vp, P(np.int32), P(np.int32), P(np.int32), P(np.float64),
                                      P(np.float64), P(np.int32)]
    lib.orc_get_grains.argtypes = [vp, P(np.float64), P(np.float64)]
    lib.orc_get_claims.argtypes = [vp, P(np.int32), P(np.int32), P(np.uint8)]
    lib.orc_get_sites.argtypes = [vp, P(np.int32)]
    lib.orc_load_state.argtypes = [vp, C.c_int32, P(np.float64), P(np.float64), C.c_int64,
                                   P(np.int32), P(np.int32), P(np.int32), P(np.float64),
                                   P(np.int32), C.c_int64, P(np.int32), P(np.int32), P(np.uint8),
                                   C.c_int32, P(np.int32), C.c_double, C.c_int64]
    lib.orc_load_state.restype = C.c_int32
    lib.orc_grain_map.argtypes = [vp, P(np.int32), P(np.float64), P(np.float64), P(np.uint32)]
    lib.orc_deposit_counts.argtypes = [vp, P(np.int32), P(np.float64), P(np.float64),
                                       P(np.uint32)]
    lib.orc_f32_deposit.argtypes = [C.c_int64, P(np.int32), P(np.int32), P(np.float32),
                                    P(np.int32), P(np.float32), P(np.float32), P(np.uint32)]
    lib.orc_f32_cells.argtypes = [C.c_int64, P(np.float32), P(np.float32), C.c_float,
                                  P(np.int32), P(np.int32)]
    lib.orc_f32_contain.argtypes = [C.c_int64, P(np.float32), P(np.int32), P(np.uint8),
                                    C.c_float, P(np.uint8)]
    lib.orc_adjoint_record.argtypes = [vp, C.c_double, C.c_int32, P(np.int32)]
    lib.orc_adjoint_record.restype = C.c_int32
    lib.orc_adjoint_replay.argtypes = [vp, P(np.float64), C.c_double, C.c_int64, P(np.int32),
                                       P(np.int32), P(np.int32), P(np.float64), P(np.int32),
                                       C.c_double, C.c_double, C.c_int32, P(np.float64)]
    lib.orc_adjoint_replay.restype = C.c_int32
    lib.orc_adjoint_grad.argtypes = [vp, C.c_int64, P(np.int32), P(np.int32), P(np.int32),
                                     P(np.float64), P(np.int32), C.c_double, C.c_double,
                                     C.c_int32, P(np.float64), P(np.float64)]
    lib.orc_adjoint_grad.restype = C.c_int32
    _lib = lib
    return lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One oracle simulation state."""

    def __init__(self, lo, hi, lambda0, h, rc, a, b, theta=0.0, branching=1, box_exit=1,
                 periodic=0):
        self.lib = _load()
        p = _Params()
        p.lo[:] = list(lo)
        p.hi[:] = list(hi)
        p.lambda0, p.h, p.rc = lambda0, h, rc
        p.a[:] = list(a)
        p.b[:] = list(b)
        p.theta = theta
        p.branching = int(branching)
        p.box_exit = int(box_exit)
        p.periodic = int(periodic)
        self.params = p
        self.h = self.lib.orc_create(C.byref(p))
        self._keep = []

    @classmethod
    def from_workload(cls, w, init=True):
        o = cls(w.lo, w.hi, w.lambda0, w.h, w.rc, w.a, w.b, w.theta, w.branching, w.box_exit,
                w.periodic)
        o.set_field(w.field)
        if init:
            if len(w.grain_centre):
                o.init_grains(w.grain_centre, w.grain_quat, w.grain_shell)
            if len(w.site_xyz):
                o.nucleate(w.site_xyz, w.site_dTn, w.site_quat)
        return o

    def __del__(self):
        try:
            if self.h:
                self.lib.orc_destroy(self.h)
        except Exception:
            pass

    # ------------------------------------------------------------ setup --
    def set_field(self, f):
        fs = _Field()
        fs.kind = f.kind
        fs.dT, fs.dT0, fs.rate = f.dT, f.dT0, f.rate
        fs.grad[:] = list(f.grad)
        fs.n[:] = list(f.n)
        fs.origin[:] = list(f.origin)
        fs.spacing[:] = list(f.spacing)
        if f.data is not None:
            arr = np.ascontiguousarray(f.data, dtype=np.float32)
            self._keep.append(arr)
            fs.data = arr.ctypes.data_as(C.POINTER(C.c_float))
        for k in ("q", "U", "alpha", "x_start", "x_end", "ys", "zs", "r_min", "dT_min"):
            setattr(fs, k, getattr(f, k))
        if getattr(f, "T", None) is not None:
            for k in ("T", "w"):
                arr = np.ascontiguousarray(getattr(f, k), dtype=np.float64)
                self._keep.append(arr)
                setattr(fs, k, arr.ctypes.data_as(C.POINTER(C.c_double)))
            fs.liq_T, fs.liq_m = f.liq_T, f.liq_m
        rc = self.lib.orc_set_field(self.h, C.byref(fs))
        if rc != 0:
            raise ValueError(f"orc_set_field failed: {rc}")

    def field_value(self, x, t=0.0):
        """Undercooling field (without theta) and its gradient at points x [n, 3]."""
        x = _f64(x).reshape(-1, 3)
        out = np.zeros(len(x))
        grad = np.zeros((len(x), 3))
        self.lib.orc_field_value(self.h, len(x), x, float(t), out, grad)
        return out, grad

    def set_theta(self, theta):
        self.lib.orc_set_theta(self.h, float(theta))

    def set_kinetics(self, a):
        self.lib.orc_set_kinetics(self.h, _f64(a))

    def set_branching(self, on):
        self.lib.orc_set_branching(self.h, int(on))

    def set_melting(self, on):
        self.lib.orc_set_melting(self.h, int(on))

    def melt_stats(self):
        out = np.zeros(4, np.int64)
        self.lib.orc_melt_stats(self.h, out)
        return dict(zip(("melted", "removed", "reactivated", "grains_melted"), out.tolist()))

    def init_grains(self, centre, quat, shell_r):
        centre, quat, shell_r = _f64(centre).reshape(-1, 3), _f64(quat).reshape(-1, 4), _i32(shell_r)
        rc = self.lib.orc_init_grains(self.h, len(shell_r), centre, quat, shell_r)
        if rc != 0:
            raise ValueError(rc)

    def nucleate(self, xyz, dTn, quat):
        xyz, dTn, quat = _f64(xyz).reshape(-1, 3), _f64(dTn), _f64(quat).reshape(-1, 4)
        rc = self.lib.orc_nucleate(self.h, len(dTn), xyz, dTn, quat)
        if rc != 0:
            raise ValueError(rc)

    # ------------------------------------------------------------- run ---
    def step(self, dt, n=1):
        return self.lib.orc_step(self.h, float(dt), int(n))

    def phase(self, ph, dt=0.0):
        return self.lib.orc_phase(self.h, int(ph), float(dt))

    @property
    def error(self):
        return self.lib.orc_error(self.h)

    @property
    def time(self):
        return self.lib.orc_time(self.h)

    def count(self, what):
        return self.lib.orc_count(self.h, what)

    def n_active(self):
        return self.count(1)

    def last_stats(self):
        out = np.zeros(6, np.int64)
        ms = C.c_double()
        self.lib.orc_last_stats(self.h, out, C.byref(ms))
        keys = ("advanced", "exited", "spawners", "children", "contained", "nucleated")
        d = dict(zip(keys, out.tolist()))
        d["max_step"] = ms.value
        return d

    # ----------------------------------------------------------- export --
    def particles(self):
        n = self.count(0)
        g = np.zeros(n, np.int32)
        site = np.zeros(3 * n, np.int32)
        d = np.zeros(n, np.int32)
        s = np.zeros(n, np.float64)
        x = np.zeros(3 * n, np.float64)
        st = np.zeros(n, np.int32)
        self.lib.orc_get_particles(self.h, g, site, d, s, x, st)
        return dict(grain=g, site=site.reshape(-1, 3), dir=d, s=s, x=x.reshape(-1, 3), state=st)

    def grains(self):
        n = self.count(4)
        c = np.zeros(3 * n)
        R = np.zeros(9 * n)
        self.lib.orc_get_grains(self.h, c, R)
        return c.reshape(-1, 3), R.reshape(-1, 3, 3)

    def claims(self):
        n = self.count(5)
        g = np.zeros(n, np.int32)
        s = np.zeros(3 * n, np.int32)
        f = np.zeros(n, np.uint8)
        self.lib.orc_get_claims(self.h, g, s, f)
        return dict(grain=g, site=s.reshape(-1, 3), flags=f)

    def site_states(self):
        n = self.count(6)
        st = np.zeros(n, np.int32)
        self.lib.orc_get_sites(self.h, st)
        return st

    def load_state(self, grain_centre, grain_quat, parts, claims, site_state, t, step):
        gc, gq = _f64(grain_centre).reshape(-1, 3), _f64(grain_quat).reshape(-1, 4)
        site_state = _i32(site_state)
        rc = self.lib.orc_load_state(
            self.h, len(gc), gc, gq, len(parts["grain"]), _i32(parts["grain"]),
            _i32(parts["site"]).reshape(-1), _i32(parts["dir"]), _f64(parts["s"]),
            _i32(parts["state"]), len(claims["grain"]), _i32(claims["grain"]),
            _i32(claims["site"]).reshape(-1), np.ascontiguousarray(claims["flags"], np.uint8),
            len(site_state), site_state, float(t), int(step))
        if rc != 0:
            raise ValueError(f"orc_load_state failed: {rc}")

    def contain_decisions(self, method=0):
        out = np.zeros(self.count(0), np.uint8)
        self.lib.orc_contain_decisions(self.h, int(method), out)
        return out

    def deposit_counts(self, n, origin, spacing):
        """Reached lattice sites per node-centred cell, shape (n2, n1, n0) (FP64)."""
        n = _i32(n)
        out = np.zeros(int(np.prod(n)), np.uint32)
        self.lib.orc_deposit_counts(self.h, n, _f64(origin), _f64(spacing), out)
        return out.reshape(n[2], n[1], n[0])

    def grain_map(self, n, origin, spacing):
        n = _i32(n)
        out = np.zeros(int(np.prod(n)), np.uint32)
        self.lib.orc_grain_map(self.h, n, _f64(origin), _f64(spacing), out)
        return out.reshape(n[2], n[1], n[0])

    # ---------------------------------------------------------- adjoint --
    def adjoint_record(self, dt, n_steps):
        nact = np.zeros(self.count(0), np.int32)
        rc = self.lib.orc_adjoint_record(self.h, float(dt), int(n_steps), nact)
        if rc != 0:
            raise ValueError(f"orc_adjoint_record failed: {rc}")
        return nact

    def adjoint_replay(self, a, theta, parts, nact, t0, dt, n_steps):
        n = len(parts["grain"])
        xN = np.zeros(3 * n)
        rc = self.lib.orc_adjoint_replay(
            self.h, _f64(a), float(theta), n, _i32(parts["grain"]), _i32(parts["site"]).reshape(-1),
            _i32(parts["dir"]), _f64(parts["s"]), _i32(nact), float(t0), float(dt), int(n_steps), xN)
        if rc != 0:
            raise ValueError(rc)
        return xN.reshape(-1, 3)

    def adjoint_grad(self, parts, nact, t0, dt, n_steps, dLdx):
        n = len(parts["grain"])
        g = np.zeros(3)
        rc = self.lib.orc_adjoint_grad(
            self.h, n, _i32(parts["grain"]), _i32(parts["site"]).reshape(-1), _i32(parts["dir"]),
            _f64(parts["s"]), _i32(nact), float(t0), float(dt), int(n_steps),
            _f64(dLdx).reshape(-1), g)
        if rc != 0:
            raise ValueError(rc)
        return g


def threads():
    return _load().orc_threads()


def set_threads(n):
    """Threads of the oracle's parallel loops from now on (0: one per processor)."""
    _load().orc_set_threads(int(n))


def f32_cells(xyz, lo, inv_h, ncell):
    lib = _load()
    xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1)
    out = np.zeros(xyz.size, np.int32)
    lib.orc_f32_cells(xyz.size // 3, xyz, np.ascontiguousarray(lo, np.float32),
                      np.float32(inv_h), _i32(ncell), out)
    return out.reshape(-1, 3)


def f32_deposit(grain, site, gtab, n, origin, inv_spacing):
    """FP32 checker of the deposition counts of reached sites (grain, site)
    from FP32 grain rows gtab [n_grains, 24]."""
    lib = _load()
    grain = _i32(grain)
    site = _i32(site).reshape(-1)
    n = _i32(n)
    out = np.zeros(int(np.prod(n)), np.uint32)
    lib.orc_f32_deposit(len(grain), grain, site,
                        np.ascontiguousarray(gtab, np.float32).reshape(-1), n,
                        np.ascontiguousarray(origin, np.float32),
                        np.ascontiguousarray(inv_spacing, np.float32), out)
    return out.reshape(n[2], n[1], n[0])


def f32_contain(xyz, grain, role, rc2):
    lib = _load()
    xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1)
    out = np.zeros(xyz.size // 3, np.uint8)
    lib.orc_f32_contain(xyz.size // 3, xyz, _i32(grain), np.ascontiguousarray(role, np.uint8),
                        np.float32(rc2), out)
    return out
