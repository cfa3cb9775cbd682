"""Python binding of libgrainenv: argument marshalling over the C ABI.

Every step of the method runs in the library's HIP kernels.  PyTorch supplies
the device workspace and the stream; numpy arrays carry host inputs.  The
binding fails loudly when the library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrainenv.so")

GE_OK, GE_EINVAL, GE_ECAPACITY, GE_ENUMERIC, GE_ECFL, GE_EDEVICE, GE_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ECAPACITY", -3: "ENUMERIC", -4: "ECFL",
                -5: "EDEVICE", -6: "ESTATE"}
FIELD_UNIFORM, FIELD_LINEAR, FIELD_GRID, FIELD_ROSENTHAL, FIELD_SOLUTE = 0, 1, 2, 3, 4
(QUERY_COUNTS, QUERY_PARTICLES, QUERY_GRAIN_MAP, QUERY_CLAIMS, QUERY_SITES, QUERY_GRAINS,
 QUERY_DIGEST, QUERY_MUSHY_COUNTS, QUERY_MUSHY) = range(9)
ACTIVE, STOPPED, RETIRED = 0, 1, 2

PARTICLE_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("s", "<f4"),
                           ("site", "<i4", 3), ("grain", "<u4"), ("dir", "u1"), ("state", "u1"),
                           ("pad", "<u2"), ("cell", "<i4", 3)])
CLAIM_DTYPE = np.dtype([("grain", "<u4"), ("site", "<i4", 3), ("flags", "<u4")])
ADJOINT_DTYPE = np.dtype([("grain", "<u4"), ("site", "<i4", 3), ("dir", "u1"), ("state0", "u1"),
                          ("pad", "<u2"), ("s0", "<f4"), ("s_final", "<f4"), ("nact", "<i4")])
assert PARTICLE_DTYPE.itemsize == 48 and CLAIM_DTYPE.itemsize == 20


class GrainEnvError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ge_params(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("lambda0", C.c_double),
                ("h", C.c_double), ("rc", C.c_double), ("a", C.c_double * 2),
                ("b", C.c_double * 2), ("theta", C.c_double), ("branching", C.c_int32),
                ("box_exit", C.c_int32), ("cap_particles", C.c_int64),
                ("cap_stopped", C.c_int64), ("cap_grains", C.c_int32), ("cap_sites", C.c_int32),
                ("cap_claim_bricks", C.c_int64), ("field_n", C.c_int32 * 3),
                ("resort_every", C.c_int32), ("periodic", C.c_int32)]


class ge_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dT", C.c_double), ("dT0", C.c_double),
                ("grad", C.c_double * 3), ("rate", C.c_double), ("n", C.c_int32 * 3),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("data", C.c_void_p), ("data_on_device", C.c_int32), ("q", C.c_double),
                ("U", C.c_double), ("alpha", C.c_double), ("x_start", C.c_double),
                ("x_end", C.c_double), ("ys", C.c_double), ("zs", C.c_double),
                ("r_min", C.c_double), ("dT_min", C.c_double), ("T", C.c_void_p),
                ("w", C.c_void_p), ("liq_T", C.c_double), ("liq_m", C.c_double)]


class ge_step_stats(C.Structure):
    _fields_ = [("n_active", C.c_int64), ("n_stopped", C.c_int64), ("n_grains", C.c_int64),
                ("n_claim_bricks", C.c_int64), ("advanced", C.c_int64), ("exited", C.c_int64),
                ("spawners", C.c_int64), ("children", C.c_int64), ("contained", C.c_int64),
                ("nucleated", C.c_int64), ("max_step", C.c_double), ("t", C.c_double),
                ("step", C.c_int64), ("pair_tests", C.c_int64), ("dirty_tests", C.c_int64),
                ("melted", C.c_int64), ("removed", C.c_int64), ("reactivated", C.c_int64),
                ("grains_melted", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ge_query_args(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


class ge_state_in(C.Structure):
    _fields_ = [("n_grains", C.c_int32), ("centre", C.c_void_p), ("quat", C.c_void_p),
                ("n_particles", C.c_int64), ("grain", C.c_void_p), ("site", C.c_void_p),
                ("dir", C.c_void_p), ("s", C.c_void_p), ("state", C.c_void_p),
                ("n_claims", C.c_int64), ("c_grain", C.c_void_p), ("c_site", C.c_void_p),
                ("c_flags", C.c_void_p), ("n_sites", C.c_int32), ("site_state", C.c_void_p),
                ("t", C.c_double), ("step", C.c_int64)]


class ge_state_header(C.Structure):
    _fields_ = [("magic", C.c_uint32), ("version", C.c_uint32), ("bytes", C.c_uint64),
                ("checksum", C.c_uint64), ("lambda0", C.c_double), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("t", C.c_double), ("step", C.c_int64),
                ("n_grains", C.c_int64), ("n_sites", C.c_int64), ("n_particles", C.c_int64),
                ("n_claim_bricks", C.c_int64)]


STATE_MAGIC, STATE_VERSION = 0x54534547, 1
assert C.sizeof(ge_state_header) == 128

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libgrainenv.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback path)")
    # torch's HIP runtime is loaded before the library's: loaded the other way
    # round, the library's runtime finds no device in a process that then
    # imports torch.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, P = C.c_void_p, C.POINTER
    sig = {
        "ge_workspace_size": ([P(ge_params), P(C.c_size_t)], C.c_int32),
        "ge_validate_params": ([P(ge_params)], C.c_int32),
        "ge_create": ([P(ge_params), vp, C.c_size_t, vp, P(vp)], C.c_int32),
        "ge_destroy": ([vp], C.c_int32),
        "ge_last_error": ([vp], C.c_char_p),
        "ge_init_grains": ([vp, C.c_int32, vp, vp, vp, P(C.c_uint32)], C.c_int32),
        "ge_set_thermal_field": ([vp, P(ge_field)], C.c_int32),
        "ge_set_deposition_grid": ([vp, vp, vp, vp], C.c_int32),
        "ge_set_melting": ([vp, C.c_int32], C.c_int32),
        "ge_nucleate": ([vp, C.c_int32, vp, vp, vp], C.c_int32),
        "ge_step": ([vp, C.c_double, C.c_int32, P(ge_step_stats)], C.c_int32),
        "ge_query_envelope": ([vp, C.c_int32, P(ge_query_args), vp, C.c_size_t,
                               P(C.c_size_t)], C.c_int32),
        "ge_load_state": ([vp, P(ge_state_in)], C.c_int32),
        "ge_query_particles_noalloc": ([vp, P(ge_query_args), vp, C.c_size_t, P(C.c_size_t)],
                                       C.c_int32),
        "ge_save_state": ([vp, vp, C.c_size_t, P(C.c_size_t)], C.c_int32),
        "ge_state_check": ([vp, C.c_size_t, P(ge_state_header)], C.c_int32),
        "ge_restore_state": ([vp, vp, C.c_size_t], C.c_int32),
        "ge_profile": ([vp, C.c_int32], C.c_int32),
        "ge_profile_read": ([vp, P(C.c_double), P(C.c_int64)], C.c_int32),
        "ge_profile_phase": ([vp, C.c_int32], C.c_int32),
        "ge_phase_name": ([C.c_int32], C.c_char_p),
        "ge_get_schedule": ([vp, P(C.c_int32)], C.c_int32),
        "ge_set_schedule": ([vp, P(C.c_int32)], C.c_int32),
        "ge_autotune": ([vp, C.c_double, C.c_int32, vp, C.c_size_t, P(C.c_int32)], C.c_int32),
        "ge_tunable_name": ([C.c_int32], C.c_char_p),
        "ge_use_graphs": ([vp, C.c_int32], C.c_int32),
        "ge_prepare_step": ([vp, C.c_double], C.c_int32),
        "ge_hold": ([vp, C.c_int32], C.c_int32),
        "ge_batch_workspace_size": ([C.c_int32, P(ge_params), P(C.c_size_t)], C.c_int32),
        "ge_batch_create": ([C.c_int32, P(ge_params), vp, C.c_size_t, vp, P(vp)], C.c_int32),
        "ge_batch_destroy": ([vp], C.c_int32),
        "ge_batch_member": ([vp, C.c_int32, P(vp)], C.c_int32),
        "ge_batch_last_error": ([vp], C.c_char_p),
        "ge_batch_step": ([vp, C.c_double, C.c_int32, P(ge_step_stats)], C.c_int32),
        "ge_batch_use_graphs": ([vp, C.c_int32], C.c_int32),
        "ge_batch_get_blocks": ([vp, P(C.c_int32)], C.c_int32),
        "ge_batch_set_blocks": ([vp, P(C.c_int32)], C.c_int32),
        "ge_batch_autotune": ([vp, C.c_double, C.c_int32, vp, C.c_size_t, P(C.c_int32)],
                              C.c_int32),
        "ge_set_model": ([vp, P(C.c_double), P(C.c_double), C.c_double, C.c_int32], C.c_int32),
        "ge_adjoint_workspace_size": ([vp, C.c_int32, C.c_int32, P(C.c_size_t)], C.c_int32),
        "ge_adjoint_forward": ([vp, C.c_double, C.c_int32, C.c_int32, vp, C.c_size_t,
                                P(C.c_int64)], C.c_int32),
        "ge_adjoint_positions": ([vp, vp, C.c_size_t, C.c_int32], C.c_int32),
        "ge_adjoint_tracked": ([vp, vp, C.c_size_t], C.c_int32),
        "ge_adjoint_backward": ([vp, vp, C.c_int32, P(C.c_double)], C.c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


EXPORTED = ("ge_workspace_size", "ge_validate_params", "ge_create", "ge_destroy",
            "ge_last_error", "ge_init_grains", "ge_set_thermal_field", "ge_set_deposition_grid",
            "ge_set_melting",
            "ge_nucleate", "ge_step",
            "ge_query_envelope", "ge_query_particles_noalloc", "ge_load_state",
            "ge_save_state", "ge_state_check",
            "ge_restore_state", "ge_profile", "ge_profile_read", "ge_profile_phase",
            "ge_phase_name", "ge_get_schedule", "ge_set_schedule", "ge_autotune",
            "ge_tunable_name", "ge_set_model", "ge_adjoint_workspace_size", "ge_adjoint_forward",
            "ge_adjoint_positions", "ge_adjoint_tracked", "ge_adjoint_backward",
            "ge_use_graphs", "ge_prepare_step", "ge_hold", "ge_batch_workspace_size", "ge_batch_create", "ge_batch_destroy",
            "ge_batch_member", "ge_batch_last_error", "ge_batch_step", "ge_batch_use_graphs",
            "ge_batch_get_blocks", "ge_batch_set_blocks", "ge_batch_autotune")
N_PHASES = 12
N_TUNABLE = 8
MAX_BLOCKS = 2048


def make_params(lo, hi, lambda0, h, rc, a, b, theta=0.0, branching=1, box_exit=1,
                cap_particles=1 << 20, cap_stopped=1 << 20, cap_grains=1 << 12,
                cap_sites=1 << 12, cap_claim_bricks=1 << 16, field_n=(0, 0, 0),
                resort_every=0, periodic=0) -> ge_params:
    p = ge_params()
    p.lo[:] = [float(v) for v in lo]
    p.hi[:] = [float(v) for v in hi]
    p.lambda0, p.h, p.rc = float(lambda0), float(h), float(rc)
    p.a[:] = [float(v) for v in a]
    p.b[:] = [float(v) for v in b]
    p.theta = float(theta)
    p.branching, p.box_exit = int(branching), int(box_exit)
    p.cap_particles, p.cap_stopped = int(cap_particles), int(cap_stopped)
    p.cap_grains, p.cap_sites = int(cap_grains), int(cap_sites)
    p.cap_claim_bricks = int(cap_claim_bricks)
    p.field_n[:] = [int(v) for v in field_n]
    p.resort_every = int(resort_every)
    p.periodic = int(periodic)
    return p


def params_from_workload(w, **caps) -> ge_params:
    fn = (tuple(w.field.n) if w.field.kind in (FIELD_GRID, FIELD_ROSENTHAL, FIELD_SOLUTE)
          else (0, 0, 0))
    caps.setdefault("field_n", fn)
    caps.setdefault("cap_sites", max(len(w.site_dTn), 1))
    caps.setdefault("periodic", w.periodic)
    return make_params(w.lo, w.hi, w.lambda0, w.h, w.rc, w.a, w.b, w.theta, w.branching,
                       w.box_exit, **caps)


def workspace_size(p: ge_params) -> int:
    lib = load_library()
    n = C.c_size_t()
    rc = lib.ge_workspace_size(C.byref(p), C.byref(n))
    if rc != GE_OK:
        raise GrainEnvError(rc, "invalid parameters")
    return n.value


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def state_check(blob) -> dict:
    """Header of a saved state after checking the blob (no device needed);
    raises GrainEnvError(EINVAL) for a blob that is not a valid saved state."""
    lib = load_library()
    blob = np.ascontiguousarray(blob, np.uint8)
    h = ge_state_header()
    rc = lib.ge_state_check(_ptr(blob), blob.nbytes, C.byref(h))
    if rc != GE_OK:
        raise GrainEnvError(rc, "not a valid saved state")
    return {k: (list(getattr(h, k)) if k in ("lo", "hi") else getattr(h, k)) for k, _ in h._fields_}


class Context:
    """A grain-envelope simulation on one GPU (the C context plus its
    workspace, a torch uint8 tensor)."""

    def __init__(self, params: ge_params, device="cuda:0", stream=None):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.params = params
        nbytes = workspace_size(params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        rc = self.lib.ge_create(C.byref(params), C.c_void_p(self.workspace.data_ptr()),
                                nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if rc != GE_OK:
            msg = self.lib.ge_last_error(None)
            raise GrainEnvError(rc, f"ge_create failed: {msg.decode() if msg else ''}")
        self.ctx = ctx
        self.n_sites = 0

    @classmethod
    def from_workload(cls, w, device="cuda:0", init=True, **caps):
        c = cls(params_from_workload(w, **caps), device=device)
        c.init_from_workload(w, init)
        return c

    def init_from_workload(self, w, init=True):
        """Field, grains and nucleation sites of a workload."""
        self.set_thermal_field(w.field)
        if init:
            if len(w.grain_centre):
                self.init_grains(w.grain_centre, w.grain_quat, w.grain_shell)
            if len(w.site_dTn):
                self.nucleate(w.site_xyz, w.site_dTn, w.site_quat)

    @classmethod
    def borrowed(cls, ctx_ptr, params, owner, device="cuda:0"):
        """A view of a context owned by a batch (not destroyed by close())."""
        import torch
        c = cls.__new__(cls)
        c.lib = load_library()
        c.torch = torch
        c.device = torch.device(device)
        c.params = params
        c.workspace = None
        c.stream = owner.stream
        c.ctx = ctx_ptr
        c.n_sites = 0
        c._owner = owner
        return c

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self.ctx = None
            return
        if getattr(self, "ctx", None):
            self.lib.ge_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != GE_OK:
            msg = self.lib.ge_last_error(self.ctx)
            raise GrainEnvError(rc, f"{what}: {msg.decode() if msg else ''}")

    # ------------------------------------------------------------ C ABI ---
    def init_grains(self, centre, quat, shell_r):
        centre = np.ascontiguousarray(centre, np.float64).reshape(-1, 3)
        quat = np.ascontiguousarray(quat, np.float64).reshape(-1, 4)
        shell = np.ascontiguousarray(shell_r, np.int32).reshape(-1)
        first = C.c_uint32()
        self._check(self.lib.ge_init_grains(self.ctx, len(shell), _ptr(centre), _ptr(quat),
                                            _ptr(shell), C.byref(first)), "ge_init_grains")
        return first.value

    def set_thermal_field(self, f):
        fs = ge_field()
        fs.kind = f.kind
        fs.dT, fs.dT0, fs.rate = f.dT, f.dT0, f.rate
        fs.grad[:] = list(f.grad)
        fs.n[:] = list(f.n)
        fs.origin[:] = list(f.origin)
        fs.spacing[:] = list(f.spacing)
        keep = []

        n_nodes = int(np.prod(list(f.n)))

        def nodes(a, dtype):
            """Pointer to node values (numpy: host; torch: host or device);
            a missing array passes NULL, which the library rejects."""
            if a is None:
                return None, 0
            if hasattr(a, "data_ptr"):
                t = a.contiguous()
                if t.element_size() != np.dtype(dtype).itemsize or not t.is_floating_point():
                    raise ValueError(f"node values must be {np.dtype(dtype).name}")
                if t.numel() != n_nodes:
                    raise ValueError(f"{t.numel()} node values for a grid of {n_nodes} nodes")
                keep.append(t)
                return t.data_ptr(), 1 if t.is_cuda else 0
            arr = np.ascontiguousarray(a, dtype)
            if arr.size != n_nodes:
                raise ValueError(f"{arr.size} node values for a grid of {n_nodes} nodes")
            keep.append(arr)
            return arr.ctypes.data, 0

        if f.kind == FIELD_GRID:
            fs.data, fs.data_on_device = nodes(f.data, np.float32)
        elif f.kind == FIELD_SOLUTE:
            fs.T, on_t = nodes(f.T, np.float64)
            fs.w, on_w = nodes(f.w, np.float64)
            if on_t != on_w:
                raise ValueError("SOLUTE: T and w must both be host or both device arrays")
            fs.data_on_device = on_t
            fs.liq_T, fs.liq_m = float(f.liq_T), float(f.liq_m)
        for k in ("q", "U", "alpha", "x_start", "x_end", "ys", "zs", "r_min", "dT_min"):
            setattr(fs, k, float(getattr(f, k)))
        self._check(self.lib.ge_set_thermal_field(self.ctx, C.byref(fs)), "ge_set_thermal_field")
        del keep

    def set_melting(self, on):
        """Melting by walk-back at the start of every step (off by default)."""
        self._check(self.lib.ge_set_melting(self.ctx, int(bool(on))), "ge_set_melting")

    def set_deposition_grid(self, n, origin=None, spacing=None):
        """Mushy-zone deposition grid (node-centred cells); n = None: off."""
        if n is None:
            self._check(self.lib.ge_set_deposition_grid(self.ctx, None, None, None),
                        "ge_set_deposition_grid")
            self.dep_n = None
            return
        nn = np.ascontiguousarray(n, np.int32)
        o = np.ascontiguousarray(origin, np.float64)
        sp = np.ascontiguousarray(spacing, np.float64)
        self._check(self.lib.ge_set_deposition_grid(self.ctx, _ptr(nn), _ptr(o), _ptr(sp)),
                    "ge_set_deposition_grid")
        self.dep_n = tuple(int(v) for v in nn)

    def mushy_counts(self) -> np.ndarray:
        """Reached lattice sites per deposition cell, shape (n2, n1, n0)."""
        n0, n1, n2 = self.dep_n
        out = np.zeros((n2, n1, n0), np.uint32)
        self.query_envelope(QUERY_MUSHY_COUNTS, out)
        return out

    def mushy_fraction(self) -> np.ndarray:
        """Mushy-zone fraction g^m per deposition cell, shape (n2, n1, n0)."""
        n0, n1, n2 = self.dep_n
        out = np.zeros((n2, n1, n0), np.float32)
        self.query_envelope(QUERY_MUSHY, out)
        return out

    def nucleate(self, xyz, dT_nuc, quat):
        xyz = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
        dT = np.ascontiguousarray(dT_nuc, np.float64).reshape(-1)
        quat = np.ascontiguousarray(quat, np.float64).reshape(-1, 4)
        self._check(self.lib.ge_nucleate(self.ctx, len(dT), _ptr(xyz), _ptr(dT), _ptr(quat)),
                    "ge_nucleate")
        self.n_sites += len(dT)

    def step(self, dt, n_steps=1, stats=True):
        st = ge_step_stats()
        rc = self.lib.ge_step(self.ctx, float(dt), int(n_steps), C.byref(st) if stats else None)
        self._check(rc, "ge_step")
        return st.as_dict() if stats else None

    def query_envelope(self, kind, out=None, args: Optional[ge_query_args] = None):
        """Raw query: returns the needed byte count, fills `out` (numpy array
        or torch tensor) when given."""
        need = C.c_size_t()
        if out is None:
            self._check(self.lib.ge_query_envelope(self.ctx, kind, C.byref(args) if args else None,
                                                   None, 0, C.byref(need)), "ge_query_envelope")
            return need.value
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else out.ctypes.data
        nbytes = out.numel() * out.element_size() if hasattr(out, "numel") else out.nbytes
        self._check(self.lib.ge_query_envelope(self.ctx, kind, C.byref(args) if args else None,
                                               C.c_void_p(ptr), nbytes, C.byref(need)),
                    "ge_query_envelope")
        return need.value

    def load_state(self, grain_centre, grain_quat, parts, claims, site_state, t, step):
        gc = np.ascontiguousarray(grain_centre, np.float64).reshape(-1, 3)
        gq = np.ascontiguousarray(grain_quat, np.float64).reshape(-1, 4)
        pg = np.ascontiguousarray(parts["grain"], np.int32)
        ps = np.ascontiguousarray(parts["site"], np.int32).reshape(-1, 3)
        pdir = np.ascontiguousarray(parts["dir"], np.int32)
        pss = np.ascontiguousarray(parts["s"], np.float32)
        pst = np.ascontiguousarray(parts["state"], np.int32)
        cg = np.ascontiguousarray(claims["grain"], np.int32)
        cs = np.ascontiguousarray(claims["site"], np.int32).reshape(-1, 3)
        cf = np.ascontiguousarray(claims["flags"], np.uint8)
        ss = np.ascontiguousarray(site_state, np.int32)
        st = ge_state_in()
        st.n_grains = len(gc)
        st.centre, st.quat = _ptr(gc), _ptr(gq)
        st.n_particles = len(pg)
        st.grain, st.site, st.dir, st.s, st.state = _ptr(pg), _ptr(ps), _ptr(pdir), _ptr(pss), _ptr(pst)
        st.n_claims = len(cg)
        st.c_grain, st.c_site, st.c_flags = _ptr(cg), _ptr(cs), _ptr(cf)
        st.n_sites = len(ss)
        st.site_state = _ptr(ss)
        st.t, st.step = float(t), int(step)
        self._check(self.lib.ge_load_state(self.ctx, C.byref(st)), "ge_load_state")

    def save_state(self) -> np.ndarray:
        """The whole state as a versioned blob (uint8 array in host memory)."""
        need = C.c_size_t()
        self._check(self.lib.ge_save_state(self.ctx, None, 0, C.byref(need)), "ge_save_state")
        out = np.zeros(need.value, np.uint8)
        self._check(self.lib.ge_save_state(self.ctx, _ptr(out), out.nbytes, C.byref(need)),
                    "ge_save_state")
        return out

    def restore_state(self, blob: np.ndarray):
        blob = np.ascontiguousarray(blob, np.uint8)
        self._check(self.lib.ge_restore_state(self.ctx, _ptr(blob), blob.nbytes),
                    "ge_restore_state")
        self.n_sites = state_check(blob)["n_sites"]

    def profile(self, on):
        self._check(self.lib.ge_profile(self.ctx, int(on)), "ge_profile")

    def profile_phase(self, phase):
        """Times one phase (by name or index; None stops) in every step,
        recorded step sequences included."""
        if phase is None:
            k = -1
        elif isinstance(phase, str):
            names = [self.lib.ge_phase_name(i).decode() for i in range(N_PHASES)]
            k = names.index(phase)
        else:
            k = int(phase)
        self._check(self.lib.ge_profile_phase(self.ctx, k), "ge_profile_phase")

    def profile_read(self):
        ms = (C.c_double * N_PHASES)()
        steps = C.c_int64()
        self._check(self.lib.ge_profile_read(self.ctx, ms, C.byref(steps)), "ge_profile_read")
        names = [self.lib.ge_phase_name(k).decode() for k in range(N_PHASES)]
        return dict(zip(names, list(ms))), steps.value

    def schedule(self):
        """Blocks per launch of each tunable kernel, by kernel name."""
        b = (C.c_int32 * N_TUNABLE)()
        self._check(self.lib.ge_get_schedule(self.ctx, b), "ge_get_schedule")
        names = [self.lib.ge_tunable_name(k).decode() for k in range(N_TUNABLE)]
        return dict(zip(names, list(b)))

    def set_schedule(self, blocks):
        """blocks: {kernel name: blocks}; kernels not named keep theirs."""
        names = [self.lib.ge_tunable_name(k).decode() for k in range(N_TUNABLE)]
        unknown = set(blocks) - set(names)
        if unknown:
            raise ValueError(f"unknown kernels {sorted(unknown)}")
        b = (C.c_int32 * N_TUNABLE)(*[int(blocks.get(n, 0)) for n in names])
        self._check(self.lib.ge_set_schedule(self.ctx, b), "ge_set_schedule")

    def use_graphs(self, on):
        self._check(self.lib.ge_use_graphs(self.ctx, int(bool(on))), "ge_use_graphs")

    def prepare_step(self, dt):
        self._check(self.lib.ge_prepare_step(self.ctx, float(dt)), "ge_prepare_step")

    def hold(self, on):
        self._check(self.lib.ge_hold(self.ctx, int(bool(on))), "ge_hold")

    def digest(self):
        """(active, stopped, claims) order-independent state digests."""
        out = np.zeros(3, np.uint64)
        self.query_envelope(QUERY_DIGEST, out)
        return tuple(int(v) for v in out)

    def set_model(self, a, b, theta, branching):
        av = (C.c_double * 2)(*[float(v) for v in a])
        bv = (C.c_double * 2)(*[float(v) for v in b])
        self._check(self.lib.ge_set_model(self.ctx, av, bv, float(theta), int(branching)),
                    "ge_set_model")

    # ---------------------------------------------------------- adjoint ---
    def adjoint_forward(self, dt, n_steps, ckpt_every=50):
        """Recorded run of n_steps steps (branching must be off); returns the
        number of tracked particles.  The adjoint workspace (a torch uint8
        tensor) is kept on the context until the next recorded run."""
        nbytes = C.c_size_t()
        self._check(self.lib.ge_adjoint_workspace_size(self.ctx, int(n_steps), int(ckpt_every),
                                                       C.byref(nbytes)),
                    "ge_adjoint_workspace_size")
        ws = getattr(self, "adj_workspace", None)
        if ws is None or ws.numel() < nbytes.value:
            self.adj_workspace = ws = self.torch.empty(nbytes.value, dtype=self.torch.uint8,
                                                       device=self.device)
        n = C.c_int64()
        self._check(self.lib.ge_adjoint_forward(self.ctx, float(dt), int(n_steps), int(ckpt_every),
                                                C.c_void_p(ws.data_ptr()), ws.numel(),
                                                C.byref(n)), "ge_adjoint_forward")
        self.adj_n = n.value
        return n.value

    def adjoint_positions(self):
        """Final positions of the tracked particles: torch float32 [n, 3] on the device."""
        out = self.torch.empty((self.adj_n, 3), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.ge_adjoint_positions(self.ctx, C.c_void_p(out.data_ptr()),
                                                  4 * out.numel(), 1), "ge_adjoint_positions")
        return out

    def adjoint_tracked(self) -> np.ndarray:
        out = np.zeros(self.adj_n, ADJOINT_DTYPE)
        self._check(self.lib.ge_adjoint_tracked(self.ctx, _ptr(out), out.nbytes),
                    "ge_adjoint_tracked")
        return out

    def adjoint_backward(self, dLdx):
        """(dL/da0, dL/da1, dL/dtheta) for dL/dx_N = dLdx, a torch float32
        [n, 3] tensor on the device or a numpy array."""
        g = (C.c_double * 3)()
        if isinstance(dLdx, np.ndarray):
            arr = np.ascontiguousarray(dLdx, np.float32).reshape(-1, 3)
            assert len(arr) == self.adj_n
            rc = self.lib.ge_adjoint_backward(self.ctx, _ptr(arr), 0, g)
        else:
            t = dLdx.detach().to(device=self.device, dtype=self.torch.float32).contiguous()
            assert tuple(t.shape) == (self.adj_n, 3)
            rc = self.lib.ge_adjoint_backward(self.ctx, C.c_void_p(t.data_ptr()), 1, g)
        self._check(rc, "ge_adjoint_backward")
        return tuple(g)

    def autotune(self, dt, steps_per_trial=2, restore=True):
        """Autotunes the launch schedule; with restore, every trial starts from
        the current state and the state is left unchanged (a device snapshot
        of the workspace's size is held during the call)."""
        b = (C.c_int32 * N_TUNABLE)()
        snap, ptr, n = None, None, 0
        if restore:
            n = workspace_size(self.params)
            snap = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
            ptr = C.c_void_p(snap.data_ptr())
        rc = self.lib.ge_autotune(self.ctx, float(dt), int(steps_per_trial), ptr, n, b)
        del snap
        self._check(rc, "ge_autotune")
        names = [self.lib.ge_tunable_name(k).decode() for k in range(N_TUNABLE)]
        return dict(zip(names, list(b)))

    # ---------------------------------------------------------- helpers ---
    def counts(self):
        st = ge_step_stats()
        buf = np.zeros(C.sizeof(ge_step_stats), np.uint8)
        self.query_envelope(QUERY_COUNTS, buf)
        C.memmove(C.addressof(st), buf.ctypes.data, C.sizeof(st))
        return st.as_dict()

    @staticmethod
    def _window(window):
        if window is None:
            return None
        lo, hi = window
        a = ge_query_args()
        a.n[:] = [1, 1, 1]
        a.origin[:] = [float(v) for v in lo]
        a.spacing[:] = [float(h - l) for l, h in zip(lo, hi)]
        return a

    def particles(self, window=None) -> np.ndarray:
        """Active and stopped particles; window = (lo, hi) restricts to a box."""
        a = self._window(window)
        need = self.query_envelope(QUERY_PARTICLES, args=a)
        out = np.zeros(need // PARTICLE_DTYPE.itemsize, PARTICLE_DTYPE)
        if need:
            self.query_envelope(QUERY_PARTICLES, out, args=a)
        return out

    def particles_noalloc(self, window=None, out=None):
        """Particles of a window through the allocation-free entry point
        (the library's static staging).  out: a host numpy array or a device
        tensor of PARTICLE_DTYPE records (uint8 bytes for a tensor), or None
        for a new host array."""
        a = self._window(window)
        need = C.c_size_t()
        self._check(self.lib.ge_query_particles_noalloc(
            self.ctx, C.byref(a) if a is not None else None, None, 0, C.byref(need)),
            "ge_query_particles_noalloc")
        n = need.value // PARTICLE_DTYPE.itemsize
        if out is None:
            out = np.zeros(n, PARTICLE_DTYPE)
        if isinstance(out, np.ndarray):
            ptr, nbytes = _ptr(out), out.nbytes
        else:
            ptr, nbytes = C.c_void_p(out.data_ptr()), out.numel() * out.element_size()
        self._check(self.lib.ge_query_particles_noalloc(
            self.ctx, C.byref(a) if a is not None else None, ptr, nbytes, C.byref(need)),
            "ge_query_particles_noalloc")
        return out, n

    def claims(self, window=None) -> np.ndarray:
        a = self._window(window)
        need = self.query_envelope(QUERY_CLAIMS, args=a)
        out = np.zeros(need // CLAIM_DTYPE.itemsize, CLAIM_DTYPE)
        if need:
            self.query_envelope(QUERY_CLAIMS, out, args=a)
        return out

    def site_states(self) -> np.ndarray:
        out = np.zeros(self.n_sites, np.int32)
        if self.n_sites:
            self.query_envelope(QUERY_SITES, out)
        return out

    def grains(self) -> np.ndarray:
        need = self.query_envelope(QUERY_GRAINS)
        out = np.zeros(need // 4, np.float32)
        if need:
            self.query_envelope(QUERY_GRAINS, out)
        return out.reshape(-1, 24)

    def grain_map(self, n, origin, spacing, device_out=False):
        a = ge_query_args()
        a.n[:] = [int(v) for v in n]
        a.origin[:] = [float(v) for v in origin]
        a.spacing[:] = [float(v) for v in spacing]
        if device_out:
            out = self.torch.zeros(int(np.prod(n)), dtype=self.torch.int32, device=self.device)
        else:
            out = np.zeros(int(np.prod(n)), np.uint32)
        self.query_envelope(QUERY_GRAIN_MAP, out, a)
        return out.reshape(int(n[2]), int(n[1]), int(n[0]))


class Batch:
    """Many contexts in one device workspace, advanced together by batched
    launches (ge_batch_*).  members[i] is a borrowed Context."""

    def __init__(self, params_list, device="cuda:0", stream=None):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        n = len(params_list)
        arr = (ge_params * n)(*params_list)
        nbytes = C.c_size_t()
        rc = self.lib.ge_batch_workspace_size(n, arr, C.byref(nbytes))
        if rc != GE_OK:
            raise GrainEnvError(rc, "ge_batch_workspace_size: invalid parameters")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = C.c_void_p()
        rc = self.lib.ge_batch_create(n, arr, C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                      C.c_void_p(self.stream.cuda_stream), C.byref(b))
        if rc != GE_OK:
            raise GrainEnvError(rc, "ge_batch_create failed")
        self.b = b
        self.members = []
        for i in range(n):
            p = C.c_void_p()
            self._check(self.lib.ge_batch_member(self.b, i, C.byref(p)), "ge_batch_member")
            self.members.append(Context.borrowed(p, params_list[i], self, device))

    def _check(self, rc, what):
        if rc != GE_OK:
            msg = self.lib.ge_batch_last_error(self.b)
            raise GrainEnvError(rc, f"{what}: {msg.decode() if msg else ''}")

    def step(self, dt, n_steps=1):
        st = (ge_step_stats * len(self.members))()
        self._check(self.lib.ge_batch_step(self.b, float(dt), int(n_steps), st), "ge_batch_step")
        return [s.as_dict() for s in st]

    def use_graphs(self, on):
        self._check(self.lib.ge_batch_use_graphs(self.b, int(bool(on))), "ge_batch_use_graphs")

    def blocks(self):
        b = (C.c_int32 * N_TUNABLE)()
        self._check(self.lib.ge_batch_get_blocks(self.b, b), "ge_batch_get_blocks")
        names = [self.lib.ge_tunable_name(k).decode() for k in range(N_TUNABLE)]
        return dict(zip(names, list(b)))

    def set_blocks(self, blocks):
        names = [self.lib.ge_tunable_name(k).decode() for k in range(N_TUNABLE)]
        b = (C.c_int32 * N_TUNABLE)(*[int(blocks.get(n, 0)) for n in names])
        self._check(self.lib.ge_batch_set_blocks(self.b, b), "ge_batch_set_blocks")

    def autotune(self, dt, steps_per_trial=1, restore=True):
        """Autotunes the shared launches; with restore, from a snapshot of the
        batch workspace that is restored at the end."""
        b = (C.c_int32 * N_TUNABLE)()
        snap, ptr, n = None, None, 0
        if restore:
            n = self.workspace.numel()
            snap = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
            ptr = C.c_void_p(snap.data_ptr())
        rc = self.lib.ge_batch_autotune(self.b, float(dt), int(steps_per_trial), ptr, n, b)
        del snap
        self._check(rc, "ge_batch_autotune")
        names = [self.lib.ge_tunable_name(k).decode() for k in range(N_TUNABLE)]
        return dict(zip(names, list(b)))

    def close(self):
        if getattr(self, "b", None):
            for m in self.members:
                m.ctx = None
            self.lib.ge_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
