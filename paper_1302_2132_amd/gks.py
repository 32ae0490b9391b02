"""ctypes binding of libgks.so with the same names as the C ABI (include/gks.h).

Argument marshalling only: no arithmetic of the scheme happens here.  Device memory
(workspaces) comes from PyTorch tensors and streams are PyTorch's HIP streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libgks.so")

GKS_OK, GKS_ERR_ARG, GKS_ERR_NONPHYSICAL, GKS_ERR_NOMEM, GKS_ERR_DEVICE, GKS_ERR_STATE = range(6)
_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_NONPHYSICAL", 3: "ERR_NOMEM", 4: "ERR_DEVICE", 5: "ERR_STATE"}
BC = {"periodic": 0, "wall": 1, "dirichlet": 2, "profile": 3, "outflow": 4}
PRECISION = {"fp64": 0, "fp32_flux": 1}
FIELD = {"cons": 0, "prim": 1, "strain": 2, "turb": 3, "eps": 4, "tau": 5, "turb_cons": 6}
EPS_MODE = {"dt": 0, "tauhat": 1}
RECON = {"muscl2": 0, "muscl3": 1, "weno5": 2}

# every entry point declared in include/gks.h
EXPORTED = (
    "gks_workspace_bytes", "gks_init", "gks_step", "gks_residual", "gks_fields",
    "gks_state_device_ptr", "gks_destroy", "gks_last_error", "gks_face_flops", "gks_kw_face_flops",
    "gks_face_flops_multid", "gks_face_flops_recon",
    "gks_set_timing", "gks_kernel_times",
    "gks_batch_workspace_bytes", "gks_batch_create", "gks_batch_set_members", "gks_batch_step",
    "gks_batch_capture", "gks_batch_set_launch", "gks_batch_status", "gks_batch_destroy",
    "gks_batch_create_static", "gks_batch_capture_steps", "gks_resume",
)
GKS_BATCH_STATIC_CAPACITY = 256


class GksError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"gks {_NAMES.get(status, status)}: {msg}")
        self.status = status


class gks_config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("n", C.c_int64 * 3),
        ("xf", C.c_void_p * 3),
        ("bc", (C.c_int32 * 2) * 3),
        ("bc_data", (C.c_void_p * 2) * 3),
        ("gamma", C.c_double), ("prandtl", C.c_double), ("mu", C.c_double), ("c_a", C.c_double),
        ("c_mu", C.c_double), ("cfl", C.c_double), ("t_end", C.c_double),
        ("precision", C.c_int32),
        ("max_steps", C.c_int64),
        ("turb_transport", C.c_int32),
        ("eps_mode", C.c_int32),
        ("recon", C.c_int32),
        ("multi_d", C.c_int32),
        ("res_tol", C.c_double),
    ]


_lib = None


def lib():
    """Load libgks.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise RuntimeError(f"libgks.so not found at {lib_path}: build it with "
                               "`python -m paper_1302_2132_amd.build` (hipcc, gfx950)")
        # Load torch's HIP runtime first: libgks.so then binds to the same runtime (its
        # libamdhip64.so.7 dependency matches the already loaded soname).  Loaded the other
        # way round, torch would bring a second runtime into the process and device
        # pointers and streams would not be shared between the two.
        import torch  # noqa: F401
        L = C.CDLL(lib_path)
        vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
        sz = C.POINTER(C.c_size_t)
        L.gks_workspace_bytes.argtypes = [C.POINTER(gks_config), sz]
        L.gks_init.argtypes = [C.POINTER(gks_config), vp, C.c_size_t, vp, dp, dp, dp, C.POINTER(vp)]
        L.gks_step.argtypes = [vp, i32]
        L.gks_residual.argtypes = [vp, dp, dp, dp, dp, C.POINTER(i64)]
        L.gks_fields.argtypes = [vp, i32, dp]
        L.gks_state_device_ptr.argtypes = [vp, C.POINTER(vp)]
        L.gks_resume.argtypes = [vp, dp, dp, C.c_double, C.c_double, i64, dp]
        L.gks_destroy.argtypes = [vp]
        L.gks_last_error.argtypes = [vp]
        L.gks_last_error.restype = C.c_char_p
        L.gks_face_flops.argtypes = [i32, i32, dp]
        L.gks_kw_face_flops.argtypes = [dp]
        L.gks_face_flops_multid.argtypes = [i32, dp]
        L.gks_face_flops_recon.argtypes = [i32, i32, dp]
        L.gks_set_timing.argtypes = [vp, i32]
        L.gks_kernel_times.argtypes = [vp, dp, C.POINTER(i64)]
        L.gks_batch_workspace_bytes.argtypes = [i32, sz]
        L.gks_batch_create.argtypes = [C.POINTER(vp), i32, i32, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.gks_batch_set_members.argtypes = [vp, C.POINTER(vp), i32]
        L.gks_batch_step.argtypes = [vp, i32]
        L.gks_batch_capture.argtypes = [vp]
        L.gks_batch_set_launch.argtypes = [vp, i32, i32, i32]
        L.gks_batch_status.argtypes = [vp, C.POINTER(i64), dp, dp, dp, C.POINTER(i32)]
        L.gks_batch_destroy.argtypes = [vp]
        L.gks_batch_create_static.argtypes = [C.POINTER(vp), i32, i32, vp, C.POINTER(vp)]
        L.gks_batch_capture_steps.argtypes = [vp, i32]
        for nm in EXPORTED:
            if nm != "gks_last_error":
                getattr(L, nm).restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(st, h=None):
    if st != GKS_OK:
        msg = lib().gks_last_error(h).decode(errors="replace")
        raise GksError(st, msg)


class _Cfg:
    """A gks_config plus the host arrays its pointers refer to."""

    def __init__(self, case):
        self.keep = []
        c = gks_config()
        c.dim = case.dim
        for d in range(3):
            c.n[d] = int(case.n[d]) if d < case.dim else 1
        for d in range(case.dim):
            xf = np.ascontiguousarray(case.xf[d], dtype=np.float64)
            self.keep.append(xf)
            c.xf[d] = xf.ctypes.data
            for s in range(2):
                c.bc[d][s] = BC[case.bc[d][s]]
                bd = case.bc_data[d][s]
                if bd is not None:
                    bd = np.ascontiguousarray(bd, dtype=np.float64)
                    self.keep.append(bd)
                    c.bc_data[d][s] = bd.ctypes.data
        c.gamma, c.prandtl, c.mu, c.c_a = case.gamma, case.prandtl, case.mu, case.c_a
        c.c_mu, c.cfl, c.t_end = case.c_mu, case.cfl, case.t_end
        c.precision = PRECISION[case.precision]
        c.max_steps = int(getattr(case, "max_steps", 0) or 0)
        c.turb_transport = 1 if getattr(case, "kw_transport", False) else 0
        c.eps_mode = EPS_MODE[getattr(case, "eps_mode", "dt")]
        c.recon = RECON[getattr(case, "recon", "muscl2")]
        c.multi_d = 1 if getattr(case, "multi_d", False) else 0
        c.res_tol = float(getattr(case, "res_tol", 0.0) or 0.0)
        self.c = c


def config_from_case(case):
    return _Cfg(case)


# ----------------------------------------------------------------------------------
# thin wrappers with the C names
# ----------------------------------------------------------------------------------
def gks_workspace_bytes(cfg):
    out = C.c_size_t(0)
    _check(lib().gks_workspace_bytes(C.byref(cfg.c), C.byref(out)))
    return int(out.value)


def gks_init(cfg, workspace_ptr, nbytes, stream_ptr, W, k, omega):
    W = np.ascontiguousarray(W, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().gks_init(C.byref(cfg.c), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream_ptr),
                          _dp(W), _dp(k), _dp(omega), C.byref(h)))
    return h


def gks_step(h, nsteps):
    _check(lib().gks_step(h, int(nsteps)), h)


def gks_residual(h, nv):
    res, res1 = np.zeros(nv), np.zeros(nv)
    dt, t = C.c_double(0), C.c_double(0)
    steps = C.c_int64(0)
    st = lib().gks_residual(h, _dp(res), _dp(res1), C.byref(dt), C.byref(t), C.byref(steps))
    _check(st, h)
    return {"res": res, "res_first": res1, "dt": dt.value, "t": t.value, "steps": int(steps.value)}


def gks_fields(h, which, shape):
    out = np.zeros(shape, dtype=np.float64)
    _check(lib().gks_fields(h, FIELD[which], _dp(out)), h)
    return out


def gks_resume(h, res, res_first, dt_last, t, steps_done, turb_cons=None):
    res = None if res is None else np.ascontiguousarray(res, dtype=np.float64)
    res_first = None if res_first is None else np.ascontiguousarray(res_first, dtype=np.float64)
    tc = None if turb_cons is None else np.ascontiguousarray(turb_cons, dtype=np.float64)
    _check(lib().gks_resume(h, None if res is None else _dp(res), None if res_first is None else _dp(res_first),
                            float(dt_last), float(t), int(steps_done), None if tc is None else _dp(tc)), h)


def gks_state_device_ptr(h):
    p = C.c_void_p()
    _check(lib().gks_state_device_ptr(h, C.byref(p)), h)
    return int(p.value)


def gks_destroy(h):
    return lib().gks_destroy(h)


def gks_last_error(h=None):
    return lib().gks_last_error(h).decode(errors="replace")


def gks_face_flops(dim, precision="fp64"):
    out = C.c_double(0)
    _check(lib().gks_face_flops(int(dim), PRECISION[precision], C.byref(out)))
    return out.value


def gks_face_flops_multid(dim):
    out = C.c_double(0)
    _check(lib().gks_face_flops_multid(int(dim), C.byref(out)))
    return out.value


def gks_face_flops_recon(dim, recon):
    out = C.c_double(0)
    _check(lib().gks_face_flops_recon(int(dim), RECON[recon], C.byref(out)))
    return out.value


def gks_kw_face_flops():
    out = C.c_double(0)
    _check(lib().gks_kw_face_flops(C.byref(out)))
    return out.value


def gks_set_timing(h, enable):
    _check(lib().gks_set_timing(h, 1 if enable else 0), h)


def gks_kernel_times(h):
    ms = np.zeros(4)
    n = C.c_int64(0)
    _check(lib().gks_kernel_times(h, _dp(ms), C.byref(n)), h)
    return {"strain_ms": ms[0], "face_ms": ms[1], "update_ms": ms[2], "finish_ms": ms[3], "steps": int(n.value)}


def gks_batch_workspace_bytes(capacity):
    out = C.c_size_t(0)
    _check(lib().gks_batch_workspace_bytes(int(capacity), C.byref(out)))
    return int(out.value)


def _handles(hs):
    arr = (C.c_void_p * max(len(hs), 1))()
    for i, h in enumerate(hs):
        arr[i] = h.value if isinstance(h, C.c_void_p) else h
    return arr


def gks_batch_create(hs, capacity, workspace_ptr, nbytes, stream_ptr):
    b = C.c_void_p()
    _check(lib().gks_batch_create(_handles(hs), len(hs), int(capacity), C.c_void_p(workspace_ptr), nbytes,
                                  C.c_void_p(stream_ptr), C.byref(b)))
    return b


def gks_batch_create_static(hs, capacity, stream_ptr):
    b = C.c_void_p()
    _check(lib().gks_batch_create_static(_handles(hs), len(hs), int(capacity), C.c_void_p(stream_ptr),
                                         C.byref(b)))
    return b


def gks_batch_set_members(b, hs):
    _check(lib().gks_batch_set_members(b, _handles(hs), len(hs)))


def gks_batch_step(b, nsteps):
    _check(lib().gks_batch_step(b, int(nsteps)))


def gks_batch_capture(b):
    _check(lib().gks_batch_capture(b))


def gks_batch_capture_steps(b, steps):
    _check(lib().gks_batch_capture_steps(b, int(steps)))


def gks_batch_set_launch(b, kind, grid, tile=0):
    _check(lib().gks_batch_set_launch(b, int(kind), int(grid), int(tile)))


def gks_batch_status(b, count):
    steps = np.zeros(max(count, 1), dtype=np.int64)
    res = np.zeros(5 * max(count, 1))
    res1 = np.zeros(5 * max(count, 1))
    t = np.zeros(max(count, 1))
    state = np.zeros(max(count, 1), dtype=np.int32)
    _check(lib().gks_batch_status(b, steps.ctypes.data_as(C.POINTER(C.c_int64)), _dp(res), _dp(res1), _dp(t),
                                  state.ctypes.data_as(C.POINTER(C.c_int32))))
    return {"steps": steps[:count], "res": res[:5 * count].reshape(count, 5),
            "res_first": res1[:5 * count].reshape(count, 5), "t": t[:count], "state": state[:count]}


def gks_batch_destroy(b):
    return lib().gks_batch_destroy(b)


# ----------------------------------------------------------------------------------
# convenience objects (torch for device memory and streams)
# ----------------------------------------------------------------------------------
def _torch_stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream, int(stream.cuda_stream)


class Solver:
    """One solve: workspace tensor + handle.  `case` is an inputs.cases.Case."""

    def __init__(self, case, device="cuda:0", stream=None, resume=None):
        """`resume`: a dict from checkpoint() of a solve of the same case; the new solve
        continues it exactly."""
        import torch
        lib()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required (no CPU fallback)")
        self.case = case
        self.cfg = config_from_case(case)
        self.nbytes = gks_workspace_bytes(self.cfg)
        self.h = None
        W = case.W if resume is None else resume["W"]
        with torch.cuda.device(device):
            self.stream, sp = _torch_stream(stream)
            self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
            self.h = gks_init(self.cfg, self.ws.data_ptr(), self.nbytes, sp, W, case.k, case.omega)
            if resume is not None:
                gks_resume(self.h, resume["res"], resume["res_first"], resume["dt"], resume["t"], resume["steps"],
                           resume.get("turb_cons"))
        self.nv = case.nvar

    def checkpoint(self):
        """What a resumed solve needs: the conservative state, with transport rho k and rho
        omega, and the time, step count and residuals."""
        ck = dict(self.residual())
        ck["W"] = self.fields("cons")
        if getattr(self.case, "kw_transport", False):
            ck["turb_cons"] = self.fields("turb_cons")
        return ck

    def step(self, n=1):
        gks_step(self.h, n)

    def residual(self):
        return gks_residual(self.h, self.nv)

    def fields(self, which="cons"):
        """cons / prim: (nvar, nz, ny, nx); strain, eps, tau: (nz, ny, nx); turb: (2, nz, ny, nx), k and omega."""
        shape = {"strain": self.case.k.shape, "eps": self.case.k.shape, "tau": self.case.k.shape,
                 "turb": (2,) + self.case.k.shape, "turb_cons": (2,) + self.case.k.shape}.get(which, self.case.W.shape)
        return gks_fields(self.h, which, shape)

    def close(self):
        if self.h is not None:
            st = gks_destroy(self.h)
            self.h = None
            return st
        return GKS_OK

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Persistent-kernel batch over existing Solvers (their handles and workspaces).  With
    static=True the batch takes no workspace of its own (gks_batch_create_static)."""

    def __init__(self, solvers, capacity=None, device="cuda:0", stream=None, static=False):
        import torch
        self.solvers = list(solvers)
        self.capacity = capacity or max(len(self.solvers), 1)
        with torch.cuda.device(device):
            # a stream of its own: the null stream cannot be captured into a graph
            if stream is None:
                stream = torch.cuda.Stream(device=device)
            self.stream, sp = _torch_stream(stream)
            if static:
                self.ws = None
                self.b = gks_batch_create_static([s.h for s in self.solvers], self.capacity, sp)
            else:
                nbytes = gks_batch_workspace_bytes(self.capacity)
                self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
                self.b = gks_batch_create([s.h for s in self.solvers], self.capacity, self.ws.data_ptr(), nbytes,
                                          sp)

    def set_members(self, solvers):
        self.solvers = list(solvers)
        gks_batch_set_members(self.b, [s.h for s in self.solvers])

    def capture(self, steps=1):
        """Capture `steps` consecutive steps as one graph (replayed by step())."""
        if steps == 1:
            gks_batch_capture(self.b)
        else:
            gks_batch_capture_steps(self.b, steps)

    def set_launch(self, kind, grid, tile=0):
        gks_batch_set_launch(self.b, kind, grid, tile)

    def step(self, n=1):
        gks_batch_step(self.b, n)

    def status(self):
        return gks_batch_status(self.b, len(self.solvers))

    def close(self):
        if self.b is not None:
            gks_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
