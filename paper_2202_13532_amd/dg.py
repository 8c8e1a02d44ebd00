"""Thin ctypes binding of the C ABI in include/dg.h (same names, marshalling only).

Device memory and streams come from PyTorch; every computation runs in the
HIP library ``libdg.so`` built next to this file.  If the library is missing
the binding raises -- there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK, DG_ERR_INVALID, DG_ERR_UNSUPPORTED, DG_ERR_OOM, DG_ERR_DEVICE, DG_ERR_CFL, DG_ERR_NONFINITE = range(7)
DG_F32, DG_F64 = 0, 1
DG_VBC_PERIODIC, DG_VBC_ZERO_INFLOW = 0, 1
STATUS_NAMES = {0: "DG_OK", 1: "DG_ERR_INVALID", 2: "DG_ERR_UNSUPPORTED", 3: "DG_ERR_OOM",
                4: "DG_ERR_DEVICE", 5: "DG_ERR_CFL", 6: "DG_ERR_NONFINITE"}

EXPORTED = ["dg_workspace_bytes", "dg_init", "dg_destroy", "dg_rhs", "dg_poisson", "dg_rk_step",
            "dg_diagnostics", "dg_profile_step", "dg_dt_max", "dg_node_coords", "dg_last_error", "dg_basis",
            "dg_connection_tensor", "dg_courant_number", "dg_batch_workspace_bytes", "dg_batch_init",
            "dg_batch_destroy", "dg_batch_rk_step", "dg_batch_tune", "dg_batch_grid", "dg_batch_last_error"]


class dg_config(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("n", ctypes.c_int32), ("nelem", ctypes.c_int32 * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("omega_c", ctypes.c_double),
                ("pmax", ctypes.c_int32), ("storage", ctypes.c_int32), ("vbc", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class dg_diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("mass", ctypes.c_double), ("field_energy", ctypes.c_double),
                ("kinetic_energy", ctypes.c_double), ("l2sq", ctypes.c_double), ("max_abs_E", ctypes.c_double),
                ("finite", ctypes.c_int32), ("step", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """Load libdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdg.so not built at %s (run __graft_entry__.build())" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    cfgp = ctypes.POINTER(dg_config)
    diagp = ctypes.POINTER(dg_diag)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "dg_workspace_bytes": (S, [cfgp]),
        "dg_init": (I, [cfgp, P, S, P, ctypes.POINTER(P)]),
        "dg_destroy": (I, [P]),
        "dg_rhs": (I, [P, P, P, P]),
        "dg_poisson": (I, [P, P, P, P]),
        "dg_rk_step": (I, [P, P, D, I, diagp]),
        "dg_diagnostics": (I, [P, P, diagp]),
        "dg_profile_step": (I, [P, P, D, I, dp]),
        "dg_dt_max": (D, [P, D]),
        "dg_node_coords": (I, [P, I, dp]),
        "dg_last_error": (ctypes.c_char_p, [P]),
        "dg_basis": (I, [I, dp, dp, dp, dp, dp]),
        "dg_connection_tensor": (I, [I, I, D, D, I, dp]),
        "dg_courant_number": (D, [I]),
        "dg_batch_workspace_bytes": (S, [cfgp, I]),
        "dg_batch_init": (I, [cfgp, I, P, S, P, ctypes.POINTER(P)]),
        "dg_batch_destroy": (I, [P]),
        "dg_batch_rk_step": (I, [P, ctypes.POINTER(P), dp, I, diagp]),
        "dg_batch_tune": (I, [P, ctypes.POINTER(P), dp, I, dp]),
        "dg_batch_grid": (I, [P]),
        "dg_batch_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status, ctx=None):
    if status != DG_OK:
        msg = lib().dg_last_error(ctx).decode()
        raise DGError(status, msg)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_config(nv, n, nelem, lo, hi, omega_c=0.0, pmax=0, storage="f32", vbc="periodic"):
    c = dg_config()
    c.nv, c.n = nv, n
    for a in range(3):
        c.nelem[a] = int(nelem[a]) if a < len(nelem) else 0
        c.lo[a] = float(lo[a]) if a < len(lo) else 0.0
        c.hi[a] = float(hi[a]) if a < len(hi) else 0.0
    c.omega_c = float(omega_c)
    c.pmax = int(pmax)
    c.storage = DG_F64 if storage in ("f64", DG_F64) else DG_F32
    c.vbc = DG_VBC_ZERO_INFLOW if vbc in ("zero_inflow", DG_VBC_ZERO_INFLOW) else DG_VBC_PERIODIC
    c.reserved = 0
    return c


# ---------------- C ABI, same names ----------------

def dg_workspace_bytes(cfg):
    return int(lib().dg_workspace_bytes(ctypes.byref(cfg)))


def dg_init(cfg, workspace, stream=None):
    ctx = ctypes.c_void_p()
    st = lib().dg_init(ctypes.byref(cfg), _ptr(workspace), workspace.numel() * workspace.element_size(),
                       ctypes.c_void_p(stream), ctypes.byref(ctx))
    _check(st, None)
    return ctx


def dg_destroy(ctx):
    _check(lib().dg_destroy(ctx), None)


def dg_rhs(ctx, f, E, rhs):
    _check(lib().dg_rhs(ctx, _ptr(f), _ptr(E), _ptr(rhs)), ctx)


def dg_poisson(ctx, f, E, coeffs=None):
    _check(lib().dg_poisson(ctx, _ptr(f), _ptr(E), _ptr(coeffs)), ctx)


def dg_rk_step(ctx, f, dt, nsteps, diag=False):
    recs = (dg_diag * nsteps)() if (diag and nsteps > 0) else None
    st = lib().dg_rk_step(ctx, _ptr(f), float(dt), int(nsteps), recs)
    _check(st, ctx)
    return [r.as_dict() for r in recs] if recs is not None else None


def dg_profile_step(ctx, f, dt, nsteps):
    ms = np.zeros(6 * max(int(nsteps), 0), dtype=np.float64)
    _check(lib().dg_profile_step(ctx, _ptr(f), float(dt), int(nsteps), _dptr(ms)), ctx)
    return ms.reshape(-1, 6)


def dg_diagnostics(ctx, f):
    d = dg_diag()
    _check(lib().dg_diagnostics(ctx, _ptr(f), ctypes.byref(d)), ctx)
    return d.as_dict()


def dg_dt_max(ctx, max_abs_E):
    return float(lib().dg_dt_max(ctx, float(max_abs_E)))


def dg_node_coords(ctx, axis, count):
    out = np.zeros(count, dtype=np.float64)
    _check(lib().dg_node_coords(ctx, int(axis), _dptr(out)), ctx)
    return out


def dg_last_error(ctx=None):
    return lib().dg_last_error(ctx).decode()


def dg_basis(n):
    xi, w = np.zeros(n), np.zeros(n)
    ups, xf, dm = np.zeros(n * n), np.zeros(2 * n), np.zeros(n * n)
    _check(lib().dg_basis(n, _dptr(xi), _dptr(w), _dptr(ups), _dptr(xf), _dptr(dm)))
    return {"xi": xi, "w": w, "Ups": ups.reshape(n, n), "Xi": xf.reshape(n, 2), "D": dm.reshape(n, n)}


def dg_connection_tensor(n, nelem, lo, hi, pmax):
    out = np.zeros(2 * pmax * nelem * n)
    _check(lib().dg_connection_tensor(n, nelem, lo, hi, pmax, _dptr(out)))
    c = out.reshape(pmax, nelem, n, 2)
    return c[..., 0] + 1j * c[..., 1]


def dg_courant_number(n):
    return float(lib().dg_courant_number(n))


# ---------------- convenience wrapper (memory + stream plumbing) ----------------

class Solver:
    """Owns a device workspace (torch uint8) and a library context."""

    def __init__(self, nv, n, nelem, lo, hi, omega_c=0.0, pmax=0, storage="f32", vbc="periodic",
                 device="cuda"):
        import torch
        self.torch = torch
        self.cfg = make_config(nv, n, nelem, lo, hi, omega_c, pmax, storage, vbc)
        nbytes = dg_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise DGError(DG_ERR_INVALID, "invalid configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + nbytes]
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.ctx = dg_init(self.cfg, self.ws, stream)
        self.nv, self.n = nv, n
        self.nelem = list(nelem[: 1 + nv])
        self.shape = tuple(s for N in self.nelem for s in (N, n))
        self.dtype = torch.float64 if storage in ("f64", DG_F64) else torch.float32
        self.pmax = pmax if pmax > 0 else nelem[0]

    def close(self):
        if getattr(self, "ctx", None) is not None:
            dg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_state(self, f):
        t = self.torch
        if not isinstance(f, t.Tensor) or f.device.type != "cuda":
            raise DGError(DG_ERR_INVALID, "state must be a device tensor")
        if f.dtype != self.dtype or not f.is_contiguous() or tuple(f.shape) != self.shape:
            raise DGError(DG_ERR_INVALID, "state must be contiguous %s of shape %s" % (self.dtype, self.shape))

    def nodes(self, axis):
        return dg_node_coords(self.ctx, axis, self.nelem[axis] * self.n).reshape(self.nelem[axis], self.n)

    def empty_state(self):
        return self.torch.empty(self.shape, dtype=self.dtype, device=self.device)

    def rhs(self, f, E=None, out=None):
        self._check_state(f)
        out = self.empty_state() if out is None else out
        self._check_state(out)
        dg_rhs(self.ctx, f, E, out)
        return out

    def poisson(self, f, coeffs=False):
        self._check_state(f)
        E = self.torch.empty(self.nelem[0] * self.n, dtype=self.torch.float64, device=self.device)
        c = self.torch.empty(2 * self.pmax, dtype=self.torch.float64, device=self.device) if coeffs else None
        dg_poisson(self.ctx, f, E, c)
        return (E, c) if coeffs else E

    def step(self, f, dt, nsteps=1, diag=False):
        self._check_state(f)
        return dg_rk_step(self.ctx, f, dt, nsteps, diag)

    def profile_step(self, f, dt, nsteps=1):
        self._check_state(f)
        return dg_profile_step(self.ctx, f, dt, nsteps)

    def diagnostics(self, f):
        self._check_state(f)
        return dg_diagnostics(self.ctx, f)

    def dt_max(self, max_abs_E=0.0):
        return dg_dt_max(self.ctx, max_abs_E)


# ---------------- batches ----------------

def _bcheck(status, b=None):
    if status != DG_OK:
        raise DGError(status, lib().dg_batch_last_error(b).decode())


def dg_batch_workspace_bytes(cfgs):
    arr = (dg_config * len(cfgs))(*cfgs)
    return int(lib().dg_batch_workspace_bytes(arr, len(cfgs)))


def dg_batch_init(cfgs, workspace, stream=None):
    arr = (dg_config * len(cfgs))(*cfgs)
    b = ctypes.c_void_p()
    st = lib().dg_batch_init(arr, len(cfgs), _ptr(workspace), workspace.numel() * workspace.element_size(),
                             ctypes.c_void_p(stream), ctypes.byref(b))
    _bcheck(st, None)
    return b


def dg_batch_destroy(b):
    _bcheck(lib().dg_batch_destroy(b), None)


def _ptr_array(states):
    return (ctypes.c_void_p * len(states))(*[t.data_ptr() for t in states])


def dg_batch_rk_step(b, states, dts, nsteps, diag=False):
    dt = np.ascontiguousarray(dts, dtype=np.float64)
    recs = (dg_diag * (len(states) * nsteps))() if (diag and nsteps > 0) else None
    _bcheck(lib().dg_batch_rk_step(b, _ptr_array(states), _dptr(dt), int(nsteps), recs), b)
    if recs is None:
        return None
    return [[recs[r * nsteps + k].as_dict() for k in range(nsteps)] for r in range(len(states))]


def dg_batch_tune(b, states, dts, reps):
    dt = np.ascontiguousarray(dts, dtype=np.float64)
    best = np.zeros(1)
    _bcheck(lib().dg_batch_tune(b, _ptr_array(states), _dptr(dt), int(reps), _dptr(best)), b)
    return float(best[0])


def dg_batch_grid(b):
    return int(lib().dg_batch_grid(b))


class Batch:
    """Many independent runs stepped by one persistent launch per RK stage."""

    def __init__(self, configs, device="cuda"):
        import torch
        self.torch = torch
        self.cfgs = list(configs)
        nbytes = dg_batch_workspace_bytes(self.cfgs)
        if nbytes == 0:
            raise DGError(DG_ERR_INVALID, "invalid batch configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + nbytes]
        self.b = dg_batch_init(self.cfgs, self.ws, torch.cuda.current_stream(self.device).cuda_stream)
        self.shapes = []
        for c in self.cfgs:
            ne = [c.nelem[a] for a in range(1 + c.nv)]
            self.shapes.append(tuple(x for N in ne for x in (N, c.n)))

    def close(self):
        if getattr(self, "b", None) is not None:
            dg_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, states):
        if len(states) != len(self.cfgs):
            raise DGError(DG_ERR_INVALID, "one state per run")
        for t, shp in zip(states, self.shapes):
            if t.dtype != self.torch.float32 or not t.is_contiguous() or tuple(t.shape) != shp or t.device.type != "cuda":
                raise DGError(DG_ERR_INVALID, "state must be contiguous float32 of shape %s" % (shp,))

    def step(self, states, dts, nsteps=1, diag=False):
        self._check(states)
        return dg_batch_rk_step(self.b, states, dts, nsteps, diag)

    def tune(self, states, dts, reps=3):
        self._check(states)
        return dg_batch_tune(self.b, states, dts, reps)

    @property
    def grid(self):
        return dg_batch_grid(self.b)
