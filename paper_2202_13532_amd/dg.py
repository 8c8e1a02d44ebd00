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
DG_LAYOUT_DENSE, DG_LAYOUT_VPAD = 0, 1
STATUS_NAMES = {0: "DG_OK", 1: "DG_ERR_INVALID", 2: "DG_ERR_UNSUPPORTED", 3: "DG_ERR_OOM",
                4: "DG_ERR_DEVICE", 5: "DG_ERR_CFL", 6: "DG_ERR_NONFINITE"}

EXPORTED = ["dg_workspace_bytes", "dg_init", "dg_destroy", "dg_rhs", "dg_poisson", "dg_rk_step",
            "dg_diagnostics", "dg_profile_step", "dg_dt_max", "dg_node_coords", "dg_last_error", "dg_basis",
            "dg_connection_tensor", "dg_courant_number", "dg_batch_workspace_bytes", "dg_batch_init",
            "dg_batch_destroy", "dg_batch_rk_step", "dg_batch_tune", "dg_batch_grid", "dg_batch_last_error",
            "dg_nn_workspace_bytes", "dg_nn_init", "dg_nn_destroy", "dg_nn_param_count", "dg_nn_input_ld",
            "dg_nn_set_params", "dg_nn_get_params", "dg_nn_forward", "dg_nn_loss_grad", "dg_nn_adamw",
            "dg_projection_matrix", "dg_project", "dg_nn_features", "dg_nn_features_raw", "dg_nn_to_elements",
            "dg_nn_column_stats", "dg_nn_rk_step", "dg_nn_last_error", "dg_state_elems", "dg_state_pack",
            "dg_state_unpack", "dg_rhs_static", "dg_set_background", "dg_fourier", "dg_filter_x",
            "dg_profile_copy", "dg_batch_choice", "dg_batch_set_choice", "dg_nn_set_fused"]


class dg_config(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("n", ctypes.c_int32), ("nelem", ctypes.c_int32 * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("omega_c", ctypes.c_double),
                ("pmax", ctypes.c_int32), ("storage", ctypes.c_int32), ("vbc", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


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
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(ctypes.c_int32)
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
        "dg_nn_workspace_bytes": (S, [ip, I, I]),
        "dg_nn_init": (I, [ip, I, I, P, S, P, ctypes.POINTER(P)]),
        "dg_nn_destroy": (I, [P]),
        "dg_nn_param_count": (ctypes.c_int64, [P]),
        "dg_nn_input_ld": (I, [P]),
        "dg_nn_set_params": (I, [P, fp]),
        "dg_nn_get_params": (I, [P, fp]),
        "dg_nn_forward": (I, [P, P, I, P]),
        "dg_nn_set_fused": (I, [P, I]),
        "dg_nn_loss_grad": (I, [P, P, P, I, dp, fp]),
        "dg_nn_adamw": (I, [P, ctypes.c_float, ctypes.c_float]),
        "dg_projection_matrix": (I, [I, I, I, dp]),
        "dg_project": (I, [P, P, P, P]),
        "dg_nn_features": (I, [P, P, P, P, P, P, P]),
        "dg_nn_features_raw": (I, [P, P, P, I, P]),
        "dg_nn_to_elements": (I, [P, P, P, ctypes.c_float, I, P]),
        "dg_nn_column_stats": (I, [P, P, ctypes.c_int64, I, dp, dp]),
        "dg_nn_rk_step": (I, [P, P, P, P, ctypes.c_float, P, D, I, diagp]),
        "dg_nn_last_error": (ctypes.c_char_p, [P]),
        "dg_state_elems": (S, [P]),
        "dg_state_pack": (I, [P, P, P]),
        "dg_state_unpack": (I, [P, P, P]),
        "dg_rhs_static": (I, [cfgp, P, P, P, P]),
        "dg_set_background": (I, [P, dp]),
        "dg_fourier": (I, [P, P, P]),
        "dg_filter_x": (I, [P, dp, P, P]),
        "dg_profile_copy": (I, [P, P, P, I, I, dp]),
        "dg_batch_choice": (I, [P, ip]),
        "dg_batch_set_choice": (I, [P, ip, I]),
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


def make_config(nv, n, nelem, lo, hi, omega_c=0.0, pmax=0, storage="f32", vbc="periodic", layout="dense"):
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
    c.layout = DG_LAYOUT_VPAD if layout in ("vpad", DG_LAYOUT_VPAD) else DG_LAYOUT_DENSE
    return c


def state_shape(cfg):
    """Tensor shape of a state of cfg's layout: [N0, n, N1, n, ...] dense, or
    [Nx, n, Nu, n, 64 C] with padded v rows (C = ceil(Nv / floor(64 / n)))."""
    ne = [cfg.nelem[a] for a in range(1 + cfg.nv)]
    if cfg.layout == DG_LAYOUT_VPAD:
        tv = 64 // cfg.n
        return (ne[0], cfg.n, ne[1], cfg.n, 64 * ((ne[2] + tv - 1) // tv))
    return tuple(x for N in ne for x in (N, cfg.n))


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


def dg_rhs_static(cfg, f, E, rhs, stream=None):
    _check(lib().dg_rhs_static(ctypes.byref(cfg), _ptr(f), _ptr(E), _ptr(rhs), ctypes.c_void_p(stream)), None)


def dg_profile_copy(ctx, f_in, f_out, pattern, reps):
    ms = np.zeros(1)
    _check(lib().dg_profile_copy(ctx, _ptr(f_in), _ptr(f_out), int(pattern), int(reps), _dptr(ms)), ctx)
    return float(ms[0])


def dg_fourier(ctx, g, coeffs):
    _check(lib().dg_fourier(ctx, _ptr(g), _ptr(coeffs)), ctx)


def dg_filter_x(ctx, sigma, f_in, f_out):
    sg = np.ascontiguousarray(sigma, dtype=np.float64)
    _check(lib().dg_filter_x(ctx, _dptr(sg), _ptr(f_in), _ptr(f_out)), ctx)


def dg_set_background(ctx, f0=None):
    if f0 is None:
        _check(lib().dg_set_background(ctx, None), ctx)
        return
    a = np.ascontiguousarray(f0, dtype=np.float64)
    _check(lib().dg_set_background(ctx, _dptr(a)), ctx)


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


def dg_state_elems(ctx):
    return int(lib().dg_state_elems(ctx))


def dg_state_pack(ctx, dense, state):
    _check(lib().dg_state_pack(ctx, _ptr(dense), _ptr(state)), ctx)


def dg_state_unpack(ctx, state, dense):
    _check(lib().dg_state_unpack(ctx, _ptr(state), _ptr(dense)), ctx)


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
                 device="cuda", layout="dense"):
        import torch
        self.torch = torch
        self.cfg = make_config(nv, n, nelem, lo, hi, omega_c, pmax, storage, vbc, layout)
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
        self.dense_shape = tuple(s for N in self.nelem for s in (N, n))
        self.shape = state_shape(self.cfg)   # shape of this context's state arrays
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

    def pack(self, dense):
        """Dense state (dense_shape) -> a state of this context's layout."""
        t = self.torch
        if dense.dtype != self.dtype or not dense.is_contiguous() or tuple(dense.shape) != self.dense_shape:
            raise DGError(DG_ERR_INVALID, "dense state must be contiguous %s of shape %s" % (self.dtype, self.dense_shape))
        out = self.empty_state()
        dg_state_pack(self.ctx, dense, out)
        return out

    def unpack(self, f):
        """State of this context's layout -> dense state (dense_shape)."""
        self._check_state(f)
        out = self.torch.empty(self.dense_shape, dtype=self.dtype, device=self.device)
        dg_state_unpack(self.ctx, f, out)
        return out

    def _check_field(self, E):
        t = self.torch
        nx = self.nelem[0] * self.n
        if (not isinstance(E, t.Tensor) or E.device.type != "cuda" or E.dtype != t.float64
                or not E.is_contiguous() or E.numel() != nx):
            raise DGError(DG_ERR_INVALID, "E must be a contiguous float64 device tensor of %d values" % nx)

    def rhs(self, f, E=None, out=None):
        self._check_state(f)
        if E is not None:
            self._check_field(E)
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

    def profile_copy(self, f, pattern, reps=20):
        """Mean ms of a copy of state f: pattern 0 streaming, 1 the stage kernel's tile pattern;
        pattern 2 times an empty dependent launch instead (f untouched); pattern 3 is
        pattern 1 held to the stage-1 kernel's residency per CU."""
        self._check_state(f)
        out = self.empty_state()
        return dg_profile_copy(self.ctx, f, out, pattern, reps)

    def profile_step(self, f, dt, nsteps=1):
        self._check_state(f)
        return dg_profile_step(self.ctx, f, dt, nsteps)

    def diagnostics(self, f):
        self._check_state(f)
        return dg_diagnostics(self.ctx, f)

    def dt_max(self, max_abs_E=0.0):
        return dg_dt_max(self.ctx, max_abs_E)

    def fourier(self, g):
        """c_p, p = 1..pmax (complex numpy array), of nodal values g (device float64, Nx*n) on the x grid."""
        t = self.torch
        if (not isinstance(g, t.Tensor) or g.device.type != "cuda" or g.dtype != t.float64
                or not g.is_contiguous() or g.numel() != self.nelem[0] * self.n):
            raise DGError(DG_ERR_INVALID, "g must be a contiguous float64 device tensor of Nx*n values")
        c = t.empty(2 * self.pmax, dtype=t.float64, device=self.device)
        dg_fourier(self.ctx, g, c)
        h = c.cpu().numpy().reshape(-1, 2)
        return h[:, 0] + 1j * h[:, 1]

    def filter_x(self, f, sigma, out=None):
        """Global x filter of a state: modes p = 1..pmax weighted by sigma (host array of pmax)."""
        self._check_state(f)
        sigma = np.asarray(sigma, dtype=np.float64).reshape(-1)
        if sigma.size != self.pmax:
            raise DGError(DG_ERR_INVALID, "sigma needs pmax = %d weights" % self.pmax)
        out = self.empty_state() if out is None else out
        self._check_state(out)
        dg_filter_x(self.ctx, sigma, f, out)
        return out

    def set_background(self, f0=None):
        """x-uniform background f0 (host, [Nu*n, Nv*n] or [Nv*n]); states then hold f - f0."""
        if f0 is not None:
            nvn = self.nelem[-1] * self.n
            nu = self.nelem[1] * self.n if self.nv == 2 else 1
            f0 = np.asarray(f0, dtype=np.float64).reshape(nu, nvn) if self.nv == 2 else \
                np.asarray(f0, dtype=np.float64).reshape(nvn)
        dg_set_background(self.ctx, f0)


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


def _batch_dts(states, dts):
    dt = np.ascontiguousarray(dts, dtype=np.float64).reshape(-1)
    if dt.size != len(states):
        raise DGError(DG_ERR_INVALID, "need one dt per run (%d runs, %d dt values)" % (len(states), dt.size))
    return dt


def dg_batch_rk_step(b, states, dts, nsteps, diag=False):
    dt = _batch_dts(states, dts)
    recs = (dg_diag * (len(states) * nsteps))() if (diag and nsteps > 0) else None
    _bcheck(lib().dg_batch_rk_step(b, _ptr_array(states), _dptr(dt), int(nsteps), recs), b)
    if recs is None:
        return None
    return [[recs[r * nsteps + k].as_dict() for k in range(nsteps)] for r in range(len(states))]


def dg_batch_tune(b, states, dts, reps):
    dt = _batch_dts(states, dts)
    best = np.zeros(1)
    _bcheck(lib().dg_batch_tune(b, _ptr_array(states), _dptr(dt), int(reps), _dptr(best)), b)
    return float(best[0])


def dg_batch_grid(b):
    return int(lib().dg_batch_grid(b))


def dg_batch_choice(b):
    """The batch's launch choices; per kind wg_per_cu is the persistent grid
    in work-groups per CU, 0 for one work-group per tile."""
    k = int(lib().dg_batch_choice(b, None))
    out = (ctypes.c_int32 * (2 + 4 * k))()
    lib().dg_batch_choice(b, out)
    kinds = [{"n": out[2 + 4 * q], "nv": out[3 + 4 * q], "wg_per_cu": out[4 + 4 * q], "grid": out[5 + 4 * q]}
             for q in range(k)]
    return {"concurrent": bool(out[0]), "order": "run-interleaved" if out[1] else "cost-sorted", "kinds": kinds}


def dg_batch_set_choice(b, choice):
    k = len(choice["kinds"])
    arr = (ctypes.c_int32 * (2 + 4 * k))()
    arr[0] = 1 if choice["concurrent"] else 0
    arr[1] = 1 if choice["order"] == "run-interleaved" else 0
    for q, kd in enumerate(choice["kinds"]):
        arr[2 + 4 * q], arr[3 + 4 * q], arr[4 + 4 * q], arr[5 + 4 * q] = kd["n"], kd["nv"], kd["wg_per_cu"], 0
    _bcheck(lib().dg_batch_set_choice(b, arr, 2 + 4 * k), b)


class Batch:
    """Many independent runs (FP32) stepped together: per RK stage one launch
    per kind (the 1D2V runs of one node count; all 1D1V runs), each a
    persistent grid or one work-group per tile as the tuner chose, then one
    batched field solve, replayed from a captured graph."""

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
        self.shapes = [state_shape(c) for c in self.cfgs]

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

    @property
    def choice(self):
        return dg_batch_choice(self.b)

    @choice.setter
    def choice(self, c):
        dg_batch_set_choice(self.b, c)


# ---------------- learned coarse-grid correction ----------------

def _ncheck(status, nn=None):
    if status != DG_OK:
        raise DGError(status, lib().dg_nn_last_error(nn).decode())


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _sizes(sizes):
    return (ctypes.c_int32 * len(sizes))(*[int(x) for x in sizes])


def dg_nn_workspace_bytes(sizes, max_rows):
    return int(lib().dg_nn_workspace_bytes(_sizes(sizes), len(sizes) - 1, int(max_rows)))


def dg_nn_init(sizes, max_rows, workspace, stream=None):
    nn = ctypes.c_void_p()
    st = lib().dg_nn_init(_sizes(sizes), len(sizes) - 1, int(max_rows), _ptr(workspace),
                          workspace.numel() * workspace.element_size(), ctypes.c_void_p(stream), ctypes.byref(nn))
    _ncheck(st, None)
    return nn


def dg_nn_destroy(nn):
    _ncheck(lib().dg_nn_destroy(nn), None)


def dg_nn_param_count(nn):
    return int(lib().dg_nn_param_count(nn))


def dg_nn_input_ld(nn):
    return int(lib().dg_nn_input_ld(nn))


def dg_nn_set_params(nn, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _ncheck(lib().dg_nn_set_params(nn, _fptr(a)), nn)


def dg_nn_get_params(nn):
    a = np.zeros(dg_nn_param_count(nn), dtype=np.float32)
    _ncheck(lib().dg_nn_get_params(nn, _fptr(a)), nn)
    return a


def dg_nn_forward(nn, X, rows, Y):
    _ncheck(lib().dg_nn_forward(nn, _ptr(X), int(rows), _ptr(Y)), nn)


def dg_nn_set_fused(nn, on):
    _ncheck(lib().dg_nn_set_fused(nn, 1 if on else 0), nn)


def dg_nn_loss_grad(nn, X, T, rows, want_loss=True, want_grads=False):
    loss = np.zeros(1)
    g = np.zeros(dg_nn_param_count(nn), dtype=np.float32) if want_grads else None
    _ncheck(lib().dg_nn_loss_grad(nn, _ptr(X), _ptr(T), int(rows), _dptr(loss) if want_loss else None,
                                  _fptr(g) if want_grads else None), nn)
    return (float(loss[0]) if want_loss else None), g


def dg_nn_adamw(nn, lr, weight_decay=0.0):
    _ncheck(lib().dg_nn_adamw(nn, float(lr), float(weight_decay)), nn)


def dg_nn_column_stats(nn, X, rows, cols):
    s, q = np.zeros(cols), np.zeros(cols)
    _ncheck(lib().dg_nn_column_stats(nn, _ptr(X), int(rows), int(cols), _dptr(s), _dptr(q)), nn)
    return s, q


def dg_nn_last_error(nn=None):
    return lib().dg_nn_last_error(nn).decode()


def dg_projection_matrix(nc, nf, r):
    out = np.zeros(nc * r * nf)
    _check(lib().dg_projection_matrix(int(nc), int(nf), int(r), _dptr(out)))
    return out.reshape(nc, r * nf)


def dg_project(fine_ctx, coarse_ctx, f_fine, f_coarse):
    _check(lib().dg_project(fine_ctx, coarse_ctx, _ptr(f_fine), _ptr(f_coarse)), coarse_ctx)


def dg_nn_features(coarse_ctx, nn, f, E, mean, inv_std, X):
    _check(lib().dg_nn_features(coarse_ctx, nn, _ptr(f), _ptr(E), _ptr(mean), _ptr(inv_std), _ptr(X)), coarse_ctx)


def dg_nn_features_raw(coarse_ctx, f, E, out, fluct=False):
    _check(lib().dg_nn_features_raw(coarse_ctx, _ptr(f), _ptr(E), 1 if fluct else 0, _ptr(out)), coarse_ctx)


def dg_nn_to_elements(coarse_ctx, x, sub, scale, out, fluct=False):
    _check(lib().dg_nn_to_elements(coarse_ctx, _ptr(x), _ptr(sub), float(scale), 1 if fluct else 0, _ptr(out)), coarse_ctx)


def dg_nn_rk_step(coarse_ctx, nn, mean, inv_std, out_scale, f, dt, nsteps, diag=False):
    recs = (dg_diag * nsteps)() if (diag and nsteps > 0) else None
    st = lib().dg_nn_rk_step(coarse_ctx, nn, _ptr(mean), _ptr(inv_std), float(out_scale), _ptr(f), float(dt),
                             int(nsteps), recs)
    _check(st, coarse_ctx)
    return [r.as_dict() for r in recs] if recs is not None else None


class Network:
    """Per-element MLP of the learned correction; owns its device workspace."""

    def __init__(self, sizes, max_rows, device="cuda"):
        import torch
        self.torch = torch
        self.sizes = [int(x) for x in sizes]
        self.max_rows = int(max_rows)
        nbytes = dg_nn_workspace_bytes(self.sizes, self.max_rows)
        if nbytes == 0:
            raise DGError(DG_ERR_INVALID, "invalid network configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + nbytes]
        self.nn = dg_nn_init(self.sizes, self.max_rows, self.ws, torch.cuda.current_stream(self.device).cuda_stream)
        self.ld = dg_nn_input_ld(self.nn)
        self.nparam = dg_nn_param_count(self.nn)

    def close(self):
        if getattr(self, "nn", None) is not None:
            dg_nn_destroy(self.nn)
            self.nn = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        dg_nn_set_params(self.nn, flat)

    def get_params(self):
        return dg_nn_get_params(self.nn)

    def unflatten(self, flat):
        out, o = [], 0
        for a, b in zip(self.sizes[:-1], self.sizes[1:]):
            out.append(np.asarray(flat[o:o + a * b]).reshape(a, b))
            o += a * b
            out.append(np.asarray(flat[o:o + b]))
            o += b
        return out

    @staticmethod
    def flatten(params):
        return np.concatenate([np.asarray(p, dtype=np.float32).ravel() for p in params])

    def _rows(self, X):
        t = self.torch
        if (not isinstance(X, t.Tensor) or X.device.type != "cuda" or X.dtype != t.int16 or X.dim() != 2
                or X.shape[1] != self.ld or not X.is_contiguous()):
            raise DGError(DG_ERR_INVALID, "X must be a contiguous int16 (BF16 bits) device tensor of shape (rows, %d)"
                          % self.ld)
        return X.shape[0]

    def forward(self, X, out=None):
        rows = self._rows(X)
        t = self.torch
        if out is None:
            Y = t.empty((rows, self.sizes[-1]), dtype=t.float32, device=self.device)
        else:
            if (not isinstance(out, t.Tensor) or out.device.type != "cuda" or out.dtype != t.float32
                    or tuple(out.shape) != (rows, self.sizes[-1]) or not out.is_contiguous()):
                raise DGError(DG_ERR_INVALID, "out must be a contiguous float32 device tensor of shape (%d, %d)"
                              % (rows, self.sizes[-1]))
            Y = out
        dg_nn_forward(self.nn, X, rows, Y)
        return Y

    def set_fused(self, on):
        """Inference form: the fused single launch (default, where the shape
        allows it) or one GEMM launch per layer."""
        dg_nn_set_fused(self.nn, on)

    def loss_grad(self, X, T, want_loss=True, want_grads=False):
        rows = self._rows(X)
        if T.dtype != self.torch.float32 or tuple(T.shape) != (rows, self.sizes[-1]) or not T.is_contiguous():
            raise DGError(DG_ERR_INVALID, "T must be contiguous float32 of shape (rows, %d)" % self.sizes[-1])
        return dg_nn_loss_grad(self.nn, X, T, rows, want_loss, want_grads)

    def adamw(self, lr, weight_decay=0.0):
        dg_nn_adamw(self.nn, lr, weight_decay)

    def column_stats(self, X):
        rows, cols = X.shape
        return dg_nn_column_stats(self.nn, X, rows, cols)
