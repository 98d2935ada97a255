"""ctypes binding of liblbm.so (include/lbm.h): the same entry points under
the same names, argument marshalling only.  PyTorch supplies device memory
(the workspace) and the stream; every step of the method runs in the
library's HIP kernels.  There is no fallback: if the library or a GPU is
missing, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY may name another build of the same library (e.g. a tuning
# variant); the default is the in-tree build.
LIB_PATH = os.environ.get("LBM_LIBRARY", os.path.join(_HERE, "liblbm.so"))

LBM_OK, LBM_EINVAL, LBM_ENOSPACE, LBM_EHIP, LBM_ESTATE, LBM_EUNSTABLE = 0, -1, -2, -3, -4, -5
LBM_FP64, LBM_FP32_OFFSET, LBM_FP16_OFFSET = 0, 1, 2
LBM_BGK, LBM_MRT = 0, 1
LBM_LATERAL_WALLS, LBM_LATERAL_PERIODIC = 0, 1
LBM_X_INOUT, LBM_X_PERIODIC = 0, 1
LBM_OUT_ZOUHE, LBM_OUT_NN = 0, 1


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("lateral", ctypes.c_int32), ("xbc", ctypes.c_int32),
                ("tau", ctypes.c_double), ("s_e", ctypes.c_double),
                ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
                ("u_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("noise_amp", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("history_cap", ctypes.c_int64), ("stream", ctypes.c_void_p)]


class lbm_force_out(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("fx_sum", ctypes.c_double), ("fy_sum", ctypes.c_double),
                ("mass", ctypes.c_double), ("step", ctypes.c_int64),
                ("n_fallback", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_FP = ctypes.POINTER(ctypes.c_float)


class lbm_mlp(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_h1", ctypes.c_int32),
                ("n_h2", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("w1", _FP), ("b1", _FP), ("w2", _FP), ("b2", _FP), ("w3", _FP), ("b3", _FP),
                ("mu_in", _FP), ("sd_in", _FP), ("mu_out", _FP), ("sd_out", _FP),
                ("mass_bound", ctypes.c_double)]


class LbmError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


_lib = None


def library():
    """Load liblbm.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run python -m paper_2506_05293_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        P, VP, I32, I64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        DP = P(ctypes.c_double)
        sig = {
            "lbm_workspace_bytes": (ctypes.c_size_t, [P(lbm_params)]),
            "lbm_create": (I32, [P(lbm_params), VP, ctypes.c_size_t, P(VP)]),
            "lbm_destroy": (I32, [VP]),
            "lbm_set_geometry": (I32, [VP, P(ctypes.c_uint8)]),
            "lbm_init_fields": (I32, [VP, DP, DP, DP]),
            "lbm_set_inlet_profile": (I32, [VP, DP]),
            "lbm_step": (I32, [VP, I64]),
            "lbm_forces": (I32, [VP, P(lbm_force_out)]),
            "lbm_force_history": (I32, [VP, DP, DP, I64, P(I64)]),
            "lbm_set_outflow_model": (I32, [VP, I32, P(lbm_mlp)]),
            "lbm_read_populations": (I32, [VP, DP]),
            "lbm_write_populations": (I32, [VP, DP]),
            "lbm_sync": (I32, [VP]),
            "lbm_mlp_forward": (I32, [VP, VP, VP, I64]),
            "lbm_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = res, args
        _lib = lib
    return _lib


def _check(status, where):
    if status < 0:
        raise LbmError(status, where, library().lbm_last_error().decode())
    return status


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c_f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


# --- the C entry points ----------------------------------------------------------

def lbm_workspace_bytes(params):
    n = library().lbm_workspace_bytes(ctypes.byref(params))
    if n == 0:
        raise LbmError(LBM_EINVAL, "lbm_workspace_bytes", library().lbm_last_error().decode())
    return n


def lbm_create(params, workspace_ptr, nbytes):
    ctx = ctypes.c_void_p()
    _check(library().lbm_create(ctypes.byref(params), ctypes.c_void_p(workspace_ptr), nbytes,
                                ctypes.byref(ctx)), "lbm_create")
    return ctx


def lbm_destroy(ctx):
    return _check(library().lbm_destroy(ctx), "lbm_destroy")


def lbm_set_geometry(ctx, mask):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return _check(library().lbm_set_geometry(ctx, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
                  "lbm_set_geometry")


def lbm_init_fields(ctx, rho, ux, uy):
    shape = np.shape(rho)
    r, u, v = _c_f64(rho, shape), _c_f64(ux, shape), _c_f64(uy, shape)
    return _check(library().lbm_init_fields(ctx, _dptr(r), _dptr(u), _dptr(v)), "lbm_init_fields")


def lbm_set_inlet_profile(ctx, ux):
    if ux is None:
        return _check(library().lbm_set_inlet_profile(ctx, None), "lbm_set_inlet_profile")
    u = np.ascontiguousarray(ux, dtype=np.float64)
    return _check(library().lbm_set_inlet_profile(ctx, _dptr(u)), "lbm_set_inlet_profile")


def lbm_step(ctx, nsteps):
    return _check(library().lbm_step(ctx, int(nsteps)), "lbm_step")


def lbm_forces(ctx, allow_unstable=False):
    out = lbm_force_out()
    st = library().lbm_forces(ctx, ctypes.byref(out))
    if not (allow_unstable and st == LBM_EUNSTABLE):
        _check(st, "lbm_forces")
    return out


def lbm_force_history(ctx, cap):
    fx, fy = np.zeros(cap), np.zeros(cap)
    n = ctypes.c_int64()
    _check(library().lbm_force_history(ctx, _dptr(fx), _dptr(fy), cap, ctypes.byref(n)),
           "lbm_force_history")
    return fx[:n.value], fy[:n.value]


def _mlp_struct(P, mass_bound):
    keep = {k: np.ascontiguousarray(P[k], dtype=np.float32).reshape(-1)
            for k in ("w1", "b1", "w2", "b2", "w3", "b3", "mu_in", "sd_in", "mu_out", "sd_out")}
    s = lbm_mlp(27, 64, 64, 3, *[keep[k].ctypes.data_as(_FP) for k in
                                 ("w1", "b1", "w2", "b2", "w3", "b3", "mu_in", "sd_in",
                                  "mu_out", "sd_out")], float(mass_bound))
    return s, keep


def lbm_set_outflow_model(ctx, kind, P=None, mass_bound=1e-2):
    if kind == LBM_OUT_ZOUHE or P is None:
        return _check(library().lbm_set_outflow_model(ctx, kind, None), "lbm_set_outflow_model")
    s, keep = _mlp_struct(P, mass_bound)
    st = library().lbm_set_outflow_model(ctx, kind, ctypes.byref(s))
    del keep
    return _check(st, "lbm_set_outflow_model")


def lbm_read_populations(ctx, nx, ny):
    out = np.empty((9, ny, nx))
    _check(library().lbm_read_populations(ctx, _dptr(out)), "lbm_read_populations")
    return out


def lbm_write_populations(ctx, f):
    a = np.ascontiguousarray(f, dtype=np.float64)
    return _check(library().lbm_write_populations(ctx, _dptr(a)), "lbm_write_populations")


def lbm_sync(ctx):
    return _check(library().lbm_sync(ctx), "lbm_sync")


def lbm_mlp_forward(ctx, x_ptr, s_ptr, n):
    return _check(library().lbm_mlp_forward(ctx, ctypes.c_void_p(x_ptr), ctypes.c_void_p(s_ptr), n),
                  "lbm_mlp_forward")


def lbm_last_error():
    return library().lbm_last_error().decode()


# --- convenience: one lattice with a torch-owned workspace --------------------------

_PREC = {"fp64": LBM_FP64, "fp32": LBM_FP32_OFFSET, "fp16": LBM_FP16_OFFSET}
_COLL = {"bgk": LBM_BGK, "mrt": LBM_MRT}
_LAT = {"walls": LBM_LATERAL_WALLS, "periodic": LBM_LATERAL_PERIODIC}
_XBC = {"inout": LBM_X_INOUT, "periodic": LBM_X_PERIODIC}


class Lattice:
    """A lattice on the current CUDA (HIP) device.  The workspace is a torch
    uint8 tensor and the stream is torch's current stream."""

    def __init__(self, mask, tau, *, precision="fp32", collision="bgk", lateral="walls",
                 xbc="inout", u_in=0.05, rho_out=1.0, s_e=1.0, s_eps=1.0, s_q=0.0,
                 noise_amp=0.0, seed=0, history_cap=0, device="cuda"):
        import torch
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.ny, self.nx = mask.shape
        self.stream = torch.cuda.current_stream(device)
        self.params = lbm_params(self.nx, self.ny, _PREC[precision], _COLL[collision],
                                 _LAT[lateral], _XBC[xbc], tau, s_e, s_eps, s_q, u_in,
                                 rho_out, noise_amp, seed, history_cap,
                                 ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = lbm_workspace_bytes(self.params)
        # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert self.workspace.data_ptr() % 256 == 0
        self.ctx = lbm_create(self.params, self.workspace.data_ptr(), nbytes)
        lbm_set_geometry(self.ctx, mask)
        self.history_cap = history_cap

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and _lib is not None:
            _lib.lbm_destroy(ctx)
            self.ctx = None

    def step(self, n=1):
        lbm_step(self.ctx, n)
        return self

    def forces(self, allow_unstable=False):
        return lbm_forces(self.ctx, allow_unstable)

    def force_history(self):
        return lbm_force_history(self.ctx, self.history_cap)

    def populations(self):
        return lbm_read_populations(self.ctx, self.nx, self.ny)

    def write_populations(self, f):
        lbm_write_populations(self.ctx, f)

    def init_fields(self, rho, ux, uy):
        lbm_init_fields(self.ctx, rho, ux, uy)

    def set_inlet_profile(self, ux):
        lbm_set_inlet_profile(self.ctx, ux)

    def set_outflow_nn(self, P, mass_bound=1e-2):
        lbm_set_outflow_model(self.ctx, LBM_OUT_NN, P, mass_bound)

    def set_outflow_zouhe(self):
        lbm_set_outflow_model(self.ctx, LBM_OUT_ZOUHE)

    def macroscopic(self):
        f = self.populations()
        rho = f.sum(0)
        cxv = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)[:, None, None]
        cyv = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)[:, None, None]
        return rho, (cxv * f).sum(0) / rho, (cyv * f).sum(0) / rho

    def sync(self):
        lbm_sync(self.ctx)
