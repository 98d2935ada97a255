"""ctypes binding of liblbm.so (include/lbm.h): the same entry points under
the same names, argument marshalling only.  PyTorch supplies device memory
(the workspace) and the stream; every step of the method runs in the
library's HIP kernels.  There is no fallback: if the library or a GPU is
missing, the calls raise.
"""
import atexit
import ctypes
import os
import weakref

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
LBM_OUT_ZOUHE, LBM_OUT_NN, LBM_OUT_CBC = 0, 1, 2
LBM_LAUNCH_AUTO, LBM_LAUNCH_SINGLE, LBM_LAUNCH_PAIRS_PLAIN, LBM_LAUNCH_PAIRS_HELD = 0, 1, 2, 3
LBM_LAUNCH_TRIPLES, LBM_LAUNCH_PAIRS, LBM_LAUNCH_TRIPLES_PLAIN, LBM_LAUNCH_TRIPLES_HELD = 4, 5, 6, 7
LBM_PATH_AUTO, LBM_PATH_SCALAR, LBM_PATH_VECTOR = 0, 1, 2
LBM_BATCH_PER_STEP, LBM_BATCH_PERSISTENT = 0, 1


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("lateral", ctypes.c_int32), ("xbc", ctypes.c_int32),
                ("launch", ctypes.c_int32), ("bulk_path", ctypes.c_int32),
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


class lbm_cbc_net(ctypes.Structure):
    _fields_ = [("w1", _FP), ("b1", _FP), ("w2", _FP), ("b2", _FP), ("w3", _FP), ("b3", _FP),
                ("mu_in", _FP), ("sd_in", _FP), ("leaky_slope", ctypes.c_double),
                ("sigma_scale", ctypes.c_double), ("sigma_shift", ctypes.c_double),
                ("kappa_scale", ctypes.c_double), ("kappa_shift", ctypes.c_double)]


class lbm_cbc(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("kappa2", ctypes.c_double),
                ("mach", ctypes.c_double), ("length", ctypes.c_double),
                ("rho_inf", ctypes.c_double), ("net", ctypes.POINTER(lbm_cbc_net))]


class lbm_nn9_net(ctypes.Structure):
    _fields_ = [(k, ctypes.POINTER(ctypes.c_float)) for k in ("w1", "b1", "w2", "b2", "w3", "b3")] + \
               [("mu_in", ctypes.c_float * 9), ("sd_in", ctypes.c_float * 9),
                ("mu_out", ctypes.c_float * 3), ("sd_out", ctypes.c_float * 3)]


class lbm_cbc_train_params(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int32), ("n_max", ctypes.c_int32), ("n_seg", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tau", ctypes.c_double), ("mach", ctypes.c_double),
                ("length", ctypes.c_double), ("rho_inf", ctypes.c_double), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class lbm3d_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("lateral_y", ctypes.c_int32),
                ("lateral_z", ctypes.c_int32), ("xbc", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tau", ctypes.c_double), ("u_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("history_cap", ctypes.c_int64), ("stream", ctypes.c_void_p)]


class lbm3d_force_out(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("fz", ctypes.c_double),
                ("dmass", ctypes.c_double), ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class lbm_train_params(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_void_p)]


class lbm_mlp_host(ctypes.Structure):
    _fields_ = [(k, _FP) for k in ("w1", "b1", "w2", "b2", "w3", "b3",
                                   "mu_in", "sd_in", "mu_out", "sd_out")]


class lbm_batch_lattice(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("u_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("mask", ctypes.POINTER(ctypes.c_uint8)), ("seed", ctypes.c_uint64),
                ("log_role", ctypes.c_int32), ("log_x", ctypes.c_int32),
                ("log_row0", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lbm_batch_params(ctypes.Structure):
    _fields_ = [("collision", ctypes.c_int32), ("lateral", ctypes.c_int32),
                ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
                ("noise_amp", ctypes.c_double), ("history_cap", ctypes.c_int64),
                ("log_start", ctypes.c_int64), ("log_every", ctypes.c_int64),
                ("log_slots", ctypes.c_int64), ("log_rows", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("stream", ctypes.c_void_p)]


PARAM_SHAPES = {"w1": (64, 27), "b1": (64,), "w2": (64, 64), "b2": (64,), "w3": (3, 64), "b3": (3,)}
N_PARAMS = 6147
CBC_PARAM_SHAPES = {"w1": (20, 9), "b1": (20,), "w2": (20, 20), "b2": (20,), "w3": (2, 20),
                    "b3": (2,)}
LBM_CBC_NPARAMS = 662
LBM_NN9_NPARAMS = 683
NN9_PARAM_SHAPES = {"w1": (20, 9), "b1": (20,), "w2": (20, 20), "b2": (20,), "w3": (3, 20),
                    "b3": (3,)}


class LbmError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


_lib = None
# Native objects still alive; closed at interpreter exit, before torch and the
# HIP runtime are torn down, so no launch is still running then.
_live = weakref.WeakSet()


@atexit.register
def _close_live():
    for obj in list(_live):
        obj.close()


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
            "lbm_set_outflow_cbc": (I32, [VP, P(lbm_cbc)]),
            "lbm_read_populations": (I32, [VP, DP]),
            "lbm_read_macroscopic": (I32, [VP, DP, DP, DP]),
            "lbm_write_populations": (I32, [VP, DP]),
            "lbm_sync": (I32, [VP]),
            "lbm_mlp_forward": (I32, [VP, VP, VP, I64]),
            "lbm_last_error": (ctypes.c_char_p, []),
            "lbm_batch_workspace_bytes": (ctypes.c_size_t, [P(lbm_batch_params), P(lbm_batch_lattice),
                                                            ctypes.c_int32]),
            "lbm_batch_create": (I32, [P(lbm_batch_params), P(lbm_batch_lattice), ctypes.c_int32, VP,
                                       ctypes.c_size_t, P(VP)]),
            "lbm_batch_destroy": (I32, [VP]),
            "lbm_batch_step": (I32, [VP, I64]),
            "lbm_batch_forces": (I32, [VP, ctypes.c_int32, P(lbm_force_out)]),
            "lbm_batch_force_history": (I32, [VP, ctypes.c_int32, DP, DP, I64, P(I64)]),
            "lbm_batch_read_populations": (I32, [VP, ctypes.c_int32, DP]),
            "lbm_batch_retired": (I32, [VP, P(ctypes.c_int32)]),
            "lbm_batch_dataset": (I32, [VP, P(VP), P(VP), P(VP), P(I64)]),
            "lbm_train_workspace_bytes": (ctypes.c_size_t, [P(lbm_train_params)]),
            "lbm_train_create": (I32, [P(lbm_train_params), VP, ctypes.c_size_t, P(VP)]),
            "lbm_train_destroy": (I32, [VP]),
            "lbm_train_set_data": (I32, [VP, VP, VP, I64]),
            "lbm_train_set_weights": (I32, [VP, P(lbm_mlp)]),
            "lbm_train_step": (I32, [VP, I64]),
            "lbm_train_loss": (I32, [VP, DP]),
            "lbm_train_get_weights": (I32, [VP, P(lbm_mlp_host)]),
            "lbm_train_gradient": (I32, [VP, VP, ctypes.c_int32, _FP, DP]),
            "lbm_train_sample_rows": (I32, [VP, I64, P(ctypes.c_int32)]),
            "lbm_mlp_gradient_noalloc": (I32, [P(lbm_mlp), VP, VP, VP, ctypes.c_int32, _FP, DP,
                                               VP]),
            "lbm3d_workspace_bytes": (ctypes.c_size_t, [P(lbm3d_params)]),
            "lbm3d_create": (I32, [P(lbm3d_params), VP, ctypes.c_size_t, P(VP)]),
            "lbm3d_destroy": (I32, [VP]),
            "lbm3d_set_geometry": (I32, [VP, P(ctypes.c_uint8)]),
            "lbm3d_init_fields": (I32, [VP, DP, DP]),
            "lbm3d_step": (I32, [VP, I64]),
            "lbm3d_forces": (I32, [VP, P(lbm3d_force_out)]),
            "lbm3d_force_history": (I32, [VP, DP, DP, DP, I64, P(I64)]),
            "lbm3d_read_populations": (I32, [VP, DP]),
            "lbm3d_write_populations": (I32, [VP, DP]),
            "lbm3d_sync": (I32, [VP]),
            "lbm_cbc_train_workspace_bytes": (ctypes.c_size_t, [P(lbm_cbc_train_params)]),
            "lbm_cbc_train_create": (I32, [P(lbm_cbc_train_params), VP, ctypes.c_size_t, P(VP)]),
            "lbm_cbc_train_destroy": (I32, [VP]),
            "lbm_cbc_train_set_segments": (I32, [VP, DP, DP, P(ctypes.c_int32)]),
            "lbm_cbc_train_set_net": (I32, [VP, P(lbm_cbc_net)]),
            "lbm_cbc_train_set_nn": (I32, [VP, P(lbm_nn9_net)]),
            "lbm_cbc_train_set_segment_params": (I32, [VP, DP, DP]),
            "lbm_cbc_train_gradient": (I32, [VP, DP, DP]),
            "lbm_cbc_train_step": (I32, [VP, I64]),
            "lbm_cbc_train_loss": (I32, [VP, DP]),
            "lbm_cbc_train_get_weights": (I32, [VP, _FP]),
            "lbm_cbc_train_final_state": (I32, [VP, ctypes.c_int32, DP]),
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
    h1, n_in = np.shape(P["w1"])
    h2 = np.shape(P["w2"])[0]
    s = lbm_mlp(n_in, h1, h2, 3, *[keep[k].ctypes.data_as(_FP) for k in
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


def _cbc_net_struct(net):
    """lbm_cbc_net for a dict of weights and maps; returns the struct and the
    FP32 arrays it points into (keep them alive during the call)."""
    keep = {k: np.ascontiguousarray(net[k], dtype=np.float32).reshape(-1)
            for k in ("w1", "b1", "w2", "b2", "w3", "b3", "mu_in", "sd_in")}
    n = lbm_cbc_net(*[keep[k].ctypes.data_as(_FP) for k in
                      ("w1", "b1", "w2", "b2", "w3", "b3", "mu_in", "sd_in")],
                    float(net.get("leaky_slope", 0.01)), float(net["sigma_scale"]),
                    float(net["sigma_shift"]), float(net["kappa_scale"]),
                    float(net["kappa_shift"]))
    return n, keep


def lbm_set_outflow_cbc(ctx, sigma=0.0, kappa2=0.0, mach=0.0, length=1.0, rho_inf=1.0,
                        net=None):
    keep = None
    p = lbm_cbc(sigma, kappa2, mach, length, rho_inf, None)
    if net is not None:
        n, keep = _cbc_net_struct(net)
        p.net = ctypes.pointer(n)
    st = library().lbm_set_outflow_cbc(ctx, ctypes.byref(p))
    del keep
    return _check(st, "lbm_set_outflow_cbc")


def lbm_read_populations(ctx, nx, ny):
    out = np.empty((9, ny, nx))
    _check(library().lbm_read_populations(ctx, _dptr(out)), "lbm_read_populations")
    return out


def lbm_read_macroscopic(ctx, nx, ny):
    rho, ux, uy = (np.empty((ny, nx)) for _ in range(3))
    _check(library().lbm_read_macroscopic(ctx, _dptr(rho), _dptr(ux), _dptr(uy)),
           "lbm_read_macroscopic")
    return rho, ux, uy


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


# --- batched lattices (include/lbm_batch.h) -----------------------------------------

def _lattice_array(lattices):
    arr = (lbm_batch_lattice * len(lattices))()
    masks = []
    for i, L in enumerate(lattices):
        m = np.ascontiguousarray(L["mask"], dtype=np.uint8)
        masks.append(m)
        ny, nx = m.shape
        arr[i] = lbm_batch_lattice(nx, ny, L["tau"], L.get("u_in", 0.05), L.get("rho_out", 1.0),
                                   m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), L.get("seed", 0),
                                   L.get("log_role", 0), L.get("log_x", 0), L.get("log_row0", 0), 0)
    return arr, masks


def lbm_batch_workspace_bytes(params, lattices):
    arr, masks = _lattice_array(lattices)
    n = library().lbm_batch_workspace_bytes(ctypes.byref(params), arr, len(lattices))
    if n == 0:
        raise LbmError(LBM_EINVAL, "lbm_batch_workspace_bytes", library().lbm_last_error().decode())
    return n


def lbm_batch_create(params, lattices, workspace_ptr, nbytes):
    arr, masks = _lattice_array(lattices)
    b = ctypes.c_void_p()
    _check(library().lbm_batch_create(ctypes.byref(params), arr, len(lattices),
                                      ctypes.c_void_p(workspace_ptr), nbytes, ctypes.byref(b)),
           "lbm_batch_create")
    return b


def lbm_batch_destroy(b):
    return _check(library().lbm_batch_destroy(b), "lbm_batch_destroy")


def lbm_batch_step(b, nsteps):
    return _check(library().lbm_batch_step(b, int(nsteps)), "lbm_batch_step")


def lbm_batch_forces(b, lattice, allow_unstable=False):
    out = lbm_force_out()
    st = library().lbm_batch_forces(b, lattice, ctypes.byref(out))
    if not (allow_unstable and st == LBM_EUNSTABLE):
        _check(st, "lbm_batch_forces")
    return out


def lbm_batch_force_history(b, lattice, cap):
    fx, fy = np.zeros(cap), np.zeros(cap)
    n = ctypes.c_int64()
    _check(library().lbm_batch_force_history(b, lattice, _dptr(fx), _dptr(fy), cap, ctypes.byref(n)),
           "lbm_batch_force_history")
    return fx[:n.value], fy[:n.value]


def lbm_batch_read_populations(b, lattice, nx, ny):
    out = np.empty((9, ny, nx))
    _check(library().lbm_batch_read_populations(b, lattice, _dptr(out)), "lbm_batch_read_populations")
    return out


def lbm_batch_retired(b, n):
    flags = np.zeros(n, np.int32)
    _check(library().lbm_batch_retired(b, flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "lbm_batch_retired")
    return flags


def lbm_batch_dataset(b):
    x, xa, t = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    n = ctypes.c_int64()
    _check(library().lbm_batch_dataset(b, ctypes.byref(x), ctypes.byref(xa), ctypes.byref(t),
                                       ctypes.byref(n)), "lbm_batch_dataset")
    return x.value, xa.value, t.value, n.value


class Batch:
    """Many lattices advanced together; `lattices` is a list of dicts with
    mask, tau and optionally u_in, rho_out, seed, log_role, log_x, log_row0."""

    def __init__(self, lattices, *, collision="mrt", lateral="periodic", s_e=1.0, s_eps=1.0, s_q=0.0,
                 noise_amp=0.0, history_cap=0, log_start=0, log_every=1, log_slots=0, log_rows=0,
                 spin_limit=0, launch="per_step", groups_per_cu=0, device="cuda"):
        import torch
        self.lattices = lattices
        self.shapes = [np.shape(L["mask"]) for L in lattices]
        self.stream = torch.cuda.current_stream(device)
        self.params = lbm_batch_params(_COLL[collision], _LAT[lateral], s_e, s_eps, s_q, noise_amp,
                                       history_cap, log_start, log_every, log_slots, log_rows,
                                       spin_limit, _LAUNCH[launch], groups_per_cu,
                                       ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = lbm_batch_workspace_bytes(self.params, lattices)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.b = lbm_batch_create(self.params, lattices, self.workspace.data_ptr(), nbytes)
        _live.add(self)
        self.history_cap = history_cap

    def close(self):
        """Wait for the queued work and release the native object (also at
        interpreter exit and on garbage collection)."""
        h = getattr(self, "b", None)
        if h is not None and _lib is not None:
            _lib.lbm_batch_destroy(h)
        self.b = None

    __del__ = close

    def step(self, n=1):
        lbm_batch_step(self.b, n)

    def populations(self, i):
        ny, nx = self.shapes[i]
        return lbm_batch_read_populations(self.b, i, nx, ny)

    def forces(self, i, allow_unstable=False):
        return lbm_batch_forces(self.b, i, allow_unstable)

    def force_history(self, i):
        return lbm_batch_force_history(self.b, i, self.history_cap)

    def retired(self):
        return lbm_batch_retired(self.b, len(self.lattices))

    def dataset(self):
        """(x, x_ablation, t) as torch tensors viewing the workspace."""
        import torch
        xp, xap, tp, n = lbm_batch_dataset(self.b)
        base = self.workspace.data_ptr()
        def view(ptr, cols):
            off = ptr - base
            return self.workspace[off:off + n * cols * 4].view(torch.float32).view(n, cols)
        return view(xp, 27), view(xap, 27), view(tp, 3)


# --- training of the outflow network (include/lbm_train.h) -----------------------

def lbm_train_workspace_bytes(params):
    n = library().lbm_train_workspace_bytes(ctypes.byref(params))
    if n == 0:
        raise LbmError(LBM_EINVAL, "lbm_train_workspace_bytes", library().lbm_last_error().decode())
    return n


def lbm_train_create(params, workspace_ptr, nbytes):
    tr = ctypes.c_void_p()
    _check(library().lbm_train_create(ctypes.byref(params), ctypes.c_void_p(workspace_ptr), nbytes,
                                      ctypes.byref(tr)), "lbm_train_create")
    return tr


def lbm_train_destroy(tr):
    return _check(library().lbm_train_destroy(tr), "lbm_train_destroy")


def lbm_train_set_data(tr, x_ptr, t_ptr, n):
    return _check(library().lbm_train_set_data(tr, ctypes.c_void_p(x_ptr), ctypes.c_void_p(t_ptr), n),
                  "lbm_train_set_data")


def lbm_train_set_weights(tr, P):
    full = dict(P)
    for k in ("mu_in", "sd_in", "mu_out", "sd_out"):
        full.setdefault(k, np.zeros(27 if k.endswith("in") else 3))
    s, keep = _mlp_struct(full, 0.0)
    st = library().lbm_train_set_weights(tr, ctypes.byref(s))
    del keep
    return _check(st, "lbm_train_set_weights")


def lbm_train_step(tr, nsteps):
    return _check(library().lbm_train_step(tr, int(nsteps)), "lbm_train_step")


def lbm_train_loss(tr):
    v = ctypes.c_double()
    _check(library().lbm_train_loss(tr, ctypes.byref(v)), "lbm_train_loss")
    return v.value


def lbm_train_get_weights(tr):
    out = {k: np.zeros(v, np.float32) for k, v in PARAM_SHAPES.items()}
    out.update(mu_in=np.zeros(27, np.float32), sd_in=np.zeros(27, np.float32),
               mu_out=np.zeros(3, np.float32), sd_out=np.zeros(3, np.float32))
    h = lbm_mlp_host(*[out[k].ctypes.data_as(_FP) for k in
                       ("w1", "b1", "w2", "b2", "w3", "b3", "mu_in", "sd_in", "mu_out", "sd_out")])
    _check(library().lbm_train_get_weights(tr, ctypes.byref(h)), "lbm_train_get_weights")
    return out


def lbm_train_gradient(tr, rows_ptr, n_rows):
    g = np.zeros(N_PARAMS, np.float32)
    loss = ctypes.c_double()
    _check(library().lbm_train_gradient(tr, ctypes.c_void_p(rows_ptr), n_rows, g.ctypes.data_as(_FP),
                                        ctypes.byref(loss)), "lbm_train_gradient")
    return g, loss.value


def lbm_mlp_gradient_noalloc(P, x_ptr, t_ptr, rows_ptr, n_rows, stream_ptr):
    """Loss and gradient of network P (a 27-64-64-3 dict with its
    standardisation) on device samples at device rows, with no workspace."""
    s, keep = _mlp_struct(P, 0.0)
    g = np.zeros(N_PARAMS, np.float32)
    loss = ctypes.c_double()
    _check(library().lbm_mlp_gradient_noalloc(ctypes.byref(s), ctypes.c_void_p(x_ptr),
                                              ctypes.c_void_p(t_ptr), ctypes.c_void_p(rows_ptr),
                                              n_rows, g.ctypes.data_as(_FP), ctypes.byref(loss),
                                              ctypes.c_void_p(stream_ptr)), "lbm_mlp_gradient_noalloc")
    del keep
    return g, loss.value


def lbm_train_sample_rows(tr, step, batch):
    rows = np.zeros(batch, np.int32)
    _check(library().lbm_train_sample_rows(tr, step, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "lbm_train_sample_rows")
    return rows


def unflatten_params(g):
    """Split a flat 6147-vector (w1, b1, w2, b2, w3, b3 order) into arrays."""
    out, o = {}, 0
    for k, shp in PARAM_SHAPES.items():
        n = int(np.prod(shp))
        out[k] = np.asarray(g[o:o + n]).reshape(shp)
        o += n
    return out


class Trainer:
    """Training state on the current device; x [n][27] and t [n][3] are
    float32 torch tensors on that device, kept alive by this object."""

    def __init__(self, x, t, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        import torch
        self.x, self.t = x.contiguous(), t.contiguous()
        self.stream = torch.cuda.current_stream(x.device)
        self.params = lbm_train_params(batch, lr, beta1, beta2, eps, seed,
                                       ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = lbm_train_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        self.tr = lbm_train_create(self.params, self.workspace.data_ptr(), nbytes)
        _live.add(self)
        lbm_train_set_data(self.tr, self.x.data_ptr(), self.t.data_ptr(), self.x.shape[0])
        self.batch = batch

    def close(self):
        """Wait for the queued work and release the native object (also at
        interpreter exit and on garbage collection)."""
        h = getattr(self, "tr", None)
        if h is not None and _lib is not None:
            _lib.lbm_train_destroy(h)
        self.tr = None

    __del__ = close

    def set_weights(self, P):
        lbm_train_set_weights(self.tr, P)

    def step(self, n=1):
        lbm_train_step(self.tr, n)

    def loss(self):
        return lbm_train_loss(self.tr)

    def weights(self):
        return lbm_train_get_weights(self.tr)

    def gradient(self, rows):
        import torch
        r = torch.as_tensor(np.asarray(rows, np.int32), device=self.x.device)
        return lbm_train_gradient(self.tr, r.data_ptr(), len(rows))

    def sample_rows(self, step):
        return lbm_train_sample_rows(self.tr, step, self.batch)


# --- closed-loop training of the CBC tuning network (include/lbm_cbc_train.h) -----

def lbm_cbc_train_workspace_bytes(params):
    n = library().lbm_cbc_train_workspace_bytes(ctypes.byref(params))
    if n == 0:
        raise LbmError(LBM_EINVAL, "lbm_cbc_train_workspace_bytes",
                       library().lbm_last_error().decode())
    return n


def lbm_cbc_train_create(params, workspace_ptr, nbytes):
    t = ctypes.c_void_p()
    _check(library().lbm_cbc_train_create(ctypes.byref(params), ctypes.c_void_p(workspace_ptr),
                                          nbytes, ctypes.byref(t)), "lbm_cbc_train_create")
    return t


def lbm_cbc_train_destroy(t):
    return _check(library().lbm_cbc_train_destroy(t), "lbm_cbc_train_destroy")


def lbm_cbc_train_set_segments(t, a0, ref, n_t):
    a0 = np.ascontiguousarray(a0, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    n_t = np.ascontiguousarray(n_t, dtype=np.int32)
    return _check(library().lbm_cbc_train_set_segments(
        t, _dptr(a0), _dptr(ref), n_t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
        "lbm_cbc_train_set_segments")


def lbm_cbc_train_set_segment_params(t, tau=None, mach=None):
    keep = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (tau, mach)]
    ptrs = [None if a is None else _dptr(a) for a in keep]
    return _check(library().lbm_cbc_train_set_segment_params(t, *ptrs),
                  "lbm_cbc_train_set_segment_params")


def lbm_cbc_train_set_net(t, net):
    n, keep = _cbc_net_struct(net)
    st = library().lbm_cbc_train_set_net(t, ctypes.byref(n))
    del keep
    return _check(st, "lbm_cbc_train_set_net")


def lbm_cbc_train_set_nn(t, net):
    """The Eq. 16 network (dict w1 .. b3, mu_in, sd_in, mu_out, sd_out)."""
    keep = {k: np.ascontiguousarray(net[k], dtype=np.float32).reshape(-1)
            for k in ("w1", "b1", "w2", "b2", "w3", "b3")}
    n = lbm_nn9_net(*[keep[k].ctypes.data_as(_FP) for k in ("w1", "b1", "w2", "b2", "w3", "b3")],
                    (ctypes.c_float * 9)(*np.asarray(net["mu_in"], np.float32)),
                    (ctypes.c_float * 9)(*np.asarray(net["sd_in"], np.float32)),
                    (ctypes.c_float * 3)(*np.asarray(net["mu_out"], np.float32)),
                    (ctypes.c_float * 3)(*np.asarray(net["sd_out"], np.float32)))
    st = library().lbm_cbc_train_set_nn(t, ctypes.byref(n))
    del keep
    return _check(st, "lbm_cbc_train_set_nn")


def lbm_cbc_train_gradient(t, nparams=LBM_CBC_NPARAMS):
    g = np.zeros(nparams)
    loss = ctypes.c_double()
    _check(library().lbm_cbc_train_gradient(t, ctypes.byref(loss), _dptr(g)),
           "lbm_cbc_train_gradient")
    return loss.value, g


def lbm_cbc_train_step(t, nsteps):
    return _check(library().lbm_cbc_train_step(t, int(nsteps)), "lbm_cbc_train_step")


def lbm_cbc_train_loss(t):
    v = ctypes.c_double()
    _check(library().lbm_cbc_train_loss(t, ctypes.byref(v)), "lbm_cbc_train_loss")
    return v.value


def lbm_cbc_train_get_weights(t, nparams=LBM_CBC_NPARAMS):
    w = np.zeros(nparams, np.float32)
    _check(library().lbm_cbc_train_get_weights(t, w.ctypes.data_as(_FP)),
           "lbm_cbc_train_get_weights")
    return w


def lbm_cbc_train_final_state(t, seg, ny, width):
    out = np.empty((9, ny, width))
    _check(library().lbm_cbc_train_final_state(t, int(seg), _dptr(out)),
           "lbm_cbc_train_final_state")
    return out


def cbc_unflatten(v, shapes=None):
    """Split a flat parameter vector (w1, b1, w2, b2, w3, b3 order: 662 for
    the tuning network, 683 with NN9_PARAM_SHAPES) into arrays."""
    out, o = {}, 0
    for k, shp in (shapes or CBC_PARAM_SHAPES).items():
        n = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + n]).reshape(shp)
        o += n
    return out


class CbcTrainer:
    """Closed-loop trainer on the current device: of the CBC tuning network
    (outlet "cbc") or of the Eq. 16 reconstruction network (outlet "nn").

    a0 [n_seg][9][ny][2 n_max + 3]: start states of the segments (the last
    columns of the truncated lattice); ref [n_seg][3][ny][n_max]: reference
    rho, u, v at step n_t, right-aligned; n_t [n_seg]."""

    def __init__(self, a0, ref, n_t, net, *, tau, mach=0.0, length=1.0, rho_inf=1.0,
                 precision="fp32", lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, outlet="cbc"):
        import torch
        a0 = np.asarray(a0)
        n_seg, _, ny, width = a0.shape
        n_max = (width - 3) // 2
        if width != 2 * n_max + 3 or np.shape(ref) != (n_seg, 3, ny, n_max):
            raise ValueError("a0 must be [n_seg][9][ny][2 n_max + 3], ref [n_seg][3][ny][n_max]")
        self.ny, self.width, self.n_max, self.n_seg = ny, width, n_max, n_seg
        self.stream = torch.cuda.current_stream()
        self.params = lbm_cbc_train_params(ny, n_max, n_seg, _PREC[precision], tau, mach, length,
                                           rho_inf, lr, beta1, beta2, eps,
                                           ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = lbm_cbc_train_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.t = lbm_cbc_train_create(self.params, self.workspace.data_ptr(), nbytes)
        _live.add(self)
        lbm_cbc_train_set_segments(self.t, a0, ref, n_t)
        self.outlet = outlet
        self.set_net(net)

    def close(self):
        """Wait for the queued work and release the native object (also at
        interpreter exit and on garbage collection)."""
        h = getattr(self, "t", None)
        if h is not None and _lib is not None:
            _lib.lbm_cbc_train_destroy(h)
        self.t = None

    __del__ = close

    def set_net(self, net):
        if self.outlet == "nn":
            lbm_cbc_train_set_nn(self.t, net)
        else:
            lbm_cbc_train_set_net(self.t, net)

    def _shapes(self):
        return (NN9_PARAM_SHAPES, LBM_NN9_NPARAMS) if self.outlet == "nn" else \
            (CBC_PARAM_SHAPES, LBM_CBC_NPARAMS)

    def set_segment_params(self, tau=None, mach=None):
        """Per-segment relaxation time and Mach number (arrays of n_seg)."""
        lbm_cbc_train_set_segment_params(self.t, tau, mach)

    def gradient(self):
        """(loss, {w1: .., b3: ..}) of the current weights."""
        shapes, n = self._shapes()
        loss, g = lbm_cbc_train_gradient(self.t, n)
        return loss, cbc_unflatten(g, shapes)

    def step(self, n=1):
        lbm_cbc_train_step(self.t, n)

    def loss(self):
        return lbm_cbc_train_loss(self.t)

    def weights(self):
        shapes, n = self._shapes()
        return cbc_unflatten(lbm_cbc_train_get_weights(self.t, n), shapes)

    def final_state(self, seg):
        return lbm_cbc_train_final_state(self.t, seg, self.ny, self.width)


# --- the D3Q19 step (include/lbm3d.h) -----------------------------------------------

def lbm3d_workspace_bytes(params):
    n = library().lbm3d_workspace_bytes(ctypes.byref(params))
    if n == 0:
        raise LbmError(LBM_EINVAL, "lbm3d_workspace_bytes", library().lbm_last_error().decode())
    return n


def lbm3d_create(params, workspace_ptr, nbytes):
    c = ctypes.c_void_p()
    _check(library().lbm3d_create(ctypes.byref(params), ctypes.c_void_p(workspace_ptr), nbytes,
                                  ctypes.byref(c)), "lbm3d_create")
    return c


def lbm3d_destroy(c):
    return _check(library().lbm3d_destroy(c), "lbm3d_destroy")


def lbm3d_set_geometry(c, mask):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return _check(library().lbm3d_set_geometry(c, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
                  "lbm3d_set_geometry")


def lbm3d_init_fields(c, rho, u):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    return _check(library().lbm3d_init_fields(c, _dptr(rho), _dptr(u)), "lbm3d_init_fields")


def lbm3d_step(c, nsteps):
    return _check(library().lbm3d_step(c, int(nsteps)), "lbm3d_step")


def lbm3d_forces(c, allow_unstable=False):
    out = lbm3d_force_out()
    st = library().lbm3d_forces(c, ctypes.byref(out))
    if not (allow_unstable and st == LBM_EUNSTABLE):
        _check(st, "lbm3d_forces")
    return out


def lbm3d_force_history(c, cap):
    fx, fy, fz = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    n = ctypes.c_int64()
    _check(library().lbm3d_force_history(c, _dptr(fx), _dptr(fy), _dptr(fz), cap, ctypes.byref(n)),
           "lbm3d_force_history")
    return fx[:n.value], fy[:n.value], fz[:n.value]


def lbm3d_read_populations(c, nx, ny, nz):
    out = np.empty((19, nz, ny, nx))
    _check(library().lbm3d_read_populations(c, _dptr(out)), "lbm3d_read_populations")
    return out


def lbm3d_write_populations(c, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return _check(library().lbm3d_write_populations(c, _dptr(f)), "lbm3d_write_populations")


def lbm3d_sync(c):
    return _check(library().lbm3d_sync(c), "lbm3d_sync")


class Lattice3D:
    """One D3Q19 lattice on the current device; mask (nz, ny, nx) with 0 fluid
    and 1 body; lateral 'walls' / 'periodic' or a (y, z) pair."""

    def __init__(self, mask, tau, *, precision="fp32", lateral="walls", xbc="inout", u_in=0.05,
                 rho_out=1.0, history_cap=0):
        import torch
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.nz, self.ny, self.nx = mask.shape
        lat_y, lat_z = (lateral, lateral) if isinstance(lateral, str) else lateral
        self.stream = torch.cuda.current_stream()
        self.params = lbm3d_params(self.nx, self.ny, self.nz, _PREC[precision], _LAT[lat_y],
                                   _LAT[lat_z], _XBC[xbc], 0, tau, u_in, rho_out, history_cap,
                                   ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = lbm3d_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.ctx = lbm3d_create(self.params, self.workspace.data_ptr(), nbytes)
        _live.add(self)
        lbm3d_set_geometry(self.ctx, mask)
        self.history_cap = history_cap

    def close(self):
        """Wait for the queued work and release the native object (also at
        interpreter exit and on garbage collection)."""
        h = getattr(self, "ctx", None)
        if h is not None and _lib is not None:
            _lib.lbm3d_destroy(h)
        self.ctx = None

    __del__ = close

    def init_fields(self, rho, u):
        lbm3d_init_fields(self.ctx, rho, u)

    def step(self, n=1):
        lbm3d_step(self.ctx, n)

    def sync(self):
        lbm3d_sync(self.ctx)

    def forces(self, allow_unstable=False):
        return lbm3d_forces(self.ctx, allow_unstable)

    def force_history(self):
        return lbm3d_force_history(self.ctx, self.history_cap)

    def populations(self):
        return lbm3d_read_populations(self.ctx, self.nx, self.ny, self.nz)

    def write_populations(self, f):
        lbm3d_write_populations(self.ctx, f)


# --- convenience: one lattice with a torch-owned workspace --------------------------

_PREC = {"fp64": LBM_FP64, "fp32": LBM_FP32_OFFSET, "fp16": LBM_FP16_OFFSET}
_COLL = {"bgk": LBM_BGK, "mrt": LBM_MRT}
_LAT = {"walls": LBM_LATERAL_WALLS, "periodic": LBM_LATERAL_PERIODIC}
_XBC = {"inout": LBM_X_INOUT, "periodic": LBM_X_PERIODIC}
_LAUNCH = {"persistent": LBM_BATCH_PERSISTENT, "per_step": LBM_BATCH_PER_STEP}


_STEP_LAUNCH = {"auto": LBM_LAUNCH_AUTO, "pairs": LBM_LAUNCH_PAIRS, "single": LBM_LAUNCH_SINGLE,
                "pairs_plain": LBM_LAUNCH_PAIRS_PLAIN, "pairs_held": LBM_LAUNCH_PAIRS_HELD,
                "triples": LBM_LAUNCH_TRIPLES, "triples_plain": LBM_LAUNCH_TRIPLES_PLAIN,
                "triples_held": LBM_LAUNCH_TRIPLES_HELD}
_PATH = {"auto": LBM_PATH_AUTO, "scalar": LBM_PATH_SCALAR, "vector": LBM_PATH_VECTOR}
# Kernel schedule of Lattice objects created without explicit launch /
# bulk_path arguments (passed to the library in lbm_params).
LATTICE_DEFAULTS = {"launch": "auto", "bulk_path": "auto"}


class Lattice:
    """A lattice on the current CUDA (HIP) device.  The workspace is a torch
    uint8 tensor and the stream is torch's current stream."""

    def __init__(self, mask, tau, *, precision="fp32", collision="bgk", lateral="walls",
                 xbc="inout", u_in=0.05, rho_out=1.0, s_e=1.0, s_eps=1.0, s_q=0.0,
                 noise_amp=0.0, seed=0, history_cap=0, launch=None, bulk_path=None,
                 device="cuda"):
        import torch
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.ny, self.nx = mask.shape
        self.stream = torch.cuda.current_stream(device)
        launch = LATTICE_DEFAULTS["launch"] if launch is None else launch
        bulk_path = LATTICE_DEFAULTS["bulk_path"] if bulk_path is None else bulk_path
        self.params = lbm_params(self.nx, self.ny, _PREC[precision], _COLL[collision],
                                 _LAT[lateral], _XBC[xbc], _STEP_LAUNCH[launch], _PATH[bulk_path],
                                 tau, s_e, s_eps, s_q, u_in,
                                 rho_out, noise_amp, seed, history_cap,
                                 ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = lbm_workspace_bytes(self.params)
        # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert self.workspace.data_ptr() % 256 == 0
        self.ctx = lbm_create(self.params, self.workspace.data_ptr(), nbytes)
        _live.add(self)
        lbm_set_geometry(self.ctx, mask)
        self.history_cap = history_cap

    def close(self):
        """Wait for the queued work and release the native object (also at
        interpreter exit and on garbage collection)."""
        h = getattr(self, "ctx", None)
        if h is not None and _lib is not None:
            _lib.lbm_destroy(h)
        self.ctx = None

    __del__ = close

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

    def set_outflow_cbc(self, sigma=0.0, kappa2=0.0, mach=0.0, length=None, rho_inf=1.0,
                        net=None):
        """Characteristic outflow (lbm_set_outflow_cbc); length defaults to nx."""
        lbm_set_outflow_cbc(self.ctx, sigma, kappa2, mach,
                            float(self.nx if length is None else length), rho_inf, net)

    def macroscopic(self):
        return lbm_read_macroscopic(self.ctx, self.nx, self.ny)

    def sync(self):
        lbm_sync(self.ctx)
