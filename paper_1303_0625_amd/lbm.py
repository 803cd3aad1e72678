"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every function of the header is exposed under the same name; ``Lattice``
wraps a context whose device workspace and stream come from PyTorch.  All
arithmetic of the time step, the forces and the fields runs in the HIP
kernels of liblbm.so: there is no host fallback, and loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ESIZE, LBM_EDEVICE, LBM_ENUMERIC, LBM_ESTATE, LBM_EGEOM = 0, -1, -2, -3, -4, -5, -6
LBM_F64, LBM_F32, LBM_F16, LBM_BF16 = 0, 1, 2, 3
LBM_CME, LBM_GME = 0, 1
LBM_REFILL_A1, LBM_REFILL_A2, LBM_REFILL_A3 = 0, 1, 2
LBM_DISC, LBM_BOX = 0, 1

STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ESIZE", -3: "LBM_EDEVICE",
                -4: "LBM_ENUMERIC", -5: "LBM_ESTATE", -6: "LBM_EGEOM"}
DTYPES = {"f64": LBM_F64, "f32": LBM_F32, "f16": LBM_F16, "bf16": LBM_BF16}


class lbm_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("walls_y", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("refill", ctypes.c_int32),
                ("rho_w_local", ctypes.c_int32), ("rho0", ctypes.c_double),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("u0x", ctypes.c_double),
                ("u0y", ctypes.c_double), ("wall_vx", ctypes.c_double),
                ("wall_vy", ctypes.c_double)]


class lbm_nn_config(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("w", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("ch", ctypes.c_int32 * 4), ("rho_scale", ctypes.c_double)]


class lbm_solid(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("moves", ctypes.c_int32), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("vx", ctypes.c_double), ("vy", ctypes.c_double)]


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
class lbm3d_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("duct", ctypes.c_int32), ("refill", ctypes.c_int32),
                ("R", ctypes.c_double), ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("u0", ctypes.c_double * 3)]


class lbm3d_sphere(ctypes.Structure):
    _fields_ = [("X", ctypes.c_double * 3), ("r", ctypes.c_double), ("V", ctypes.c_double * 3),
                ("omega", ctypes.c_double * 3), ("moves", ctypes.c_int32), ("pad", ctypes.c_int32)]


_SIG = {
    "lbm_abi_version": (_I32, []),
    "lbm_workspace_bytes": (_I32, [ctypes.POINTER(lbm_grid), ctypes.POINTER(lbm_solid), _I32, _I64,
                                   ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_create": (_I32, [ctypes.POINTER(lbm_grid), ctypes.c_double, ctypes.POINTER(lbm_solid), _I32,
                          _I64, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lbm_create_static": (_I32, [ctypes.POINTER(lbm_grid), ctypes.c_double, ctypes.POINTER(lbm_solid), _I32,
                                 _I64, _VP, ctypes.POINTER(_VP)]),
    "lbm_step": (_I32, [_VP, _I64]),
    "lbm_time": (_I64, [_VP]),
    "lbm_force": (_I32, [_VP, _I32, _I32, ctypes.POINTER(ctypes.c_double)]),
    "lbm_force_history": (_I32, [_VP, _I64, _I64, _VP]),
    "lbm_fields": (_I32, [_VP, _VP, _VP, _VP, _I32, _VP]),
    "lbm_init_fields": (_I32, [_VP, _VP, _VP, _VP, _I32]),
    "lbm_populations": (_I32, [_VP, _VP]),
    "lbm_link_forces": (_I32, [_VP, _VP, _I64, ctypes.POINTER(_I64)]),
    "lbm_checkpoint_bytes": (_I32, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_save": (_I32, [_VP, _VP, ctypes.c_size_t]),
    "lbm_load": (_I32, [_VP, _VP, ctypes.c_size_t]),
    "lbm_profile": (_I32, [_VP, _I32]),
    "lbm_profile_read": (_I32, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "lbm_status_check": (_I32, [_VP]),
    "lbm_destroy": (None, [_VP]),
    "lbm_last_error": (ctypes.c_char_p, [_VP]),
    "lbm_batch_workspace_bytes": (_I32, [ctypes.POINTER(lbm_grid), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(lbm_solid), ctypes.POINTER(_I32), _I32,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_batch_create": (_I32, [ctypes.POINTER(lbm_grid), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(lbm_solid), ctypes.POINTER(_I32), _I32, _VP,
                                ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lbm_batch_autotune": (_I32, [_VP, ctypes.c_char_p]),
    "lbm_batch_tiling": (_I32, [_VP, ctypes.POINTER(_I32)]),
    "lbm_batch_set_tiling": (_I32, [_VP, _I32, _I32]),
    "lbm_batch_set_graph": (_I32, [_VP, _I32]),
    "lbm_batch_step": (_I32, [_VP, _I64]),
    "lbm_batch_monitor": (_I32, [_VP, ctypes.c_double]),
    "lbm_batch_run": (_I32, [_VP, _I64, ctypes.c_double, _I32, ctypes.POINTER(_I64)]),
    "lbm_batch_status": (_I32, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "lbm_batch_force": (_I32, [_VP, _I32, _I32, _I32, ctypes.POINTER(ctypes.c_double)]),
    "lbm_batch_fields": (_I32, [_VP, _I32, _VP, _VP, _VP, _I32, _VP]),
    "lbm_batch_init_poiseuille": (_I32, [_VP, _I32]),
    "lbm_batch_set_active": (_I32, [_VP, _I32, _I32]),
    "lbm_init_poiseuille": (_I32, [_VP]),
    "lbm_set_collision": (_I32, [_VP, _I32, _VP]),
    "lbm_set_boundary": (_I32, [_VP, _I32]),
    "lbm_set_free_body": (_I32, [_VP, _I32, ctypes.c_double, ctypes.c_double]),
    "lbm_set_gravity": (_I32, [_VP, ctypes.c_double, ctypes.c_double, _I32]),
    "lbm_body_state": (_I32, [_VP, _I32, _VP]),
    "lbm_batch_init_fields": (_I32, [_VP, _I32, _VP, _VP, _VP, _I32]),
    "lbm_batch_time": (_I64, [_VP]),
    "lbm_batch_destroy": (None, [_VP]),
    "lbm_batch_last_error": (ctypes.c_char_p, [_VP]),
    "lbm_nn_workspace_bytes": (_I32, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_nn_create": (_I32, [_VP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lbm_nn_param_count": (_I64, [_VP]),
    "lbm_nn_set_params": (_I32, [_VP, _VP]),
    "lbm_nn_get_params": (_I32, [_VP, _VP]),
    "lbm_nn_get_grads": (_I32, [_VP, _VP]),
    "lbm_nn_forward": (_I32, [_VP, _VP, _I32, _VP]),
    "lbm_nn_backward": (_I32, [_VP, _VP]),
    "lbm_nn_layer_wgrad": (_I32, [_VP, _I32, _I32, _VP, _I32, _VP, _I32, _VP]),
    "lbm_nn_layer_forward": (_I32, [_VP, _I32, _I32, _VP, _I32, _VP, _I32]),
    "lbm_nn_adam": (_I32, [_VP, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lbm_nn_train_step": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I32, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double)]),
    "lbm_nn_eval": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I32,
                           ctypes.POINTER(ctypes.c_double)]),
    "lbm_nn_infer": (_I32, [_VP, _VP, _VP, _VP, _VP, _I32, _VP, _VP, _VP]),
    "lbm_warm_project": (_I32, [_I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP]),
    "lbm_warm_check": (_I32, [_I32, _I32, _I32, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_double, _VP, _VP]),
    "lbm_nn_destroy": (None, [_VP]),
    "lbm_nn_last_error": (ctypes.c_char_p, [_VP]),
    "lbm3d_workspace_bytes": (_I32, [ctypes.POINTER(lbm3d_grid), ctypes.POINTER(lbm3d_sphere), _I32, _I64,
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "lbm3d_create": (_I32, [ctypes.POINTER(lbm3d_grid), ctypes.POINTER(lbm3d_sphere), _I32, _I64, _VP,
                            ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lbm3d_step": (_I32, [_VP, _I64]),
    "lbm3d_time": (_I64, [_VP]),
    "lbm3d_force": (_I32, [_VP, _I32, _I32, _I64, ctypes.POINTER(ctypes.c_double)]),
    "lbm3d_force_history": (_I32, [_VP, _I64, _I64, _VP]),
    "lbm3d_fields": (_I32, [_VP, _VP, _VP, _VP]),
    "lbm3d_link_count": (_I64, [_VP]),
    "lbm3d_set_free": (_I32, [_VP, _I32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "lbm3d_set_gravity": (_I32, [_VP, ctypes.POINTER(ctypes.c_double), _I32]),
    "lbm3d_body_state": (_I32, [_VP, _I32, ctypes.POINTER(ctypes.c_double)]),
    "lbm3d_set_force_average": (_I32, [_VP, _I32]),
    "lbm3d_set_pressure": (_I32, [_VP, ctypes.c_double, ctypes.c_double]),
    "lbm3d_set_boundary": (_I32, [_VP, _I32]),
    "lbm3d_status_check": (_I32, [_VP]),
    "lbm3d_profile": (_I32, [_VP, _I32]),
    "lbm3d_profile_read": (_I32, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "lbm3d_destroy": (None, [_VP]),
    "lbm3d_last_error": (ctypes.c_char_p, [_VP]),
}


def load_library(path: str = LIB_PATH):
    """Load liblbm.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_1303_0625_amd.build.build_library()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIG.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIG)


def _check(status, ctx=None):
    if status != LBM_OK:
        msg = load_library().lbm_last_error(ctx)
        raise LBMError(status, msg.decode() if msg else "")


# ---- thin wrappers with the header's names --------------------------------
def lbm_abi_version() -> int:
    return load_library().lbm_abi_version()


def lbm_workspace_bytes(grid: lbm_grid, solids, history_steps: int) -> int:
    arr, n = _solid_array(solids)
    out = ctypes.c_size_t(0)
    _check(load_library().lbm_workspace_bytes(ctypes.byref(grid), arr, n, history_steps,
                                              ctypes.byref(out)))
    return out.value


def lbm_create(grid: lbm_grid, tau: float, solids, history_steps: int, d_workspace: int,
               nbytes: int, stream: int):
    arr, n = _solid_array(solids)
    ctx = _VP()
    _check(load_library().lbm_create(ctypes.byref(grid), tau, arr, n, history_steps, d_workspace,
                                     nbytes, stream, ctypes.byref(ctx)))
    return ctx


def lbm_create_static(grid: lbm_grid, tau: float, solids, history_steps: int, stream: int):
    """lbm_create with the context in the library's static scratch (no device
    allocation); one such context per device at a time."""
    arr, n = _solid_array(solids)
    ctx = _VP()
    _check(load_library().lbm_create_static(ctypes.byref(grid), tau, arr, n, history_steps, stream,
                                            ctypes.byref(ctx)))
    return ctx


def lbm_step(ctx, n: int) -> None:
    _check(load_library().lbm_step(ctx, n), ctx)


def lbm_time(ctx) -> int:
    return load_library().lbm_time(ctx)


def lbm_force(ctx, solid_id: int, scheme: int):
    out = (ctypes.c_double * 3)()
    _check(load_library().lbm_force(ctx, solid_id, scheme, out), ctx)
    return list(out)


def lbm_force_history(ctx, first: int, count: int, d_out: int) -> None:
    _check(load_library().lbm_force_history(ctx, first, count, d_out), ctx)


def lbm_fields(ctx, d_rho, d_ux, d_uy, out_dtype: int, d_owner) -> None:
    _check(load_library().lbm_fields(ctx, d_rho, d_ux, d_uy, out_dtype, d_owner), ctx)


def lbm_init_fields(ctx, d_rho, d_ux, d_uy, in_dtype: int) -> None:
    _check(load_library().lbm_init_fields(ctx, d_rho, d_ux, d_uy, in_dtype), ctx)


def lbm_populations(ctx, d_out) -> None:
    _check(load_library().lbm_populations(ctx, d_out), ctx)


def lbm_link_forces(ctx, d_out, max_records: int) -> int:
    n = _I64(0)
    _check(load_library().lbm_link_forces(ctx, d_out, max_records, ctypes.byref(n)), ctx)
    return n.value


def lbm_checkpoint_bytes(ctx) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().lbm_checkpoint_bytes(ctx, ctypes.byref(out)), ctx)
    return out.value


def lbm_save(ctx, d_dst, nbytes: int) -> None:
    _check(load_library().lbm_save(ctx, d_dst, nbytes), ctx)


def lbm_load(ctx, d_src, nbytes: int) -> None:
    _check(load_library().lbm_load(ctx, d_src, nbytes), ctx)


def lbm_profile(ctx, enable: bool) -> None:
    _check(load_library().lbm_profile(ctx, int(bool(enable))), ctx)


def lbm_profile_read(ctx):
    ms = ctypes.c_double(0.0)
    n = _I64(0)
    _check(load_library().lbm_profile_read(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def lbm_status_check(ctx) -> None:
    _check(load_library().lbm_status_check(ctx), ctx)


def lbm_destroy(ctx) -> None:
    load_library().lbm_destroy(ctx)


def lbm_last_error(ctx=None) -> str:
    m = load_library().lbm_last_error(ctx)
    return m.decode() if m else ""


# ---- batched steady-state solver -------------------------------------------
def _bcheck(status, b=None):
    if status != LBM_OK:
        msg = load_library().lbm_batch_last_error(b)
        raise LBMError(status, msg.decode() if msg else "")


def _batch_arrays(grids, taus, solids_per_case):
    n = len(grids)
    garr = (lbm_grid * n)(*grids)
    tarr = (ctypes.c_double * n)(*[float(t) for t in taus])
    flat = [b for case in solids_per_case for b in case]
    sarr, _ = _solid_array(flat)
    narr = (_I32 * n)(*[len(case) for case in solids_per_case])
    return garr, tarr, sarr, narr, n


def lbm_batch_workspace_bytes(grids, taus, solids_per_case) -> int:
    garr, tarr, sarr, narr, n = _batch_arrays(grids, taus, solids_per_case)
    out = ctypes.c_size_t(0)
    _bcheck(load_library().lbm_batch_workspace_bytes(garr, tarr, sarr, narr, n, ctypes.byref(out)))
    return out.value


def lbm_batch_create(grids, taus, solids_per_case, d_workspace: int, nbytes: int, stream: int):
    garr, tarr, sarr, narr, n = _batch_arrays(grids, taus, solids_per_case)
    b = _VP()
    _bcheck(load_library().lbm_batch_create(garr, tarr, sarr, narr, n, d_workspace, nbytes, stream,
                                            ctypes.byref(b)))
    return b


def lbm_batch_autotune(b, cache_path=None) -> None:
    _bcheck(load_library().lbm_batch_autotune(b, cache_path.encode() if cache_path else None), b)


def lbm_batch_tiling(b):
    nt = _I32(0)
    w = load_library().lbm_batch_tiling(b, ctypes.byref(nt))
    return w, nt.value


def lbm_batch_set_tiling(b, waves: int, nontemporal: bool) -> None:
    _bcheck(load_library().lbm_batch_set_tiling(b, int(waves), int(bool(nontemporal))), b)


def lbm_batch_set_graph(b, enable: bool) -> None:
    _bcheck(load_library().lbm_batch_set_graph(b, int(bool(enable))), b)


def lbm_batch_step(b, n: int) -> None:
    _bcheck(load_library().lbm_batch_step(b, n), b)


def lbm_batch_monitor(b, tol: float) -> None:
    _bcheck(load_library().lbm_batch_monitor(b, tol), b)


def lbm_batch_run(b, max_steps: int, tol: float, check_every: int) -> int:
    done = _I64(0)
    _bcheck(load_library().lbm_batch_run(b, max_steps, tol, check_every, ctypes.byref(done)), b)
    return done.value


def lbm_batch_status(b, n_cases: int):
    conv = (_I32 * n_cases)()
    steps = (_I64 * n_cases)()
    res = (ctypes.c_double * n_cases)()
    drag = (ctypes.c_double * (2 * n_cases))()
    _bcheck(load_library().lbm_batch_status(b, conv, steps, res, drag), b)
    return list(conv), list(steps), list(res), [(drag[2 * k], drag[2 * k + 1]) for k in range(n_cases)]


def lbm_batch_force(b, case_id: int, solid_id: int, scheme: int):
    out = (ctypes.c_double * 3)()
    _bcheck(load_library().lbm_batch_force(b, case_id, solid_id, scheme, out), b)
    return list(out)


def lbm_batch_fields(b, case_id: int, d_rho, d_ux, d_uy, out_dtype: int, d_owner=None) -> None:
    _bcheck(load_library().lbm_batch_fields(b, case_id, d_rho, d_ux, d_uy, out_dtype, d_owner), b)


def lbm_batch_set_active(b, case_id: int, active: bool) -> None:
    _bcheck(load_library().lbm_batch_set_active(b, case_id, int(bool(active))), b)


def lbm_batch_init_poiseuille(b, case_id: int) -> None:
    _bcheck(load_library().lbm_batch_init_poiseuille(b, case_id), b)


LBM_BGK, LBM_MRT = 0, 1
LBM_HALFWAY, LBM_INTERPOLATED = 0, 1


def lbm_set_boundary(ctx, rule: int) -> None:
    _check(load_library().lbm_set_boundary(ctx, int(rule)), ctx)
# relaxation rates (s_e, s_eps, s_q) of the paper's MRT simulations (Sec. IV)
PAPER_MRT_RATES = (1.64, 1.54, 1.9)


def lbm_set_collision(ctx, model: int, rates=None) -> None:
    arr = (ctypes.c_double * 3)(*(rates if rates is not None else (0.0, 0.0, 0.0)))
    _check(load_library().lbm_set_collision(ctx, int(model), arr), ctx)


def lbm_set_free_body(ctx, solid_id: int, rho_s: float, omega0: float = 0.0) -> None:
    _check(load_library().lbm_set_free_body(ctx, int(solid_id), float(rho_s), float(omega0)), ctx)


def lbm_set_gravity(ctx, gx: float, gy: float, scheme: int) -> None:
    _check(load_library().lbm_set_gravity(ctx, float(gx), float(gy), int(scheme)), ctx)


def lbm_body_state(ctx, solid_id: int):
    out = (ctypes.c_double * 5)()
    _check(load_library().lbm_body_state(ctx, int(solid_id), out), ctx)
    return list(out)


def lbm_init_poiseuille(ctx) -> None:
    _check(load_library().lbm_init_poiseuille(ctx), ctx)


def lbm_batch_init_fields(b, case_id: int, d_rho, d_ux, d_uy, in_dtype: int) -> None:
    _bcheck(load_library().lbm_batch_init_fields(b, case_id, d_rho, d_ux, d_uy, in_dtype), b)


def lbm_batch_time(b) -> int:
    return load_library().lbm_batch_time(b)


def lbm_batch_destroy(b) -> None:
    load_library().lbm_batch_destroy(b)


def lbm_batch_last_error(b=None) -> str:
    m = load_library().lbm_batch_last_error(b)
    return m.decode() if m else ""


# ---- warm-start network ----------------------------------------------------
def _ncheck(status, n=None):
    if status != LBM_OK:
        msg = load_library().lbm_nn_last_error(n)
        raise LBMError(status, msg.decode() if msg else "")


def lbm_nn_workspace_bytes(cfg: lbm_nn_config) -> int:
    out = ctypes.c_size_t(0)
    _ncheck(load_library().lbm_nn_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def lbm_nn_create(cfg: lbm_nn_config, d_workspace: int, nbytes: int, stream: int):
    n = _VP()
    _ncheck(load_library().lbm_nn_create(ctypes.byref(cfg), d_workspace, nbytes, stream, ctypes.byref(n)))
    return n


def lbm_nn_param_count(n) -> int:
    return load_library().lbm_nn_param_count(n)


def lbm_nn_set_params(n, d_params) -> None:
    _ncheck(load_library().lbm_nn_set_params(n, d_params), n)


def lbm_nn_get_params(n, d_out) -> None:
    _ncheck(load_library().lbm_nn_get_params(n, d_out), n)


def lbm_nn_get_grads(n, d_out) -> None:
    _ncheck(load_library().lbm_nn_get_grads(n, d_out), n)


def lbm_nn_forward(n, d_x, batch: int, d_y) -> None:
    _ncheck(load_library().lbm_nn_forward(n, d_x, batch, d_y), n)


def lbm_nn_backward(n, d_gy) -> None:
    _ncheck(load_library().lbm_nn_backward(n, d_gy), n)


def lbm_nn_layer_forward(n, layer, batch, d_x, x_cs, d_y, y_cs) -> None:
    _ncheck(load_library().lbm_nn_layer_forward(n, layer, batch, d_x, x_cs, d_y, y_cs), n)


def lbm_nn_layer_wgrad(n, layer, batch, d_x, x_cs, d_g, g_cs, d_grad) -> None:
    _ncheck(load_library().lbm_nn_layer_wgrad(n, layer, batch, d_x, x_cs, d_g, g_cs, d_grad), n)


def lbm_nn_adam(n, lr, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    _ncheck(load_library().lbm_nn_adam(n, lr, beta1, beta2, eps), n)


def lbm_nn_train_step(n, d_solid, d_rho, d_ux, d_uy, d_re, d_gx, d_tau, d_idx, d_aug, batch: int, lr: float,
                      want_loss: bool = False):
    loss = ctypes.c_double(0.0)
    _ncheck(load_library().lbm_nn_train_step(n, d_solid, d_rho, d_ux, d_uy, d_re, d_gx, d_tau, d_idx, d_aug, batch,
                                             lr, ctypes.byref(loss) if want_loss else None), n)
    return loss.value if want_loss else None


def lbm_nn_eval(n, d_solid, d_rho, d_ux, d_uy, d_re, d_gx, d_tau, d_idx, batch: int) -> float:
    loss = ctypes.c_double(0.0)
    _ncheck(load_library().lbm_nn_eval(n, d_solid, d_rho, d_ux, d_uy, d_re, d_gx, d_tau, d_idx, batch,
                                       ctypes.byref(loss)), n)
    return loss.value


def lbm_nn_infer(n, d_solid, d_re, d_gx, d_tau, batch: int, d_rho, d_ux, d_uy) -> None:
    _ncheck(load_library().lbm_nn_infer(n, d_solid, d_re, d_gx, d_tau, batch, d_rho, d_ux, d_uy), n)


def lbm_warm_project(nx: int, ny: int, n_fields: int, d_owner, d_rho, d_ux, d_uy, d_rho2, d_ux2, d_uy2,
                     rho0: float, stream) -> None:
    _ncheck(load_library().lbm_warm_project(nx, ny, n_fields, d_owner, d_rho, d_ux, d_uy, d_rho2, d_ux2, d_uy2,
                                            rho0, stream))


def warm_project(owner, rho, ux, uy, rho0=1.0, second=None):
    """In-place projection of warm-start fields (torch CUDA tensors
    [n][ny][nx]: owner uint8, rho/ux/uy float32) on the current stream;
    second = (rho2, ux2, uy2) averages that set in first."""
    import torch

    for t in (owner, rho, ux, uy) + (tuple(second) if second else ()):
        assert t.is_contiguous() and t.is_cuda
    n, ny, nx = rho.shape
    p2 = [t.data_ptr() for t in second] if second else [None, None, None]
    lbm_warm_project(nx, ny, n, owner.data_ptr(), rho.data_ptr(), ux.data_ptr(), uy.data_ptr(), *p2, rho0,
                     torch.cuda.current_stream(rho.device).cuda_stream)


def lbm_warm_check(nx: int, ny: int, n_fields: int, d_owner, d_rho, d_ux, d_uy, rho0: float, u_max: float,
                   d_ok, hip_stream) -> None:
    _ncheck(load_library().lbm_warm_check(nx, ny, n_fields, d_owner, d_rho, d_ux, d_uy, rho0, u_max, d_ok,
                                          hip_stream), None)


def warm_check(owner, rho, ux, uy, rho0=1.0, u_max=0.3):
    """Per channel, whether warm-start fields (torch CUDA tensors [n][ny][nx]:
    owner uint8, rho/ux/uy float32) are safe to start from: int32 tensor [n],
    1 when every fluid node has a finite density in (0, 2 rho0) and a finite
    speed <= u_max."""
    import torch

    for t in (owner, rho, ux, uy):
        assert t.is_contiguous() and t.is_cuda
    n, ny, nx = rho.shape
    ok = torch.empty(n, dtype=torch.int32, device=rho.device)
    lbm_warm_check(nx, ny, n, owner.data_ptr(), rho.data_ptr(), ux.data_ptr(), uy.data_ptr(), rho0, u_max,
                   ok.data_ptr(), torch.cuda.current_stream(rho.device).cuda_stream)
    return ok


def lbm_nn_destroy(n) -> None:
    load_library().lbm_nn_destroy(n)


def lbm_nn_last_error(n=None) -> str:
    m = load_library().lbm_nn_last_error(n)
    return m.decode() if m else ""


# ---- helpers ---------------------------------------------------------------
def _solid_array(solids):
    solids = list(solids)
    n = len(solids)
    arr = (lbm_solid * max(n, 1))()
    for k, b in enumerate(solids):
        if isinstance(b, lbm_solid):
            arr[k] = b
            continue
        kind = b.get("kind", "disc")
        box = kind in ("box", LBM_BOX)
        arr[k].shape = LBM_BOX if box else LBM_DISC
        arr[k].moves = int(bool(b.get("moves", False)))
        arr[k].cx = float(b["cx"])
        arr[k].cy = float(b["cy"])
        arr[k].a = float(b["hx"] if box else b["r"])
        arr[k].b = float(b.get("hy", 0.0)) if box else 0.0
        arr[k].vx = float(b.get("vx", 0.0))
        arr[k].vy = float(b.get("vy", 0.0))
    return arr, n


def make_grid(case: dict, dtype="f64") -> lbm_grid:
    g = lbm_grid()
    g.nx, g.ny = case["nx"], case["ny"]
    g.walls_y = int(case.get("walls_y", False))
    g.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    g.refill = int(case.get("refill", 0))
    g.rho_w_local = 0
    g.rho0 = float(case.get("rho0", 1.0))
    g.gx, g.gy = float(case.get("gx", 0.0)), float(case.get("gy", 0.0))
    u0 = case.get("u0", (0.0, 0.0))
    g.u0x, g.u0y = float(u0[0]), float(u0[1])
    wv = case.get("wall_v", (0.0, 0.0))
    g.wall_vx, g.wall_vy = float(wv[0]), float(wv[1])
    return g


class Lattice:
    """One simulation on the current CUDA (HIP) device.

    The workspace is a torch uint8 tensor; kernels are enqueued on torch's
    current stream at creation time.
    """

    def __init__(self, case: dict, dtype="f64", history_steps=None, device="cuda", stream=None, mrt=None,
                 static=False):
        """mrt: None for the BGK operator, else the MRT rates (s_e, s_eps, s_q).
        static: the context lives in the library's static scratch
        (lbm_create_static) instead of a workspace tensor."""
        import torch

        self.torch = torch
        self.case = case
        self.dtype = dtype
        self.nx, self.ny = case["nx"], case["ny"]
        self.n_solids = len(case.get("bodies", ()))
        self.grid = make_grid(case, dtype)
        if history_steps is None:
            history_steps = max(1, int(case.get("steps", 0)) or 1024)
        self.history_steps = int(history_steps)
        solids = case.get("bodies", ())
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._destroy = load_library().lbm_destroy  # usable at interpreter exit
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        if static:
            self.workspace = None  # the library's static scratch holds the context
            self.ctx = lbm_create_static(self.grid, float(case["tau"]), solids, self.history_steps,
                                         self.stream.cuda_stream)
        else:
            nbytes = lbm_workspace_bytes(self.grid, solids, self.history_steps)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            self.ctx = lbm_create(self.grid, float(case["tau"]), solids, self.history_steps,
                                  self._ws_ptr, nbytes, self.stream.cuda_stream)
        if mrt is not None:
            lbm_set_collision(self.ctx, LBM_MRT, tuple(float(r) for r in mrt))

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            self._destroy(ctx)
            self.ctx = None

    @property
    def t(self) -> int:
        return lbm_time(self.ctx)

    def step(self, n: int = 1) -> None:
        lbm_step(self.ctx, int(n))

    def force(self, solid_id: int, scheme: int):
        return lbm_force(self.ctx, solid_id, scheme)

    def force_history(self, first=0, count=None):
        """float64 tensor [count][n_solids+1][6] (CME Fx Fy Tz, GME Fx Fy Tz)."""
        t = self.t
        if count is None:
            count = t - first
        out = self.torch.empty((count, self.n_solids + 1, 6), dtype=self.torch.float64,
                               device=self.device)
        lbm_force_history(self.ctx, first, count, out.data_ptr())
        return out

    def fields(self, out_dtype="f64"):
        tdt = self.torch.float64 if out_dtype == "f64" else self.torch.float32
        shp = (self.ny, self.nx)
        dev = self.device
        rho = self.torch.empty(shp, dtype=tdt, device=dev)
        ux = self.torch.empty(shp, dtype=tdt, device=dev)
        uy = self.torch.empty(shp, dtype=tdt, device=dev)
        own = self.torch.empty(shp, dtype=self.torch.uint8, device=dev)
        lbm_fields(self.ctx, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(), DTYPES[out_dtype],
                   own.data_ptr())
        return rho, ux, uy, own

    def init_fields(self, rho, ux, uy):
        dt = LBM_F64 if rho.dtype == self.torch.float64 else LBM_F32
        rho, ux, uy = (a.contiguous() for a in (rho, ux, uy))
        lbm_init_fields(self.ctx, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(), dt)
        self._keep = (rho, ux, uy)

    def init_poiseuille(self) -> None:
        lbm_init_poiseuille(self.ctx)

    def set_free(self, solid_id: int, rho_s: float, omega0: float = 0.0) -> None:
        """Body solid_id (a disc created with moves=True) becomes a free particle."""
        lbm_set_free_body(self.ctx, solid_id, rho_s, omega0)

    def set_gravity(self, G, scheme: int = 1) -> None:
        lbm_set_gravity(self.ctx, G[0], G[1], scheme)

    def set_boundary(self, interpolated: bool = True) -> None:
        """Interpolated (True) or half-way (False) bounce-back on body links."""
        lbm_set_boundary(self.ctx, LBM_INTERPOLATED if interpolated else LBM_HALFWAY)

    def body_state(self, solid_id: int):
        """[X, Y, V_x, V_y, Omega] of a body at the current step."""
        return lbm_body_state(self.ctx, solid_id)

    def populations(self):
        out = self.torch.empty((9, self.ny, self.nx), dtype=self.torch.float64,
                               device=self.device)
        lbm_populations(self.ctx, out.data_ptr())
        return out

    def link_forces(self):
        """float64 tensor [n_links][8] of the links the next step evaluates."""
        lib = load_library()
        n = _I64(0)
        st = lib.lbm_link_forces(self.ctx, None, 0, ctypes.byref(n))
        if st not in (LBM_OK, LBM_ESIZE):
            _check(st, self.ctx)
        out = self.torch.empty((max(n.value, 1), 8), dtype=self.torch.float64,
                               device=self.device)
        got = lbm_link_forces(self.ctx, out.data_ptr(), out.shape[0])
        return out[:got]

    def checkpoint_bytes(self) -> int:
        return lbm_checkpoint_bytes(self.ctx)

    def save(self):
        nb = self.checkpoint_bytes()
        buf = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        lbm_save(self.ctx, buf.data_ptr(), nb)
        return buf

    def load(self, buf) -> None:
        lbm_load(self.ctx, buf.data_ptr(), buf.numel())

    def check(self) -> None:
        lbm_status_check(self.ctx)

    def profile(self, enable: bool = True) -> None:
        lbm_profile(self.ctx, enable)

    def profile_read(self):
        """(summed ms, launches) of the lattice-update kernel since profile()."""
        return lbm_profile_read(self.ctx)


class LatticeBatch:
    """Many fixed-geometry lattices advanced together to steady state.

    ``cases`` is a list of case dicts (as for ``Lattice``; bodies must not
    move), all with one storage dtype.  The workspace is a torch uint8 tensor.
    """

    def __init__(self, cases, dtype="f32", device="cuda", stream=None):
        import torch

        self.torch = torch
        self.cases = list(cases)
        self.n = len(self.cases)
        self.dtype = dtype
        self.grids = [make_grid(c, dtype) for c in self.cases]
        self.taus = [float(c["tau"]) for c in self.cases]
        solids = [list(c.get("bodies", ())) for c in self.cases]
        self.n_solids = [len(s) for s in solids]
        nbytes = lbm_batch_workspace_bytes(self.grids, self.taus, solids)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._destroy = load_library().lbm_batch_destroy  # usable at interpreter exit
        self.b = lbm_batch_create(self.grids, self.taus, solids, self._ws_ptr, nbytes,
                                  self.stream.cuda_stream)

    def __del__(self):
        b = getattr(self, "b", None)
        if b:
            self._destroy(b)
            self.b = None

    @property
    def t(self) -> int:
        return lbm_batch_time(self.b)

    def autotune(self, cache_path=None) -> None:
        lbm_batch_autotune(self.b, cache_path)

    def tiling(self):
        return lbm_batch_tiling(self.b)

    def set_tiling(self, waves: int, nontemporal: bool = False) -> None:
        lbm_batch_set_tiling(self.b, waves, nontemporal)

    def set_graph(self, enable: bool) -> None:
        lbm_batch_set_graph(self.b, enable)

    def step(self, n: int = 1) -> None:
        lbm_batch_step(self.b, int(n))

    def monitor(self, tol: float = -1.0) -> None:
        lbm_batch_monitor(self.b, float(tol))

    def run(self, max_steps: int, tol: float, check_every: int = 100) -> int:
        return lbm_batch_run(self.b, int(max_steps), float(tol), int(check_every))

    def status(self):
        """(converged, steps, residual, [(CME drag, GME drag)]) per case."""
        return lbm_batch_status(self.b, self.n)

    def force(self, case_id: int, solid_id: int, scheme: int):
        return lbm_batch_force(self.b, case_id, solid_id, scheme)

    def fields(self, case_id: int, out_dtype="f64", owner=False):
        """rho, ux, uy [ny][nx] (and the uint8 owner map when owner=True)."""
        c = self.cases[case_id]
        tdt = self.torch.float64 if out_dtype == "f64" else self.torch.float32
        shp = (c["ny"], c["nx"])
        dev = self.workspace.device
        rho, ux, uy = (self.torch.empty(shp, dtype=tdt, device=dev) for _ in range(3))
        own = self.torch.empty(shp, dtype=self.torch.uint8, device=dev) if owner else None
        lbm_batch_fields(self.b, case_id, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(), DTYPES[out_dtype],
                         own.data_ptr() if owner else None)
        return (rho, ux, uy, own) if owner else (rho, ux, uy)

    def init_poiseuille(self, case_id: int) -> None:
        lbm_batch_init_poiseuille(self.b, case_id)

    def set_active(self, case_id: int, active: bool) -> None:
        lbm_batch_set_active(self.b, case_id, active)

    def init_fields(self, case_id: int, rho, ux, uy) -> None:
        dt = LBM_F64 if rho.dtype == self.torch.float64 else LBM_F32
        rho, ux, uy = (a.contiguous() for a in (rho, ux, uy))
        lbm_batch_init_fields(self.b, case_id, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(), dt)

    def init_cold(self, case_id: int) -> None:
        """Case case_id back to the cold start it was created with."""
        lbm_batch_init_fields(self.b, case_id, None, None, None, LBM_F32)


class WarmStartNet:
    """The warm-start U-Net on the current device.  Tensors passed in are torch
    CUDA tensors (contiguous, of the dtypes the header names)."""

    def __init__(self, h, w, max_batch, dtype="bf16", ch=(32, 64, 128, 256), rho_scale=1.0, device="cuda",
                 stream=None):
        import torch

        self.torch = torch
        self.h, self.w, self.max_batch = int(h), int(w), int(max_batch)
        self.cfg = lbm_nn_config()
        self.cfg.h, self.cfg.w, self.cfg.max_batch = self.h, self.w, self.max_batch
        self.cfg.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        for k in range(4):
            self.cfg.ch[k] = int(ch[k])
        self.cfg.rho_scale = float(rho_scale)
        nbytes = lbm_nn_workspace_bytes(self.cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._destroy = load_library().lbm_nn_destroy
        self.n = lbm_nn_create(self.cfg, self._ws_ptr, nbytes, self.stream.cuda_stream)
        self.n_params = lbm_nn_param_count(self.n)
        self.ch = tuple(int(c) for c in ch)

    # level of each layer's input (0: h x w, k: h / 2^k x w / 2^k)
    LAYER_LEVELS = (0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0)

    def layer_shapes(self):
        """(c_out, c_in) of the 15 convolutions in parameter order."""
        c0, c1, c2, c3 = self.ch
        cin = (2, c0, c0, c1, c1, c2, c2, c3, 2 * c3 + c2, c2, c2 + c1, c1, c1 + c0, c0, c0)
        cout = (c0, c0, c1, c1, c2, c2, c3, c3, c2, c2, c1, c1, c0, c0, 3)
        return list(zip(cout, cin))

    def __del__(self):
        n = getattr(self, "n", None)
        if n:
            self._destroy(n)
            self.n = None

    def _f32(self, t):
        return t.to(device=self.workspace.device, dtype=self.torch.float32).contiguous()

    def set_params(self, params) -> None:
        p = self._f32(self.torch.as_tensor(params))
        assert p.numel() == self.n_params
        lbm_nn_set_params(self.n, p.data_ptr())
        self.stream.synchronize()

    def params(self):
        out = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.workspace.device)
        lbm_nn_get_params(self.n, out.data_ptr())
        return out

    def grads(self):
        out = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.workspace.device)
        lbm_nn_get_grads(self.n, out.data_ptr())
        return out

    def forward(self, x):
        """x [B][h][w][2] -> y [B][h][w][3] (float32)."""
        x = self._f32(x)
        y = self.torch.empty(x.shape[:3] + (3,), dtype=self.torch.float32, device=x.device)
        lbm_nn_forward(self.n, x.data_ptr(), x.shape[0], y.data_ptr())
        self._keep = x
        return y

    def backward(self, gy) -> None:
        gy = self._f32(gy)
        lbm_nn_backward(self.n, gy.data_ptr())
        self._keep_g = gy

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        lbm_nn_adam(self.n, lr, beta1, beta2, eps)

    def layer_forward(self, layer, x):
        """ReLU(conv(x) + b) of one layer (1..13) on x [B][h_l][w_l][x_cs]
        (device tensor of the compute type) -> [B][h_l][w_l][cout]."""
        cout, cin = self.layer_shapes()[layer]
        x = x.contiguous()
        y = self.torch.zeros(x.shape[:3] + (cout,), dtype=x.dtype, device=x.device)
        lbm_nn_layer_forward(self.n, layer, x.shape[0], x.data_ptr(), x.shape[-1], y.data_ptr(), cout)
        return y

    def layer_wgrad(self, layer, x, g):
        """Weight and bias gradient of one layer from its input x
        [B][h_l][w_l][x_cs] and pre-activation gradient g [B][h_l][w_l][g_cs]
        (device tensors of the compute type) -> float32 [cout * 9 * cin + cout]."""
        cout, cin = self.layer_shapes()[layer]
        out = self.torch.empty(cout * 9 * cin + cout, dtype=self.torch.float32, device=x.device)
        x = x.contiguous()
        g = g.contiguous()
        lbm_nn_layer_wgrad(self.n, layer, x.shape[0], x.data_ptr(), x.shape[-1], g.data_ptr(), g.shape[-1],
                           out.data_ptr())
        return out

    def train_step(self, data, idx, lr, want_loss=False, aug=None):
        """data: dict of device tensors solid, rho, ux, uy, re, gx, tau; idx
        int32 [B]; aug (optional) int32 [B] augmentation codes."""
        d = data
        return lbm_nn_train_step(self.n, d["solid"].data_ptr(), d["rho"].data_ptr(), d["ux"].data_ptr(),
                                 d["uy"].data_ptr(), d["re"].data_ptr(), d["gx"].data_ptr(), d["tau"].data_ptr(),
                                 idx.data_ptr(), aug.data_ptr() if aug is not None else None, idx.numel(), lr,
                                 want_loss)

    def eval(self, data, idx) -> float:
        d = data
        return lbm_nn_eval(self.n, d["solid"].data_ptr(), d["rho"].data_ptr(), d["ux"].data_ptr(),
                           d["uy"].data_ptr(), d["re"].data_ptr(), d["gx"].data_ptr(), d["tau"].data_ptr(),
                           idx.data_ptr(), idx.numel())

    def infer(self, solid, re, gx, tau):
        """solid u8 [B][h][w], re/gx/tau float64 [B] (device) -> rho, ux, uy [B][h][w] float32."""
        B = solid.shape[0]
        dev = self.workspace.device
        outs = [self.torch.empty((B, self.h, self.w), dtype=self.torch.float32, device=dev) for _ in range(3)]
        lbm_nn_infer(self.n, solid.data_ptr(), re.data_ptr(), gx.data_ptr(), tau.data_ptr(), B,
                     *(o.data_ptr() for o in outs))
        return outs


# ---- three dimensions (Sec. IV.D) -------------------------------------------
LBM3D_OPEN, LBM3D_TUBE, LBM3D_PLANES = 0, 1, 2


def _check3(status, ctx=None):
    if status != LBM_OK:
        msg = load_library().lbm3d_last_error(ctx)
        raise LBMError(status, msg.decode() if msg else "")


def make_grid3(case: dict, dtype="f64") -> lbm3d_grid:
    g = lbm3d_grid()
    g.nx, g.ny, g.nz = int(case["nx"]), int(case["ny"]), int(case["nz"])
    g.dtype = {"f64": LBM_F64, "f32": LBM_F32}[dtype]
    g.duct = int(case.get("duct", LBM3D_OPEN))
    g.R = float(case.get("R", 0.0))
    g.refill = int(case.get("refill", 0))
    g.tau = float(case["tau"])
    g.rho0 = float(case.get("rho0", 1.0))
    for d in range(3):
        g.g[d] = float(case.get("g", (0.0, 0.0, 0.0))[d])
        g.u0[d] = float(case.get("u0", (0.0, 0.0, 0.0))[d])
    return g


def _spheres(spheres):
    n = len(spheres)
    arr = (lbm3d_sphere * max(1, n))()
    for k, sp in enumerate(spheres):
        arr[k].X[:] = [float(sp["cx"]), float(sp["cy"]), float(sp["cz"])]
        arr[k].r = float(sp["r"])
        arr[k].V[:] = [float(v) for v in sp.get("v", (0.0, 0.0, 0.0))]
        arr[k].omega[:] = [float(v) for v in sp.get("omega", (0.0, 0.0, 0.0))]
        arr[k].moves = int(bool(sp.get("moves", False)))
    return arr, n


def lbm3d_workspace_bytes(grid, spheres, history_steps: int) -> int:
    arr, n = _spheres(spheres)
    out = ctypes.c_size_t()
    _check3(load_library().lbm3d_workspace_bytes(ctypes.byref(grid), arr, n, int(history_steps),
                                                 ctypes.byref(out)))
    return out.value


def lbm3d_create(grid, spheres, history_steps: int, d_workspace: int, nbytes: int, stream: int):
    arr, n = _spheres(spheres)
    ctx = ctypes.c_void_p()
    _check3(load_library().lbm3d_create(ctypes.byref(grid), arr, n, int(history_steps), d_workspace, nbytes,
                                        stream, ctypes.byref(ctx)))
    return ctx


def lbm3d_step(ctx, n: int) -> None:
    _check3(load_library().lbm3d_step(ctx, int(n)), ctx)


def lbm3d_force(ctx, solid: int, scheme: int, step: int = -1):
    out = (ctypes.c_double * 6)()
    _check3(load_library().lbm3d_force(ctx, int(solid), int(scheme), int(step), out), ctx)
    return list(out)


class Lattice3D:
    """One D3Q19 lattice on the current device (workspace: a torch uint8
    tensor; kernels on torch's current stream).  case keys: nx, ny, nz, tau,
    duct, R, rho0, g, u0, refill, spheres (dicts cx, cy, cz, r, v, omega,
    moves)."""

    def __init__(self, case: dict, dtype="f64", history_steps=1024, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.case = case
        self.nx, self.ny, self.nz = case["nx"], case["ny"], case["nz"]
        self.spheres = list(case.get("spheres", ()))
        self.ns = len(self.spheres)
        self.grid = make_grid3(case, dtype)
        self.history_steps = int(history_steps)
        nbytes = lbm3d_workspace_bytes(self.grid, self.spheres, self.history_steps)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._destroy = load_library().lbm3d_destroy
        self.ctx = lbm3d_create(self.grid, self.spheres, self.history_steps, self._ws_ptr, nbytes,
                                self.stream.cuda_stream)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            self._destroy(ctx)
            self.ctx = None

    @property
    def t(self) -> int:
        return load_library().lbm3d_time(self.ctx)

    def step(self, n: int = 1) -> None:
        lbm3d_step(self.ctx, n)

    def force(self, solid: int, scheme: int, step: int = -1):
        return lbm3d_force(self.ctx, solid, scheme, step)

    def force_history(self):
        """[t][ns + 1][12] (CME F, T, GME F, T) of the steps still in the ring."""
        t = self.t
        first = max(0, t - self.history_steps)
        out = self.torch.empty((t - first, self.ns + 1, 12), dtype=self.torch.float64, device=self.workspace.device)
        if t > first:
            _check3(load_library().lbm3d_force_history(self.ctx, first, t - first, out.data_ptr()), self.ctx)
        self.stream.synchronize()
        return out

    def fields(self):
        """rho [nz, ny, nx], u [3, nz, ny, nx], owner [nz, ny, nx] (device tensors)."""
        T = self.torch
        shp = (self.nz, self.ny, self.nx)
        dev = self.workspace.device
        rho = T.empty(shp, dtype=T.float64, device=dev)
        u = T.empty((3,) + shp, dtype=T.float64, device=dev)
        own = T.empty(shp, dtype=T.int32, device=dev)
        _check3(load_library().lbm3d_fields(self.ctx, rho.data_ptr(), u.data_ptr(), own.data_ptr()), self.ctx)
        self.stream.synchronize()
        return rho, u, own

    def link_count(self) -> int:
        return load_library().lbm3d_link_count(self.ctx)

    def set_free(self, sphere: int, rho_s: float, omega0=(0.0, 0.0, 0.0)) -> None:
        """Sphere `sphere` (created with moves=True) becomes a free particle."""
        om = (ctypes.c_double * 3)(*[float(v) for v in omega0])
        _check3(load_library().lbm3d_set_free(self.ctx, int(sphere), float(rho_s), om), self.ctx)

    def set_gravity(self, G, scheme: int = 1) -> None:
        g = (ctypes.c_double * 3)(*[float(v) for v in G])
        _check3(load_library().lbm3d_set_gravity(self.ctx, g, int(scheme)), self.ctx)

    def set_boundary(self, interpolated: bool = True) -> None:
        """Interpolated (True) or half-way (False) bounce-back on sphere links."""
        _check3(load_library().lbm3d_set_boundary(self.ctx, LBM_INTERPOLATED if interpolated else LBM_HALFWAY),
                self.ctx)

    def set_pressure(self, rho_in: float, rho_out: float) -> None:
        """Pressure inlet (x = 0) and outlet (x = nx - 1) densities."""
        _check3(load_library().lbm3d_set_pressure(self.ctx, float(rho_in), float(rho_out)), self.ctx)

    def set_force_average(self, enable: bool = True) -> None:
        """Free spheres take the mean force of the last two steps."""
        _check3(load_library().lbm3d_set_force_average(self.ctx, int(bool(enable))), self.ctx)

    def body_state(self, sphere: int):
        """[X (3), V (3), Omega (3)] of a sphere at the current step."""
        out = (ctypes.c_double * 9)()
        _check3(load_library().lbm3d_body_state(self.ctx, int(sphere), out), self.ctx)
        return list(out)

    def check(self) -> None:
        _check3(load_library().lbm3d_status_check(self.ctx), self.ctx)

    def profile(self, enable: bool) -> None:
        _check3(load_library().lbm3d_profile(self.ctx, int(bool(enable))), self.ctx)

    def profile_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check3(load_library().lbm3d_profile_read(self.ctx, ctypes.byref(ms), ctypes.byref(n)), self.ctx)
        return ms.value, n.value
