"""FP64 CPU oracle for the D2Q9 momentum-exchange path (test infrastructure).

This package is the independent reference for the GPU library: only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.  The
arithmetic lives in ``lbm_oracle.c`` (plain C, built with ``-O2
-ffp-contract=off``); this module only marshals arrays through ctypes.  It
shares no code with the GPU path.

Method: Wen et al., arXiv:1303.0625 -- LBE collision/advection (Sec. II,
Eqs. 1-3), Eq. 8 equilibrium, half-way bounce-back with the moving-boundary
term (Sec. III.A), CME (Eq. 4) and GME (Eq. 5) link forces, total force and
torque (Eqs. 6-7), newborn refill A1/A2/A3 (Sec. IV.B); the D3Q19 step of
Sec. IV.D (``lbm3d_oracle.c``, fixed geometry: spheres with a rigid surface
motion in a tube or between planes).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRC3 = os.path.join(_HERE, "lbm3d_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
# The same sources built with OpenMP: the per-node collision and advection
# loops split over threads, every result identical (used to time the oracle on
# all of a host's cores; the tests use the single-threaded build).
_LIB_OMP = os.path.join(_HERE, "liblbm_oracle_omp.so")

DISC, BOX = 0, 1
CME, GME = 0, 1
A1, A2, A3 = 0, 1, 2

# D2Q9 set in the order of Sec. III.C (the oracle's own copy; tests use it to
# build inputs and closed forms).
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
OPP = (0, 3, 4, 1, 2, 7, 8, 5, 6)
W = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (and its multi-threaded
    timing build from the same sources); returns the path of the first."""
    newest = max(os.path.getmtime(p) for p in (_SRC, _SRC3))
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < newest:
            cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared", *extra,
                   "-o", lib + ".tmp", _SRC, _SRC3, "-lm"]
            subprocess.check_call(cmd)
            os.replace(lib + ".tmp", lib)
    return _LIB


class _Body(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("moves", ctypes.c_int),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("vx", ctypes.c_double), ("vy", ctypes.c_double)]


_lib = None
_lib_omp = None


def _load(omp: bool = False):
    """The oracle library; omp: its multi-threaded timing build."""
    global _lib, _lib_omp
    if omp:
        if _lib_omp is None:
            build(force=False)
            _lib_omp = _bind(ctypes.CDLL(_LIB_OMP))
        return _lib_omp
    if _lib is not None:
        return _lib
    build(force=False)
    _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(_Body)]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
    lib.orc_time.argtypes = [ctypes.c_void_p]
    lib.orc_time.restype = ctypes.c_long
    lib.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, ip]
    lib.orc_force.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_int, ctypes.c_int, dp]
    lib.orc_force.restype = ctypes.c_int
    lib.orc_links.argtypes = [ctypes.c_void_p, ctypes.c_long, dp]
    lib.orc_links.restype = ctypes.c_long
    lib.orc_get_f.argtypes = [ctypes.c_void_p, dp]
    lib.orc_set_f.argtypes = [ctypes.c_void_p, dp]
    lib.orc_init_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
    lib.orc_feq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    lib.orc_link_force.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
    lib.orc_collide_node.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    lib.orc_refill_node.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ip,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp]
    lib.orc_refill_node.restype = ctypes.c_int
    lib.orc_set_mrt.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.orc_collide_node_mrt.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
    lib.orc_mrt_matrix.argtypes = [dp]
    lib.orc_mrt_inverse.argtypes = [dp]
    lib.orc_set_free.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.orc_set_free.restype = ctypes.c_int
    lib.orc_set_gravity.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.orc_body_state.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    lib.orc_body_state.restype = ctypes.c_int
    lib.orc_set_ibb.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_link_q.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_int]
    lib.orc_link_q.restype = ctypes.c_double
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    """Eq. 8 equilibrium, nine directions."""
    out = np.zeros(9)
    _load().orc_feq(rho, ux, uy, _dp(out))
    return out


def link_force(i: int, a: float, b: float, vx: float, vy: float, scheme: int) -> np.ndarray:
    """Eq. 4 (CME) or Eq. 5 (GME) for one link in direction i."""
    out = np.zeros(2)
    _load().orc_link_force(i, a, b, vx, vy, scheme, _dp(out))
    return out


def collide_node(f, tau: float, gx: float = 0.0, gy: float = 0.0) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    _load().orc_collide_node(_dp(f), tau, gx, gy, _dp(out))
    return out


def collide_node_mrt(f, s, gx: float = 0.0, gy: float = 0.0) -> np.ndarray:
    """MRT collision of one node with the nine moment rates s (moments rho,
    e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros(9)
    _load().orc_collide_node_mrt(_dp(f), _dp(s), gx, gy, _dp(out))
    return out


def mrt_matrix() -> np.ndarray:
    out = np.zeros(81)
    _load().orc_mrt_matrix(_dp(out))
    return out.reshape(9, 9)


def mrt_inverse() -> np.ndarray:
    out = np.zeros(81)
    _load().orc_mrt_inverse(_dp(out))
    return out.reshape(9, 9)


def refill_node(fpost: np.ndarray, oldfluid: np.ndarray, x: int, y: int, scheme: int,
                walls_y: bool = False, rho0: float = 1.0, v=(0.0, 0.0)):
    """Refill of one newborn node; returns (f[9], number of participating links)."""
    fpost = np.ascontiguousarray(fpost, dtype=np.float64)
    oldfluid = np.ascontiguousarray(oldfluid, dtype=np.int32)
    _, ny, nx = fpost.shape
    out = np.zeros(9)
    n = _load().orc_refill_node(nx, ny, int(walls_y), _dp(fpost), _ip(oldfluid), x, y, scheme,
                                rho0, v[0], v[1], _dp(out))
    return out, n


class OracleSim:
    """One D2Q9 simulation held by the C oracle.

    ``bodies`` is a sequence of dicts with keys kind ('disc'|'box' or 0|1),
    cx, cy, r (or hx), hy, vx, vy, moves.  ``omp``: run on the multi-threaded
    build (OMP_NUM_THREADS threads; the same results).
    """

    def __init__(self, nx, ny, tau, *, walls_y=False, rho0=1.0, gx=0.0, gy=0.0, u0=(0.0, 0.0),
                 wall_v=(0.0, 0.0), refill=A1, rho_w_local=False, bodies=(), mrt=None, omp=False):
        lib = _load(omp)
        self.nx, self.ny = int(nx), int(ny)
        self.nb = len(bodies)
        arr = (_Body * max(1, self.nb))()
        for k, b in enumerate(bodies):
            kind = b.get("kind", DISC)
            if isinstance(kind, str):
                kind = DISC if kind == "disc" else BOX
            arr[k].kind = kind
            arr[k].moves = int(b.get("moves", 0))
            arr[k].cx = float(b["cx"])
            arr[k].cy = float(b["cy"])
            arr[k].a = float(b.get("r", b.get("hx", 0.0)))
            arr[k].b = float(b.get("hy", 0.0))
            arr[k].vx = float(b.get("vx", 0.0))
            arr[k].vy = float(b.get("vy", 0.0))
        self._lib = lib
        self._h = lib.orc_create(self.nx, self.ny, int(walls_y), tau, rho0, gx, gy, u0[0], u0[1],
                                 wall_v[0], wall_v[1], int(refill), int(rho_w_local), self.nb, arr)
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        if mrt is not None:
            # (s_e, s_eps, s_q); the shear rates are 1/tau
            lib.orc_set_mrt(self._h, float(mrt[0]), float(mrt[1]), float(mrt[2]))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def set_free(self, body: int, rho_s: float, omega0: float = 0.0) -> None:
        """Body `body` (1-based disc) becomes a free particle of density rho_s."""
        if self._lib.orc_set_free(self._h, int(body), float(rho_s), float(omega0)) != 0:
            raise ValueError("oracle rejected the free body")

    def set_ibb(self, on: bool = True) -> None:
        """Interpolated bounce-back on body links."""
        self._lib.orc_set_ibb(self._h, int(bool(on)))

    def link_q(self, body: int, x: int, y: int, i: int) -> float:
        return self._lib.orc_link_q(self._h, int(body), int(x), int(y), int(i))

    def set_gravity(self, G, scheme: int) -> None:
        self._lib.orc_set_gravity(self._h, float(G[0]), float(G[1]), int(scheme))

    def body_state(self, body: int) -> np.ndarray:
        """{X, Y, V_x, V_y, Omega} of body `body` now."""
        out = np.zeros(5)
        if self._lib.orc_body_state(self._h, int(body), _dp(out)) != 0:
            raise IndexError(body)
        return out

    @property
    def t(self) -> int:
        return self._lib.orc_time(self._h)

    def step(self, n: int = 1) -> None:
        self._lib.orc_step(self._h, int(n))

    def fields(self):
        shp = (self.ny, self.nx)
        rho, ux, uy = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        own = np.zeros(shp, dtype=np.int32)
        self._lib.orc_fields(self._h, _dp(rho), _dp(ux), _dp(uy), _ip(own))
        return rho, ux, uy, own

    def force(self, solid: int, scheme: int, step: int | None = None) -> np.ndarray:
        out = np.zeros(3)
        if step is None:
            step = self.t - 1
        if self._lib.orc_force(self._h, int(step), int(solid), int(scheme), _dp(out)) != 0:
            raise IndexError("no force record for that step/solid")
        return out

    def force_history(self, scheme: int) -> np.ndarray:
        """[steps][n_bodies+1][3] array of {Fx, Fy, Tz}."""
        T = self.t
        h = np.zeros((T, self.nb + 1, 3))
        for st in range(T):
            for s in range(self.nb + 1):
                h[st, s] = self.force(s, scheme, st)
        return h

    def links(self) -> np.ndarray:
        n = self._lib.orc_links(self._h, 0, None)
        rec = np.zeros((max(n, 1), 8))
        self._lib.orc_links(self._h, n, _dp(rec))
        return rec[:n]

    def get_f(self) -> np.ndarray:
        f = np.zeros((9, self.ny, self.nx))
        self._lib.orc_get_f(self._h, _dp(f))
        return f

    def set_f(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self._lib.orc_set_f(self._h, _dp(f))

    def init_fields(self, rho, ux, uy) -> None:
        rho, ux, uy = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy))
        self._lib.orc_init_fields(self._h, _dp(rho), _dp(ux), _dp(uy))


# ------------------------------------------------------------------ D3Q19 (Sec. IV.D)
OPEN3, TUBE3, PLANES3 = 0, 1, 2
# the oracle's velocity set: rest, six axis directions, twelve edge diagonals
E3 = ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
      (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
      (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1))


def _load3():
    lib = _load()
    if getattr(lib, "_orc3_bound", False):
        return lib
    dp = ctypes.POINTER(ctypes.c_double)
    lib.orc3_create.restype = ctypes.c_void_p
    lib.orc3_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp]
    lib.orc3_destroy.argtypes = [ctypes.c_void_p]
    lib.orc3_time.argtypes = [ctypes.c_void_p]
    lib.orc3_time.restype = ctypes.c_long
    lib.orc3_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
    lib.orc3_fields.argtypes = [ctypes.c_void_p, dp, dp, ctypes.POINTER(ctypes.c_int)]
    lib.orc3_force.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_int, ctypes.c_int, dp]
    lib.orc3_force.restype = ctypes.c_int
    lib.orc3_feq.argtypes = [ctypes.c_double, dp, dp]
    lib.orc3_collide_node.argtypes = [dp, ctypes.c_double, dp, dp]
    lib.orc3_link_force.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int, dp]
    lib.orc3_get_f.argtypes = [ctypes.c_void_p, dp]
    lib.orc3_set_f.argtypes = [ctypes.c_void_p, dp]
    lib.orc3_get_ft.argtypes = [ctypes.c_void_p, dp]
    lib.orc3_set_moving.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc3_set_moving.restype = ctypes.c_int
    lib.orc3_error.argtypes = [ctypes.c_void_p]
    lib.orc3_error.restype = ctypes.c_int
    lib.orc3_set_free.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, dp]
    lib.orc3_set_free.restype = ctypes.c_int
    lib.orc3_set_gravity.argtypes = [ctypes.c_void_p, dp, ctypes.c_int]
    lib.orc3_set_force_average.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc3_set_pressure.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    lib.orc3_set_ibb.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc3_link_q.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc3_link_q.restype = ctypes.c_double
    lib.orc3_tube_q.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc3_tube_q.restype = ctypes.c_double
    lib.orc3_set_pressure.restype = ctypes.c_int
    lib.orc3_body_state.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    lib.orc3_body_state.restype = ctypes.c_int
    lib.orc3_record_links.argtypes = [ctypes.c_void_p, ctypes.c_long]
    lib.orc3_links.argtypes = [ctypes.c_void_p, dp, ctypes.c_long]
    lib.orc3_links.restype = ctypes.c_long
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.orc3_refill_node.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, u8p, u8p, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
    lib._orc3_bound = True
    return lib


def _vec(v, n=3):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))


def feq3(rho: float, u) -> np.ndarray:
    out = np.zeros(19)
    _load3().orc3_feq(float(rho), _dp(_vec(u)), _dp(out))
    return out


def collide_node3(f, tau: float, g=(0.0, 0.0, 0.0)) -> np.ndarray:
    f = _vec(f, 19)
    out = np.zeros(19)
    _load3().orc3_collide_node(_dp(f), float(tau), _dp(_vec(g)), _dp(out))
    return out


def link_force3(i: int, a: float, b: float, v, scheme: int) -> np.ndarray:
    out = np.zeros(3)
    _load3().orc3_link_force(int(i), float(a), float(b), _dp(_vec(v)), int(scheme), _dp(out))
    return out


def refill_node3(fn, own_t, own_n, x, y, z, scheme):
    """Refill of a newborn node from post-advection values fn [19, nz, ny, nx]
    and the owner maps of steps t and t + 1; (values, participant count)."""
    fn = np.ascontiguousarray(fn, dtype=np.float64)
    ot = np.ascontiguousarray(own_t, dtype=np.uint8)
    on = np.ascontiguousarray(own_n, dtype=np.uint8)
    _, nz, ny, nx = fn.shape
    out = np.zeros(19)
    npart = ctypes.c_int()
    u8p = ctypes.POINTER(ctypes.c_uint8)
    _load3().orc3_refill_node(nx, ny, nz, _dp(fn), ot.ctypes.data_as(u8p), on.ctypes.data_as(u8p), int(x), int(y),
                              int(z), int(scheme), ctypes.byref(npart), _dp(out))
    return out, npart.value


class OracleSim3D:
    """One D3Q19 simulation held by the C oracle.  spheres: dicts with keys
    cx, cy, cz, r and optional v (3), omega (3)."""

    def __init__(self, nx, ny, nz, tau, *, rho0=1.0, g=(0.0, 0.0, 0.0), u0=(0.0, 0.0, 0.0),
                 duct=OPEN3, R=0.0, spheres=()):
        lib = _load3()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.ns = len(spheres)
        rec = np.zeros((max(1, self.ns), 10))
        for k, sp in enumerate(spheres):
            rec[k, :4] = (sp["cx"], sp["cy"], sp["cz"], sp["r"])
            rec[k, 4:7] = sp.get("v", (0.0, 0.0, 0.0))
            rec[k, 7:10] = sp.get("omega", (0.0, 0.0, 0.0))
        rec = np.ascontiguousarray(rec)
        self._lib = lib
        self._h = lib.orc3_create(self.nx, self.ny, self.nz, float(tau), float(rho0), _dp(_vec(g)),
                                  _dp(_vec(u0)), int(duct), float(R), self.ns, _dp(rec))
        if not self._h:
            raise ValueError("oracle rejected the 3D configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc3_destroy(h)
            self._h = None

    def set_moving(self, sphere: int, moving: bool = True, refill: int = 0) -> None:
        """Sphere `sphere` (1-based) translates at its v; refill A1/A2/A3 (0/1/2)."""
        if self._lib.orc3_set_moving(self._h, int(sphere), int(bool(moving)), int(refill)) != 0:
            raise ValueError("oracle rejected the moving sphere")

    def set_free(self, sphere: int, rho_s: float, omega0=(0.0, 0.0, 0.0)) -> None:
        """Sphere `sphere` (set moving first) becomes free with density rho_s."""
        if self._lib.orc3_set_free(self._h, int(sphere), float(rho_s), _dp(_vec(omega0))) != 0:
            raise ValueError("oracle rejected the free sphere")

    def set_gravity(self, G, scheme: int) -> None:
        self._lib.orc3_set_gravity(self._h, _dp(_vec(G)), int(scheme))

    def set_ibb(self, on: bool = True) -> None:
        """Interpolated bounce-back on sphere links."""
        self._lib.orc3_set_ibb(self._h, int(bool(on)))

    def link_q(self, sphere: int, x: int, y: int, z: int, i: int) -> float:
        return self._lib.orc3_link_q(self._h, int(sphere), int(x), int(y), int(z), int(i))

    def tube_q(self, y: int, z: int, i: int) -> float:
        return self._lib.orc3_tube_q(self._h, int(y), int(z), int(i))

    def record_links(self, cap: int) -> None:
        """Keep per-link records (at most cap links per step) from now on."""
        self._lib.orc3_record_links(self._h, int(cap))
        self._rec_cap = int(cap)

    def links(self) -> np.ndarray:
        """Link records of the last step: [n][11] = x, y, z, i, solid (0 the
        duct), CME force (3), GME force (3)."""
        cap = getattr(self, "_rec_cap", 0)
        out = np.zeros((max(cap, 1), 11))
        n = self._lib.orc3_links(self._h, _dp(out), cap)
        return out[:n]

    def set_pressure(self, rho_in: float, rho_out: float) -> None:
        """Pressure inlet (x = 0) and outlet (x = nx - 1) densities."""
        if self._lib.orc3_set_pressure(self._h, float(rho_in), float(rho_out)) != 0:
            raise ValueError("oracle rejected the pressure boundary")

    def set_force_average(self, on: bool = True) -> None:
        """Free spheres take the mean force of the last two steps."""
        self._lib.orc3_set_force_average(self._h, int(bool(on)))

    def body_state(self, sphere: int) -> np.ndarray:
        """{X (3), V (3), Omega (3)} of sphere `sphere` now."""
        out = np.zeros(9)
        if self._lib.orc3_body_state(self._h, int(sphere), _dp(out)) != 0:
            raise IndexError(sphere)
        return out

    @property
    def error(self) -> int:
        return self._lib.orc3_error(self._h)

    @property
    def t(self) -> int:
        return self._lib.orc3_time(self._h)

    def step(self, n: int = 1) -> None:
        self._lib.orc3_step(self._h, int(n))

    def fields(self):
        """rho [nz, ny, nx], u [3, nz, ny, nx] (Guo velocity), owner [nz, ny, nx]."""
        shp = (self.nz, self.ny, self.nx)
        rho = np.zeros(shp)
        u = np.zeros((3,) + shp)
        own = np.zeros(shp, dtype=np.int32)
        self._lib.orc3_fields(self._h, _dp(rho), _dp(u), _ip(own))
        return rho, u, own

    def force(self, solid: int, scheme: int, step: int | None = None) -> np.ndarray:
        """{F_x, F_y, F_z, T_x, T_y, T_z} of solid (0 duct, k sphere k)."""
        out = np.zeros(6)
        if step is None:
            step = self.t - 1
        if self._lib.orc3_force(self._h, int(step), int(solid), int(scheme), _dp(out)) != 0:
            raise IndexError("no force record for that step/solid")
        return out

    def force_history(self, scheme: int) -> np.ndarray:
        h = np.zeros((self.t, self.ns + 1, 6))
        for st in range(self.t):
            for s in range(self.ns + 1):
                h[st, s] = self.force(s, scheme, st)
        return h

    def get_f(self) -> np.ndarray:
        f = np.zeros((19, self.nz, self.ny, self.nx))
        self._lib.orc3_get_f(self._h, _dp(f))
        return f

    def get_ft(self) -> np.ndarray:
        """Post-collision populations of the last step [19][nz][ny][nx]
        (the pressure planes' extrapolated state included)."""
        f = np.zeros((19, self.nz, self.ny, self.nx))
        self._lib.orc3_get_ft(self._h, _dp(f))
        return f
