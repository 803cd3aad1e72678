"""Seeded synthetic workloads shared by the oracle tests and the GPU path.

This module only draws and places inputs (grid sizes, relaxation times, body
forces, cylinder radii, centres and velocities).  It holds none of the lattice
Boltzmann arithmetic: rasterisation, collision, streaming, bounce-back, refill
and force evaluation are implemented separately by the oracle and by the GPU
library.

A case is a plain dict:
    nx, ny          lattice size
    walls_y         half-way walls at y = -1/2 and ny - 1/2 (else periodic in y)
    tau, rho0       BGK relaxation time, reference density
    gx, gy          body-force acceleration (force density rho*g)
    u0              initial uniform velocity (populations start at f_eq(rho0, u0))
    wall_v          velocity of the walls (solid id 0)
    refill          0 = A1, 1 = A2, 2 = A3 (Sec. IV.B)
    bodies          list of {kind: 'disc'|'box', cx, cy, r | (hx, hy), vx, vy, moves}
    steps           number of time steps of the workload
"""
from __future__ import annotations

import math

import numpy as np

A1, A2, A3 = 0, 1, 2


def make_case(nx, ny, tau, *, walls_y=False, rho0=1.0, gx=0.0, gy=0.0, u0=(0.0, 0.0),
              wall_v=(0.0, 0.0), refill=A1, bodies=(), steps=0, name=""):
    return {
        "name": name, "nx": int(nx), "ny": int(ny), "walls_y": bool(walls_y), "tau": float(tau),
        "rho0": float(rho0), "gx": float(gx), "gy": float(gy),
        "u0": (float(u0[0]), float(u0[1])), "wall_v": (float(wall_v[0]), float(wall_v[1])),
        "refill": int(refill), "bodies": [dict(b) for b in bodies], "steps": int(steps),
    }


def disc(cx, cy, r, vx=0.0, vy=0.0, moves=False):
    return {"kind": "disc", "cx": float(cx), "cy": float(cy), "r": float(r),
            "vx": float(vx), "vy": float(vy), "moves": bool(moves)}


def box(cx, cy, hx, hy, vx=0.0, vy=0.0, moves=False):
    return {"kind": "box", "cx": float(cx), "cy": float(cy), "hx": float(hx), "hy": float(hy),
            "vx": float(vx), "vy": float(vy), "moves": bool(moves)}


# --------------------------------------------------------------------------
# Driven channel with one centred cylinder (FP64 parity workload).
# 128 x 64, walls at y, tau = 0.8, gx = 1e-6, D = 10 at (63.5, 31.5), 5000 steps.
# frame = 'rest'        everything at rest
#         'moving'      fluid starts at f_eq(1, (-U, 0)); walls and cylinder
#                       carry v = (-U, 0) with the cylinder geometry fixed
#         'translating' as 'moving' but the cylinder geometry translates at -U
# --------------------------------------------------------------------------
def channel_cylinder(frame="rest", U=0.05, nx=128, ny=64, steps=5000, r=5.0, tau=0.8, gx=1e-6):
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    if frame == "rest":
        return make_case(nx, ny, tau, walls_y=True, gx=gx, bodies=[disc(cx, cy, r)], steps=steps,
                         name=f"channel_cylinder_{nx}x{ny}_rest")
    v = -U
    moves = frame == "translating"
    if frame not in ("moving", "translating"):
        raise ValueError(frame)
    return make_case(nx, ny, tau, walls_y=True, gx=gx, u0=(v, 0.0), wall_v=(v, 0.0),
                     bodies=[disc(cx, cy, r, vx=v, moves=moves)], steps=steps,
                     name=f"channel_cylinder_{nx}x{ny}_{frame}")


def channel_empty(frame="rest", U=0.05, nx=16, ny=64, tau=0.8, gx=1e-6, steps=2000):
    """Obstacle-free driven channel, at rest or seen from a frame moving at -U."""
    v = 0.0 if frame == "rest" else -U
    return make_case(nx, ny, tau, walls_y=True, gx=gx, u0=(v, 0.0), wall_v=(v, 0.0), steps=steps,
                     name=f"channel_empty_{frame}")


# --------------------------------------------------------------------------
# Placement helpers (pure geometry of the workload, no lattice arithmetic).
# --------------------------------------------------------------------------
def _periodic_dist(a, b, n):
    d = abs(a - b) % n
    return min(d, n - d)


def _centre_gap(b1, b2, nx, ny, periodic_y):
    dx = _periodic_dist(b1["cx"], b2["cx"], nx)
    dy = _periodic_dist(b1["cy"], b2["cy"], ny) if periodic_y else abs(b1["cy"] - b2["cy"])
    return math.hypot(dx, dy) - b1["r"] - b2["r"]


def moving_cylinders(seed=2002, nx=2048, ny=1024, n_discs=32, r_range=(6.0, 12.0),
                     v_range=(0.01, 0.05), tau=0.6, steps=10_000, lane_margin=4.0, gap=4.0):
    """Channel with half fixed and half translating cylinders.

    Each mover owns an exclusive horizontal lane [cy - r - m, cy + r + m] and
    translates along x at |v| in v_range with a random sign; fixed cylinders
    stay outside every lane, with surface gaps >= `gap` to each other and to
    the walls.  Drawn with numpy.random.default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    n_move = n_discs // 2
    radii = rng.uniform(r_range[0], r_range[1], n_discs)
    movers, lanes = [], []
    tries = 0
    for k in range(n_move):
        r = float(radii[k])
        while True:
            tries += 1
            if tries > 100000:
                raise RuntimeError("could not place movers")
            cy = float(rng.uniform(r + lane_margin + 1.0, ny - 2.0 - r - lane_margin))
            lo, hi = cy - r - lane_margin, cy + r + lane_margin
            if all(hi < l0 or lo > l1 for (l0, l1) in lanes):
                break
        cx = float(rng.uniform(0.0, nx))
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        v = sign * float(rng.uniform(v_range[0], v_range[1]))
        lanes.append((lo, hi))
        movers.append(disc(cx, cy, r, vx=v, moves=True))
    fixed = []
    for k in range(n_move, n_discs):
        r = float(radii[k])
        while True:
            tries += 1
            if tries > 1000000:
                raise RuntimeError("could not place fixed cylinders")
            cx = float(rng.uniform(0.0, nx))
            cy = float(rng.uniform(r + gap + 1.0, ny - 2.0 - r - gap))
            lo, hi = cy - r - gap, cy + r + gap
            if not all(hi < l0 or lo > l1 for (l0, l1) in lanes):
                continue
            cand = disc(cx, cy, r)
            if all(_centre_gap(cand, o, nx, ny, False) >= gap for o in fixed):
                break
        fixed.append(cand)
    return make_case(nx, ny, tau, walls_y=True, bodies=movers + fixed, refill=A1, steps=steps,
                     name=f"moving_cylinders_{nx}x{ny}_seed{seed}")


def periodic_cylinders(seed=3003, n=4096, n_discs=64, r_range=(8.0, 16.0), gap=4.0, tau=0.6,
                       gx=1e-5, steps=5000):
    """Fully periodic n x n box with fixed cylinders (surface gaps >= gap,
    minimum image), driven by gx."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(r_range[0], r_range[1], n_discs)
    bodies = []
    for k in range(n_discs):
        r = float(radii[k])
        for _ in range(1000000):
            cand = disc(float(rng.uniform(0, n)), float(rng.uniform(0, n)), r)
            if all(_centre_gap(cand, o, n, n, True) >= gap for o in bodies):
                break
        else:
            raise RuntimeError("could not place cylinders")
        bodies.append(cand)
    return make_case(n, n, tau, gx=gx, bodies=bodies, steps=steps,
                     name=f"periodic_cylinders_{n}x{n}_seed{seed}")


def periodic_crop(seed=3003, n=4096, crop=256, **kw):
    """crop x crop periodic window holding only the first cylinder of
    periodic_cylinders(seed), centred in the window."""
    big = periodic_cylinders(seed=seed, n=n, **kw)
    b = dict(big["bodies"][0])
    b["cx"] = crop / 2.0 + (b["cx"] - math.floor(b["cx"]))
    b["cy"] = crop / 2.0 + (b["cy"] - math.floor(b["cy"]))
    return make_case(crop, crop, big["tau"], gx=big["gx"], bodies=[b], steps=big["steps"],
                     name=f"periodic_crop_{crop}_seed{seed}")


# --------------------------------------------------------------------------
# Reynolds-number parametrisation of the channel/cylinder cases.
# Re = U_mean * D / nu with U_mean = 0.02 nominal; tau = 3 nu + 1/2 clamped to
# [0.51, 2.0] (U_mean then follows from Re); gx = 12 nu U_mean / H^2, the
# plane-Poiseuille driving for mean velocity U_mean in a channel of height H.
# --------------------------------------------------------------------------
def re_to_tau_g(Re, D, H, u_mean=0.02, tau_lo=0.51, tau_hi=2.0):
    nu = u_mean * D / Re
    tau = 3.0 * nu + 0.5
    if tau < tau_lo or tau > tau_hi:
        tau = min(max(tau, tau_lo), tau_hi)
        nu = (tau - 0.5) / 3.0
        u_mean = Re * nu / D
    g = 12.0 * nu * u_mean / (H * H)
    return tau, g, u_mean


def uneven_channels(seed=4004, n_cases=256, nx_range=(64, 512), re_range=(1.0, 100.0)):
    """Independent channel/cylinder cases of uneven sizes: nx = 2*round(U(64, 512)),
    ny = nx/2, walls at y, one cylinder of radius U(0.05, 0.10)*ny at
    x = U(0.25, 0.5)*nx, y = y_c + U(-0.1, 0.1)*ny, Re ~ U(1, 100)."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(n_cases):
        nx = 2 * int(round(rng.uniform(nx_range[0], nx_range[1])))
        ny = nx // 2
        r = float(rng.uniform(0.05, 0.10) * ny)
        cx = float(rng.uniform(0.25, 0.5) * nx)
        cy = (ny - 1) / 2.0 + float(rng.uniform(-0.1, 0.1) * ny)
        Re = float(rng.uniform(*re_range))
        tau, g, _ = re_to_tau_g(Re, 2 * r, ny)
        c = make_case(nx, ny, tau, walls_y=True, gx=g, bodies=[disc(cx, cy, r)],
                      name=f"uneven_{k}")
        c["Re"] = Re
        cases.append(c)
    return cases


def warmstart_channels(seed=5005, n_cases=2000, nx=256, ny=128, n_range=(1, 3),
                       r_range=(6.0, 16.0), gap=4.0, re_range=(1.0, 100.0)):
    """256 x 128 channels with 1-3 fixed cylinders (gaps >= 4), Re ~ U(1, 100)
    based on the largest diameter."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(n_cases):
        nb = int(rng.integers(n_range[0], n_range[1] + 1))
        bodies = []
        for _ in range(nb):
            r = float(rng.uniform(*r_range))
            for _ in range(100000):
                cand = disc(float(rng.uniform(r + gap, nx - r - gap)),
                            float(rng.uniform(r + gap + 1.0, ny - 2.0 - r - gap)), r)
                if all(_centre_gap(cand, o, nx, ny, False) >= gap for o in bodies):
                    break
            else:
                raise RuntimeError("could not place cylinders")
            bodies.append(cand)
        Re = float(rng.uniform(*re_range))
        D = 2.0 * max(b["r"] for b in bodies)
        tau, g, _ = re_to_tau_g(Re, D, ny)
        c = make_case(nx, ny, tau, walls_y=True, gx=g, bodies=bodies, name=f"warm_{seed}_{k}")
        c["Re"] = Re
        cases.append(c)
    return cases


def random_populations(shape, seed, amp=1e-3, w=None):
    """Seeded random populations around the rest weights: w_i * (1 + amp*U(-1,1))."""
    rng = np.random.default_rng(seed)
    if w is None:
        raise ValueError("weights must be supplied by the caller")
    w = np.asarray(w, dtype=np.float64).reshape((9,) + (1,) * (len(shape) - 1))
    return w * (1.0 + amp * rng.uniform(-1.0, 1.0, size=shape))
