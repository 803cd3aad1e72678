"""Shared test helpers: build oracle and GPU runs from one seeded case and
compare them.

Comparison rules.  Density: max |gpu - oracle| over fluid nodes relative to
max |rho|.  Velocity: max over both components of |gpu - oracle| relative to
the largest velocity magnitude (a component that is roundoff in a symmetric
flow is not compared with itself).  Force of a solid: relative to
max(largest force magnitude of that solid over the history, 1e-3 x the
largest body force in the case), torque additionally times the body's
half-size."""
from __future__ import annotations

import numpy as np


def oracle_sim(oracle, c, mrt=None, omp=False):
    """The oracle for case c; omp: its multi-threaded build (same results)."""
    return oracle.OracleSim(c["nx"], c["ny"], c["tau"], walls_y=c["walls_y"], rho0=c["rho0"],
                            gx=c["gx"], gy=c["gy"], u0=c["u0"], wall_v=c["wall_v"],
                            refill=c["refill"], bodies=c["bodies"], mrt=mrt, omp=omp)


def rel_field_err(gpu, ref, mask):
    g = np.asarray(gpu)[mask]
    r = np.asarray(ref)[mask]
    scale = np.abs(r).max()
    if scale == 0:
        return float(np.abs(g).max())
    return float(np.abs(g - r).max() / scale)


def rel_l2(f, F):
    """Relative L2-norm error of a history (Eq. 11), with sums for integrals."""
    f = np.asarray(f, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    return float(np.sqrt(((f - F) ** 2).sum()) / np.sqrt((F ** 2).sum()))


def oracle_history(osim, nb):
    """[steps][nb+1][6] from the oracle (CME Fx Fy Tz, GME Fx Fy Tz)."""
    T = osim.t
    h = np.zeros((T, nb + 1, 6))
    for st in range(T):
        for s in range(nb + 1):
            h[st, s, :3] = osim.force(s, 0, st)
            h[st, s, 3:] = osim.force(s, 1, st)
    return h


def field_errors(gpu_fields, oracle_fields):
    rho, ux, uy, own = gpu_fields
    orho, oux, ouy, oown = oracle_fields
    assert (np.asarray(own).astype(np.int32) == oown).all(), "owner maps differ"
    m = oown == 0
    e_rho = float(np.abs(rho - orho)[m].max() / np.abs(orho[m]).max())
    umag = np.sqrt(oux ** 2 + ouy ** 2)[m].max()
    du = max(np.abs(ux - oux)[m].max(), np.abs(uy - ouy)[m].max())
    e_u = float(du / umag) if umag > 0 else float(du)
    return e_rho, e_u


def link_load(osim, nb):
    """Per solid, the sum of |link force components| of the oracle's last step:
    the magnitude of the terms the total is summed from."""
    rec = osim.links()
    load = np.zeros(nb + 1)
    for s in range(nb + 1):
        r = rec[rec[:, 3] == s]
        load[s] = np.abs(r[:, 4:8]).sum() / 2.0
    return load


def force_errors(h, oh, case, tol=1e-10, load=None):
    """Worst force/torque error of every solid and component, normalised so
    that <= 1 passes: |gpu - oracle| <= tol * scale + 16 eps * load, where
    scale is max(largest force magnitude of the solid over the history,
    1e-3 x the largest body force) (times the half-size for torque) and the
    second term bounds the roundoff of summing the solid's link terms in a
    different order (load = sum of |link terms|).  Returns (worst normalised,
    worst relative-to-scale, where)."""
    nb = h.shape[1] - 1
    eps = np.finfo(np.float64).eps
    body_scale = [np.abs(oh[:, s, [0, 1, 3, 4]]).max() for s in range(nb + 1)]
    floor = 1e-3 * max(body_scale[1:]) if nb > 0 else 0.0
    if load is None:
        load = np.zeros(nb + 1)
    worst, worst_rel, where = 0.0, 0.0, None
    for s in range(nb + 1):
        fscale = max(body_scale[s], floor)
        size = 1.0
        if s > 0:
            b = case["bodies"][s - 1]
            size = b.get("r", max(b.get("hx", 0.0), b.get("hy", 0.0), 1.0))
        for c in range(6):
            if s == 0 and c in (2, 5):
                continue
            scale = fscale * (size if c in (2, 5) else 1.0)
            diff = float(np.abs(h[:, s, c] - oh[:, s, c]).max())
            allow = tol * scale + 16 * eps * load[s] * (size if c in (2, 5) else 1.0)
            norm = diff / allow if allow > 0 else (0.0 if diff == 0 else np.inf)
            rel = diff / scale if scale > 0 else diff
            if norm > worst:
                worst, where = norm, (s, c)
            worst_rel = max(worst_rel, rel)
    return worst, worst_rel, where


def plane_state(oracle_mod, osim, own):
    """The oracle's pressure-plane state: on x = 0 and x = nx - 1, where the
    inner neighbour is fluid, the extrapolated post-collision populations
    (what the GPU stores there in place of the streamed state, and what the
    next step streams from).  The GPU holds the post-collision state of the
    step it has reached, the oracle the streamed state before that step's
    collision, so the oracle is advanced by one step here and its
    post-collision state read (call this after every other comparison).
    Returns (rho, u, mask); g = 0."""
    osim.step(1)
    ft = osim.get_ft()
    e = np.array(oracle_mod.E3, dtype=float)
    rho = ft.sum(0)
    with np.errstate(invalid="ignore", divide="ignore"):  # solid nodes hold no populations
        u = np.einsum("id,izyx->dzyx", e, ft) / rho
    mask = np.zeros(own.shape, dtype=bool)
    mask[:, :, 0] = (own[:, :, 0] == 0) & (own[:, :, 1] == 0)
    mask[:, :, -1] = (own[:, :, -1] == 0) & (own[:, :, -2] == 0)
    return rho, u, mask
