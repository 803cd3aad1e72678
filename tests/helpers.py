"""Shared test helpers: build oracle and GPU runs from one seeded case and
compare them.  Comparisons follow one rule: per field, max |gpu - oracle| over
fluid nodes divided by max |oracle| over fluid nodes (density is compared
relative to its own size, ~rho0)."""
from __future__ import annotations

import numpy as np


def oracle_sim(oracle, c):
    return oracle.OracleSim(c["nx"], c["ny"], c["tau"], walls_y=c["walls_y"], rho0=c["rho0"],
                            gx=c["gx"], gy=c["gy"], u0=c["u0"], wall_v=c["wall_v"],
                            refill=c["refill"], bodies=c["bodies"])


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
