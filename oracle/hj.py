"""One explicit step of the Hamilton-Jacobi equation of Sec. 2.1.

TEST INFRASTRUCTURE: part of the oracle the GPU path is checked against; used only by the tests, the
smoke check and the benchmark's CPU baseline.

phi_t + v |grad phi| = 0 on the periodic node grid, first-order Godunov
upwinding (Osher-Sethian).  The paper leaves the discretisation to its
library; the reading here: nodal velocity v = mean of dJ/drho over the eight
elements around a node, normalised to max |v| = 1, time step dt = cfl * h.
v > 0 lowers phi, i.e. grows solid (phi < 0) where J increases.
"""
from __future__ import annotations

import numpy as np

from .cell import element_nodes


def nodal_velocity(n, g_rho):
    en = element_nodes(n)
    v = np.zeros(n ** 3)
    for l in range(8):
        np.add.at(v, en[:, l], g_rho)
    v /= 8.0
    vmax = np.max(np.abs(v))
    return v / vmax if vmax > 0 else v


def hj_step(n, phi, v, cfl=0.5):
    h = 1.0 / n
    dt = cfl * h
    f = np.asarray(phi, dtype=np.float64).reshape(n, n, n)   # [k][j][i]
    vv = np.asarray(v, dtype=np.float64).reshape(n, n, n)
    gp2 = np.zeros_like(f)   # |grad|^2 for v > 0
    gm2 = np.zeros_like(f)   # |grad|^2 for v < 0
    for ax in (2, 1, 0):     # x, y, z
        dm = (f - np.roll(f, 1, axis=ax)) / h      # backward difference
        dp = (np.roll(f, -1, axis=ax) - f) / h     # forward difference
        gp2 += np.maximum(dm, 0.0) ** 2 + np.minimum(dp, 0.0) ** 2
        gm2 += np.minimum(dm, 0.0) ** 2 + np.maximum(dp, 0.0) ** 2
    upd = np.maximum(vv, 0.0) * np.sqrt(gp2) + np.minimum(vv, 0.0) * np.sqrt(gm2)
    return (f - dt * upd).ravel()
