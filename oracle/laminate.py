"""Closed-form effective matrix of a layered cell (a pin for the whole solve).

TEST INFRASTRUCTURE: part of the oracle the GPU path is checked against; used only by the tests, the
smoke check and the benchmark's CPU baseline.

For a cell whose ersatz scale s depends only on the coordinate along one
axis, the exact solution keeps the in-plane ("t") generalised strains equal
to the macroscopic ones and the normal ("n") generalised stresses constant
across layers.  With <s> the arithmetic and s_h the harmonic mean of the
layer scales:

    M^H_nn = s_h M_nn,  M^H_nt = s_h M_nt,  M^H_tn = s_h M_tn,
    M^H_tt = <s> (M_tt - M_tn M_nn^-1 M_nt) + s_h M_tn M_nn^-1 M_nt.

The trilinear FE space contains that piecewise-linear solution when the
layers are element layers, so the discrete cell problem reproduces it
exactly (up to solver tolerance).
"""
from __future__ import annotations

import numpy as np

# indices of (normal strain, two shears containing the axis, normal field)
NORMAL = {0: [0, 4, 5, 6], 1: [1, 3, 5, 7], 2: [2, 3, 4, 8]}


def laminate_effective(M, layer_scales, axis):
    s = np.asarray(layer_scales, dtype=np.float64)
    s_a = s.mean()
    s_h = 1.0 / np.mean(1.0 / s)
    n_idx = NORMAL[axis]
    t_idx = [i for i in range(9) if i not in n_idx]
    Mnn = M[np.ix_(n_idx, n_idx)]
    Mnt = M[np.ix_(n_idx, t_idx)]
    Mtn = M[np.ix_(t_idx, n_idx)]
    Mtt = M[np.ix_(t_idx, t_idx)]
    corr = Mtn @ np.linalg.solve(Mnn, Mnt)
    out = np.zeros((9, 9))
    out[np.ix_(n_idx, n_idx)] = s_h * Mnn
    out[np.ix_(n_idx, t_idx)] = s_h * Mnt
    out[np.ix_(t_idx, n_idx)] = s_h * Mtn
    out[np.ix_(t_idx, t_idx)] = s_a * (Mtt - corr) + s_h * corr
    return out


def laminate_effective_grad(M, layer_scales, axis, n, W):
    """d<W, M^H_lam>/ds_e for an element in layer k: (1/n^2) d/ds_k (per layer)."""
    s = np.asarray(layer_scales, dtype=np.float64)
    nl = len(s)
    s_h = 1.0 / np.mean(1.0 / s)
    n_idx = NORMAL[axis]
    t_idx = [i for i in range(9) if i not in n_idx]
    Mnn = M[np.ix_(n_idx, n_idx)]
    Mnt = M[np.ix_(n_idx, t_idx)]
    Mtn = M[np.ix_(t_idx, n_idx)]
    Mtt = M[np.ix_(t_idx, t_idx)]
    corr = Mtn @ np.linalg.solve(Mnn, Mnt)
    dA = np.zeros((9, 9))   # derivative of M^H wrt <s>
    dA[np.ix_(t_idx, t_idx)] = Mtt - corr
    dH = np.zeros((9, 9))   # derivative wrt s_h
    dH[np.ix_(n_idx, n_idx)] = Mnn
    dH[np.ix_(n_idx, t_idx)] = Mnt
    dH[np.ix_(t_idx, n_idx)] = Mtn
    dH[np.ix_(t_idx, t_idx)] = corr
    ds_a = 1.0 / nl
    ds_h = s_h ** 2 / (nl * s ** 2)
    per_layer = ds_a * np.sum(W * dA) + ds_h * np.sum(W * dH)
    # each layer holds n^2 elements sharing the layer derivative equally
    return per_layer / n ** 2
