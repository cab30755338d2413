"""Figures of merit of the effective tensors (Sec. 2.3) and their gradients.

TEST INFRASTRUCTURE: part of the oracle the GPU path is checked against; used only by the tests, the
smoke check and the benchmark's CPU baseline.

Definitions (SI units, Voigt notation with engineering shear):
* S = (C^H)^-1, d = e^H S (3x6, strain coefficients),
* d_h = d_31 + d_32 + d_33 (sum over the z row of the first three columns),
* B_Voigt = (1/9) sum_{i,j<=3} C^H_ij,  B_Reuss = 1 / sum_{i,j<=3} S_ij.
The paper uses g_h and k_h without defining them; the reading taken here is
the usual hydrophone set: stress-free permittivity kappa^T = kappa^H + d e^T,
g_h = d_h / kappa^T_33, k_h = sqrt(d_h g_h B_Reuss).

Gradients are taken by the complex-step method (exact to rounding for these
analytic maps), independently of any closed form.
"""
from __future__ import annotations

import numpy as np

NAMES = ("d_h", "g_h", "B_voigt", "B_reuss", "k_h")


def foms(C, e, kappa):
    C = np.asarray(C).reshape(6, 6)
    e = np.asarray(e).reshape(3, 6)
    kappa = np.asarray(kappa).reshape(3, 3)
    S = np.linalg.inv(C)
    d = e @ S
    dh = d[2, 0] + d[2, 1] + d[2, 2]
    bv = C[:3, :3].sum() / 9.0
    br = 1.0 / S[:3, :3].sum()
    kT = kappa + d @ e.T
    gh = dh / kT[2, 2]
    kh = np.sqrt(dh * gh * br)
    return {"d_h": dh, "g_h": gh, "B_voigt": bv, "B_reuss": br, "k_h": kh}


def fom_grads(C, e, kappa, name, step=1e-30):
    """d(name)/d(C, e, kappa) by complex step, each w.r.t. all entries."""
    C = np.asarray(C, dtype=np.complex128).reshape(6, 6)
    e = np.asarray(e, dtype=np.complex128).reshape(3, 6)
    kappa = np.asarray(kappa, dtype=np.complex128).reshape(3, 3)
    out = []
    for arr in (C, e, kappa):
        g = np.zeros(arr.shape)
        scale = np.max(np.abs(arr.real)) or 1.0
        hstep = step * scale
        for idx in np.ndindex(arr.shape):
            orig = arr[idx]
            arr[idx] = orig + 1j * hstep
            g[idx] = foms(C, e, kappa)[name].imag / hstep
            arr[idx] = orig
        out.append(g)
    return out
