"""Material matrix, units, trilinear hex8 element and density map (FP64).

TEST INFRASTRUCTURE: part of the oracle the GPU path is checked against; used only by the tests, the
smoke check and the benchmark's CPU baseline.

Sec. 2.2 (constitutive laws): sigma = C eps - e^T E, D = e eps + kappa E,
eps = sym grad u, E = -grad phi.  With the generalised strain
g = (eps_xx, eps_yy, eps_zz, gamma_yz, gamma_xz, gamma_xy, E_x, E_y, E_z)
(engineering shear, Voigt order of Sec. 2.3) and generalised stress
tau = (sigma, -D), the laws read tau = M g with the symmetric 9x9

    M = [[ C, -e^T],
         [-e, -kappa]].
"""
from __future__ import annotations

import numpy as np

# Non-dimensionalisation (Sec. 2.2 says a scaling is used but does not print
# it).  Reading: stress scale C0, charge scale E0; permittivity scale E0^2/C0.
C0 = 1.0e9
E0 = 1.0
K0 = E0 ** 2 / C0


def material_matrix(C, e, kappa):
    """The 9x9 generalised material matrix M = [[C, -e^T], [-e, -kappa]]."""
    M = np.zeros((9, 9))
    M[:6, :6] = C
    M[:6, 6:] = -np.asarray(e).T
    M[6:, :6] = -np.asarray(e)
    M[6:, 6:] = -np.asarray(kappa)
    return M


def nondim_matrix(mat):
    """M built from the material scaled to C/C0, e/E0, kappa/K0."""
    return material_matrix(mat.C / C0, mat.e / E0, mat.kappa / K0)


def split_effective(MH, dimensional=True):
    """Split a 9x9 effective matrix into (C^H, e^H, kappa^H).

    C^H = MH[:6,:6], e^H = -MH[6:,:6] (mean D under strain loads),
    kappa^H = -MH[6:,6:] (mean D under field loads).  With dimensional=True
    the non-dimensional blocks are rescaled to SI.
    """
    C = MH[:6, :6].copy()
    e = -MH[6:, :6].copy()
    k = -MH[6:, 6:].copy()
    if dimensional:
        C *= C0
        e *= E0
        k *= K0
    return C, e, k


# ---------------------------------------------------------------- element
# Local node l = a + 2b + 4c sits at (a, b, c) * h of the element [0, h]^3.
LOCAL = np.array([[l & 1, (l >> 1) & 1, (l >> 2) & 1] for l in range(8)], dtype=np.int64)


def shape_grads(xi):
    """Gradients (8, 3) of the trilinear shape functions on [0,1]^3 at xi."""
    G = np.zeros((8, 3))
    for l in range(8):
        f = [xi[d] if LOCAL[l, d] else 1.0 - xi[d] for d in range(3)]
        df = [1.0 if LOCAL[l, d] else -1.0 for d in range(3)]
        G[l, 0] = df[0] * f[1] * f[2]
        G[l, 1] = f[0] * df[1] * f[2]
        G[l, 2] = f[0] * f[1] * df[2]
    return G


def shape_values(xi):
    """Values (8,) of the trilinear shape functions on [0,1]^3 at xi."""
    return np.array([np.prod([xi[d] if LOCAL[l, d] else 1.0 - xi[d] for d in range(3)]) for l in range(8)])


def bmat(xi, h):
    """9x32 map from element dofs (4l + f, f = ux, uy, uz, phi) to g at xi."""
    G = shape_grads(xi) / h            # physical gradients
    B = np.zeros((9, 32))
    for l in range(8):
        dx, dy, dz = G[l]
        c = 4 * l
        B[0, c + 0] = dx
        B[1, c + 1] = dy
        B[2, c + 2] = dz
        B[3, c + 1] = dz                # gamma_yz = du_y/dz + du_z/dy
        B[3, c + 2] = dy
        B[4, c + 0] = dz                # gamma_xz = du_x/dz + du_z/dx
        B[4, c + 2] = dx
        B[5, c + 0] = dy                # gamma_xy = du_x/dy + du_y/dx
        B[5, c + 1] = dx
        B[6, c + 3] = -dx               # E = -grad phi
        B[7, c + 3] = -dy
        B[8, c + 3] = -dz
    return B


def gauss_rule(npts):
    """Tensor Gauss-Legendre rule on [0,1]^3: points (q,3), weights (q,)."""
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for k in range(npts):
        for j in range(npts):
            for i in range(npts):
                pts.append((x[i], x[j], x[k]))
                wts.append(w[i] * w[j] * w[k])
    return np.array(pts), np.array(wts)


def element_bmats(h, npts=2):
    """Bmat at each Gauss point and the physical weights (volume h^3 total)."""
    pts, wts = gauss_rule(npts)
    Bs = np.array([bmat(p, h) for p in pts])
    return Bs, wts * h ** 3


def element_matrices(M, h, npts=2):
    """Element stiffness K (32x32) and load matrix F (32x9) for material M.

    K = sum_q w_q B_q^T M B_q and F = sum_q w_q B_q^T M, so that the weak form
    of Sec. 2.2 on one element with macroscopic field e_L and fluctuation x
    contributes v^T (F e_L + K x).  Linear in M, so an ersatz element with
    material s*M has matrices s*K, s*F.
    """
    Bs, w = element_bmats(h, npts)
    K = np.einsum("q,qai,ab,qbj->ij", w, Bs, M, Bs)
    F = np.einsum("q,qai,ab->ib", w, Bs, M)
    return K, F


def element_matrices_qp(M, h, npts=2):
    """The terms of element_matrices per Gauss point: K_q = w_q B_q^T M B_q (q, 32, 32) and
    F_q = w_q B_q^T M (q, 32, 9), so that an element whose material is s_q M at point q has matrices
    sum_q s_q K_q and sum_q s_q F_q (the quadrature-point interpolation of the material)."""
    Bs, w = element_bmats(h, npts)
    K = np.einsum("q,qai,ab,qbj->qij", w, Bs, M, Bs)
    F = np.einsum("q,qai,ab->qib", w, Bs, M)
    return K, F


# ---------------------------------------------------------------- density
def smoothed_heaviside(t, eta):
    """Sinusoidal smoothed Heaviside of half-width eta (Sec. 2.6 smoothing)."""
    t = np.asarray(t, dtype=np.float64)
    H = np.where(t > eta, 1.0, 0.0)
    band = np.abs(t) <= eta
    tb = t[band]
    H = H.astype(np.float64)
    H[band] = 0.5 * (1.0 + tb / eta + np.sin(np.pi * tb / eta) / np.pi)
    return H


def smoothed_heaviside_deriv(t, eta):
    t = np.asarray(t, dtype=np.float64)
    d = np.zeros_like(t)
    band = np.abs(t) <= eta
    d[band] = (1.0 + np.cos(np.pi * t[band] / eta)) / (2.0 * eta)
    return d


def element_mean(n, nodal):
    """Mean of an element's 8 nodal values; element (i,j,k) -> nodes i..i+1 etc."""
    f = np.asarray(nodal).reshape(n, n, n)     # [k][j][i]
    acc = np.zeros_like(f)
    for a, b, c in LOCAL:
        acc += np.roll(f, shift=(-c, -b, -a), axis=(0, 1, 2))
    return (acc / 8.0).ravel()


def density_from_levelset(n, phi, width_elems=2.0):
    """rho_e = 1 - H_eta(mean_e phi) with eta = width_elems * h (phi < 0 solid)."""
    eta = width_elems / n
    return 1.0 - smoothed_heaviside(element_mean(n, phi), eta)


def levelset_at_gauss(n, phi, npts=2):
    """Trilinear interpolation of the nodal level set at every element's Gauss points: (n^3, npts^3),
    points in gauss_rule's order."""
    pts, _ = gauss_rule(npts)
    f = np.asarray(phi, dtype=np.float64).reshape(n, n, n)     # [k][j][i]
    corner = [np.roll(f, shift=(-c, -b, -a), axis=(0, 1, 2)).ravel() for a, b, c in LOCAL]
    Nv = np.array([shape_values(p) for p in pts])                # (q, 8)
    return np.stack(corner, axis=1) @ Nv.T                        # (ne, q)


def density_qp(n, phi, width_elems=2.0, npts=2):
    """rho at each Gauss point, 1 - H_eta(phi interpolated there): the smoothing evaluated at the
    quadrature points instead of once per element (phi < 0 solid)."""
    return 1.0 - smoothed_heaviside(levelset_at_gauss(n, phi, npts), width_elems / n)


def ersatz_scale(rho, void_scale):
    """s = eps_v + (1 - eps_v) rho, applied to C, e and kappa alike."""
    return void_scale + (1.0 - void_scale) * np.asarray(rho, dtype=np.float64)
