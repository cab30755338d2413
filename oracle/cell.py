"""Periodic cell problem: assembly, pinned direct solve, effective tensors.

TEST INFRASTRUCTURE: part of the oracle the GPU path is checked against; used only by the tests, the
smoke check and the benchmark's CPU baseline.

Sec. 2.2: for each of the nine unit macroscopic fields g_L (six engineering
strains, three electric fields) find the periodic fluctuation x^L with

    sum_e s_e int_e (B v)^T M (g_L + B x^L) = 0   for all periodic v,

i.e.  K x^L = -F e_L  with K, F assembled from the element matrices.  The
effective matrix is the cell average of tau = s M (g_L + B x^L) over the unit
cell (Vol(D) = 1), which is the paper's formulas for the homogenised C, e and
kappa written for all nine loads at once (flux form).

Periodicity leaves the four constant fields (three translations, constant
potential) in the kernel; they do not change any tensor.  The oracle fixes
them by deleting node 0's four dofs (pin), a reading the paper leaves open.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe


def element_nodes(n):
    """(n^3, 8) global node of each element corner, element order = node order."""
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    out = np.empty((n ** 3, 8), dtype=np.int64)
    for l, (a, b, c) in enumerate(fe.LOCAL):
        out[:, l] = ((i + a) % n) + n * (((j + b) % n) + n * ((k + c) % n))
    return out


def element_dofs(n):
    en = element_nodes(n)
    return (4 * en[:, :, None] + np.arange(4)[None, None, :]).reshape(-1, 32)


def assemble(n, s, M, npts=2):
    """Global K (CSR, 4n^3 square) and F (dense 4n^3 x 9) for scales s: one per element (n^3,), or
    one per element and Gauss point (n^3, npts^3) for the quadrature-point material."""
    h = 1.0 / n
    s = np.asarray(s, dtype=np.float64)
    dofs = element_dofs(n)
    ne = n ** 3
    nd = 4 * ne
    rows = np.repeat(dofs, 32, axis=1).ravel()
    cols = np.tile(dofs, (1, 32)).ravel()
    if s.ndim == 1:
        Ke, Fe = fe.element_matrices(M, h, npts)
        vals = (s[:, None] * Ke.ravel()[None, :]).ravel()
        contrib = s[:, None, None] * Fe[None, :, :]
    else:
        Kq, Fq = fe.element_matrices_qp(M, h, npts)
        vals = np.einsum("eq,qij->eij", s, Kq).ravel()
        contrib = np.einsum("eq,qil->eil", s, Fq)
    K = sp.coo_matrix((vals, (rows, cols)), shape=(nd, nd)).tocsr()
    K.sum_duplicates()
    F = np.zeros((nd, 9))
    np.add.at(F, dofs.ravel(), contrib.reshape(-1, 9))
    return K, F


def assemble_loops(n, s, M, npts=2):
    """Same as assemble() but dense and with explicit Python loops (tiny n only)."""
    h = 1.0 / n
    Ke, Fe = fe.element_matrices(M, h, npts)
    nd = 4 * n ** 3
    K = np.zeros((nd, nd))
    F = np.zeros((nd, 9))
    e = 0
    for k in range(n):
        for j in range(n):
            for i in range(n):
                gd = []
                for a, b, c in fe.LOCAL:
                    node = ((i + a) % n) + n * (((j + b) % n) + n * ((k + c) % n))
                    gd.extend(4 * node + f for f in range(4))
                for p in range(32):
                    F[gd[p], :] += s[e] * Fe[p, :]
                    for q in range(32):
                        K[gd[p], gd[q]] += s[e] * Ke[p, q]
                e += 1
    return K, F


def solve_pinned(K, F):
    """Solve K X = -F with node 0's four dofs fixed to zero (sparse LU)."""
    nd = K.shape[0]
    free = np.arange(4, nd)
    Kf = K[free][:, free].tocsc()
    lu = spla.splu(Kf, permc_spec="MMD_AT_PLUS_A")
    X = np.zeros((nd, F.shape[1]))
    X[free] = lu.solve(-F[free])
    return X


def solve_dense_pinned(K, F):
    K = np.asarray(K.todense()) if sp.issparse(K) else np.asarray(K)
    X = np.zeros((K.shape[0], F.shape[1]))
    X[4:] = np.linalg.solve(K[4:, 4:], -F[4:])
    return X


def solve_dense_minnorm(K, F):
    K = np.asarray(K.todense()) if sp.issparse(K) else np.asarray(K)
    X, *_ = np.linalg.lstsq(K, -F, rcond=1e-13)
    return X


def _gauss_g(n, X, npts=2):
    """g_q,e^L = e_L + B_q x_e^L: array (q, n^3, 9 comps, 9 loads) and weights."""
    h = 1.0 / n
    Bs, w = fe.element_bmats(h, npts)
    Xe = X[element_dofs(n)]                       # (ne, 32, 9)
    g = np.einsum("qai,eil->qeal", Bs, Xe)
    g += np.eye(9)[None, None, :, :]
    return g, w


def _point_scales(s, nq):
    """Scales per (element, Gauss point): per-element scales repeat at every point."""
    s = np.asarray(s, dtype=np.float64)
    return np.repeat(s[:, None], nq, axis=1) if s.ndim == 1 else s


def effective_flux(n, s, M, X, npts=2):
    """M^H[:, L] = sum_e sum_q w_q s_eq M (e_L + B_q x_e^L)  (mean generalised stress)."""
    g, w = _gauss_g(n, X, npts)
    mean_g = np.einsum("q,eq,qeal->al", w, _point_scales(s, len(w)), g)
    return M @ mean_g


def effective_energy(n, s, M, X, npts=2):
    """M^H_en[K, L] = sum_e sum_q w_q s_eq (e_K + B x^K) . M (e_L + B x^L)."""
    g, w = _gauss_g(n, X, npts)
    return np.einsum("q,eq,qeak,ab,qebl->kl", w, _point_scales(s, len(w)), g, M, g, optimize=True)


def element_energy_matrices(n, X, M, npts=2):
    """G_e[K, L] = sum_q w_q (e_K + B x_e^K) . M (e_L + B x_e^L): (ne, 9, 9).

    With M^H = sum_e s_e G_e at the discrete solution (Galerkin
    orthogonality), dM^H/ds_e = G_e and dM^H/drho_e = (1 - eps_v) G_e.
    """
    g, w = _gauss_g(n, X, npts)
    return np.einsum("q,qeak,ab,qebl->ekl", w, g, M, g, optimize=True)


def rhs_compatibility(n, F):
    """Sum of the load vector over all nodes, per field and load (must be 0)."""
    return F.reshape(n ** 3, 4, 9).sum(axis=0)


class Result(dict):
    __getattr__ = dict.__getitem__


def homogenise(n, mat, phi=None, rho=None, width_elems=2.0, solver="lu", want_x=True, smoothing="element"):
    """Full oracle pipeline for one cell: density -> solve -> tensors.

    Give either the nodal level set phi (length n^3) or per-element rho.  smoothing = "qp" evaluates
    the smoothed Heaviside at every Gauss point of the level set's trilinear interpolation (rho and s
    then have one value per element and point).
    Returns a dict with s, rho, X (4n^3 x 9, node-major dofs 4*node + f),
    MH (non-dimensional flux form), MH_energy, and SI tensors C, e, kappa.
    """
    M = fe.nondim_matrix(mat)
    if rho is None:
        rho = fe.density_qp(n, phi, width_elems) if smoothing == "qp" else fe.density_from_levelset(n, phi, width_elems)
    s = fe.ersatz_scale(rho, mat.void_scale)
    K, F = assemble(n, s, M)
    if solver == "lu":
        X = solve_pinned(K, F)
    elif solver == "dense":
        X = solve_dense_pinned(K, F)
    else:
        raise ValueError(solver)
    MH = effective_flux(n, s, M, X)
    MHe = effective_energy(n, s, M, X)
    C, e, k = fe.split_effective(MH)
    r = Result(s=s, rho=rho, MH=MH, MH_energy=MHe, C=C, e=e, kappa=k, M=M)
    if want_x:
        r["X"] = X
        r["K"] = K
        r["F"] = F
    return r


def grad_rho(n, mat, X, W_nd):
    """dJ/drho_e = (1 - eps_v) <W, G_e> for W = dJ/dM^H (non-dimensional)."""
    M = fe.nondim_matrix(mat)
    G = element_energy_matrices(n, X, M)
    return (1.0 - mat.void_scale) * np.einsum("ekl,kl->e", G, W_nd)


def grad_phi_from_rho(n, phi, g_rho, width_elems=2.0):
    """Chain rule to nodal phi: rho_e = 1 - H(mean_e phi), so
    dJ/dphi_n = -(1/8) sum_{e containing n} H'(mean_e phi) dJ/drho_e."""
    eta = width_elems / n
    t = fe.element_mean(n, phi)
    ge = -fe.smoothed_heaviside_deriv(t, eta) * g_rho / 8.0
    en = element_nodes(n)
    out = np.zeros(n ** 3)
    for l in range(8):
        np.add.at(out, en[:, l], ge)
    return out


def element_energy_matrices_qp(n, X, M, npts=2):
    """Per element and Gauss point, G_ep[K, L] = w_p (e_K + B_p x_e^K) . M (e_L + B_p x_e^L):
    (ne, q, 9, 9).  With the material at the points, M^H = sum_e sum_p s_ep G_ep at the discrete
    solution, so dM^H/ds_ep = G_ep."""
    g, w = _gauss_g(n, X, npts)
    return np.einsum("q,qeak,ab,qebl->eqkl", w, g, M, g, optimize=True)


def grad_rho_qp(n, mat, X, W_nd):
    """dJ/drho_ep = (1 - eps_v) <W, G_ep> (ne, q) for W = dJ/dM^H."""
    M = fe.nondim_matrix(mat)
    G = element_energy_matrices_qp(n, X, M)
    return (1.0 - mat.void_scale) * np.einsum("eqkl,kl->eq", G, W_nd)


def grad_phi_from_rho_qp(n, phi, g_rho, width_elems=2.0, npts=2):
    """Chain rule of the point densities rho_ep = 1 - H(phi(x_p)), phi(x_p) = sum_l N_l(xi_p) phi_l:
    dJ/dphi_n = -sum over (e, p) with n = corner l of e of H'(phi(x_p)) N_l(xi_p) dJ/drho_ep."""
    eta = width_elems / n
    pts, _ = fe.gauss_rule(npts)
    Nv = np.array([fe.shape_values(p) for p in pts])                 # (q, 8)
    gp = -fe.smoothed_heaviside_deriv(fe.levelset_at_gauss(n, phi, npts), eta) * g_rho     # (ne, q)
    contrib = gp @ Nv                                                  # (ne, 8 corners)
    en = element_nodes(n)
    out = np.zeros(n ** 3)
    for l in range(8):
        np.add.at(out, en[:, l], contrib[:, l])
    return out


def W_from_tensor_grads(gC, ge, gk):
    """Map gradients w.r.t. SI (C^H, e^H, kappa^H) to W = dJ/dM^H (non-dim).

    C^H = C0 MH[:6,:6], e^H = -E0 MH[6:,:6], kappa^H = -K0 MH[6:,6:].
    """
    W = np.zeros((9, 9))
    W[:6, :6] = fe.C0 * np.asarray(gC).reshape(6, 6)
    W[6:, :6] = -fe.E0 * np.asarray(ge).reshape(3, 6)
    W[6:, 6:] = -fe.K0 * np.asarray(gk).reshape(3, 3)
    return W
