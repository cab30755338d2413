"""Oracle checks at full problem sizes (64^3 to 256^3), where assembling and
factorising the cell matrix is out of reach.  TEST INFRASTRUCTURE ONLY.

Everything here is the definition of Sec. 2.2 written element by element:
the operator is K x = sum_e s_e P_e^T Ke P_e x and the load vectors are
F = sum_e s_e P_e^T Fe, with the element matrices Ke, Fe of oracle.fe
(2 x 2 x 2 Gauss quadrature of B^T M B and B^T M).  From a solution X that
someone else computed, these functions give

  * the full residual K X + F (every node; vectorised over elements),
  * residual rows at chosen nodes, each row summed from the eight elements
    around the node (cost independent of the grid size),
  * the per-element sensitivity (1 - eps_v) <W, G_e> at chosen elements,
    G_e[K, L] = sum_q w_q (e_K + B_q x_e^K) . M (e_L + B_q x_e^L),

so that a GPU solve can be checked where the oracle cannot solve.  The
residual bounds the tensors: the flux form is M^H = <s> M + F^T X, and with
F e_K = -K x^K and K symmetric the flux-form error of entry (K, L) is
-(x^K)^T r^L, at most ||x^K|| ||r^L|| in magnitude.
"""
from __future__ import annotations

import numpy as np

from . import fe
from .cell import element_nodes


def load_vectors(n, s, M):
    """F = sum_e s_e P_e^T Fe, (4 n^3, 9), node-major dofs 4 node + field."""
    _, Fe = fe.element_matrices(M, 1.0 / n)
    en = element_nodes(n)
    F = np.zeros((n ** 3, 4, 9))
    s = np.asarray(s, dtype=np.float64)
    for c in range(8):
        # every node is corner c of exactly one element: en[:, c] is a permutation
        F[en[:, c]] += s[:, None, None] * Fe[4 * c:4 * c + 4][None, :, :]
    return F.reshape(-1, 9)


def element_apply(n, s, M, X):
    """K X for X (4 n^3, k) without assembling K."""
    Ke, _ = fe.element_matrices(M, 1.0 / n)
    en = element_nodes(n)
    X = np.asarray(X, dtype=np.float64)
    k = X.shape[1]
    Xn = X.reshape(n ** 3, 4, k)
    s = np.asarray(s, dtype=np.float64)
    Y = np.zeros((n ** 3, 4, k))
    # element inputs (ne, 32, k), dof 4 l + f
    Xe = Xn[en].reshape(n ** 3, 32, k)
    for c in range(8):
        Y[en[:, c]] += s[:, None, None] * np.einsum("ij,ejk->eik", Ke[4 * c:4 * c + 4], Xe)
    return Y.reshape(-1, k)


def residual_norms(n, s, M, X):
    """Per load ||K x^L + F^L|| / ||F^L|| (0 where F^L = 0)."""
    F = load_vectors(n, s, M)
    R = element_apply(n, s, M, X) + F
    nf = np.linalg.norm(F, axis=0)
    return np.where(nf > 0, np.linalg.norm(R, axis=0) / np.where(nf > 0, nf, 1.0), 0.0)


def residual_rows(n, s, M, X, nodes):
    """(K X + F) at the given nodes: (len(nodes), 4, 9), each row summed over
    the eight elements that have the node as a corner."""
    Ke, Fe = fe.element_matrices(M, 1.0 / n)
    X = np.asarray(X, dtype=np.float64).reshape(n ** 3, 4, -1)
    s = np.asarray(s, dtype=np.float64)
    nodes = np.asarray(nodes, dtype=np.int64)
    i, j, k = nodes % n, (nodes // n) % n, nodes // (n * n)
    out = np.zeros((len(nodes), 4, X.shape[2]))
    for c, (a, b, cc) in enumerate(fe.LOCAL):
        # the element whose corner c is the node has origin node - (a, b, cc)
        e = ((i - a) % n) + n * (((j - b) % n) + n * ((k - cc) % n))
        xe = np.concatenate([X[((i - a + a2) % n) + n * (((j - b + b2) % n) + n * ((k - cc + c2) % n))]
                             for (a2, b2, c2) in fe.LOCAL], axis=1)     # (m, 32, k)
        out += s[e][:, None, None] * (np.einsum("ij,mjk->mik", Ke[4 * c:4 * c + 4], xe)
                                      + Fe[4 * c:4 * c + 4][None, :, :])
    return out


def element_sensitivity(n, mat, X, W, elems):
    """(1 - eps_v) <W, G_e> at the given elements (W non-dimensional, 9 x 9)."""
    M = fe.nondim_matrix(mat)
    h = 1.0 / n
    Bs, w = fe.element_bmats(h)
    X = np.asarray(X, dtype=np.float64).reshape(n ** 3, 4, 9)
    elems = np.asarray(elems, dtype=np.int64)
    i, j, k = elems % n, (elems // n) % n, elems // (n * n)
    xe = np.concatenate([X[((i + a) % n) + n * (((j + b) % n) + n * ((k + c) % n))]
                         for (a, b, c) in fe.LOCAL], axis=1)            # (m, 32, 9)
    g = np.einsum("qai,mil->qmal", Bs, xe) + np.eye(9)[None, None]
    G = np.einsum("q,qmak,ab,qmbl->mkl", w, g, M, g, optimize=True)
    return (1.0 - mat.void_scale) * np.einsum("mkl,kl->m", G, np.asarray(W))
