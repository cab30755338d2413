"""Textbook right-preconditioned GMRES with the Schur preconditioner of Sec. 2.5.3.

TEST INFRASTRUCTURE: part of the oracle the GPU path is checked against; used only by the tests, the
smoke check and the benchmark's CPU baseline.

The block system of Sec. 2.5 orders unknowns as (x, y) = (displacements,
potential):  calA = [[A, B^T], [B, -C]].  The preconditioner is the block
lower-triangular  P = [[A, 0], [B, -S]]  (the paper's P_SCP written for calA
instead of its sign-flipped twin), with either the exact Schur complement
S = C + B A^-1 B^T or the element-wise approximation

    S_bar = sum_e C_e + B_e (A_e + delta I)^-1 B_e^T,   delta = 1e-10,

assembled like any other element matrix.  (The printed formula transposes B;
the reading taken is the one whose dimensions agree with B in R^{m x n}.)
Applying P^-1 to (r_x, r_y):  z_x = A^-1 r_x,  z_y = S^-1 (B z_x - r_y).

Everything here is dense or scipy-sparse on pinned (node 0 removed) systems
and exists to pin the preconditioner's structure, not to be fast.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe
from .cell import element_dofs


def field_split(nd):
    """Index arrays of the displacement and potential dofs among 0..nd-1."""
    d = np.arange(nd)
    return d[d % 4 != 3], d[d % 4 == 3]


def schur_elementwise(n, s, M, delta=1e-10):
    """Assembled S_bar over potential dofs (n^3 square, CSR)."""
    h = 1.0 / n
    Ke, _ = fe.element_matrices(M, h)
    ui = [4 * l + f for l in range(8) for f in range(3)]
    pi = [4 * l + 3 for l in range(8)]
    A0 = Ke[np.ix_(ui, ui)]
    B0 = Ke[np.ix_(pi, ui)]
    C0 = -Ke[np.ix_(pi, pi)]
    en = element_dofs(n)[:, 3::4] // 4          # element -> global node (= potential index)
    rows, cols, vals = [], [], []
    for e in range(n ** 3):
        Ae = s[e] * A0 + delta * np.eye(24)
        Be = s[e] * B0
        Se = s[e] * C0 + Be @ np.linalg.solve(Ae, Be.T)
        rows.append(np.repeat(en[e], 8))
        cols.append(np.tile(en[e], 8))
        vals.append(Se.ravel())
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n ** 3, n ** 3)).tocsr()
    S.sum_duplicates()
    return S


class SchurPreconditioner:
    """z = P^-1 r for P = [[A, 0], [B, -S]] on the pinned system (dense solves)."""

    def __init__(self, K, free, S=None):
        Kd = np.asarray(K.todense()) if sp.issparse(K) else np.asarray(K)
        Kf = Kd[np.ix_(free, free)]
        is_u = (free % 4) != 3
        self.iu = np.nonzero(is_u)[0]
        self.ip = np.nonzero(~is_u)[0]
        self.A = Kf[np.ix_(self.iu, self.iu)]
        self.B = Kf[np.ix_(self.ip, self.iu)]
        C = -Kf[np.ix_(self.ip, self.ip)]
        if S is None:
            S = C + self.B @ np.linalg.solve(self.A, self.B.T)
        self.S = S

    def apply(self, r):
        z = np.zeros_like(r)
        zu = np.linalg.solve(self.A, r[self.iu])
        z[self.iu] = zu
        z[self.ip] = np.linalg.solve(self.S, self.B @ zu - r[self.ip])
        return z


def gmres_right(Aop, b, Pinv, rtol=1e-12, restart=50, maxit=500):
    """Right-preconditioned restarted GMRES (modified Gram-Schmidt, Givens).

    Solves Aop(x) = b as Aop(P^-1 t) = b, x = P^-1 t.  Returns x and the list
    of true relative residual norms at each inner step.
    """
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = []
    if nb == 0.0:
        return x, [0.0]
    it = 0
    while it < maxit:
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        hist.append(beta / nb)
        if beta / nb <= rtol:
            break
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k_used = 0
        for j in range(restart):
            w = Aop(Pinv(V[j]))
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k_used = j + 1
            it += 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) / nb <= rtol or H[j, j] == 0.0 or it >= maxit:
                break
            V.append(w / hn if hn != 0 else w)
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        t = sum(y[i] * V[i] for i in range(k_used))
        x = x + Pinv(t)
        if hist[-1] <= rtol:
            r = b - Aop(x)
            hist.append(np.linalg.norm(r) / nb)
            if hist[-1] <= rtol * 10:
                break
    return x, hist


def solve_scp(K, F, n=None, s=None, M=None, exact=True, rtol=1e-12, restart=50):
    """Pinned solve of K X = -F by SCP-GMRES, one load column at a time."""
    nd = K.shape[0]
    free = np.arange(4, nd)
    Kf = K[free][:, free]
    S = None
    if not exact:
        Sbar = schur_elementwise(n, s, M).toarray()
        S = Sbar[1:, 1:]                       # potential of node 0 pinned
    P = SchurPreconditioner(K, free, S)
    X = np.zeros((nd, F.shape[1]))
    hists = []
    for L in range(F.shape[1]):
        x, h = gmres_right(lambda v: Kf @ v, -F[free, L], P.apply, rtol=rtol, restart=restart)
        X[free, L] = x
        hists.append(h)
    return X, hists
