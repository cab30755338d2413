"""TriCG, the short-recurrence Krylov method the paper compares for its symmetric quasi-definite block
system (Sec. 2.5, Sec. 2.5.2; Montoison and Orban, SIAM J. Sci. Comput. 43, 2021).

TEST INFRASTRUCTURE: the oracle of the GPU path, used only by the tests.

The system [[E, A], [A^T, -F]] [x; y] = [b; c] has E and F symmetric positive definite (on the periodic
cell: on the subspace of zero field means).  For the piezoelectric block system of Sec. 2.5,
calA = [[A, B^T], [B, -C]], the roles are E = A, the coupling A = B^T, F = C.

The method, as written here:

* Orthogonal tridiagonalisation with the E- and F-inner products (the Saunders-Simon-Yip process):
  beta_1 E u_1 = b and gamma_1 F v_1 = c with ||u_1||_E = ||v_1||_F = 1; then for k = 1, 2, ...
      A v_k   = gamma_k E u_{k-1} + alpha_k E u_k + beta_{k+1}  E u_{k+1},
      A^T u_k = beta_k  F v_{k-1} + alpha_k F v_k + gamma_{k+1} F v_{k+1},
  alpha_k = u_k^T A v_k, and beta_{k+1}, gamma_{k+1} normalise the new vectors.  With U_k, V_k the
  bases and T_k the tridiagonal matrix (diagonal alpha, below it beta_2.., above it gamma_2..):
  U^T E U = I, V^T F V = I, U^T A V = T.
* Galerkin condition: x_k = U_k xi, y_k = V_k eta with the residual orthogonal to both bases, i.e.
      [[I, T_k], [T_k^T, -I]] [xi; eta] = [beta_1 e_1; gamma_1 e_1].
  Interleaving (xi_1, eta_1, xi_2, eta_2, ...) makes this block tridiagonal with 2 x 2 blocks:
  diagonal [[1, alpha_k], [alpha_k, -1]], below the diagonal [[0, beta_k], [gamma_k, 0]].  It is a
  symmetric permutation of a quasi-definite matrix, so the block LDL^T factorisation exists without
  pivoting: D_1 = Delta_1, L_k = Gamma_k D_{k-1}^-1, D_k = Delta_k - L_k Gamma_k^T.
* Short recurrences: with d_1 = (beta_1, gamma_1), d_k = -L_k d_{k-1}, z_k = D_k^-1 d_k and the two
  direction columns G_k = P_k - G_{k-1} L_k^T (P_k has (u_k, 0) and (0, v_k) as columns), the iterate is
  updated by (x, y) += G_k z_k.  The last block of (xi, eta) is z_k, and the residual is
  (-eta_k beta_{k+1} E u_{k+1}, -xi_k gamma_{k+1} F v_{k+1}), so its norm costs nothing extra.
* A right-hand side with one zero block cannot start the process.  Reading taken (the paper reports a
  load whose blocks are both nonzero): for c = 0 start from y_0 = F^-1 A^T E^-1 b (if that is zero,
  (E^-1 b, 0) is the solution), for b = 0 from x_0 = -E^-1 A F^-1 c (if zero, (0, -F^-1 c) is), and run
  TriCG on the residual of that start.  On the piezoelectric cell this happens: for the z-poled
  material of the workloads the in-plane shear load has no potential part.
* Breakdown: when beta_{k+1} or gamma_{k+1} falls below 1e-10 of the largest one so far, one of the
  two Krylov spaces is exhausted and the process cannot continue (it happens right after the start
  above).  The cycle stops at its last iterate, and the solve restarts from the true residual of the
  accumulated solution.  A residual block below 1e-12 of the other, or below min(1e-13, rtol / 10) of
  the right-hand side (rounding noise, negligible against the target), counts as zero there and takes
  the start above (on the cell, the in-plane shear load's potential residual is exact after a cycle).
  Cycles also end when the recurrence's residual reaches the tolerance; the solve ends when the true
  residual does.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def tricg(Aop, Atop, Einv, Finv, b, c, rtol=1e-10, maxit=500, record=False):
    """Solve [[E, A], [A^T, -F]] [x; y] = [b; c] given x -> A x, y -> A^T y, E^-1 and F^-1.

    Stops when the residual (from the recurrence) is at most rtol ||(b, c)|| or at a breakdown.  Returns
    (x, y, info); info has 'iters', 'est' (residual norms per iteration), 'breakdown' and, with record,
    'iterates', 'U', 'V', 'alpha', 'beta', 'gamma'.
    """
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    bnorm = np.sqrt(b @ b + c @ c)
    x, y = np.zeros_like(b), np.zeros_like(c)
    info = {"iters": 0, "est": [], "breakdown": False}
    if bnorm == 0.0:
        return x, y, info
    Eb, Fc = Einv(b), Finv(c)
    beta, gamma = np.sqrt(b @ Eb), np.sqrt(c @ Fc)
    if not (beta > 0.0 and gamma > 0.0):
        raise ValueError("TriCG needs both right-hand-side blocks nonzero")
    u, Eu, v, Fv = Eb / beta, b / beta, Fc / gamma, c / gamma
    Eu_prev, Fv_prev = np.zeros_like(b), np.zeros_like(c)
    g1x, g2x, g1y, g2y = np.zeros_like(b), np.zeros_like(b), np.zeros_like(c), np.zeros_like(c)
    d = np.array([beta, gamma])
    D = None
    bmax, gmax = beta, gamma
    if record:
        info.update(iterates=[], U=[u], V=[v], alpha=[], beta=[beta], gamma=[gamma])
    for k in range(1, maxit + 1):
        # tridiagonalisation step k
        q = Aop(v) - gamma * Eu_prev
        p = Atop(u) - beta * Fv_prev
        alpha = u @ q
        q -= alpha * Eu
        p -= alpha * Fv
        Eq, Fp = Einv(q), Finv(p)
        beta_n, gamma_n = np.sqrt(max(q @ Eq, 0.0)), np.sqrt(max(p @ Fp, 0.0))
        # block LDL^T step k
        Delta = np.array([[1.0, alpha], [alpha, -1.0]])
        if D is None:
            L = np.zeros((2, 2))
            D = Delta
        else:
            Gamma = np.array([[0.0, beta], [gamma, 0.0]])
            L = Gamma @ np.linalg.inv(D)
            D = Delta - L @ Gamma.T
            d = -L @ d
        z = np.linalg.solve(D, d)
        # directions and iterate
        g1x, g2x = u - (L[0, 0] * g1x + L[0, 1] * g2x), -(L[1, 0] * g1x + L[1, 1] * g2x)
        g1y, g2y = -(L[0, 0] * g1y + L[0, 1] * g2y), v - (L[1, 0] * g1y + L[1, 1] * g2y)
        x = x + z[0] * g1x + z[1] * g2x
        y = y + z[0] * g1y + z[1] * g2y
        est = np.sqrt((z[1] * np.linalg.norm(q)) ** 2 + (z[0] * np.linalg.norm(p)) ** 2)
        info["est"].append(est / bnorm)
        info["iters"] = k
        if record:
            info["iterates"].append((x.copy(), y.copy()))
            info["alpha"].append(alpha)
        if est <= rtol * bnorm:
            break
        bmax, gmax = max(bmax, beta_n), max(gmax, gamma_n)
        if not (beta_n > 1e-10 * bmax and gamma_n > 1e-10 * gmax):
            info["breakdown"] = True
            break
        Eu_prev, Fv_prev = Eu, Fv
        u, Eu, v, Fv = Eq / beta_n, q / beta_n, Fp / gamma_n, p / gamma_n
        beta, gamma = beta_n, gamma_n
        if record:
            info["U"].append(u)
            info["V"].append(v)
            info["beta"].append(beta)
            info["gamma"].append(gamma)
    return x, y, info


def galerkin_iterate(U, V, alpha, beta, gamma, k):
    """The k-th TriCG iterate by its definition: solve the Galerkin system of the first k basis vectors
    densely and expand (an independent check of the short recurrences)."""
    T = np.diag(alpha[:k])
    for i in range(1, k):
        T[i, i - 1] = beta[i]
        T[i - 1, i] = gamma[i]
    M = np.block([[np.eye(k), T], [T.T, -np.eye(k)]])
    rhs = np.zeros(2 * k)
    rhs[0], rhs[k] = beta[0], gamma[0]
    sol = np.linalg.solve(M, rhs)
    x = sum(sol[i] * U[i] for i in range(k))
    y = sum(sol[k + i] * V[i] for i in range(k))
    return x, y


def pinned_inverse(M, F):
    """x -> M^+ x for a periodic-cell block M (node-major, F fields per node) whose kernel is the
    per-field constants: solve with the first node's F dofs removed, then remove each field's mean
    (the zero-mean solution for a zero-mean right-hand side)."""
    M = sp.csc_matrix(M)
    n = M.shape[0]
    keep = np.arange(F, n)
    lu = spla.splu(M[keep][:, keep].tocsc())

    def apply(r):
        out = np.zeros(n)
        out[keep] = lu.solve(np.asarray(r, dtype=np.float64)[keep])
        out = out.reshape(-1, F)
        return (out - out.mean(axis=0)).ravel()

    return apply


def piezo_blocks(K):
    """(A, B^T, C) of the assembled cell matrix K (dofs 4 node + field): calA = [[A, B^T], [B, -C]]."""
    K = sp.csr_matrix(K)
    d = np.arange(K.shape[0])
    iu, ip = d[d % 4 < 3], d[d % 4 == 3]
    A = K[iu][:, iu]
    Bt = K[iu][:, ip]
    C = -K[ip][:, ip]
    return A, Bt, C, iu, ip


def start(b, c, Aop, Atop, Einv, Finv):
    """The start (x_0, y_0) for a right-hand side with a zero block (zeros otherwise), and whether it is
    already the solution."""
    zb, zc = not np.any(b), not np.any(c)
    x0, y0 = np.zeros_like(b), np.zeros_like(c)
    if zb and zc:
        return x0, y0, True
    if zc:
        xh = Einv(b)
        y0 = Finv(Atop(xh))
        if not np.any(y0):
            return xh, y0, True
    elif zb:
        yh = Finv(c)
        x0 = -Einv(Aop(yh))
        if not np.any(x0):
            return x0, -yh, True
    return x0, y0, False


def solve_restarted(Kop, Aop, Atop, Einv, Finv, b, c, rtol=1e-10, maxit=500, max_cycles=60):
    """TriCG cycles from the true residual (Kop: (x, y) -> K (x, y) as a pair) with the zero-block start
    and restarts after breakdowns.  Returns (x, y, TriCG iterations over all cycles, cycles)."""
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    x, y = np.zeros_like(b), np.zeros_like(c)
    n0 = np.sqrt(b @ b + c @ c)
    total = cycles = 0
    while cycles < max_cycles and total < maxit:
        kx, ky = Kop(x, y)
        rx, ry = b - kx, c - ky
        nx, ny = np.linalg.norm(rx), np.linalg.norm(ry)
        rn = np.hypot(nx, ny)
        if rn <= rtol * n0:
            break
        cycles += 1
        tiny = min(1e-13, 0.1 * rtol) * n0
        if ny <= 1e-12 * nx or ny <= tiny:
            ry = np.zeros_like(ry)
        elif nx <= 1e-12 * ny or nx <= tiny:
            rx = np.zeros_like(rx)
        x0, y0, done = start(rx, ry, Aop, Atop, Einv, Finv)
        if done or np.any(x0) or np.any(y0):
            x, y = x + x0, y + y0
            continue
        dx, dy, info = tricg(Aop, Atop, Einv, Finv, rx, ry, rtol * n0 / rn, maxit - total)
        x, y = x + dx, y + dy
        total += info["iters"]
    return x, y, total, cycles


def solve_tricg(K, rhs, rtol=1e-10, maxit=500):
    """TriCG with exact block inverses on the cell system K X = rhs, one load column at a time
    (solve_restarted).  Returns (X with zero field means, iterations per column)."""
    A, Bt, C, iu, ip = piezo_blocks(K)
    B = sp.csr_matrix(Bt.T)
    K = sp.csr_matrix(K)
    Einv, Finv = pinned_inverse(A, 3), pinned_inverse(C, 1)
    nd = K.shape[0]

    def Kop(x, y):
        v = np.zeros(nd)
        v[iu], v[ip] = x, y
        w = K @ v
        return w[iu], w[ip]

    rhs = np.asarray(rhs, dtype=np.float64)
    X = np.zeros_like(rhs)
    its = []
    for col in range(rhs.shape[1]):
        x, y, total, _ = solve_restarted(Kop, lambda v: Bt @ v, lambda u: B @ u, Einv, Finv, rhs[iu, col],
                                         rhs[ip, col], rtol, maxit)
        X[iu, col], X[ip, col] = x, y
        its.append(total)
    return X, its
