"""The level-set optimisation loop around the homogenisation (Sec. 2.1, Sec. 2.3, Sec. 2.6): reinitialisation
to a signed distance, the extension of the discrete sensitivities into a velocity by a Hilbert-space
projection onto the constraints' null space, and the stopping rule.

TEST INFRASTRUCTURE: the oracle of the GPU path, used only by the tests.

The paper states the problem (maximise a figure of merit under equality constraints on the volume and
on a second effective property), reinitialisation every five iterations by a standard first-order
scheme, and its stopping rule; it defers the velocity construction to the projection method of its
library.  Readings, all shared with the GPU path:

* reinitialisation: pseudo-time steps of phi_t + S(phi0) (|grad phi| - 1) = 0 with the smoothed sign
  S = phi0 / sqrt(phi0^2 + h^2), the same first-order Godunov upwinding as the HJ step, dtau = cfl h;
  or, with the subcell fix of Russo and Smereka (J. Comput. Phys. 163, 2000), still first order: the
  exact sign elsewhere, and nodes with a sign change of phi0 towards one of their six neighbours (or
  phi0 = 0) relax towards D = phi0 / |grad phi0| instead, phi <- phi - (dtau / h)(sign(phi0)|phi| - D),
  with |grad phi0| from, per direction, the largest of the central and the two one-sided differences.
  The zero level set then stays where phi0 puts it; the plain scheme moves it by a fraction of h per
  reinitialisation, which erodes features a few elements thick;
* sensitivities: j = -dJ/dphi, the exact derivative of the discrete functional with respect to the
  nodal level set (positive where lowering phi, i.e. growing solid, increases J); the HJ step lowers
  phi by cfl h v |grad phi|, so to first order J changes by cfl h (j . v) for |grad phi| = 1;
* Hilbertian extension: g = H^-1 j with H = alpha^2 K + M, the trilinear finite-element Laplace and
  mass matrices on the periodic grid (alpha = 4h by default), so that <g, w>_H = g^T H w = j . w;
* projection: with g_0 from the objective and g_i from the constraints (i = 1..m), G_ik = j_i . g_k,
  theta_J = g_0 - sum_i g_i (G^-1 b)_i, b_k = j_k . g_0 (the objective direction with the constraint
  directions removed), and theta_C = -sum_i g_i (G^-1 c)_i for the relative violations c_i (to first
  order it removes them: <g_k, theta_C>_H = -c_k);
* velocity: v = w theta_J / max|theta_J| + (gamma / (cfl h)) theta_C, scaled down to max|v| = 1 when
  larger (w = 1 unless a step control lowers it) (the objective part moves the boundary by cfl h per step, the constraint part removes a
  fraction gamma of each violation per step to first order);
* stopping: at iteration q >= 10, |J_q - J_{q-j}| / |J_q| < 0.2 h for j = 1..5 and every relative
  violation below 1e-3 (h, the element side, is the paper's epsilon_m).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe
from .cell import element_nodes


def reinit(n, phi, steps=20, cfl=0.5, subcell=False):
    """`steps` first-order pseudo-time steps of the reinitialisation equation (plain, or with the
    subcell fix at the interface nodes)."""
    h = 1.0 / n
    dt = cfl * h
    f0 = np.asarray(phi, dtype=np.float64).reshape(n, n, n)
    if subcell:
        S = np.sign(f0)
        iface = f0 == 0.0
        grad2 = np.zeros_like(f0)
        for ax in (2, 1, 0):
            lo, hi = np.roll(f0, 1, axis=ax), np.roll(f0, -1, axis=ax)
            iface |= (f0 * lo < 0.0) | (f0 * hi < 0.0)
            d = np.maximum(np.abs(hi - lo) / 2.0, np.maximum(np.abs(hi - f0), np.abs(f0 - lo)))
            grad2 += d * d
        D = np.where(grad2 > 0.0, h * f0 / np.sqrt(np.where(grad2 > 0.0, grad2, 1.0)), 0.0)
    else:
        S = f0 / np.sqrt(f0 * f0 + h * h)
    f = f0.copy()
    for _ in range(steps):
        gp2 = np.zeros_like(f)
        gm2 = np.zeros_like(f)
        for ax in (2, 1, 0):
            dm = (f - np.roll(f, 1, axis=ax)) / h
            dp = (np.roll(f, -1, axis=ax) - f) / h
            gp2 += np.maximum(dm, 0.0) ** 2 + np.minimum(dp, 0.0) ** 2
            gm2 += np.minimum(dm, 0.0) ** 2 + np.maximum(dp, 0.0) ** 2
        upd = f - dt * (np.maximum(S, 0.0) * np.sqrt(gp2) + np.minimum(S, 0.0) * np.sqrt(gm2) - S)
        if subcell:
            upd = np.where(iface, f - (dt / h) * (S * np.abs(f) - D), upd)
        f = upd
    return f.ravel()


def scalar_element_matrices(h, npts=2):
    """Trilinear element Laplace K (grad . grad) and mass M, 8 x 8 (2-point Gauss is exact)."""
    pts, wts = fe.gauss_rule(npts)
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    for p, w in zip(pts, wts):
        G = fe.shape_grads(p) / h
        N = np.array([np.prod([p[d] if fe.LOCAL[l, d] else 1.0 - p[d] for d in range(3)]) for l in range(8)])
        K += w * h ** 3 * G @ G.T
        M += w * h ** 3 * np.outer(N, N)
    return K, M


def helmholtz_matrix(n, alpha):
    """H = alpha^2 K + M on the periodic node grid (CSR, n^3 square)."""
    Ke, Me = scalar_element_matrices(1.0 / n)
    He = alpha * alpha * Ke + Me
    en = element_nodes(n)
    rows = np.repeat(en, 8, axis=1).ravel()
    cols = np.tile(en, (1, 8)).ravel()
    vals = np.tile(He.ravel(), n ** 3)
    H = sp.coo_matrix((vals, (rows, cols)), shape=(n ** 3, n ** 3)).tocsr()
    H.sum_duplicates()
    return H


def riesz(n, j, alpha):
    """g = H^-1 j (H is symmetric positive definite: the mass part removes the constants)."""
    return spla.spsolve(helmholtz_matrix(n, alpha).tocsc(), np.asarray(j, dtype=np.float64))


def hpm_velocity(n, j_obj, j_cons, viol, alpha=None, cfl=0.5, gamma=0.5, obj_weight=1.0):
    """Velocity of one optimisation step (readings in the module docstring)."""
    h = 1.0 / n
    alpha = 4.0 * h if alpha is None else alpha
    g0 = riesz(n, j_obj, alpha)
    gs = [riesz(n, j, alpha) for j in j_cons]
    m = len(gs)
    if m:
        G = np.array([[np.dot(j_cons[i], gs[k]) for k in range(m)] for i in range(m)])
        b = np.array([np.dot(j_cons[k], g0) for k in range(m)])
        lam_b = np.linalg.solve(G, b)
        lam_c = np.linalg.solve(G, np.asarray(viol, dtype=np.float64))
        thJ = g0 - sum(lam_b[i] * gs[i] for i in range(m))
        thC = -sum(lam_c[i] * gs[i] for i in range(m))
    else:
        thJ, thC = g0, np.zeros_like(g0)
    v = obj_weight * thJ / np.max(np.abs(thJ)) + (gamma / (cfl * h)) * thC
    vm = np.max(np.abs(v))
    return v / vm if vm > 1.0 else v


def volume(n, phi, width_elems=2.0):
    """Vol(Omega) = the cell mean of the smoothed density."""
    return float(np.mean(fe.density_from_levelset(n, phi, width_elems)))


def should_stop(J_hist, viol_hist, h):
    """The paper's stopping rule (Sec. 2.6) on the objective and relative-violation histories."""
    q = len(J_hist) - 1
    if q < 10:
        return False
    Jq = J_hist[q]
    if any(abs(Jq - J_hist[q - j]) >= 0.2 * h * abs(Jq) for j in range(1, 6)):
        return False
    return all(abs(c) < 1e-3 for c in viol_hist[q])
