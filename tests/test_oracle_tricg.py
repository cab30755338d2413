"""Pins of the oracle's TriCG: its short recurrences against the Galerkin projection they stand for,
the tridiagonalisation's orthogonality, the residual it reports, and the direct solve."""
import numpy as np

import synth
from oracle import cell, fe, tricg


def random_sqd(n=12, m=7, seed=5):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    H = rng.standard_normal((m, m))
    E = G @ G.T + n * np.eye(n)
    F = H @ H.T + m * np.eye(m)
    A = rng.standard_normal((n, m))
    return E, F, A, rng.standard_normal(n), rng.standard_normal(m)


def run(E, F, A, b, c, **kw):
    return tricg.tricg(lambda v: A @ v, lambda u: A.T @ u, lambda r: np.linalg.solve(E, r),
                       lambda r: np.linalg.solve(F, r), b, c, **kw)


def test_short_recurrences_equal_the_galerkin_solution():
    """Every iterate equals the dense solve of the Galerkin system [[I, T], [T^T, -I]] built from the
    stored bases and coefficients (a dropped or mis-signed term in the LDL^T updates fails this)."""
    E, F, A, b, c = random_sqd()
    x, y, info = run(E, F, A, b, c, rtol=1e-30, maxit=10, record=True)
    for k in range(1, info["iters"] + 1):
        xg, yg = tricg.galerkin_iterate(info["U"], info["V"], info["alpha"], info["beta"], info["gamma"], k)
        xk, yk = info["iterates"][k - 1]
        scale = np.abs(np.concatenate([xg, yg])).max()
        assert np.abs(np.concatenate([xk - xg, yk - yg])).max() < 1e-11 * scale, k


def test_tridiagonalisation_is_orthonormal_and_projects():
    """U^T E U = I, V^T F V = I and U^T A V = T for the first six steps."""
    E, F, A, b, c = random_sqd()
    _, _, info = run(E, F, A, b, c, rtol=1e-30, maxit=6, record=True)
    k = 6
    U, V = np.array(info["U"][:k]).T, np.array(info["V"][:k]).T
    T = np.diag(info["alpha"][:k])
    for i in range(1, k):
        T[i, i - 1], T[i - 1, i] = info["beta"][i], info["gamma"][i]
    assert np.abs(U.T @ E @ U - np.eye(k)).max() < 1e-12
    assert np.abs(V.T @ F @ V - np.eye(k)).max() < 1e-12
    assert np.abs(U.T @ A @ V - T).max() < 1e-11 * np.abs(T).max()


def test_reported_residual_is_the_true_residual_and_it_converges():
    """The residual norm from the recurrence equals ||(b, c) - K (x, y)|| at every step of a cycle; a
    cycle ends at the breakdown once the smaller space (dimension m = 7) is exhausted, and the
    restarted solve reaches the direct solution."""
    E, F, A, b, c = random_sqd()
    K = np.block([[E, A], [A.T, -F]])
    rhs = np.concatenate([b, c])
    x, y, info = run(E, F, A, b, c, rtol=1e-13, maxit=40, record=True)
    for k, (xk, yk) in enumerate(info["iterates"]):
        true = np.linalg.norm(rhs - K @ np.concatenate([xk, yk])) / np.linalg.norm(rhs)
        assert abs(info["est"][k] - true) <= 1e-9 * max(true, 1e-3), (k, info["est"][k], true)
    assert info["breakdown"] and info["iters"] <= 8
    x, y, total, cycles = tricg.solve_restarted(
        lambda x, y: (E @ x + A @ y, A.T @ x - F @ y), lambda v: A @ v, lambda u: A.T @ u,
        lambda r: np.linalg.solve(E, r), lambda r: np.linalg.solve(F, r), b, c, rtol=1e-13)
    ref = np.linalg.solve(K, rhs)
    assert np.abs(np.concatenate([x, y]) - ref).max() < 1e-11 * np.abs(ref).max()
    print("iterations", total, "cycles", cycles)


def test_zero_block_starts():
    """A right-hand side with a zero block is solved through the shifted start (both orientations), and
    an uncoupled system's zero block makes the start itself the solution."""
    E, F, A, b, c = random_sqd()
    K = np.block([[E, A], [A.T, -F]])
    ops = (lambda v: A @ v, lambda u: A.T @ u, lambda r: np.linalg.solve(E, r), lambda r: np.linalg.solve(F, r))
    for bb, cc in ((b, np.zeros_like(c)), (np.zeros_like(b), c)):
        x, y, total, cycles = tricg.solve_restarted(lambda x, y: (E @ x + A @ y, A.T @ x - F @ y), *ops, bb, cc,
                                                    rtol=1e-13)
        ref = np.linalg.solve(K, np.concatenate([bb, cc]))
        assert np.abs(np.concatenate([x, y]) - ref).max() < 1e-11 * np.abs(ref).max()
    Z = np.zeros_like(A)
    x, y, done = tricg.start(b, np.zeros_like(c), lambda v: Z @ v, lambda u: Z.T @ u, ops[2], ops[3])
    assert done and np.abs(E @ x - b).max() < 1e-12 * np.abs(b).max() and not np.any(y)
    x, y, done = tricg.start(np.zeros_like(b), c, lambda v: Z @ v, lambda u: Z.T @ u, ops[2], ops[3])
    assert done and np.abs(-F @ y - c).max() < 1e-12 * np.abs(c).max() and not np.any(x)


def test_piezo_cell_matches_the_direct_solve():
    """On an 4^3 random-density cell with the workload material, TriCG with exact block inverses (A and
    C pinned at one node, field means removed) gives the direct solve's solution up to the per-field
    constants, and therefore its tensors."""
    n = 4
    mat = synth.material_workload()
    M = fe.nondim_matrix(mat)
    rho = synth.random_density(n, seed=9, low=0.2, high=1.0)
    s = fe.ersatz_scale(rho, mat.void_scale)
    K, F = cell.assemble(n, s, M)
    X, its = tricg.solve_tricg(K, -F, rtol=1e-12)
    Xd = cell.solve_pinned(K, F)
    Xd = Xd.reshape(n ** 3, 4, 9)
    Xd = (Xd - Xd.mean(axis=0)).reshape(4 * n ** 3, 9)
    assert np.abs(X - Xd).max() < 1e-9 * np.abs(Xd).max()
    MH = cell.effective_flux(n, s, M, X)
    MHd = cell.effective_flux(n, s, M, Xd)
    assert np.abs(MH - MHd).max() < 1e-10 * np.abs(MHd).max()
    print("iterations per load", its)


def test_stored_tricg_cases_match_the_direct_goldens():
    """The stored TriCG runs (tests/golden/tricg16.json, written by make_golden.py) reach the direct
    solves' tensors on both 16^3 cells, within at most 25 iterations per load."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    tc = json.load(open(os.path.join(here, "tricg16.json")))
    for name in ("grf16", "sphere16"):
        ref = np.array(json.load(open(os.path.join(here, f"{name}.json")))["MH"])
        MH = np.array(tc[name]["MH"])
        assert np.abs(MH - ref).max() < 1e-9 * np.abs(ref).max(), name
        assert max(tc[name]["iterations"]) <= 25
