"""Pins of the oracle's optimisation step (reinitialisation, Hilbertian extension, projection,
stopping rule) against closed forms, invariants and the algebra the step is defined by."""
import numpy as np
import pytest

import synth
from oracle import optim


def test_scalar_element_matrices_tensor_products():
    """Trilinear Laplace and mass element matrices equal their one-dimensional tensor-product forms
    (1D mass h/6 [[2,1],[1,2]], Laplace 1/h [[1,-1],[-1,1]]), per local corner bits (a, b, c)."""
    h = 0.125
    K, M = optim.scalar_element_matrices(h)
    m1 = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    k1 = 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])
    bits = [(l & 1, (l >> 1) & 1, (l >> 2) & 1) for l in range(8)]
    Mt = np.array([[m1[a, d] * m1[b, e] * m1[c, f] for (d, e, f) in bits] for (a, b, c) in bits])
    Kt = np.array([[k1[a, d] * m1[b, e] * m1[c, f] + m1[a, d] * k1[b, e] * m1[c, f] + m1[a, d] * m1[b, e] * k1[c, f]
                    for (d, e, f) in bits] for (a, b, c) in bits])
    assert np.abs(M - Mt).max() < 1e-15
    assert np.abs(K - Kt).max() < 1e-12


def test_riesz_constant_and_fourier_mode():
    """H 1 = h^3 1, so a constant load gives g = j / h^3; a discrete Fourier mode is an eigenvector of H
    with eigenvalue from the 1D symbols m(t) = h (2 + cos t) / 3, k(t) = 2 (1 - cos t) / h."""
    n = 8
    h = 1.0 / n
    alpha = 3.0 * h
    g = optim.riesz(n, np.full(n ** 3, 2.0), alpha)
    assert np.abs(g - 2.0 / h ** 3).max() < 1e-9 / h ** 3
    idx = np.arange(n)
    kz, ky, kx = np.meshgrid(idx, idx, idx, indexing="ij")
    wave = (1, 2, 3)
    t = [2 * np.pi * w / n for w in wave]
    j = np.cos(t[0] * kx + t[1] * ky + t[2] * kz).ravel()
    m = [h * (2 + np.cos(a)) / 3 for a in t]
    k = [2 * (1 - np.cos(a)) / h for a in t]
    lam = alpha ** 2 * (k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]) + m[0] * m[1] * m[2]
    g = optim.riesz(n, j, alpha)
    assert np.abs(g - j / lam).max() < 1e-9 * np.abs(j / lam).max()


def test_reinit_keeps_a_distance_and_signs():
    """A periodic slab distance |z - 1/2| - w is a fixed point away from its kinks.  A stretched
    distance 3 d is brought to unit slope near the interface, keeps the sign of every node farther
    than h from it, and its zero level moves by less than h/2 (the first-order scheme with a smoothed
    sign lets the interface drift by a fraction of a cell)."""
    n = 16
    h = 1.0 / n
    z = (np.arange(n ** 3) // (n * n)) * h
    d = np.abs(z - 0.5) - 0.2
    r = optim.reinit(n, d, steps=10)
    kink = (np.abs(z - 0.5) < 2.5 * h) | (z < 2.5 * h) | (z > 1 - 3.5 * h)
    assert np.abs(r - d)[~kink].max() < 1e-12
    r3 = optim.reinit(n, 3.0 * d, steps=40)
    far = np.abs(d) > h
    assert np.all(np.sign(r3[far]) == np.sign(d[far]))
    band = (np.abs(d) < 2.5 * h) & ~kink
    slope = (np.roll(r3.reshape(n, n, n), -1, axis=0) - r3.reshape(n, n, n)).ravel() / h
    inner = band & (np.abs(d) > h) & (np.roll(band.reshape(n, n, n), -1, axis=0).ravel())
    assert np.abs(np.abs(slope[inner]) - 1.0).max() < 0.05
    offset = (r3 - d)[band]
    assert np.abs(offset).max() < 0.5 * h


def test_hpm_projection_and_constraint_step():
    """With zero violations the velocity is orthogonal to every constraint sensitivity (j_k . v = 0);
    with a zero objective gradient direction removed, the constraint part removes a fraction gamma of
    each violation to first order: cfl h (j_k . v) = -gamma c_k when no scaling occurs."""
    n = 6
    h = 1.0 / n
    rng = np.random.default_rng(3)
    j0 = rng.standard_normal(n ** 3)
    jc = [rng.standard_normal(n ** 3), rng.standard_normal(n ** 3)]
    v = optim.hpm_velocity(n, j0, jc, [0.0, 0.0])
    for j in jc:
        assert abs(np.dot(j, v)) < 1e-10 * np.linalg.norm(j) * np.linalg.norm(v)
    assert abs(np.abs(v).max() - 1.0) < 1e-12
    # a small violation so that the velocity is not rescaled; take the objective along a constraint
    # direction, so its projected part vanishes up to rounding and is normalised noise: use two loads
    c = np.array([2e-4, -1e-4])
    cfl, gamma = 0.5, 0.5
    v1 = optim.hpm_velocity(n, j0, jc, c, cfl=cfl, gamma=gamma)
    v0 = optim.hpm_velocity(n, j0, jc, [0.0, 0.0], cfl=cfl, gamma=gamma)
    assert np.abs(v1).max() <= 1.0 + 1e-12
    dv = v1 - v0                       # the constraint term alone
    for j, ck in zip(jc, c):
        assert abs(cfl * h * np.dot(j, dv) + gamma * ck) < 1e-9 * abs(ck)


def test_stopping_rule():
    h = 1.0 / 100
    flat = [1.0] * 12
    assert optim.should_stop(flat, [[0.0]] * 12, h)
    assert not optim.should_stop(flat[:9], [[0.0]] * 9, h)
    assert not optim.should_stop(flat, [[0.0]] * 11 + [[2e-3]], h)
    moving = [1.0 + 0.01 * q for q in range(12)]
    assert not optim.should_stop(moving, [[0.0]] * 12, h)


def _crossings(line, h):
    """Zero crossings of a periodic node line, by linear interpolation between the nodes around each."""
    nxt = np.roll(line, -1)
    i = np.where(line * nxt < 0.0)[0]
    return (i + line[i] / (line[i] - nxt[i])) * h


def test_reinit_subcell_keeps_the_zero_crossing():
    """Subcell fix: a profile of slope 3 whose zero lies 0.3 h off the grid keeps its zero crossings
    (within 0.01 h) and reaches unit slope there; the plain scheme moves them by more than 0.1 h."""
    n = 32
    h = 1.0 / n
    x, _, _ = synth.node_coords(n)
    x0 = 0.25 + 0.3 * h
    phi0 = 3.0 * np.sin(2.0 * np.pi * (x - x0)) / (2.0 * np.pi)
    exact = np.array([x0, x0 + 0.5])
    r = optim.reinit(n, phi0, steps=30, subcell=True).reshape(n, n, n)
    line = r[5, 7, :]
    assert np.abs(_crossings(line, h) - exact).max() < 0.01 * h
    k = int(np.floor(x0 / h))
    assert abs((line[k + 1] - line[k]) / h - 1.0) < 1e-6
    plain = optim.reinit(n, phi0, steps=30).reshape(n, n, n)[5, 7, :]
    assert np.abs(_crossings(plain, h) - exact).max() > 0.1 * h


def test_reinit_subcell_sphere_distance():
    """Subcell fix on a stretched sphere distance 3 (|x - c| - R): the nodes within h of the sphere
    come within 0.1 h of the distance and those within 3 h within 0.25 h (the plain scheme misses the
    first by more than half a cell)."""
    n = 32
    h = 1.0 / n
    x, y, z = synth.node_coords(n)
    dist = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) - 0.3
    r = optim.reinit(n, 3.0 * dist, steps=40, subcell=True)
    band1, band3 = np.abs(dist) < 1.01 * h, np.abs(dist) < 3.0 * h
    assert np.abs(r - dist)[band1].max() < 0.1 * h
    assert np.abs(r - dist)[band3].max() < 0.25 * h
    plain = optim.reinit(n, 3.0 * dist, steps=40)
    assert np.abs(plain - dist)[band1].max() > 0.5 * h


def test_reinit_subcell_keeps_a_thin_member():
    """A square bar three elements thick, already a distance (in the max norm), keeps its volume within
    20% over five reinitialisations with the subcell fix; the plain scheme erodes it to nothing."""
    n = 32
    h = 1.0 / n
    x, y, _ = synth.node_coords(n)
    bar = np.maximum(np.abs(x - 0.5), np.abs(y - 0.5)) - 1.5 * h
    v0 = optim.volume(n, bar)
    a, b = bar.copy(), bar.copy()
    for _ in range(5):
        a = optim.reinit(n, a, steps=20, subcell=True)
        b = optim.reinit(n, b, steps=20)
    assert abs(optim.volume(n, a) / v0 - 1.0) < 0.2
    assert optim.volume(n, b) < 0.05 * v0


def test_objective_weight_scales_only_the_objective_part():
    """With the objective weight w the velocity is w times the objective part plus the unchanged
    constraint part (while no rescaling to max|v| = 1 occurs)."""
    n = 6
    rng = np.random.default_rng(8)
    j0 = rng.standard_normal(n ** 3)
    jc = [rng.standard_normal(n ** 3)]
    c = [1e-4]
    v1 = optim.hpm_velocity(n, j0, jc, c)
    vw = optim.hpm_velocity(n, j0, jc, c, obj_weight=0.25)
    v0 = optim.hpm_velocity(n, j0, jc, [0.0])
    assert np.abs(v1).max() <= 1.0 + 1e-12
    assert np.abs((vw - (v1 - v0)) - 0.25 * v0).max() < 1e-12
