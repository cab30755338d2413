"""Pins of the oracle's quadrature-point material interpolation (smoothing at every Gauss point of the
level set's trilinear interpolation instead of once per element)."""
import numpy as np

import synth
from oracle import cell, fe

MAT = synth.material_workload()
M = fe.nondim_matrix(MAT)


def test_equal_point_scales_reproduce_the_element_assembly():
    """Scales equal at the eight points of every element give the element form's K, F and tensors
    (the per-point matrices sum to the element's)."""
    n = 4
    s = fe.ersatz_scale(synth.random_density(n, seed=3), MAT.void_scale)
    K1, F1 = cell.assemble(n, s, M)
    K8, F8 = cell.assemble(n, np.repeat(s[:, None], 8, axis=1), M)
    assert abs(K1 - K8).max() < 1e-13 * abs(K1).max()
    assert np.abs(F1 - F8).max() < 1e-13 * np.abs(F1).max()
    X = cell.solve_pinned(K1, F1)
    a, b = cell.effective_flux(n, s, M, X), cell.effective_flux(n, np.repeat(s[:, None], 8, axis=1), M, X)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_interpolation_is_exact_for_trilinear_fields():
    """The level set at the Gauss points equals a trilinear field evaluated there (elements away from
    the periodic seam), and its Gauss-point mean is the element's nodal mean."""
    n = 6
    h = 1.0 / n
    x, y, z = synth.node_coords(n)
    field = lambda x, y, z: (0.3 + 2.0 * x) * (1.0 - 0.5 * y) * (0.2 + z) - 0.4
    phiq = fe.levelset_at_gauss(n, field(x, y, z))
    pts, _ = fe.gauss_rule(2)
    e = np.arange(n ** 3)
    i, j, k = e % n, (e // n) % n, e // (n * n)
    inner = (i < n - 1) & (j < n - 1) & (k < n - 1)
    for q, (a, b, c) in enumerate(pts):
        exact = field((i + a) * h, (j + b) * h, (k + c) * h)
        assert np.abs(phiq[inner, q] - exact[inner]).max() < 1e-14
    phi = synth.grf_levelset(n, seed=4, solid_fraction=0.5)
    assert np.abs(fe.levelset_at_gauss(n, phi).mean(axis=1) - fe.element_mean(n, phi)).max() < 1e-14


def test_laminate_equals_the_element_form_with_mean_point_scales():
    """For a level set of z alone the fluctuations depend on z alone, their strains are constant in each
    element, and the point-interpolated cell equals the element form whose scales are the elements'
    mean point scales (which the laminate pins tie to the closed form)."""
    n = 8
    _, _, z = synth.node_coords(n)
    phi = 0.18 * np.cos(2 * np.pi * z) + 0.03
    rq = fe.density_qp(n, phi)
    assert np.ptp(rq, axis=1).max() > 0.05           # the points of an element do differ
    qp = cell.homogenise(n, MAT, phi=phi, smoothing="qp", want_x=False)
    el = cell.homogenise(n, MAT, rho=rq.mean(axis=1), want_x=False)
    assert np.abs(qp.MH - el.MH).max() < 1e-10 * np.abs(el.MH).max()
    assert np.abs(qp.MH - qp.MH_energy).max() < 1e-10 * np.abs(qp.MH).max()


def test_point_smoothing_differs_from_element_smoothing_near_an_interface():
    """On a sphere the two smoothings give different cells (differing by O(h) near the interface), and a
    uniform solid level set gives the base material in both."""
    n = 8
    qp = cell.homogenise(n, MAT, phi=synth.sphere_levelset(n), smoothing="qp", want_x=False)
    el = cell.homogenise(n, MAT, phi=synth.sphere_levelset(n), want_x=False)
    d = np.abs(qp.MH - el.MH).max() / np.abs(el.MH).max()
    assert 1e-4 < d < 0.2
    solid = cell.homogenise(4, MAT, phi=np.full(64, -1.0), smoothing="qp", want_x=False)
    assert np.abs(solid.MH - M).max() < 1e-12 * np.abs(M).max()


def test_point_sensitivities_euler_identity():
    """At the discrete solution sum_e sum_p s_ep G_ep equals the flux-form tensor (Galerkin
    orthogonality), the point form of the element identity."""
    n = 4
    phi = synth.grf_levelset(n, seed=6, solid_fraction=0.5)
    r = cell.homogenise(n, MAT, phi=phi, smoothing="qp")
    G = cell.element_energy_matrices_qp(n, r.X, M)
    total = np.einsum("eq,eqkl->kl", r.s, G)
    assert np.abs(total - r.MH).max() < 1e-10 * np.abs(r.MH).max()


def test_point_sensitivities_match_finite_differences():
    """dJ/dphi by the point chain rule against central differences of the point-smoothed cell, for
    J = <W, M^H> with a fixed random W, at nodes spread over the cell."""
    n = 4
    phi = synth.grf_levelset(n, seed=6, solid_fraction=0.5) * 0.6
    W = np.random.default_rng(2).standard_normal((9, 9))
    J = lambda f: float(np.sum(W * cell.homogenise(n, MAT, phi=f, smoothing="qp", want_x=False).MH))
    r = cell.homogenise(n, MAT, phi=phi, smoothing="qp")
    g = cell.grad_phi_from_rho_qp(n, phi, cell.grad_rho_qp(n, MAT, r.X, W))
    assert np.abs(g).max() > 0
    d = 1e-6
    for node in (0, 5, 21, 42, 63):
        e = np.zeros(n ** 3)
        e[node] = d
        fd = (J(phi + e) - J(phi - e)) / (2 * d)
        assert abs(fd - g[node]) <= 1e-5 * np.abs(g).max(), (node, fd, g[node])


def test_point_chain_rule_of_the_volume():
    """The volume (mean point density) differentiated by the point chain rule with dVol/drho_ep =
    1 / (8 N^3) equals its central differences."""
    n = 4
    phi = synth.grf_levelset(n, seed=7, solid_fraction=0.5) * 0.6
    vol = lambda f: float(np.mean(fe.density_qp(n, f)))
    g = cell.grad_phi_from_rho_qp(n, phi, np.full((n ** 3, 8), 1.0 / (8 * n ** 3)))
    d = 1e-6
    for node in (1, 17, 40):
        e = np.zeros(n ** 3)
        e[node] = d
        fd = (vol(phi + e) - vol(phi - e)) / (2 * d)
        assert abs(fd - g[node]) <= 1e-7 * np.abs(g).max() + 1e-12
