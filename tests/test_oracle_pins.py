"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: special
cases with exact answers, the closed-form laminate, brute force on tiny
grids, invariances of the geometry, values printed in the paper, finite
differences.  No GPU involved.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import cell, fe, foms, hj, krylov, laminate

HERE = os.path.dirname(os.path.abspath(__file__))
MAT = synth.material_workload()
MND = fe.nondim_matrix(MAT)


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


# ------------------------------------------------------------------ element
def affine_fields(h):
    """Nodal values (32 x 9) of the affine fields whose generalised strain is e_L."""
    X = np.zeros((32, 9))
    for l, (a, b, c) in enumerate(fe.LOCAL):
        x, y, z = a * h, b * h, c * h
        d = 4 * l
        X[d + 0, 0] = x            # eps_xx = 1
        X[d + 1, 1] = y            # eps_yy = 1
        X[d + 2, 2] = z            # eps_zz = 1
        X[d + 1, 3] = z            # gamma_yz = 1 via u_y = z
        X[d + 0, 4] = z            # gamma_xz = 1 via u_x = z
        X[d + 0, 5] = y            # gamma_xy = 1 via u_x = y
        X[d + 3, 6] = -x           # E_x = 1 via phi = -x
        X[d + 3, 7] = -y
        X[d + 3, 8] = -z
    return X


def test_element_quadrature_exact():
    """2x2x2 Gauss integrates the trilinear-element integrands exactly."""
    for h in (1.0, 0.25):
        K2, F2 = fe.element_matrices(MND, h, 2)
        K3, F3 = fe.element_matrices(MND, h, 3)
        assert rel(K2, K3) < 1e-14 and rel(F2, F3) < 1e-14


def test_element_kernel_is_rigid_and_constant_potential():
    """K0 is symmetric with exactly 7 null vectors: 6 rigid modes + constant phi."""
    K, _ = fe.element_matrices(MND, 0.25)
    assert rel(K, K.T) < 1e-15
    sv = np.linalg.svd(K, compute_uv=False)
    assert np.all(sv[:25] / sv[0] > 1e-4)
    assert np.all(sv[25:] / sv[0] < 1e-13)
    # explicit rigid modes and constant potential are annihilated
    modes = []
    for f in range(4):
        v = np.zeros(32)
        v[f::4] = 1.0
        modes.append(v)
    for (p, q) in ((0, 1), (1, 2), (0, 2)):  # infinitesimal rotations
        v = np.zeros(32)
        for l, xyz in enumerate(fe.LOCAL):
            v[4 * l + p] = -xyz[q]
            v[4 * l + q] = xyz[p]
        modes.append(v)
    for v in modes:
        assert np.abs(K @ v).max() < 1e-13 * np.abs(K).max()


def test_element_load_matrix_is_stiffness_on_affine_fields():
    """F0 = K0 Xbar: the load of a unit macroscopic field equals K0 times its
    affine nodal interpolant (trilinear elements reproduce affine fields)."""
    h = 0.125
    K, F = fe.element_matrices(MND, h)
    X = affine_fields(h)
    assert rel(K @ X, F) < 1e-13
    # and the element energy of those fields is V * M
    assert rel(X.T @ K @ X, h ** 3 * MND) < 1e-13


def test_vectorised_assembly_matches_loop_assembly():
    rng = np.random.default_rng(3)
    for n in (2, 3):
        s = rng.uniform(0.01, 1.0, n ** 3)
        K, F = cell.assemble(n, s, MND)
        Kl, Fl = cell.assemble_loops(n, s, MND)
        assert rel(K.toarray(), Kl) < 1e-15
        assert rel(F, Fl) < 1e-15
        assert np.abs(cell.rhs_compatibility(n, F)).max() < 1e-14


# ------------------------------------------------------------ special cases
def test_solid_cell_returns_base_tensors():
    """P1: uniform solid cell -> no fluctuation, effective = base tensors."""
    n = 4
    r = cell.homogenise(n, MAT, rho=np.ones(n ** 3))
    assert np.abs(r.F).max() < 1e-13
    assert np.abs(r.X).max() < 1e-12
    assert rel(r.C, MAT.C) < 1e-13
    assert rel(r.e, MAT.e) < 1e-13
    assert rel(r.kappa, MAT.kappa) < 1e-13


def test_void_cell_scales_by_void_factor():
    """P2: uniform void cell -> eps_v times the base tensors."""
    n = 4
    r = cell.homogenise(n, MAT, rho=np.zeros(n ** 3))
    ev = MAT.void_scale
    assert rel(r.C, ev * MAT.C) < 1e-13
    assert rel(r.e, ev * MAT.e) < 1e-13
    assert rel(r.kappa, ev * MAT.kappa) < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_closed_form(axis):
    """P3: a layered cell reproduces the textbook laminate formula exactly."""
    n = 6
    rho = synth.laminate_density(n, axis=axis, seed=5 + axis)
    r = cell.homogenise(n, MAT, rho=rho)
    s = fe.ersatz_scale(rho, MAT.void_scale).reshape(n, n, n)
    layers = {0: s[0, 0, :], 1: s[0, :, 0], 2: s[:, 0, 0]}[axis]
    ref = laminate.laminate_effective(MND, layers, axis)
    assert rel(r.MH, ref) < 1e-12


# --------------------------------------------------------------- invariants
def test_symmetry_definiteness_and_energy_form():
    """P4: M^H symmetric, C^H and kappa^H positive definite, flux = energy."""
    n = 8
    r = cell.homogenise(n, MAT, phi=synth.grf_levelset(n, seed=21))
    assert rel(r.MH, r.MH.T) < 1e-12
    assert rel(r.MH, r.MH_energy) < 1e-12
    assert np.all(np.linalg.eigvalsh(0.5 * (r.C + r.C.T)) > 0)
    assert np.all(np.linalg.eigvalsh(0.5 * (r.kappa + r.kappa.T)) > 0)
    # stress under field loads is -e^T (the sigma-under-E block)
    assert rel(-r.MH[:6, 6:].T, r.e / fe.E0) < 1e-12


def _phi_grid(phi, n):
    return phi.reshape(n, n, n)   # [k][j][i]


def test_translation_mirror_and_swap_invariance():
    """P5: rolling by whole elements changes nothing; an x-mirror and an
    x<->y swap transform the tensors exactly (transversely isotropic base)."""
    n = 8
    phi = synth.grf_levelset(n, seed=33)
    base = cell.homogenise(n, MAT, phi=phi, want_x=False).MH
    g = _phi_grid(phi, n)
    rolled = np.roll(g, shift=(2, 3, 5), axis=(0, 1, 2)).ravel()
    assert rel(cell.homogenise(n, MAT, phi=rolled, want_x=False).MH, base) < 1e-11
    # x mirror: node i -> (n - i) % n
    idx = (-np.arange(n)) % n
    mir = g[:, :, idx].ravel()
    D = np.diag([1, 1, 1, 1, -1, -1, -1, 1, 1.0])
    assert rel(cell.homogenise(n, MAT, phi=mir, want_x=False).MH, D @ base @ D) < 1e-11
    # x <-> y swap
    sw = np.transpose(g, (0, 2, 1)).ravel()
    perm = [1, 0, 2, 4, 3, 5, 7, 6, 8]
    P = np.eye(9)[perm]
    assert rel(cell.homogenise(n, MAT, phi=sw, want_x=False).MH, P @ base @ P.T) < 1e-11


def test_sphere_cell_symmetries():
    n = 8
    r = cell.homogenise(n, MAT, phi=synth.sphere_levelset(n), want_x=False)
    C, e, k = r.C, r.e, r.kappa
    tol = 1e-11
    assert abs(C[0, 0] - C[1, 1]) < tol * C[0, 0]
    assert abs(C[0, 2] - C[1, 2]) < tol * C[0, 0]
    assert abs(C[3, 3] - C[4, 4]) < tol * C[0, 0]
    assert abs(e[2, 0] - e[2, 1]) < tol * abs(e).max()
    assert abs(e[0, 4] - e[1, 3]) < tol * abs(e).max()
    assert abs(k[0, 0] - k[1, 1]) < tol * k[0, 0]
    mask = np.ones((6, 6), bool)
    mask[:3, :3] = False
    mask[3, 3] = mask[4, 4] = mask[5, 5] = False
    assert np.abs(C[mask]).max() < tol * C[0, 0]


# -------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [2, 3, 4])
def test_brute_force_dense_solves(n):
    """P6: dense pinned solve and dense minimum-norm least squares of the
    loop-assembled system give the sparse oracle's tensors."""
    rng = np.random.default_rng(100 + n)
    rho = rng.uniform(0, 1, n ** 3)
    r = cell.homogenise(n, MAT, rho=rho)
    s = r.s
    Kl, Fl = cell.assemble_loops(n, s, MND)
    Xd = cell.solve_dense_pinned(Kl, Fl)
    Xm = cell.solve_dense_minnorm(Kl, Fl)
    for X in (Xd, Xm):
        MH = cell.effective_flux(n, s, MND, X)
        assert rel(MH, r.MH) < 1e-11


def test_units_invariance():
    """P8: solving in SI units and rescaling equals the non-dimensional solve."""
    n = 3
    rng = np.random.default_rng(8)
    rho = rng.uniform(0, 1, n ** 3)
    r = cell.homogenise(n, MAT, rho=rho)
    Msi = fe.material_matrix(MAT.C, MAT.e, MAT.kappa)
    s = fe.ersatz_scale(rho, MAT.void_scale)
    Kl, Fl = cell.assemble_loops(n, s, Msi)
    # SI system is badly scaled (1e11 vs 1e-9); solve it after symmetric
    # diagonal equilibration, which changes nothing in exact arithmetic
    d = 1.0 / np.sqrt(np.abs(np.diag(Kl)))
    Ks = d[:, None] * Kl * d[None, :]
    Y = cell.solve_dense_pinned(Ks, d[:, None] * Fl)
    X = d[:, None] * Y
    MHsi = cell.effective_flux(n, s, Msi, X)
    assert rel(MHsi[:6, :6], r.C) < 1e-10
    assert rel(-MHsi[6:, :6], r.e) < 1e-10
    assert rel(-MHsi[6:, 6:], r.kappa) < 1e-10


# ---------------------------------------------------------------- FOMs
def test_base_material_dh_matches_paper():
    """P9: the paper prints d_h = 31.7 pC/N for its PZT-5A constants."""
    pv = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
    m = synth.material_pzt5a()
    f = foms.foms(m.C, m.e, m.kappa)
    # printed to three digits (31.76 shows as 31.7, i.e. truncated)
    assert 0.0 <= f["d_h"] * 1e12 - pv["base_material_dh_pC_per_N"]["value"] < 0.1
    assert f["B_reuss"] <= f["B_voigt"]
    # a solid cell homogenises to the same numbers
    r = cell.homogenise(2, m, rho=np.ones(8), want_x=False)
    f2 = foms.foms(r.C, r.e, r.kappa)
    assert abs(f2["d_h"] - f["d_h"]) < 1e-12 * abs(f["d_h"])


def test_table3_kh_identity():
    """P9: Table 3's printed (d_h, g_h, B_Reuss) give its printed k_h under
    the reading k_h = sqrt(d_h g_h B_Reuss)."""
    pv = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
    for row in pv["table3_rows"]["rows"]:
        kh = np.sqrt(row["d_h"] * row["g_h"] * row["B_reuss"])
        assert abs(kh - row["k_h"]) < 1.5e-3


@pytest.mark.parametrize("name", foms.NAMES)
def test_fom_gradients_complex_step_vs_central_fd(name):
    m = synth.material_workload()
    r = cell.homogenise(6, m, phi=synth.grf_levelset(6, seed=2), want_x=False)
    gC, ge, gk = foms.fom_grads(r.C, r.e, r.kappa, name)
    f0 = foms.foms(r.C, r.e, r.kappa)[name]
    for arr, g, idx in ((r.C, gC, (2, 2)), (r.C, gC, (0, 1)), (r.e, ge, (2, 2)),
                        (r.e, ge, (0, 4)), (r.kappa, gk, (2, 2))):
        h = 1e-6 * abs(arr[idx]) if arr[idx] != 0 else 1e-6
        a = arr.copy(); a[idx] += h
        b = arr.copy(); b[idx] -= h
        args_p = [r.C, r.e, r.kappa]
        args_m = [r.C, r.e, r.kappa]
        which = 0 if arr is r.C else (1 if arr is r.e else 2)
        args_p[which] = a
        args_m[which] = b
        fd = (foms.foms(*args_p)[name] - foms.foms(*args_m)[name]) / (2 * h)
        scale = max(abs(g[idx]), abs(f0) / max(abs(arr).max(), 1e-300))
        assert abs(fd - g[idx]) <= 1e-6 * scale


# ---------------------------------------------------------------- gradient
def test_euler_identity_and_fd_gradient():
    """P10: sum_e s_e G_e = M^H (degree-1 homogeneity) and dM^H/drho_e
    matches central finite differences of the full solve."""
    n = 4
    rng = np.random.default_rng(12)
    rho = rng.uniform(0.05, 0.95, n ** 3)
    r = cell.homogenise(n, MAT, rho=rho)
    G = cell.element_energy_matrices(n, r.X, MND)
    assert rel(np.einsum("e,ekl->kl", r.s, G), r.MH) < 1e-12
    W = rng.standard_normal((9, 9))
    g = cell.grad_rho(n, MAT, r.X, W)
    for e in (0, 17, 63):
        h = 1e-6
        rp = rho.copy(); rp[e] += h
        rm = rho.copy(); rm[e] -= h
        Mp = cell.homogenise(n, MAT, rho=rp, want_x=False).MH
        Mm = cell.homogenise(n, MAT, rho=rm, want_x=False).MH
        fd = np.sum(W * (Mp - Mm)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-5 * max(abs(g).max(), 1e-30)


def test_laminate_gradient_closed_form():
    """P10: per-element sensitivity of a laminate equals 1/n^2 of the layer
    derivative of the closed-form laminate tensor."""
    n, axis = 4, 2
    rho = synth.laminate_density(n, axis=axis, seed=9)
    rho = 0.1 + 0.8 * rho
    r = cell.homogenise(n, MAT, rho=rho)
    W = np.random.default_rng(4).standard_normal((9, 9))
    g = cell.grad_rho(n, MAT, r.X, W)
    s = fe.ersatz_scale(rho, MAT.void_scale).reshape(n, n, n)
    layers = s[:, 0, 0]
    ref = laminate.laminate_effective_grad(MND, layers, axis, n, W) * (1 - MAT.void_scale)
    got = g.reshape(n, n, n)
    for k in range(n):
        assert np.allclose(got[k], ref[k], rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_homogeneity_of_foms():
    """P10: scaling every s by t scales M^H by t: d_h and k_h are invariant
    (degree 0) and g_h scales like 1/t (degree -1)."""
    n = 4
    rho = np.random.default_rng(5).uniform(0, 1, n ** 3)
    r = cell.homogenise(n, MAT, rho=rho, want_x=False)
    f = foms.foms(r.C, r.e, r.kappa)
    t = 1.7
    f2 = foms.foms(t * r.C, t * r.e, t * r.kappa)
    assert abs(f2["d_h"] - f["d_h"]) < 1e-12 * abs(f["d_h"])
    assert abs(f2["k_h"] - f["k_h"]) < 1e-12 * abs(f["k_h"])
    assert abs(f2["g_h"] - f["g_h"] / t) < 1e-12 * abs(f["g_h"])


# ------------------------------------------------------- Schur + GMRES
def test_exact_schur_preconditioner_converges_in_two_steps():
    """P11: with exact A^-1 and exact S, calA P^-1 - I is nilpotent of
    order 2, so right-preconditioned GMRES converges in at most 2 steps."""
    n = 3
    rho = np.random.default_rng(2).uniform(0, 1, n ** 3)
    r = cell.homogenise(n, MAT, rho=rho)
    X, hists = krylov.solve_scp(r.K, r.F, exact=True, rtol=1e-12)
    for h in hists:
        inner = [v for v in h[1:3]]
        assert min(inner) < 1e-10
    assert rel(cell.effective_flux(n, r.s, MND, X), r.MH) < 1e-9


def test_elementwise_schur_scp_gmres_reaches_direct_solution():
    """Approximate S_bar (element-wise, delta = 1e-10) changes only the
    iteration count; the converged tensors equal the direct solve's."""
    n = 4
    r = cell.homogenise(n, MAT, phi=synth.grf_levelset(n, seed=4))
    X, hists = krylov.solve_scp(r.K, r.F, n=n, s=r.s, M=MND, exact=False, rtol=1e-12)
    assert rel(cell.effective_flux(n, r.s, MND, X), r.MH) < 1e-9
    for h in hists:
        assert h[-1] < 1e-11
        # P12: the GMRES residual estimate never increases within a cycle
        assert np.all(np.diff(h[1:-1]) <= 1e-14)


# ------------------------------------------------------------------ HJ step
def test_hj_zero_velocity_and_monotone():
    n = 8
    phi = synth.grf_levelset(n, seed=6)
    assert np.array_equal(hj.hj_step(n, phi, np.zeros(n ** 3)), phi)
    v = np.random.default_rng(1).uniform(-1, 1, n ** 3)
    out = hj.hj_step(n, phi, v)
    assert out.max() <= phi.max() + 1e-15 and out.min() >= phi.min() - 1e-15


def test_hj_slab_translates_exactly():
    """P13: phi = |z - 1/2| - w with constant v moves by v dt away from kinks."""
    n = 16
    x, y, z = synth.node_coords(n)
    phi = np.abs(z - 0.5) - 0.2
    for v in (1.0, -1.0):
        out = hj.hj_step(n, phi, np.full(n ** 3, v), cfl=0.5)
        dt = 0.5 / n
        zz = z.reshape(n, n, n)[:, 0, 0]
        ok = (np.abs(zz - 0.5) > 1.5 / n) & (zz > 1.5 / n) & (zz < 1 - 1.5 / n)
        got = out.reshape(n, n, n)[:, 0, 0][ok]
        exp = phi.reshape(n, n, n)[:, 0, 0][ok] - v * dt
        assert np.abs(got - exp).max() < 1e-14


# ---------------------------------------------- full-size (matrix-free) checks
def test_fullsize_matrix_free_matches_assembled():
    """The element-by-element operator, loads and residual rows used at full
    sizes agree with the assembled (pinned) matrix on a small cell."""
    from oracle import fullsize
    n = 5
    rng = np.random.default_rng(12)
    s = fe.ersatz_scale(rng.uniform(0, 1, n ** 3), MAT.void_scale)
    K, F = cell.assemble(n, s, MND)
    X = rng.standard_normal((4 * n ** 3, 9))
    assert rel(fullsize.element_apply(n, s, MND, X), K @ X) < 1e-13
    assert rel(fullsize.load_vectors(n, s, MND), F) < 1e-13
    nodes = np.array([0, 7, 31, 62, 124])
    rows = fullsize.residual_rows(n, s, MND, X, nodes)
    R = (K @ X + F).reshape(n ** 3, 4, 9)
    assert rel(rows, R[nodes]) < 1e-13


def test_fullsize_residual_and_sensitivity_of_direct_solution():
    """At the direct solution the matrix-free residual vanishes and the
    sampled sensitivities equal the oracle's full density gradient."""
    from oracle import fullsize
    n = 6
    r = cell.homogenise(n, MAT, phi=synth.grf_levelset(n, seed=31))
    assert fullsize.residual_norms(n, r.s, MND, r.X).max() < 1e-12
    W = np.random.default_rng(4).standard_normal((9, 9))
    g = cell.grad_rho(n, MAT, r.X, W)
    elems = np.array([0, 5, 17, 100, 215])
    assert rel(fullsize.element_sensitivity(n, MAT, r.X, W, elems), g[elems]) < 1e-12
    # the residual bound on the tensors: a perturbed solution's flux-form
    # error is -(x^K)^T r^L
    dX = 1e-6 * np.random.default_rng(5).standard_normal(r.X.shape)
    Xp = r.X + dX
    Rp = fullsize.element_apply(n, r.s, MND, Xp) + fullsize.load_vectors(n, r.s, MND)
    dM = cell.effective_flux(n, r.s, MND, Xp) - r.MH
    assert rel(dM, -r.X.T @ Rp) < 1e-6


def _bf16(a):
    """Round to bfloat16, nearest even (via float32)."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7fff + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_galerkin_rows_annihilate_constants_and_compact_form():
    """The compact coarse stencils rest on Galerkin operators R M P (trilinear
    P, R = P^T) annihilating constants for every field pair: P maps a constant
    to a constant and M's rows do.  Checked on the oracle's A block and
    element-wise S_bar at 16^3, levels 0-2.  Then the compact form itself on
    level 1: off-node entries rounded to bf16 and each node's own block set to
    minus the rounded row sums keeps the constants in the kernel, and its
    error on inputs 1e4 + unit noise stays within 2^-8 of the difference form,
    which rounding every entry misses by orders of magnitude."""
    import scipy.sparse as sp
    from oracle import cell, krylov
    from test_gpu_tiled import difference_magnitude, field_index, prolongation_sparse
    mat = synth.material_workload()
    mnd = fe.nondim_matrix(mat)
    n = 16
    rho = synth.random_density(n, seed=35)
    s = fe.ersatz_scale(rho, mat.void_scale)
    K, _ = cell.assemble(n, s, mnd)
    iu = field_index(n, [0, 1, 2])
    blocks = (("A", K[iu][:, iu].tocsr(), 3), ("S_bar", krylov.schur_elementwise(n, s, mnd).tocsr(), 1))
    rng = np.random.default_rng(6)
    for name, M0, F in blocks:
        Ml, nl = M0, n
        for level in range(3):
            if level:
                Pm = prolongation_sparse(nl // 2, F)
                Ml = (Pm.T @ Ml @ Pm).tocsr()
                nl //= 2
            for fi in range(F):
                one = np.zeros(nl ** 3 * F)
                one[fi::F] = 1.0
                assert np.abs(Ml @ one).max() <= 1e-13 * abs(Ml).max(), (name, level, fi)
            if level != 1:
                continue
            C = Ml.tocoo()
            off = (C.row // F) != (C.col // F)
            vals = C.data.copy()
            vals[off] = _bf16(vals[off])
            rsum = np.zeros((Ml.shape[0], F))
            np.add.at(rsum, (C.row[off], C.col[off] % F), vals[off])
            vals[~off] = 0.0
            own = sp.csr_matrix((vals, (C.row, C.col)), shape=Ml.shape)
            Mc = own.tolil()
            for r in range(Ml.shape[0]):
                node = r // F
                for g in range(F):
                    Mc[r, node * F + g] = -rsum[r, g]
            Mc = Mc.tocsr()
            for fi in range(F):
                one = np.zeros(nl ** 3 * F)
                one[fi::F] = 1.0
                assert np.abs(Mc @ one).max() <= 1e-13 * abs(Ml).max(), (name, "compact", fi)
            x = 1e4 * (1.0 + 0.1 * np.arange(9))[None, :] + rng.standard_normal((nl ** 3 * F, 9))
            ref = Ml @ x
            bound = 2.0 ** -8 * difference_magnitude(Ml, x, F)
            assert (np.abs(Mc @ x - ref) / bound).max() < 1.0, name
            Mp = sp.csr_matrix((_bf16(C.data), (C.row, C.col)), shape=Ml.shape)
            assert (np.abs(Mp @ x - ref) / bound).max() > 100.0, name


# ------------------------------------------------ smoothing and density map
# Sec. 2.6 smooths the interface over about two elements; the reading is a
# sinusoidal H of half-width eta = 2h evaluated at each element's mean phi.
# These pins fix the shape, the symmetry and the band width of that map from
# properties any correct smoothed Heaviside of that width has.

def test_smoothed_heaviside_end_values_and_symmetry():
    eta = 0.3
    H = lambda t: fe.smoothed_heaviside(np.asarray(t, dtype=float), eta)
    dH = lambda t: fe.smoothed_heaviside_deriv(np.asarray(t, dtype=float), eta)
    assert abs(H(-eta)) < 1e-15 and abs(H(eta) - 1.0) < 1e-15 and abs(H(0.0) - 0.5) < 1e-15
    assert H(-2 * eta) == 0.0 and H(2 * eta) == 1.0
    assert abs(dH(eta)) < 1e-15 and abs(dH(-eta)) < 1e-15
    t = np.linspace(-1.5 * eta, 1.5 * eta, 2001)
    # H - step is odd: H(t) + H(-t) = 1
    assert np.abs(H(t) + H(-t) - 1.0).max() < 1e-15
    # monotone, continuous at the band edges, derivative consistent with H
    assert np.all(np.diff(H(t)) >= 0.0)
    for edge in (-eta, eta):
        assert abs(H(edge - 1e-12) - H(edge + 1e-12)) < 1e-10
    tt = np.linspace(-0.99 * eta, 0.99 * eta, 37)
    d = 1e-7
    fd = (H(tt + d) - H(tt - d)) / (2 * d)
    assert np.abs(fd - dH(tt)).max() < 1e-6 / eta
    # the integral of H' over the band is one
    q = np.linspace(-eta, eta, 200001)
    assert abs(np.trapezoid(dH(q), q) - 1.0) < 1e-9


@pytest.mark.parametrize("offset", [0.0, 0.5])
def test_slab_density_band_width_and_exact_volume(offset):
    """A slab |z - 1/2| < w as a signed distance phi = |z - 1/2| - w (phi < 0
    solid).  Each element's mean phi is the distance at its mid-plane, so the
    element layers sample the distance at spacing h.  With the interfaces on
    node planes (offset 0) the mid-planes sit at +-h/2, +-3h/2, ...; with them
    on element mid-planes (offset 0.5) at 0, +-h, +-2h.  A half-width of two
    elements puts exactly four (three) layers per interface strictly inside
    (0, 1), the rest exactly 0 or 1; and because H - step is odd the samples
    cancel in pairs, so the mean density equals the slab's exact volume 2w."""
    n = 32
    h = 1.0 / n
    w = 0.25 + offset * h
    z = np.arange(n) * h
    phi_z = np.abs(z - 0.5) - w
    phi = np.broadcast_to(phi_z[:, None, None], (n, n, n)).ravel()     # [k][j][i]
    rho = fe.density_from_levelset(n, phi).reshape(n, n, n)
    layers = rho[:, 0, 0]
    assert np.all(rho == layers[:, None, None])
    tol = 1e-14   # sin(pi) rounds to about 1e-16 at the band edges
    inside = (layers > tol) & (layers < 1.0 - tol)
    assert inside.sum() == (8 if offset == 0.0 else 6)
    # the fractional layers are the ones within 2h of an interface
    mid = (np.arange(n) + 0.5) * h
    dist = np.minimum(np.abs(mid - (0.5 - w)), np.abs(mid - (0.5 + w)))
    assert np.array_equal(inside, dist < 2 * h - 1e-12)
    # solid (phi < 0) maps to rho = 1
    assert np.all(np.abs(layers[np.abs(mid - 0.5) < w - 2 * h + 1e-12] - 1.0) < tol)
    assert np.all(np.abs(layers[np.abs(mid - 0.5) > w + 2 * h - 1e-12]) < tol)
    assert abs(layers.mean() - 2 * w) < 1e-14
    # the same slab turned to lie along x
    phi_x = np.broadcast_to(phi_z[None, None, :], (n, n, n)).ravel()
    rho_x = fe.density_from_levelset(n, phi_x).reshape(n, n, n)
    assert np.array_equal(rho_x[0, 0, :], layers)


def test_density_chain_rule_matches_finite_differences():
    """The element-form chain rule dJ/dphi_n (Sec. 2.1, Sec. 2.6 smoothing)
    against central differences of J(phi) = sum_e c_e rho_e(phi) at nodes in
    and near the band, and through the whole solve at n = 4."""
    n = 8
    rng = np.random.default_rng(31)
    phi = synth.grf_levelset(n, seed=5, solid_fraction=0.5)
    c = rng.standard_normal(n ** 3)
    g = cell.grad_phi_from_rho(n, phi, c)
    J = lambda p: float(c @ fe.density_from_levelset(n, p))
    rho = fe.density_from_levelset(n, phi)
    band_nodes = np.unique(cell.element_nodes(n)[(rho > 0) & (rho < 1)])
    assert band_nodes.size > 50
    picks = list(rng.choice(band_nodes, 24, replace=False)) + [int(np.argmax(np.abs(phi)))]
    d = 1e-6
    for node in picks:
        pp = phi.copy(); pp[node] += d
        pm = phi.copy(); pm[node] -= d
        fd = (J(pp) - J(pm)) / (2 * d)
        assert abs(fd - g[node]) <= 1e-6 * np.abs(g).max(), (node, fd, g[node])
    # and through the solve: J = <W, M^H(rho(phi))>
    n = 4
    phi = synth.grf_levelset(n, seed=8, solid_fraction=0.5) * 0.3
    r = cell.homogenise(n, MAT, phi=phi)
    W = rng.standard_normal((9, 9))
    gphi = cell.grad_phi_from_rho(n, phi, cell.grad_rho(n, MAT, r.X, W))
    d = 1e-6
    for node in (0, 9, 27, 50):
        pp = phi.copy(); pp[node] += d
        pm = phi.copy(); pm[node] -= d
        fd = np.sum(W * (cell.homogenise(n, MAT, phi=pp, want_x=False).MH
                         - cell.homogenise(n, MAT, phi=pm, want_x=False).MH)) / (2 * d)
        assert abs(fd - gphi[node]) <= 1e-5 * np.abs(gphi).max(), (node, fd, gphi[node])


# ------------------------------------------------------- bulk moduli
def test_voigt_and_reuss_bulk_moduli_isotropic_equality_and_order():
    """Sec. 2.3: B_Reuss <= B_Voigt, with equality for isotropic stiffness.
    For isotropic C (Lame lam, mu) both equal the bulk modulus lam + 2 mu / 3,
    which fixes both normalisations and B_Reuss's compliance block."""
    lam, mu = 61.0e9, 27.0e9
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[[0, 1, 2], [0, 1, 2]] = lam + 2 * mu
    C[[3, 4, 5], [3, 4, 5]] = mu
    e = np.zeros((3, 6)); e[2, :3] = 3.0
    kap = np.eye(3) * 5e-9
    f = foms.foms(C, e, kap)
    K = lam + 2 * mu / 3
    assert abs(f["B_voigt"] - K) < 1e-12 * K and abs(f["B_reuss"] - K) < 1e-12 * K
    # anisotropic: random SPD stiffness matrices and the base material
    rng = np.random.default_rng(3)
    for _ in range(20):
        A = rng.standard_normal((6, 6))
        Cr = A @ A.T + 0.1 * np.eye(6)
        fr = foms.foms(Cr, e, kap)
        assert fr["B_reuss"] <= fr["B_voigt"] * (1 + 1e-14)
    for m in (synth.material_workload(), synth.material_pzt5a()):
        fm = foms.foms(m.C, m.e, m.kappa)
        assert fm["B_reuss"] < fm["B_voigt"]
    # and on solved cells
    for seed in (1, 2):
        r = cell.homogenise(6, MAT, phi=synth.grf_levelset(6, seed=seed), want_x=False)
        fr = foms.foms(r.C, r.e, r.kappa)
        assert 0 < fr["B_reuss"] < fr["B_voigt"]


def test_table3_kh_through_the_oracle():
    """P9 through oracle.foms: tensors built to have a Table 3 row's printed
    d_h, g_h and B_Reuss give that row's printed k_h.  C is orthotropic with
    normal stiffnesses (c1, c1, c3), c1 = 10 B_Reuss, c3 chosen to give the
    row's B_Reuss, so that B_Voigt is about 2.4 B_Reuss (as for the paper's
    soft-in-z designs); e has only e31 = e32 = e33 = a, so d_h = a / B_Reuss; kappa_33 is set so
    that the stress-free permittivity gives g_h."""
    pv = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
    for row in pv["table3_rows"]["rows"]:
        c1 = 10.0 * row["B_reuss"]
        c3 = 1.0 / (1.0 / row["B_reuss"] - 2.0 / c1)
        C = np.diag([c1, c1, c3, 0.3 * c1, 0.3 * c1, 0.3 * c1])
        a = row["d_h"] * row["B_reuss"]
        e = np.zeros((3, 6)); e[2, :3] = a
        kap = np.eye(3) * 1e-9
        kap[2, 2] = row["d_h"] / row["g_h"] - a * row["d_h"]
        assert kap[2, 2] > 0
        f = foms.foms(C, e, kap)
        assert abs(f["d_h"] / row["d_h"] - 1) < 1e-12
        assert abs(f["g_h"] / row["g_h"] - 1) < 1e-12
        assert abs(f["B_reuss"] / row["B_reuss"] - 1) < 1e-12
        assert f["B_voigt"] > 2.0 * f["B_reuss"]
        assert abs(f["k_h"] - row["k_h"]) < 1.5e-3
