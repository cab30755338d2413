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
