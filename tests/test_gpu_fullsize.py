"""GPU parity at the full workload sizes, where the oracle cannot solve.

The oracle checks the GPU's solution X with its own element-by-element
operator (oracle.fullsize): the full residual ||K X + F|| / ||F|| at 64^3,
residual rows at sampled nodes at 128^3 and 256^3, the flux-form tensors
recomputed from X, and per-element sensitivities at sampled elements.  A
residual r bounds the tensors: the flux-form error of entry (K, L) is
-(x^K)^T r^L.  The mixed forms are compared with the GPU's plain FP64 solve
of the same cell.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import cell, fe, fullsize, hj as ohj

pytestmark = pytest.mark.gpu

MAT = synth.material_workload()
MND = fe.nondim_matrix(MAT)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def P():
    import paper_2410_03148_amd as P
    return P


def relmax(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def relfro(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def sample_nodes(n, count, seed):
    """Random nodes plus the first and last plane rows (periodic wrap)."""
    rng = np.random.default_rng(seed)
    edge = np.concatenate([np.arange(n), n ** 3 - 1 - np.arange(n)])
    return np.unique(np.concatenate([rng.integers(0, n ** 3, count), edge]))


def test_grf64_fp64_sequential_full_residual(torch_cuda, P):
    """64^3 random-field cell (solid fraction 0.5), plain FP64 GMRES(30) with
    the SCP/multigrid preconditioner, nine loads one at a time: the oracle's
    residual of X at every node, and the tensors it recomputes from X."""
    n = 64
    say("grf64 fp64 sequential")
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.5)
    with P.Context(n, MAT, precision=P.PHZ_FP64, batched=0, restart=30, rtol=1e-10) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        st = ctx.stats()
        print("iterations", st["iterations"], "gpu residuals", max(st["true_residual"]))
        MH, MHe = ctx.effective_nd()
        X = ctx.solution().reshape(-1, 9)
        s = ctx.scale()
    rho = fe.density_from_levelset(n, phi)
    assert relmax(s, fe.ersatz_scale(rho, MAT.void_scale)) < 1e-15
    res = fullsize.residual_norms(n, s, MND, X)
    print("oracle residuals", res)
    assert res.max() < 1e-9
    MH_o = cell.effective_flux(n, s, MND, X)
    assert relmax(MH, MH_o) < 1e-10
    # error bound of the flux tensors from the oracle's residual
    R = fullsize.element_apply(n, s, MND, X) + fullsize.load_vectors(n, s, MND)
    bound = np.abs(X.T @ R).max() / np.abs(MH).max()
    print("tensor error bound from the residual", bound)
    assert bound < 1e-8
    assert relmax(MHe, MH) < 1e-8


@pytest.mark.parametrize("vf", [0.3, 0.7])
def test_grf128_mixed_vs_fp64_and_sampled_residual(torch_cuda, P, vf):
    """128^3 random-field cell at solid fractions 0.3 and 0.7, nine loads
    batched: the split-BF16 mixed form against the GPU's FP64 solve (<= 1e-6),
    and the oracle's residual rows of the mixed solution at sampled nodes."""
    n = 128
    say("grf128 mixed vs fp64, solid fraction", vf)
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=vf)
    out = {}
    for name, prec, restart in (("mixed", P.PHZ_BF16X3_IR, 12), ("fp64", P.PHZ_FP64, 15)):
        with P.Context(n, MAT, precision=prec, restart=restart, vcycles_a=2, rtol=1e-10,
                       inner_rtol=1e-4 if prec == P.PHZ_BF16X3_IR else 1e-5) as ctx:
            ctx.set_levelset(phi)
            assert ctx.solve() == P.PHZ_OK
            st = ctx.stats()
            print(name, "iterations", max(st["iterations"]), "refinements", st["refinements"],
                  "residual", max(st["true_residual"]))
            out[name] = ctx.effective()
            if name == "mixed":
                X = ctx.solution()
                s = ctx.scale()
                bnorm = np.linalg.norm(ctx.rhs().reshape(-1, 9), axis=0)
    for a, b in zip(out["mixed"], out["fp64"]):
        assert relfro(a, b) < 1e-6
    nodes = sample_nodes(n, 3000, seed=int(vf * 10))
    rows = fullsize.residual_rows(n, s, MND, X, nodes)            # (m, 4, 9)
    worst = np.abs(rows).max(axis=(0, 1)) / bnorm
    print("sampled residual rows / ||b||", worst.max())
    assert worst.max() < 1e-9


def test_grf128_backward_sampled_and_euler(torch_cuda, P):
    """128^3 differentiation form (solid fraction 0.5): d_h's density gradient
    against the oracle's (1 - eps_v) <W, G_e> at sampled elements of the GPU
    solution, the Euler identity sum_e s_e dM/ds_e = M at full size, the
    level-set chain rule at sampled nodes, and one HJ step against the oracle's."""
    n = 128
    say("grf128 backward")
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.5)
    with P.Context(n, MAT, precision=P.PHZ_FP64, restart=15, vcycles_a=2, rtol=1e-10) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        Cm, e, k = ctx.effective()
        f, (gC, ge, gk) = P.foms(Cm, e, k, grad_of="d_h")
        # a generic upstream gradient first (degree-1 Euler identity), then d_h's
        rng = np.random.default_rng(7)
        rC, re, rk = rng.standard_normal((6, 6)) * 1e-10, rng.standard_normal((3, 6)), rng.standard_normal((3, 3)) * 1e9
        g_rand = ctx.backward(rC, re, rk)
        W_rand = cell.W_from_tensor_grads(rC, re, rk)
        g, gp = ctx.backward(gC, ge, gk, want_phi=True)
        X = ctx.solution()
        s = ctx.scale()
        MH, _ = ctx.effective_nd()
        phi_new = ctx.hj_step(None, cfl=0.5)
    W = cell.W_from_tensor_grads(gC, ge, gk)
    rng = np.random.default_rng(2412)
    rho = fe.density_from_levelset(n, phi)
    # stratified sample: solid, void and interface elements
    strata = [np.flatnonzero(rho == 1.0), np.flatnonzero(rho == 0.0), np.flatnonzero((rho > 0) & (rho < 1))]
    elems = np.concatenate([rng.choice(a, 16, replace=False) for a in strata if len(a) >= 16])
    g_o = fullsize.element_sensitivity(n, MAT, X, W, elems)
    assert relmax(g[elems], g_o) < 1e-9
    # Euler (M^H is homogeneous of degree 1 in s): sum_e s_e dJ/ds_e = <W, M^H>
    # for a linear J; d_h is of degree 0 in M^H, so its sum vanishes
    J = float(np.sum(W_rand * MH))
    euler = float(np.sum(s * g_rand)) / (1.0 - MAT.void_scale)
    print("Euler (linear J)", euler, J)
    assert abs(euler - J) < 1e-8 * abs(J)
    e0 = float(np.sum(s * g)) / float(np.sum(np.abs(s * g)))
    print("Euler (d_h, degree 0)", e0)
    assert abs(e0) < 1e-9
    # level-set chain rule at sampled nodes, from the full GPU density gradient
    nodes = sample_nodes(n, 2000, seed=3)
    gp_o = cell.grad_phi_from_rho(n, phi, g)
    assert relmax(gp[nodes], gp_o[nodes]) < 1e-12
    # one HJ step: velocity = nodal mean of dJ/drho normalised to max 1
    v = ohj.nodal_velocity(n, g)
    ref = ohj.hj_step(n, phi, v, cfl=0.5)
    assert relmax(phi_new, ref) < 1e-12


def test_grf12_gradient_vs_oracle_same_field(torch_cuda, P):
    """The 12^3 cell of the same continuous random field: the GPU density and
    level-set gradients of d_h and g_h against the oracle's direct solve."""
    n = 12
    say("grf12 gradient")
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.5)
    r = cell.homogenise(n, MAT, phi=phi)
    with P.Context(n, MAT, precision=P.PHZ_FP64, rtol=1e-12) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        Cm, e, k = ctx.effective()
        for fom in ("d_h", "g_h"):
            f, (gC, ge, gk) = P.foms(Cm, e, k, grad_of=fom)
            g, gp = ctx.backward(gC, ge, gk, want_phi=True)
            W = cell.W_from_tensor_grads(gC, ge, gk)
            g_ref = cell.grad_rho(n, MAT, r.X, W)
            gp_ref = cell.grad_phi_from_rho(n, phi, g_ref)
            print(fom, relmax(g, g_ref), relmax(gp, gp_ref))
            assert relmax(g, g_ref) < 1e-7
            assert relmax(gp, gp_ref) < 1e-7


@pytest.mark.slow
def test_gyroid256_split_bf16_vs_fp64(torch_cuda, P):
    """256^3 gyroid cell with +-5% noise: the split-BF16 form with GMRES(20)
    and a float32 Krylov basis against the GPU's FP64 solve (<= 1e-6), and the
    oracle's residual rows of the split-BF16 solution at sampled nodes."""
    n = 256
    say("gyroid256 split-bf16 vs fp64")
    phi = synth.gyroid_levelset(n, seed=2411)
    out = {}
    for name, prec in (("mixed", P.PHZ_BF16X3_IR), ("fp64", P.PHZ_FP64)):
        with P.Context(n, MAT, precision=prec, restart=20, vcycles_a=2, rtol=1e-10,
                       inner_rtol=1e-4 if prec == P.PHZ_BF16X3_IR else 1e-5) as ctx:
            ctx.set_levelset(phi)
            assert ctx.solve() == P.PHZ_OK
            st = ctx.stats()
            print(name, "iterations", max(st["iterations"]), "refinements", st["refinements"],
                  "solve ms", st["solve_ms"], "tiles", st["elem_tile"])
            out[name] = ctx.effective()
            if name == "mixed":
                X = ctx.solution()
                s = ctx.scale()
                bnorm = np.linalg.norm(ctx.rhs().reshape(-1, 9), axis=0)
    for a, b in zip(out["mixed"], out["fp64"]):
        assert relfro(a, b) < 1e-6
    nodes = sample_nodes(n, 3000, seed=11)
    rows = fullsize.residual_rows(n, s, MND, X, nodes)
    worst = np.abs(rows).max(axis=(0, 1)) / bnorm
    print("sampled residual rows / ||b||", worst.max())
    assert worst.max() < 1e-9
