"""GPU parity of the quadrature-point smoothing (the material smoothed at every Gauss point of the level
set's trilinear interpolation): the full operator and the load vectors against the oracle's assembly with
per-point scales, and solves in every precision form against the oracle's direct solves."""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import cell, fe

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
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


def to_soa(a, nn, F, K):
    return np.ascontiguousarray(np.asarray(a).reshape(nn, F, K).transpose(1, 2, 0))


def from_soa(a, nn, F, K):
    return np.asarray(a).reshape(F, K, nn).transpose(2, 0, 1).reshape(nn * F, K)


def oracle_qp(n, phi):
    sq = fe.ersatz_scale(fe.density_qp(n, phi), MAT.void_scale)
    return cell.assemble(n, sq, MND)


def test_qp_operator_and_loads_vs_oracle(torch_cuda, P):
    torch = torch_cuda
    n = 16
    say("quadrature-point operator and loads", n)
    phi = synth.grf_levelset(n, seed=31, solid_fraction=0.5)
    K, F = oracle_qp(n, phi)
    nn = n ** 3
    x = np.random.default_rng(12).standard_normal((4 * nn, 9))
    with P.Context(n, MAT, precision=P.PHZ_FP64, smoothing=P.PHZ_SMOOTH_QP) as ctx:
        ctx.set_levelset(phi)
        b = ctx.rhs().reshape(4 * nn, 9)
        print("loads error", relmax(b, -F))
        assert relmax(b, -F) < 1e-13
        for prec, dt, tol in ((P.PHZ_FP64, torch.float64, 1e-13), (P.PHZ_FP32_IR, torch.float32, 3e-6)):
            for nrhs in (1, 9):
                xs = x[:, :nrhs]
                xd = torch.tensor(to_soa(xs, nn, 4, nrhs), dtype=dt, device="cuda").contiguous()
                xr = from_soa(xd.cpu().double().numpy(), nn, 4, nrhs)
                yd = torch.zeros_like(xd)
                ctx.apply(P.OP_FULL, nrhs, prec, xd.data_ptr(), yd.data_ptr())
                torch.cuda.synchronize()
                y = from_soa(yd.cpu().double().numpy(), nn, 4, nrhs)
                err = (np.abs(y - K @ xr) / np.maximum(abs(K) @ abs(xr), 1e-300)).max()
                print("precision", prec, "columns", nrhs, "max error / term magnitude", err)
                assert err < tol, (prec, nrhs, err)


@pytest.mark.parametrize("name", ["grf16", "sphere16"])
@pytest.mark.parametrize("precision", ["fp64", "fp32ir", "bf16x3ir"])
def test_qp_solve_vs_oracle(P, name, precision):
    """Solves with the point-interpolated material reach the oracle's direct solve of the same
    discretisation; the preconditioner's element-mean blocks only change the iteration counts."""
    g = json.load(open(os.path.join(HERE, "golden", f"{name}_qp.json")))
    ge = json.load(open(os.path.join(HERE, "golden", f"{name}.json")))
    phi = synth.grf_levelset(16, seed=2410, solid_fraction=0.5) if name == "grf16" else synth.sphere_levelset(16)
    prec = {"fp64": P.PHZ_FP64, "fp32ir": P.PHZ_FP32_IR, "bf16x3ir": P.PHZ_BF16X3_IR}[precision]
    say("quadrature-point solve", name, precision)
    with P.Context(16, MAT, precision=prec, rtol=1e-10, smoothing=P.PHZ_SMOOTH_QP) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        st = ctx.stats()
        MH, MHe = ctx.effective_nd()
        print("iterations", st["iterations"], "refinements", st["refinements"], "error", relmax(MH, g["MH"]),
              "element form differs by", relmax(MH, ge["MH"]))
        assert relmax(MH, g["MH"]) < 1e-8
        assert relmax(MHe, g["MH_energy"]) < 1e-8
        assert relmax(MH, ge["MH"]) > 1e-5


def test_qp_sensitivities_vs_oracle(P):
    """The point-form backward (d_h's density gradient summed per element, and its level-set gradient)
    and the chain rule of an element gradient spread over the points, against the oracle's direct
    solve of the 12^3 cell."""
    n = 12
    say("quadrature-point sensitivities", n)
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.5)
    r = cell.homogenise(n, MAT, phi=phi, smoothing="qp")
    from oracle import foms as ofoms
    gC, ge_, gk = ofoms.fom_grads(r.C, r.e, r.kappa, "d_h")
    W = cell.W_from_tensor_grads(gC, ge_, gk)
    grq = cell.grad_rho_qp(n, MAT, r.X, W)
    gphi = cell.grad_phi_from_rho_qp(n, phi, grq)
    with P.Context(n, MAT, precision=P.PHZ_FP64, rtol=1e-12, smoothing=P.PHZ_SMOOTH_QP) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        f, (gC2, ge2, gk2) = P.foms(*ctx.effective(), grad_of="d_h")
        grho, gp = ctx.backward(gC2, ge2, gk2, want_phi=True)
        print("grad_rho error", relmax(grho, grq.sum(axis=1)), "grad_phi error", relmax(gp, gphi))
        assert relmax(grho, grq.sum(axis=1)) < 1e-8
        assert relmax(gp, gphi) < 1e-8
        g = np.random.default_rng(3).standard_normal(n ** 3)
        ref = cell.grad_phi_from_rho_qp(n, phi, np.repeat(g[:, None] / 8.0, 8, axis=1))
        assert relmax(ctx.levelset_gradient(g), ref) < 1e-13


def test_qp_switch_and_density_input(P):
    """Switching the smoothing on a set geometry recomputes its scales both ways; a cell given by
    densities has equal point scales (the element form)."""
    g = json.load(open(os.path.join(HERE, "golden", "grf16_qp.json")))
    ge = json.load(open(os.path.join(HERE, "golden", "grf16.json")))
    say("smoothing switch")
    phi = synth.grf_levelset(16, seed=2410, solid_fraction=0.5)
    with P.Context(16, MAT, precision=P.PHZ_FP64, rtol=1e-10) as ctx:
        ctx.set_levelset(phi)
        ctx.solve()
        assert relmax(ctx.effective_nd()[0], ge["MH"]) < 1e-8
        ctx.set_options(smoothing=P.PHZ_SMOOTH_QP)
        ctx.solve()
        assert relmax(ctx.effective_nd()[0], g["MH"]) < 1e-8
        ctx.set_options(smoothing=P.PHZ_SMOOTH_ELEMENT)
        ctx.solve()
        assert relmax(ctx.effective_nd()[0], ge["MH"]) < 1e-8
        rho = synth.random_density(16, seed=8)
        ctx.set_density(rho)
        ctx.solve()
        el = ctx.effective_nd()[0]
        ctx.set_options(smoothing=P.PHZ_SMOOTH_QP)
        ctx.solve()
        assert relmax(ctx.effective_nd()[0], el) < 1e-9
