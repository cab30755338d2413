"""The paper's solver comparison (Sec. 2.5) on the GPU: the block-diagonal
preconditioner diag(A, -C) (DBP-GMRES) next to the approximate Schur
complement one (SCP-GMRES), with fixed V-cycle block maps or with inexact
inner solves (conjugate gradients preconditioned by one V-cycle, to a
relative tolerance eps).  Every form converges to the same discrete
solution, so the tensors are checked against the oracle's direct solve."""
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


def test_c_block_operator(torch_cuda, P):
    """The dielectric block C (calA's (phi, phi) block is -C) against the
    oracle's assembled matrix, in the three precision forms."""
    torch = torch_cuda
    n = 16
    say("C block operator")
    rho = synth.random_density(n, seed=91)
    s = fe.ersatz_scale(rho, MAT.void_scale)
    K, _ = cell.assemble(n, s, MND)
    ip = np.arange(4 * n ** 3)[np.arange(4 * n ** 3) % 4 == 3]
    Cm = -K[ip][:, ip]
    nn = n ** 3
    x = np.random.default_rng(5).standard_normal((nn, 9))
    with P.Context(n, MAT, precision=P.PHZ_BF16X3_IR) as ctx:
        ctx.set_density(rho)
        for prec, dt, tol in ((P.PHZ_FP64, torch.float64, 1e-13), (P.PHZ_FP32_IR, torch.float32, 2e-6),
                              (P.PHZ_BF16X3_IR, torch.float32, 3e-5)):
            xd = torch.tensor(to_soa(x, nn, 1, 9), dtype=dt, device="cuda").contiguous()
            xr = from_soa(xd.cpu().double().numpy(), nn, 1, 9)
            yd = torch.zeros_like(xd)
            ctx.apply(P.OP_C, 9, prec, xd.data_ptr(), yd.data_ptr())
            torch.cuda.synchronize()
            y = from_soa(yd.cpu().double().numpy(), nn, 1, 9)
            err = (np.abs(y - Cm @ xr) / np.maximum(abs(Cm) @ abs(xr), 1e-300)).max()
            print("precision", prec, "max error / term magnitude", err)
            assert err < tol, (prec, err)


CASES = [
    ("dbp", "fp64", 0, None),
    ("dbp", "fp32ir", 0, None),
    ("scp", "fp64", 1, 1e-2),
    ("scp", "fp64", 1, 1e-8),
    ("dbp", "fp64", 1, 1e-4),
    ("scp", "bf16x3ir", 1, 1e-4),
]


@pytest.mark.parametrize("solver,form,inner,eps", CASES)
def test_solver_forms_vs_stored_oracle(P, solver, form, inner, eps):
    """Each preconditioner and block-map form reaches the oracle's tensors
    of the 16^3 random-field cell; the inexact maps report their inner
    conjugate-gradient iterations."""
    g = json.load(open(os.path.join(HERE, "golden", "grf16.json")))
    say("solver", solver, form, "inner", inner, eps)
    opts = dict(solver=P.PHZ_SOLVER_DBP if solver == "dbp" else P.PHZ_SOLVER_SCP, inner=inner, rtol=1e-10)
    if eps is not None:
        opts["inner_eps"] = eps
    prec = {"fp64": P.PHZ_FP64, "fp32ir": P.PHZ_FP32_IR, "bf16x3ir": P.PHZ_BF16X3_IR}[form]
    with P.Context(16, MAT, precision=prec, **opts) as ctx:
        ctx.set_levelset(synth.grf_levelset(16, seed=2410, solid_fraction=0.5))
        assert ctx.solve() == P.PHZ_OK
        st = ctx.stats()
        print("iterations", max(st["iterations"]), "refinements", st["refinements"],
              "inner iterations / maps", st["inner_iters"], st["inner_calls"])
        MH, _ = ctx.effective_nd()
        assert relmax(MH, np.array(g["MH"])) < 1e-8
        if inner:
            assert st["inner_calls"][0] > 0 and st["inner_calls"][1] > 0
            assert st["inner_iters"][0] >= st["inner_calls"][0]
        else:
            assert st["inner_calls"] == [0, 0]


def test_tight_inner_maps_cut_outer_iterations(P):
    """With the block maps solved to 1e-8 the preconditioner is close to its
    exact form, and SCP-GMRES needs far fewer outer iterations than with
    maps solved to 1e-2 (the trend of the paper's Table 1)."""
    say("inner tolerance trend")
    its = {}
    for eps in (1e-2, 1e-8):
        with P.Context(16, MAT, precision=P.PHZ_FP64, inner=1, inner_eps=eps, rtol=1e-10) as ctx:
            ctx.set_levelset(synth.grf_levelset(16, seed=2410, solid_fraction=0.5))
            assert ctx.solve() == P.PHZ_OK
            its[eps] = max(ctx.stats()["iterations"])
    print("outer iterations", its)
    assert its[1e-8] < its[1e-2]


def test_bt_block_operator(torch_cuda, P):
    """B^T (block 5, potential -> displacements) against the oracle's assembled coupling block, float64
    and float32."""
    torch = torch_cuda
    n = 16
    say("B^T block operator")
    rho = synth.random_density(n, seed=93)
    s = fe.ersatz_scale(rho, MAT.void_scale)
    K, _ = cell.assemble(n, s, MND)
    d = np.arange(4 * n ** 3)
    iu, ip = d[d % 4 < 3], d[d % 4 == 3]
    Bt = K[iu][:, ip]
    nn = n ** 3
    x = np.random.default_rng(6).standard_normal((nn, 9))
    with P.Context(n, MAT, precision=P.PHZ_FP64) as ctx:
        ctx.set_density(rho)
        for prec, dt, tol in ((P.PHZ_FP64, torch.float64, 1e-13), (P.PHZ_FP32_IR, torch.float32, 2e-6)):
            for nrhs in (1, 9):
                xs = x[:, :nrhs]
                xd = torch.tensor(to_soa(xs, nn, 1, nrhs), dtype=dt, device="cuda").contiguous()
                xr = from_soa(xd.cpu().double().numpy(), nn, 1, nrhs)
                yd = torch.zeros((3, nrhs, nn), dtype=dt, device="cuda")
                ctx.apply(P.OP_BT, nrhs, prec, xd.data_ptr(), yd.data_ptr())
                torch.cuda.synchronize()
                y = from_soa(yd.cpu().double().numpy(), nn, 3, nrhs)
                err = (np.abs(y - Bt @ xr) / np.maximum(abs(Bt) @ abs(xr), 1e-300)).max()
                print("precision", prec, "columns", nrhs, "max error / term magnitude", err)
                assert err < tol, (prec, nrhs, err)


TRICG = json.load(open(os.path.join(HERE, "golden", "tricg16.json")))


@pytest.mark.parametrize("name", ["grf16", "sphere16"])
@pytest.mark.parametrize("batched", [1, 0])
def test_tricg_solve(P, name, batched):
    """TriCG (float64, block maps by conjugate gradients to 1e-10) reaches the oracle's direct-solve
    tensors.  Its iterations per load are those of the oracle's TriCG with exact block inverses, up to
    a short extra cycle: inexact maps can leave the true residual above the recurrence's at the end of
    a cycle, and the solve then restarts from it (-2 to +5 iterations)."""
    g = json.load(open(os.path.join(HERE, "golden", f"{name}.json")))
    phi = synth.grf_levelset(16, seed=2410, solid_fraction=0.5) if name == "grf16" else synth.sphere_levelset(16)
    say("TriCG", name, "batched", batched)
    with P.Context(16, MAT, precision=P.PHZ_FP64, solver=P.PHZ_SOLVER_TRICG, inner_eps=1e-10, rtol=1e-10,
                   batched=batched) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        st = ctx.stats()
        print("iterations", st["iterations"], "cycles", st["restarts"], "oracle", TRICG[name]["iterations"],
              "CG per map", [st["inner_iters"][i] / max(st["inner_calls"][i], 1) for i in range(2)])
        MH, _ = ctx.effective_nd()
        ref = np.array(g["MH"])
        assert relmax(MH, ref) < 1e-8
        assert max(st["true_residual"]) <= 1e-10
        for got, want in zip(st["iterations"], TRICG[name]["iterations"]):
            assert -2 <= got - want <= 5, (st["iterations"], TRICG[name]["iterations"])


def test_tricg_loose_inner_maps(P):
    """With block maps only to 1e-4 the cycles restart from the true residual until it reaches the
    tolerance: the tensors still match the direct solve."""
    g = json.load(open(os.path.join(HERE, "golden", "grf16.json")))
    say("TriCG, inner 1e-4")
    with P.Context(16, MAT, precision=P.PHZ_FP64, solver=P.PHZ_SOLVER_TRICG, inner_eps=1e-4, rtol=1e-10,
                   max_iters=2000) as ctx:
        ctx.set_levelset(synth.grf_levelset(16, seed=2410, solid_fraction=0.5))
        assert ctx.solve() == P.PHZ_OK
        st = ctx.stats()
        print("iterations", st["iterations"], "cycles", st["restarts"])
        MH, _ = ctx.effective_nd()
        assert relmax(MH, np.array(g["MH"])) < 1e-8
