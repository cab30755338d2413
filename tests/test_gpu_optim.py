"""GPU parity of the optimisation loop's pieces (reinitialisation, chain rule, Hilbertian extension,
projected velocity) and of one whole optimisation iteration against the oracle."""
import sys

import numpy as np
import pytest

import synth
from oracle import cell, fe, foms as ofoms, hj as ohj, optim

pytestmark = pytest.mark.gpu

MAT = synth.material_workload()


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


@pytest.mark.parametrize("subcell", [False, True])
@pytest.mark.parametrize("steps", [20, 7])
def test_reinit_vs_oracle(torch_cuda, P, subcell, steps):
    n = 16
    say("reinit", n, "subcell", subcell, "steps", steps)
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.5) * 2.5
    with P.Context(n, MAT) as ctx:
        ctx.set_levelset(phi)
        r = ctx.reinit(steps=steps, cfl=0.5, subcell=subcell)
        # a second call starts from the first one's result
        r2 = ctx.reinit(steps=steps, cfl=0.5, subcell=subcell)
    ref = optim.reinit(n, phi, steps=steps, cfl=0.5, subcell=subcell)
    ref2 = optim.reinit(n, ref, steps=steps, cfl=0.5, subcell=subcell)
    print("reinit error", relmax(r, ref), relmax(r2, ref2))
    assert relmax(r, ref) < 1e-12
    assert relmax(r2, ref2) < 1e-12


def test_levelset_gradient_vs_oracle(torch_cuda, P):
    n = 12
    say("levelset gradient", n)
    phi = synth.grf_levelset(n, seed=5, solid_fraction=0.4)
    g = np.random.default_rng(2).standard_normal(n ** 3)
    with P.Context(n, MAT) as ctx:
        ctx.set_levelset(phi)
        gp = ctx.levelset_gradient(g)
    ref = cell.grad_phi_from_rho(n, phi, g)
    assert relmax(gp, ref) < 1e-13


@pytest.mark.parametrize("n,alpha_h", [(16, 4.0), (24, 4.0), (16, 0.0)])
def test_riesz_vs_oracle(torch_cuda, P, n, alpha_h):
    torch = torch_cuda
    say("riesz", n, alpha_h)
    alpha = alpha_h / n
    j = np.random.default_rng(9).standard_normal((3, n ** 3))
    with P.Context(n, MAT) as ctx:
        jd = torch.tensor(j, dtype=torch.float64, device="cuda").contiguous()
        gd = torch.zeros_like(jd)
        it = ctx.riesz(3, alpha, jd.data_ptr(), gd.data_ptr())
        torch.cuda.synchronize()
        g = gd.cpu().numpy()
        if alpha_h == 4.0 and n == 16:
            # a length scale needing more than 20000 Chebyshev steps is refused before any work
            with pytest.raises(P.PiezoError):
                ctx.riesz(3, 50.0, jd.data_ptr(), gd.data_ptr())
    print("Chebyshev steps", it)
    for k in range(3):
        ref = optim.riesz(n, j[k], alpha)
        assert relmax(g[k], ref) < 1e-10


def test_hpm_velocity_vs_oracle(torch_cuda, P):
    n = 12
    say("hpm velocity", n)
    rng = np.random.default_rng(4)
    j0 = rng.standard_normal(n ** 3)
    jc = [rng.standard_normal(n ** 3), rng.standard_normal(n ** 3)]
    with P.Context(n, MAT) as ctx:
        for viol in ([0.0, 0.0], [0.02, -0.05], [3e-4, 1e-4]):
            v = ctx.hpm_velocity(j0, jc, viol, alpha=0.0, cfl=0.5, gamma=0.5)
            ref = optim.hpm_velocity(n, j0, jc, viol, cfl=0.5, gamma=0.5)
            print("violations", viol, "error", relmax(v, ref))
            assert relmax(v, ref) < 1e-9
        v = ctx.hpm_velocity(j0)
        assert relmax(v, optim.hpm_velocity(n, j0, [], [])) < 1e-9
        # a reduced objective weight (step control)
        v = ctx.hpm_velocity(j0, jc, [0.01, -0.02], obj_weight=0.3)
        assert relmax(v, optim.hpm_velocity(n, j0, jc, [0.01, -0.02], obj_weight=0.3)) < 1e-9


def test_one_optimisation_iteration_vs_oracle(torch_cuda, P):
    """Maximise B_voigt subject to Vol = 0.5 and d_h = its initial value x 1.2 at 12^3: the level set
    after one iteration (reinitialisation, solve, three sensitivities, projected velocity, HJ step)
    against the oracle's direct solve of the same steps."""
    from paper_2410_03148_amd.optimise import optimise
    n = 12
    say("one optimisation iteration", n)
    phi0 = synth.grf_levelset(n, seed=2410, solid_fraction=0.5)
    # oracle
    phi_r = optim.reinit(n, phi0, steps=20, cfl=0.5, subcell=True)
    res = cell.homogenise(n, MAT, phi=phi_r)
    dh0 = ofoms.foms(res.C, res.e, res.kappa)["d_h"]
    target = 1.2 * dh0
    rho = fe.density_from_levelset(n, phi_r)

    def jvec(name):
        g = ofoms.fom_grads(res.C, res.e, res.kappa, name)
        W = cell.W_from_tensor_grads(*g)
        return -cell.grad_phi_from_rho(n, phi_r, cell.grad_rho(n, MAT, res.X, W))

    j0 = jvec("B_voigt")
    j_vol = -cell.grad_phi_from_rho(n, phi_r, np.full(n ** 3, 1.0 / n ** 3)) / 0.5
    j_dh = jvec("d_h") / abs(target)
    viol = [(float(np.mean(rho)) - 0.5) / 0.5, (dh0 - target) / abs(target)]
    v = optim.hpm_velocity(n, j0, [j_vol, j_dh], viol)
    ref = ohj.hj_step(n, phi_r, v, cfl=0.5)
    # GPU
    with P.Context(n, MAT, precision=P.PHZ_FP64, rtol=1e-12) as ctx:
        out = optimise(ctx, MAT, phi0, "B_voigt", [("vol", 0.5), ("d_h", target)], max_iters=1)
    print("violations", out["violations"][0], "oracle", viol)
    assert np.allclose(out["violations"][0], viol, rtol=1e-8, atol=1e-12)
    print("level set error", relmax(out["phi"], ref))
    assert relmax(out["phi"], ref) < 1e-8


def test_short_run_restores_constraints(torch_cuda, P):
    """Twelve iterations at 16^3 from a volume fraction of 0.6 towards Vol = 0.5 with the hydrostatic
    coefficient held: the volume violation shrinks and the run stays finite."""
    from paper_2410_03148_amd.optimise import optimise
    n = 16
    say("short run", n)
    phi0 = synth.grf_levelset(n, seed=2410, solid_fraction=0.6)
    with P.Context(n, MAT, precision=P.PHZ_FP32_IR, rtol=1e-10) as ctx:
        ctx.set_levelset(phi0)
        ctx.solve()
        dh = P.foms(*ctx.effective())["d_h"]
        out = optimise(ctx, MAT, phi0, "B_voigt", [("vol", 0.5), ("d_h", dh)], max_iters=12)
    vol = [v[0] for v in out["violations"]]
    print("volume violations", [f"{x:.3f}" for x in vol])
    print("objective", [f"{x:.3e}" for x in out["J"]])
    assert all(np.isfinite(out["J"]))
    assert abs(vol[-1]) < 0.5 * abs(vol[0])


def test_warm_start_matches_cold_solve(P):
    """warm_start = 1: the solve on a moved interface starts from the last solution, reaches the same
    tensors as a solve from zero, in fewer iterations."""
    n = 16
    say("warm start", n)
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.5)
    phi2 = phi + 0.01 * np.cos(2 * np.pi * synth.node_coords(n)[0])
    with P.Context(n, MAT, precision=P.PHZ_FP32_IR, rtol=1e-10) as ctx:
        ctx.set_levelset(phi2)
        assert ctx.solve() == P.PHZ_OK
        cold = sum(ctx.stats()["iterations"])
        MHc, _ = ctx.effective_nd()
    with P.Context(n, MAT, precision=P.PHZ_FP32_IR, rtol=1e-10, warm_start=1) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        ctx.set_levelset(phi2)
        assert ctx.solve() == P.PHZ_OK
        warm = sum(ctx.stats()["iterations"])
        MHw, _ = ctx.effective_nd()
    print("iterations cold", cold, "warm", warm)
    assert warm < cold
    assert np.abs(MHw - MHc).max() / np.abs(MHc).max() < 1e-8


def _oracle_loop(n, phi0, target_dh, iters, cfl=0.5, gamma=0.5):
    """The optimisation loop composed from the oracle's steps in the driver's order: reinitialisation
    (subcell fix) at iterations 0, 5, ...; the direct solve; the objective's and constraints'
    sensitivities; the step control (objective weight halved when the largest violation stays above
    1e-3 without falling by 10% over five iterations, else grown by 1.1 up to 1); the projected
    velocity and the HJ step.  Returns the objective and violation histories and the level set."""
    phi = np.asarray(phi0, dtype=np.float64)
    Js, viols, tau = [], [], 1.0
    for q in range(iters):
        if q % 5 == 0:
            phi = optim.reinit(n, phi, steps=20, cfl=cfl, subcell=True)
        res = cell.homogenise(n, MAT, phi=phi)
        f = ofoms.foms(res.C, res.e, res.kappa)

        def jvec(name):
            W = cell.W_from_tensor_grads(*ofoms.fom_grads(res.C, res.e, res.kappa, name))
            return -cell.grad_phi_from_rho(n, phi, cell.grad_rho(n, MAT, res.X, W))

        rho = fe.density_from_levelset(n, phi)
        viol = [(float(np.mean(rho)) - 0.5) / 0.5, (f["d_h"] - target_dh) / abs(target_dh)]
        jc = [-cell.grad_phi_from_rho(n, phi, np.full(n ** 3, 1.0 / n ** 3)) / 0.5, jvec("d_h") / abs(target_dh)]
        Js.append(f["B_voigt"])
        viols.append(viol)
        if q >= 5:
            now, before = max(map(abs, viol)), max(map(abs, viols[-6]))
            tau = max(0.05, 0.5 * tau) if now > 1e-3 and now > 0.9 * before else min(1.0, 1.1 * tau)
        v = optim.hpm_velocity(n, jvec("B_voigt"), jc, viol, cfl=cfl, gamma=gamma, obj_weight=tau)
        phi = ohj.hj_step(n, phi, v, cfl=cfl)
    return Js, viols, phi


def test_seven_optimisation_iterations_vs_oracle(torch_cuda, P):
    """Seven iterations of the loop at 12^3 (two reinitialisations, the step control from iteration 5)
    against the oracle's loop: objective, violations and the final level set."""
    from paper_2410_03148_amd.optimise import optimise
    n = 12
    say("seven optimisation iterations", n)
    phi0 = synth.grf_levelset(n, seed=2411, solid_fraction=0.55)
    r0 = cell.homogenise(n, MAT, phi=optim.reinit(n, phi0, steps=20, cfl=0.5, subcell=True), want_x=False)
    target = 1.3 * ofoms.foms(r0.C, r0.e, r0.kappa)["d_h"]
    Js, viols, phi = _oracle_loop(n, phi0, target, 7)
    with P.Context(n, MAT, precision=P.PHZ_FP64, rtol=1e-12) as ctx:
        out = optimise(ctx, MAT, phi0, "B_voigt", [("vol", 0.5), ("d_h", target)], max_iters=7)
    print("objective", ["%.6e" % v for v in out["J"]], "oracle", ["%.6e" % v for v in Js])
    print("objective weights", out["tau"])
    assert relmax(out["J"], Js) < 1e-8
    assert np.allclose(out["violations"], viols, rtol=1e-7, atol=1e-10)
    print("level set error", relmax(out["phi"], phi))
    assert relmax(out["phi"], phi) < 1e-7
