"""Central finite differences of the effective-tensor figures of merit at
the full 128^3 size (the differentiation configuration): directional
derivatives of d_h and g_h with respect to the element densities, from
phz_backward's gradient, against (J(rho + h d) - J(rho - h d)) / 2h of
solves to a true residual of 1e-12.

One element's perturbation is below what the tensors resolve at this size
(an element is 1/2,097,152 of the cell), so the check runs along whole
directions: a seeded random direction over all elements and stratified ones
over the solid, void and interface elements.  Each direction is
multiplicative in the density (d_e = rho_e times a factor of order one), so
a step of h changes every element's ersatz scale by a relative amount of
order h, and the densities stay inside [0, 1]: the random-field density is
mapped to [0.001, 0.999] first."""
import sys

import numpy as np
import pytest

import synth
from oracle import fe

pytestmark = pytest.mark.gpu
MAT = synth.material_workload()


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_grf128_gradient_central_differences():
    import torch
    import paper_2410_03148_amd as P
    assert torch.cuda.is_available()
    n = 128
    say("128^3 central differences of d_h and g_h")
    rho = 0.001 + 0.998 * fe.density_from_levelset(n, synth.grf_levelset(n, seed=2410, solid_fraction=0.5))
    rng = np.random.default_rng(2412)
    solid, void = rho > 0.99, rho < 0.01
    iface = ~(solid | void)
    assert solid.sum() > 1000 and void.sum() > 1000 and iface.sum() > 1000
    bump = 0.75 + 0.25 * rng.uniform(-1.0, 1.0, n ** 3)   # rho (1 + h bump) stays below 1
    dirs = {"random": rng.choice([-1.0, 1.0], n ** 3) * rho,
            "solid": np.where(solid, bump * rho, 0.0),
            "void": np.where(void, bump * rho, 0.0),
            "interface": np.where(iface, bump * rho, 0.0)}
    names = ("d_h", "g_h")
    stream = torch.cuda.current_stream().cuda_stream
    with P.Context(n, MAT, stream=stream, precision=P.PHZ_BF16X3_IR, rtol=1e-12, restart=12, vcycles_a=2,
                   inner_rtol=1e-4) as ctx:
        def J(r):
            ctx.set_density(torch.tensor(r, device="cuda"))
            assert ctx.solve() == P.PHZ_OK
            return P.foms(*ctx.effective())

        base = J(rho)
        grads = {}
        for name in names:
            f, (gC, ge, gk) = P.foms(*ctx.effective(), grad_of=name)
            grads[name] = ctx.backward(gC, ge, gk)
        worst = {}
        for dname, d in dirs.items():
            for h in (1e-3, 1e-4):
                fp, fm = J(rho + h * d), J(rho - h * d)
                for name in names:
                    an = float(grads[name] @ d)
                    fd = (fp[name] - fm[name]) / (2 * h)
                    err = abs(fd - an) / abs(an)
                    say(f"  {dname:9s} h {h:.0e} {name}: analytic {an:+.6e} fd {fd:+.6e} rel err {err:.2e} "
                        f"(|dJ| / |J| = {abs(an) * h / abs(base[name]):.1e})")
                    worst[dname, name] = min(worst.get((dname, name), np.inf), err)
    for key, err in worst.items():
        assert err <= 1e-4, (key, err)
