"""The Arnoldi orthogonalisation of the GMRES step (classical Gram-Schmidt
with a second pass only where the first leaves components above
reorth_tol): the new vector stays orthogonal to the basis to a few units of
roundoff (the invariant |V^T v| small, P12), a nearly dependent vector takes
the second pass and a well-conditioned one does not, and whole solves with
the selective rule reach the same tensors in the same iteration counts as
with the second pass always."""
import json
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
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


def _basis(n, nvec, rng):
    """nvec vectors [4][9][n^3], orthonormal per load (over the four fields)."""
    nn = n ** 3
    V = np.zeros((nvec, 4, 9, nn))
    for k in range(9):
        q, _ = np.linalg.qr(rng.standard_normal((4 * nn, nvec)))
        V[:, :, k, :] = q.T.reshape(nvec, 4, nn)
    return V


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_orthogonalisation_invariant_and_second_pass_rule(torch_cuda, P, prec):
    torch = torch_cuda
    n, nvec = 16, 7
    say("Arnoldi orthogonalisation", prec, "n", n, "basis", nvec)
    rng = np.random.default_rng(5)
    code = {"fp32": P.PHZ_FP32_IR, "fp64": P.PHZ_FP64}[prec]
    dt = {"fp32": (np.float32, torch.float32), "fp64": (np.float64, torch.float64)}[prec]
    u = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53}[prec]
    V = _basis(n, nvec, rng).astype(dt[0])
    nn = n ** 3
    # loads 0..4: random vectors; loads 5..8: the basis plus a 1e-4 (fp32)
    # or 1e-9 (fp64) perturbation, so the first pass cancels
    eps = 1e-4 if prec == "fp32" else 1e-9
    w = rng.standard_normal((4, 9, nn))
    for k in range(5, 9):
        c = rng.standard_normal(nvec)
        w[:, k, :] = np.einsum("i,ifn->fn", c, V[:, :, k, :].astype(np.float64)) + eps * w[:, k, :] / np.sqrt(4 * nn)
    w = w.astype(dt[0])
    Vd = torch.tensor(V, device="cuda")
    for tol, expect in ((0.0, [0] * 5 + [1] * 4), (-1.0, [1] * 9)):
        with P.Context(n, MAT, stream=torch.cuda.current_stream().cuda_stream, reorth_tol=tol) as ctx:
            wd = torch.tensor(w, device="cuda")
            h, n2, second = ctx.orthogonalize(code, nvec, Vd.data_ptr(), wd.data_ptr())
            w2 = wd.cpu().numpy().astype(np.float64)
        assert list(second) == expect, (tol, second)
        V64 = V.astype(np.float64)
        for k in range(9):
            wk = w[:, k, :].astype(np.float64).ravel()
            Vk = V64[:, :, k, :].reshape(nvec, -1)
            # coefficients: the exact projection of the input onto the basis
            assert np.allclose(h[:, k], Vk @ wk, rtol=0, atol=64 * u * np.linalg.norm(wk))
            r = w2[:, k, :].ravel()
            assert abs(n2[k] - r @ r) <= 1e-12 * (r @ r) + 64 * u * (r @ r)
            # the invariant: the result is orthogonal to the basis to a few
            # units of roundoff of the basis's type, relative to its own norm
            assert np.abs(Vk @ r).max() <= 64 * u * np.linalg.norm(r), (k, np.abs(Vk @ r).max() / np.linalg.norm(r))


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
def test_selective_reorthogonalisation_solves(torch_cuda, P, prec):
    """grf16: the selective rule against the second pass always."""
    g = json.load(open(os.path.join(HERE, "golden", "grf16.json")))
    code = {"bf16x3": P.PHZ_BF16X3_IR, "fp64": P.PHZ_FP64}[prec]
    phi = synth.grf_levelset(16, seed=2410, solid_fraction=0.5)
    out = {}
    for tol in (0.0, -1.0):
        say("grf16 solve", prec, "reorth_tol", tol)
        with P.Context(16, MAT, precision=code, elem_tile=1, coarse_kernel=0, rtol=1e-10, reorth_tol=tol,
                       restart=12) as ctx:
            ctx.set_levelset(phi)
            assert ctx.solve() == P.PHZ_OK
            st = ctx.stats()
            MH, _ = ctx.effective_nd()
            out[tol] = (MH, st)
            print("reorth_tol", tol, "iterations", st["iterations"], "second passes", st["reorth_passes"])
            assert np.abs(MH - np.array(g["MH"])).max() < 1e-8 * np.abs(np.array(g["MH"])).max()
    (Ms, ss), (Ma, sa) = out[0.0], out[-1.0]
    assert sa["reorth_passes"] == sum(sa["iterations"])
    assert ss["reorth_passes"] <= sa["reorth_passes"]
    assert max(ss["iterations"]) <= max(sa["iterations"]) + 1
    assert np.abs(Ms - Ma).max() <= 1e-9 * np.abs(Ma).max()
