"""The Python binding on the GPU: device arguments of the wrong type are
refused before the library sees them, and the autograd form
(Homogenise, a torch.autograd.Function whose backward calls phz_backward)
backpropagates a figure of merit's gradient to the oracle's dJ/drho."""
import sys

import numpy as np
import pytest

import synth
from oracle import cell, fe, foms as ofoms

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


def test_device_arguments_are_checked_before_the_library(torch_cuda, P):
    torch = torch_cuda
    n = 8
    nn = n ** 3
    say("binding checks, n", n)
    with P.Context(n, MAT, stream=torch.cuda.current_stream().cuda_stream) as ctx:
        bad = [torch.zeros(nn, dtype=torch.float32, device="cuda"),
               torch.zeros(nn - 1, dtype=torch.float64, device="cuda"),
               torch.zeros(2 * nn, dtype=torch.float64, device="cuda")[::2]]
        for t in bad:
            for call in (ctx.set_density, ctx.set_levelset):
                with pytest.raises(ValueError):
                    call(t)
        rho = torch.tensor(synth.random_density(n, seed=3), device="cuda")
        ctx.set_density(rho)
        assert ctx.solve() == P.PHZ_OK
        with pytest.raises(ValueError):
            ctx.solution(out=torch.zeros(nn * 36, dtype=torch.float32, device="cuda"))
        with pytest.raises(ValueError):
            ctx.set_initial_guess(torch.zeros(nn * 36 - 1, dtype=torch.float64, device="cuda"))
        gC = np.eye(6)
        with pytest.raises(ValueError):
            ctx.backward(gC, out_rho=torch.zeros(nn, dtype=torch.float32, device="cuda"))
        with pytest.raises(ValueError):
            ctx.backward(gC, out_rho=torch.zeros(nn, dtype=torch.float64, device="cuda"),
                         out_phi=np.zeros(nn))
        # the accepted forms give the same numbers on the host and the device
        X = ctx.solution()
        Xd = ctx.solution(out=torch.empty(nn * 36, dtype=torch.float64, device="cuda"))
        assert np.array_equal(Xd.cpu().numpy().reshape(nn, 4, 9), X)
        g = ctx.backward(gC)
        gd, _ = ctx.backward(gC, out_rho=torch.empty(nn, dtype=torch.float64, device="cuda"))
        assert np.array_equal(gd.cpu().numpy(), g)


def _dh_torch(torch, C, e):
    S = torch.linalg.inv(C)
    d = e @ S
    return d[2, 0] + d[2, 1] + d[2, 2]


@pytest.mark.parametrize("n", [10, 12])
def test_homogenise_autograd_matches_oracle_gradient(torch_cuda, P, n):
    """d_h computed by torch from Homogenise's outputs, backpropagated through
    phz_backward, against the oracle: the direct solve's X, W = dd_h/dM^H by
    complex step, dJ/drho_e = (1 - eps_v) <W, G_e>."""
    torch = torch_cuda
    say("Homogenise autograd, n", n)
    rho_np = fe.density_from_levelset(n, synth.grf_levelset(n, seed=2410, solid_fraction=0.5))
    ref = cell.homogenise(n, MAT, rho=rho_np)
    gC, ge, gk = ofoms.fom_grads(ref.C, ref.e, ref.kappa, "d_h")
    g_ref = cell.grad_rho(n, MAT, ref.X, cell.W_from_tensor_grads(gC, ge, gk))
    H = P.Homogenise
    with P.Context(n, MAT, stream=torch.cuda.current_stream().cuda_stream) as ctx:
        rho = torch.tensor(rho_np, device="cuda", requires_grad=True)
        C, e, k = H.apply(rho, ctx)
        dh = _dh_torch(torch, C, e)
        assert abs(dh.item() / ofoms.foms(ref.C, ref.e, ref.kappa)["d_h"] - 1) < 1e-8
        dh.backward()
        assert rho.grad.device.type == "cuda" and rho.grad.dtype == torch.float64
        g = rho.grad.cpu().numpy()
        err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
        say("  grad rel err", err)
        assert err < 1e-7
        # host densities give the same gradient on the host
        rho_h = torch.tensor(rho_np, requires_grad=True)
        C2, e2, k2 = H.apply(rho_h, ctx)
        _dh_torch(torch, C2, e2).backward()
        assert rho_h.grad.device.type == "cpu"
        assert np.abs(rho_h.grad.numpy() - g).max() <= 1e-12 * np.abs(g).max()
        # a backward after the context moved on is refused
        rho3 = torch.tensor(rho_np, device="cuda", requires_grad=True)
        C3, e3, k3 = H.apply(rho3, ctx)
        ctx.set_density(torch.tensor(np.clip(rho_np * 0.9, 0, 1), device="cuda"))
        with pytest.raises(RuntimeError):
            _dh_torch(torch, C3, e3).backward()


def test_caller_allocator_receives_every_workspace(torch_cuda, P):
    """phz_create's allocator: with PyTorch's caching allocator behind it, the
    context's workspaces come from torch (counted), every one is returned at
    destroy, and the tensors equal those of a context on hipMalloc."""
    torch = torch_cuda
    n = 16
    say("caller allocator, n", n)
    phi = torch.tensor(synth.grf_levelset(n, seed=2410, solid_fraction=0.5), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    # FP64 runs the same kernels in the same order whatever the memory (no
    # timed kernel choice), so the tensors agree bit for bit; the split-BF16
    # form times its kernel choices per context, so it agrees to its bar
    for prec in (P.PHZ_FP64, P.PHZ_BF16X3_IR):
        for name, alloc in (("hip", None), ("torch", P.TorchAllocator())):
            before = torch.cuda.memory_allocated()
            with P.Context(n, MAT, stream=stream, allocator=alloc, precision=prec) as ctx:
                ctx.set_levelset(phi)
                assert ctx.solve() == P.PHZ_OK
                out[prec, name] = ctx.effective_nd()[0]
                if alloc is not None:
                    assert alloc.allocs > 20 and alloc.frees < alloc.allocs
                    assert torch.cuda.memory_allocated() - before >= alloc.bytes_live > 0
            if alloc is not None:
                assert alloc.frees == alloc.allocs and alloc.bytes_live == 0
                assert torch.cuda.memory_allocated() == before
    assert np.array_equal(out[P.PHZ_FP64, "hip"], out[P.PHZ_FP64, "torch"])
    a, b = out[P.PHZ_BF16X3_IR, "hip"], out[P.PHZ_BF16X3_IR, "torch"]
    assert np.abs(a - b).max() <= 1e-8 * np.abs(a).max()
    # an allocator that fails makes creation (or a later call) report out of memory, not crash
    failing = P.TorchAllocator()
    failing._do_alloc_orig = failing._do_alloc
    calls = {"n": 0}

    def refuse_late(nbytes, stream_, user):
        calls["n"] += 1
        return None if calls["n"] > 3 else failing._do_alloc_orig(nbytes, stream_, user)

    failing._alloc = P.ALLOC_FN(refuse_late)
    failing.struct.alloc = failing._alloc
    with pytest.raises(P.PiezoError) as ei:
        P.Context(n, MAT, stream=stream, allocator=failing)
    assert ei.value.status == -4
    assert failing.bytes_live == 0
