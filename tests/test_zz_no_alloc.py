"""The entry point that allocates nothing (phz_hj_step_noalloc), for callers
that cannot allocate device memory: its output equals phz_hj_step's (the
context's step from the last backward) on two calls in a row, the second on
a smaller cell, through the C ABI; sizes beyond its scratch are refused."""
import ctypes as C
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
MAT = synth.material_workload()


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_noalloc_hj_step_matches_context_step():
    import torch
    import paper_2410_03148_amd as P
    assert torch.cuda.is_available()
    stream = torch.cuda.current_stream()
    for n in (12, 10):   # the second call on a smaller cell
        say("hj_step_noalloc vs phz_hj_step, n", n)
        phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.5)
        with P.Context(n, MAT, stream=stream.cuda_stream) as ctx:
            ctx.set_levelset(phi)
            assert ctx.solve() == P.PHZ_OK
            Cm, e, k = ctx.effective()
            _, (gC, ge, gk) = P.foms(Cm, e, k, grad_of="d_h")
            grho = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
            ctx.backward(gC, ge, gk, out_rho=grho)
            ref = ctx.hj_step(None, cfl=0.5)          # the context's entry point
        phi_d = torch.tensor(phi, device="cuda")
        out = torch.full((n ** 3,), np.nan, dtype=torch.float64, device="cuda")
        before = torch.cuda.memory_allocated()
        P.hj_step_noalloc(n, phi_d, grho, 0.5, out, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max(), np.abs(got - ref).max()
        assert np.abs(got - phi).max() > 0          # the step moved the level set
    # beyond the scratch: refused with a stated reason, nothing launched
    small = torch.zeros(8, dtype=torch.float64, device="cuda")
    small2 = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = P._lib.phz_hj_step_noalloc(130, C.c_void_p(small.data_ptr()), C.c_void_p(small.data_ptr()), 0.5,
                                    C.c_void_p(small2.data_ptr()), None)
    assert st == -1
    assert b"exceeds the scratch maximum" in P._lib.phz_last_error(None)
    assert P._lib.phz_hj_step_noalloc(8, C.c_void_p(small.data_ptr()), C.c_void_p(small.data_ptr()), 0.5,
                                      C.c_void_p(small.data_ptr()), None) == -1
