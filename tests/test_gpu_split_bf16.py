"""GPU parity of the split-BF16 element contraction (matrix cores) and of the
solve form that uses it, against the CPU oracle.

Error model of one product under the split x = hi + lo (hi = rne_bf16(x),
lo = rne_bf16(x - hi)): |x - hi - lo| <= 2^-18 |x|, so hi*hi + hi*lo + lo*hi
differs from K*x by at most about 3 * 2^-18 |K||x| (1.1e-5), plus float32
accumulation.  With the single term hi*hi the error is about 2 * 2^-9 |K||x|.
The tests bound the error of every output element by a multiple of
(|M| |x|)_i, the sum of the magnitudes of its terms.
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import cell, fe, krylov

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
MAT = synth.material_workload()
MND = fe.nondim_matrix(MAT)
TILES = {0: (8, 8, 4), 1: (16, 4, 4), 2: (16, 8, 2)}


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


def field_index(n, fields):
    d = np.arange(4 * n ** 3)
    return d[np.isin(d % 4, fields)]


def _blocks(P, n, s):
    K, _ = cell.assemble(n, s, MND)
    Sbar = krylov.schur_elementwise(n, s, MND)
    iu, ip = field_index(n, [0, 1, 2]), field_index(n, [3])
    return {P.OP_FULL: (K, 4, 4), P.OP_A: (K[iu][:, iu], 3, 3), P.OP_B: (K[ip][:, iu], 1, 3),
            P.OP_SBAR: (Sbar, 1, 1)}


@pytest.mark.parametrize("n,tiles", [(16, [0, 1, 2]), (24, [0])])
@pytest.mark.parametrize("terms,tol", [(3, 3e-5), (1, 6e-3)])
def test_elem_operator_blocks(torch_cuda, P, n, tiles, terms, tol):
    """Every block and tile against the oracle's assembled matrix, per output
    element relative to the magnitude sum of its terms."""
    torch = torch_cuda
    rho = synth.random_density(n, seed=40 + n)
    s = fe.ersatz_scale(rho, MAT.void_scale)
    blocks = _blocks(P, n, s)
    rng = np.random.default_rng(17)
    nn = n ** 3
    for tile in tiles:
        say("elem operator", n, "terms", terms, "tile", TILES[tile])
        with P.Context(n, MAT, precision=P.PHZ_BF16X3_IR, bf16_terms=terms, elem_tile=tile) as ctx:
            ctx.set_density(rho)
            for op, (M, fo, fi) in blocks.items():
                x = rng.standard_normal((nn * fi, 9))
                yref = M @ x
                bound = abs(M) @ abs(x)
                xd = torch.tensor(to_soa(x, nn, fi, 9), dtype=torch.float32, device="cuda").contiguous()
                yd = torch.zeros((fo, 9, nn), dtype=torch.float32, device="cuda")
                ctx.apply(op, 9, P.PHZ_BF16X3_IR, xd.data_ptr(), yd.data_ptr())
                torch.cuda.synchronize()
                y = from_soa(yd.cpu().double().numpy(), nn, fo, 9)
                err = (np.abs(y - yref) / np.maximum(bound, 1e-300)).max()
                print("op", op, "max error / term magnitude", err)
                assert err < tol, (op, tile, err)


def test_elem_operator_autotuned_matches_fixed_tile(torch_cuda, P):
    """The autotuned tile computes the same values as every fixed tile (each
    tile sums the same element products in the same corner order per node)."""
    torch = torch_cuda
    n = 16
    say("elem autotune", n)
    rho = synth.random_density(n, seed=3)
    nn = n ** 3
    x = np.random.default_rng(2).standard_normal((nn * 3, 9))
    xd = torch.tensor(to_soa(x, nn, 3, 9), dtype=torch.float32, device="cuda").contiguous()
    out = []
    for tile in (-1, 0, 1, 2):
        with P.Context(n, MAT, precision=P.PHZ_BF16X3_IR, elem_tile=tile) as ctx:
            ctx.set_density(rho)
            yd = torch.zeros((3, 9, nn), dtype=torch.float32, device="cuda")
            ctx.apply(P.OP_A, 9, P.PHZ_BF16X3_IR, xd.data_ptr(), yd.data_ptr())
            torch.cuda.synchronize()
            out.append(yd.cpu().numpy())
    for o in out[1:]:
        print("bitwise equal to the autotuned tile:", np.array_equal(o, out[0]))
        assert np.abs(o - out[0]).max() <= 1e-6 * np.abs(out[0]).max()


def test_elem_rejects_sizes_no_tile_divides(torch_cuda, P):
    torch = torch_cuda
    n = 12
    say("elem reject", n)
    with P.Context(n, MAT, precision=P.PHZ_BF16X3_IR) as ctx:
        ctx.set_density(np.ones(n ** 3))
        xd = torch.zeros((3, 9, n ** 3), dtype=torch.float32, device="cuda")
        yd = torch.zeros((3, 9, n ** 3), dtype=torch.float32, device="cuda")
        with pytest.raises(P.PiezoError) as ei:
            ctx.apply(P.OP_A, 9, P.PHZ_BF16X3_IR, xd.data_ptr(), yd.data_ptr())
        assert ei.value.status == -1


def _golden(name):
    return json.load(open(os.path.join(HERE, "golden", f"{name}.json")))


@pytest.mark.parametrize("outer,tile,pterms", [(1, 0, 1), (0, 2, 1), (1, -1, 1), (1, 0, 3), (0, -1, 3)])
def test_grf16_split_bf16_ir_vs_stored_oracle(torch_cuda, P, outer, tile, pterms):
    """The mixed form with matrix-core operators still meets the FP64 residual
    target, so the tensors match the oracle to the plain-FP64 bar.  A fixed
    tile puts every block on the matrix cores; tile -1 lets the timed choice
    keep a block on the float32 gather kernel.  The preconditioner's blocks
    run with one split product (the default) or three.  (The single-product
    GMRES operator, bf16_terms = 1, is checked as an operator only: its 2^-8
    error leaves some cells short of a 1e-10 residual.)"""
    g = _golden("grf16")
    say("grf16 bf16x3-ir outer", outer, "tile", tile, "preconditioner terms", pterms)
    with P.Context(16, MAT, precision=P.PHZ_BF16X3_IR, bf16_outer=outer, elem_tile=tile, rtol=1e-10,
                   bf16_terms_precond=pterms) as ctx:
        ctx.set_levelset(synth.grf_levelset(16, seed=2410, solid_fraction=0.5))
        status = ctx.solve()
        st = ctx.stats()
        print("status", status, "iterations", st["iterations"], "refinements", st["refinements"],
              "residual", max(st["true_residual"]), "tiles", st["elem_tile"])
        assert status == P.PHZ_OK
        MH, _ = ctx.effective_nd()
        assert max(st["true_residual"]) <= 1e-10
        assert relmax(MH, np.array(g["MH"])) < 1e-8
        if tile >= 0:
            assert st["elem_tile"][1:] == [tile] * 3
            assert st["elem_tile"][0] == (tile if outer else -1)
        else:
            assert all(t in (-1, 0, 1, 2) for t in st["elem_tile"])
            assert outer or st["elem_tile"][0] == -1


def test_laminate24_split_bf16_ir_closed_form(torch_cuda, P):
    """A size where only the 8x8x4 tile divides N (3 x 3 x 6 workgroups),
    against the closed-form laminate tensors."""
    from oracle import laminate
    n = 24
    say("laminate24 bf16x3-ir")
    rho = synth.laminate_density(n, axis=1, seed=23)
    s = fe.ersatz_scale(rho, MAT.void_scale).reshape(n, n, n)
    ref = laminate.laminate_effective(MND, s[0, :, 0], 1)
    with P.Context(n, MAT, precision=P.PHZ_BF16X3_IR, elem_tile=0, rtol=1e-10) as ctx:
        ctx.set_density(rho)
        assert ctx.solve() == P.PHZ_OK
        MH, _ = ctx.effective_nd()
        assert ctx.stats()["elem_tile"] == [0, 0, 0, 0]
        assert relmax(MH, ref) < 1e-8


@pytest.mark.parametrize("precision,batched", [("bf16x3", 1), ("fp32", 1), ("bf16x3", 0)])
def test_refinement_stall_fallback_forced(torch_cuda, P, precision, batched):
    """The refinement-stall fallback, forced from the host (ir_fallback = 2
    treats every refinement step as stalled): split-BF16 moves to float32
    kernels and then to a float64 inner GMRES, float32 directly to float64.
    The form that finished is reported, and the tensors still reach the
    stored oracle's to the plain-FP64 bar."""
    g = _golden("grf16")
    prec = {"bf16x3": P.PHZ_BF16X3_IR, "fp32": P.PHZ_FP32_IR}[precision]
    say("grf16 forced refinement fallback", precision, "batched", batched)
    phi = synth.grf_levelset(16, seed=2410, solid_fraction=0.5)
    # float cycles aiming at 1e-2 need several refinement steps, so both
    # fallbacks happen before the target is reached
    with P.Context(16, MAT, precision=prec, batched=batched, elem_tile=1, rtol=1e-10, ir_fallback=2,
                   inner_rtol=1e-2) as ctx:
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        st = ctx.stats()
        print("fallbacks", st["fallbacks"], "final", st["final_precision"], "refinements", st["refinements"])
        assert st["final_precision"] == P.PHZ_FP64
        per_block = 2 if prec == P.PHZ_BF16X3_IR else 1
        assert st["fallbacks"] == per_block * (1 if batched else 9)
        assert max(st["true_residual"]) <= 1e-10
        MH, _ = ctx.effective_nd()
        assert relmax(MH, np.array(g["MH"])) < 1e-8
        # the same context without the switch: no fallback, the configured form finishes
        ctx.set_options(ir_fallback=1)
        ctx.set_levelset(phi)
        assert ctx.solve() == P.PHZ_OK
        st = ctx.stats()
        assert st["fallbacks"] == 0 and st["final_precision"] == prec
        assert relmax(ctx.effective_nd()[0], np.array(g["MH"])) < 1e-8
