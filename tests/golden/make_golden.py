"""Write the stored oracle outputs used by the GPU parity tests.

Calls only oracle/ and synth/ (never the GPU library).  Run from the repo
root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import cell, fe, foms, tricg  # noqa: E402


def case(name, n, phi=None, rho=None, mat=None, smoothing="element"):
    mat = mat or synth.material_workload()
    t = time.perf_counter()
    r = cell.homogenise(n, mat, phi=phi, rho=rho, want_x=False, smoothing=smoothing)
    dt = time.perf_counter() - t
    out = {
        "name": name, "n": n, "oracle_seconds": dt,
        "MH": r.MH.tolist(), "MH_energy": r.MH_energy.tolist(),
        "C": r.C.tolist(), "e": r.e.tolist(), "kappa": r.kappa.tolist(),
        "foms": {k: float(v) for k, v in foms.foms(r.C, r.e, r.kappa).items()},
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, f"{dt:.1f}s")


def tricg_counts(cases, rtol=1e-10):
    """TriCG iterations per load (exact block inverses, zero-block start, restarts) on the golden cells."""
    mat = synth.material_workload()
    M = fe.nondim_matrix(mat)
    out = {"rtol": rtol}
    for name, n, phi in cases:
        t = time.perf_counter()
        s = fe.ersatz_scale(fe.density_from_levelset(n, phi), mat.void_scale)
        K, F = cell.assemble(n, s, M)
        X, its = tricg.solve_tricg(K, -F, rtol=rtol)
        MH = cell.effective_flux(n, s, M, X)
        out[name] = {"iterations": its, "MH": MH.tolist()}
        print(name, "tricg", its, f"{time.perf_counter() - t:.1f}s")
    with open(os.path.join(HERE, "tricg16.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    # 16^3 void sphere of radius 0.3 (signed distance), workload material
    case("sphere16", 16, phi=synth.sphere_levelset(16))
    # 16^3 Gaussian random field, seed 2410, 50% solid
    case("grf16", 16, phi=synth.grf_levelset(16, seed=2410, solid_fraction=0.5))
    # the same two cells with the smoothing at the quadrature points
    case("sphere16_qp", 16, phi=synth.sphere_levelset(16), smoothing="qp")
    case("grf16_qp", 16, phi=synth.grf_levelset(16, seed=2410, solid_fraction=0.5), smoothing="qp")
    tricg_counts([("grf16", 16, synth.grf_levelset(16, seed=2410, solid_fraction=0.5)),
                  ("sphere16", 16, synth.sphere_levelset(16))])
