"""Benchmark: 128^3 nine-load periodic piezoelectric homogenisation on one MI355X.

One step = the whole hot path on device-resident input: level set -> element
scales -> load vectors -> preconditioner set-up (Galerkin multigrid,
Chebyshev bounds, coarsest factorisation) -> SCP-GMRES for all nine loads
(one 9-column block; by default the fine-level operators as split-BF16
element contractions on the matrix cores with FP32 vectors and Krylov basis,
inside FP64 iterative refinement to a true FP64 residual of 1e-10) ->
effective tensors -> figures of merit -> density sensitivities of d_h -> one
Hamilton-Jacobi step of the level set.

Prints one JSON line: the throughput, the dominant kernel against its
roofline, the outer operator's bandwidth, the other solve forms on the same
cell (FP32 operators in FP64 refinement, FP64 batched, FP64 one load at a
time) and the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic work per node of a fine-level operator launch, by timing label
# (fine_<block>_k<K>_<f32|f64>[_cheby] for the direct gather kernels,
# tiled_<block>_k9_f32[_cheby] for the LDS-tiled gather, and
# elem_<block>_k<K>_bf16x<T>[_cheby] for the element contraction on MFMA).
# Gather form: flops = 2 (64 FO FI + 27 FO FI K) (block build + apply).
# Element form: T split products of the element block, 2 T (8 FO)(8 FI) K per
# element (one element per node).  Bytes, both forms: the input columns x
# (FI K), the scale s, the output y (FO K), plus the y_in read (FO K) of the
# blocks that run as residual updates (A, B, S: y = y_in - A x); the full
# operator runs as y = A x.  The fused Chebyshev step adds the Jacobi block
# (FO^2), the iterate read and write (2 FO K) and the new correction (FO K),
# with 2 FO^2 K + 4 FO K flops.
OPS = {"full": (4, 4), "A": (3, 3), "B": (1, 3), "S": (1, 1)}


def per_node(name):
    parts = name.split("_")
    form, op, k, prec = parts[0], parts[1], parts[2], parts[3]
    cheby = len(parts) > 4 and parts[4] == "cheby"
    fo, fi = OPS[op]
    K = int(k[1:])
    if form == "elem":
        terms = int(prec[len("bf16x"):])
        w = 4
        flops = 2 * terms * (8 * fo) * (8 * fi) * K
    else:
        w = 4 if prec == "f32" else 8
        flops = 2 * (64 * fo * fi + 27 * fo * fi * K)
    words = fi * K + 1 + fo * K + (fo * K if op != "full" else 0)
    if cheby:
        flops += 2 * fo * fo * K + 4 * fo * K
        words += fo * fo + 3 * fo * K
    return flops, words * w, prec


def measured_traffic(label, tile=None):
    """HBM bytes per launch of a timing label from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy kernel), or None
    when the kernel source has changed since the counters were taken or, for
    the element contraction, the run used another workgroup tile."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec["kernels"].get(label)
    if k is None or k.get("tile") != tile:
        return None
    with open(os.path.join(ROOT, k["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != k["source_sha256"]:
            return None
    return k["bytes_per_launch"]


def _traffic_label(name, grid):
    """Timing label of a counted kernel (None for kernels the record does not list) and the element tile."""
    import re
    # (the counter files may keep the element kernels' names mangled: their
    # bf16 operand type defeats the demangler)
    mm = re.search(r"k_elem_mfmaI((?:L[ib]\d+E)+)E", name)
    if mm:
        vals = [("true" if v == "1" else "false") if t == "b" else v for t, v in re.findall(r"L([ib])(\d+)E", mm[1])]
        name = "k_elem_mfma<" + ", ".join(vals) + ">"
    m = re.search(r"k_elem_mfma<(\d+), (\d+), 9, (\d+), (true|false), (\d+), (\d+), (\d+)>", name)
    if m:
        fo, fi, terms, cheby = int(m[1]), int(m[2]), int(m[3]), m[4] == "true"
        block = {(4, 4): "full", (3, 3): "A", (1, 3): "B", (1, 1): "S"}[(fo, fi)]
        tile = {(8, 8, 4): 0, (16, 4, 4): 1, (16, 8, 2): 2}[(int(m[5]), int(m[6]), int(m[7]))]
        return f"elem_{block}_k9_bf16x{terms}" + ("_cheby" if cheby else ""), tile
    m = re.search(r"k_stencil_tiled<(\d), (true|false), false, true>", name)
    if m:
        n = round(grid ** (1 / 3))
        return f"coarse_tiledbf_{'A' if m[1] == '3' else 'S'}_f32" + ("_cheby" if m[2] == "true" else "") + f"@{n}", None
    m = re.search(r"k_fine_tiled<1, 1, 9, (true|false)>", name)
    if m:
        return "tiled_S_k9_f32" + ("_cheby" if m[1] == "true" else ""), None
    m = re.search(r"k_fine_apply<double, (\d), (\d), 1,", name)
    if m:
        return {"3": "fine_A_k1_f64", "1": "fine_S_k1_f64"}[m[1]], None
    return None, None


def traffic_summary(fetch_dir, write_dir, path=None):
    """HBM bytes per launch from two rocprofv3 --pmc runs of the bench workload with --copy-calibration
    (FETCH_SIZE in one, WRITE_SIZE in the other): each counter is scaled by what it reads for the plain copy
    kernel (y = -x) of known size.  Updates the measured fields and source hashes of the kernels that
    profiles/hbm_traffic.json lists and prints its table rows."""
    import csv, glob, hashlib
    def load(d, counter):
        rows = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as f:
                rows += [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
        return rows
    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    path = path or os.path.join(ROOT, "profiles", "hbm_traffic.json")
    with open(path) as f:
        rec = json.load(f)
    cal = rec["calibration"]
    copy_f = [float(r["Counter_Value"]) for r in fetch if "neg" in r["Kernel_Name"]]
    copy_w = [float(r["Counter_Value"]) for r in write if "neg" in r["Kernel_Name"]]
    cal["copy_fetch_kib"], cal["copy_write_kib"] = float(np.mean(copy_f)), float(np.mean(copy_w))
    cal["fetch_bytes_per_kib"] = cal["copy_bytes_read"] / cal["copy_fetch_kib"]
    cal["write_bytes_per_kib"] = cal["copy_bytes_written"] / cal["copy_write_kib"]
    def per_label(rows):
        acc = {}
        for r in rows:
            label, tile = _traffic_label(r["Kernel_Name"], int(r["Grid_Size"]))
            if label is not None:
                acc.setdefault((label, tile), []).append(float(r["Counter_Value"]))
        return acc
    pf, pw = per_label(fetch), per_label(write)
    out = []
    for label, k in rec["kernels"].items():
        key = (label, k.get("tile"))
        if key not in pf or key not in pw:
            continue
        with open(os.path.join(ROOT, k["source"]), "rb") as f:
            k["source_sha256"] = hashlib.sha256(f.read()).hexdigest()
        k["dispatches"] = len(pf[key])
        k["fetch_kib"], k["write_kib"] = float(np.mean(pf[key])), float(np.mean(pw[key]))
        k["fetch_bytes"] = round(k["fetch_kib"] * cal["fetch_bytes_per_kib"])
        k["write_bytes"] = round(k["write_kib"] * cal["write_bytes_per_kib"])
        k["bytes_per_launch"] = k["fetch_bytes"] + k["write_bytes"]
        out.append(f"| {label} | `{k['kernel']}` | {k['dispatches']} | {k['fetch_kib']:,.0f} | {k['write_kib']:,.0f} | "
                   f"{k['bytes_per_launch'] / 1e6:,.1f} MB | {k['algorithmic_bytes'] / 1e6:,.1f} MB | "
                   f"{k['bytes_per_launch'] / k['algorithmic_bytes']:.2f} |")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print("\n".join(out))
    return out


def measure_peaks(torch, dev):
    """Achievable rates on this GPU, to read the roofline fractions against (device library kernels, not the
    solver's): HBM copy, read-only and write-only bandwidth over 4 GiB buffers (far above the 256 MB last-level
    cache), and dense GEMM throughput in bf16, fp32 and fp64 at n = 8192.  Medians of 10 timed launches after
    3 warm-ups, timed with HIP events on the current stream."""
    def timed(fn, reps=10, warm=3):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(); fn(); b.record(); torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return float(np.median(ts))
    out = {}
    nb = 4 << 30
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    out["copy_GBps"] = 2 * nb / timed(lambda: dst.copy_(src)) / 1e9
    red = torch.empty((), dtype=torch.float32, device=dev)
    out["read_GBps"] = nb / timed(lambda: torch.sum(src, dim=0, out=red)) / 1e9
    out["write_GBps"] = nb / timed(lambda: dst.fill_(1.0)) / 1e9
    del src, dst
    n = 8192
    for dt, name in ((torch.bfloat16, "gemm_bf16_TFLOPs"), (torch.float32, "gemm_fp32_TFLOPs"),
                     (torch.float64, "gemm_fp64_TFLOPs")):
        a = torch.randn((n, n), dtype=dt, device=dev)
        b = torch.randn((n, n), dtype=dt, device=dev).contiguous()
        c = torch.empty((n, n), dtype=dt, device=dev)
        out[name] = 2 * n ** 3 / timed(lambda: torch.matmul(a, b, out=c)) / 1e12
        del a, b, c
    out["published"] = {"hbm_GBps": 8000, "bf16_TFLOPs": 2500, "fp32_TFLOPs": 157.3, "fp64_TFLOPs": 78.6}
    return out


_CPU_ENV = dict(OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")


def _cpu_child(code, timeout=3600):
    """Run oracle timing code in a single-threaded child process; returns its
    last stdout line parsed as JSON."""
    env = dict(os.environ, **_CPU_ENV)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=timeout)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


def cpu_solve_seconds(n, reps):
    """Wall seconds of the oracle's whole homogenisation (assembly, sparse LU,
    nine solves, reduction) of the n^3 random-field cell, one per repetition."""
    code = (
        "import time,sys,json; sys.path.insert(0, %r)\n"
        "import synth\nfrom oracle import cell\n"
        "m = synth.material_workload()\n"
        "phi = synth.grf_levelset(%d, seed=2410, solid_fraction=0.3)\n"
        "ts = []\n"
        "for _ in range(%d):\n"
        "    t = time.perf_counter(); cell.homogenise(%d, m, phi=phi, want_x=False)\n"
        "    ts.append(time.perf_counter() - t)\n"
        "print(json.dumps(ts))\n" % (ROOT, n, reps, n))
    return _cpu_child(code)


def cpu_apply_seconds(n, reps, csr=False):
    """Wall seconds of one oracle operator apply K X on nine columns at n^3:
    the matrix-free element form (oracle.fullsize), or with csr=True the
    assembled CSR matrix (oracle.cell.assemble, assembly not timed).  The
    second value is the CSR's stored nonzeros (0 for the element form)."""
    code = (
        "import time,sys,json; sys.path.insert(0, %r)\n"
        "import numpy as np\nimport synth\nfrom oracle import cell, fe, fullsize\n"
        "m = synth.material_workload(); M = fe.nondim_matrix(m); n = %d\n"
        "s = fe.ersatz_scale(fe.density_from_levelset(n, synth.grf_levelset(n, seed=2410, solid_fraction=0.3)),"
        " m.void_scale)\n"
        "X = np.random.default_rng(0).standard_normal((4 * n ** 3, 9))\n"
        "nnz = 0\n"
        "if %r:\n"
        "    K, _ = cell.assemble(n, s, M); nnz = int(K.nnz)\n"
        "    f = lambda: K @ X\n"
        "else:\n"
        "    f = lambda: fullsize.element_apply(n, s, M, X)\n"
        "ts = []\n"
        "for _ in range(%d):\n"
        "    t = time.perf_counter(); f(); ts.append(time.perf_counter() - t)\n"
        "print(json.dumps([ts, nnz]))\n" % (ROOT, n, bool(csr), reps))
    return _cpu_child(code)


def cpu_baseline(n, iterations, fine_launches_per_iteration):
    """The CPU oracle on bounded samples of the workload, timed on this host's
    cores in single-threaded children: whole homogenisations at 12^3 and 16^3
    (median of 3; their ratio gives the growth exponent of the direct solve),
    the assembled CSR operator applied to nine columns at 32^3 (median of 3,
    assembly not timed) and the matrix-free operator apply at the full size
    (once).  No n^3 oracle solve is run (a direct one would take hours); two
    labelled estimates stand in for it, and `value` is the one more
    favourable to the CPU:
      direct: the 16^3 time grown to n^3 with the measured exponent;
      iterative: the CSR apply grown to n^3 in proportion to its nonzeros
      (linear in the cell's nodes), times the GPU solve's operator-apply count
      (iterations x fine-level applies per iteration): the oracle's fastest
      operator running the GPU path's iteration count."""
    t12 = float(np.median(cpu_solve_seconds(12, 3)))
    t16 = float(np.median(cpu_solve_seconds(16, 3)))
    p = float(np.log(t16 / t12) / np.log(16 ** 3 / 12 ** 3))
    ts, nnz32 = cpu_apply_seconds(32, 3, csr=True)
    t_csr32 = float(np.median(ts))
    t_csr = t_csr32 * (n / 32) ** 3
    ts, _ = cpu_apply_seconds(n, 1)
    t_apply = float(ts[0])
    t_direct = t16 * (n ** 3 / 16 ** 3) ** p
    t_iter = min(t_csr, t_apply) * iterations * fine_launches_per_iteration
    best = min(t_direct, t_iter)
    return {
        "value": 1.0 / best, "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle (numpy/scipy, one thread) timed on this host: nine-load homogenisations (sparse LU) at "
                   f"12^3 {t12:.2f} s and 16^3 {t16:.2f} s (median of 3), growth exponent {p:.2f} in dofs; CSR "
                   f"operator on nine columns at 32^3 {t_csr32 * 1e3:.1f} ms ({nnz32} nonzeros, median of 3), "
                   f"{t_csr:.2f} s grown to {n}^3; matrix-free apply at {n}^3 {t_apply:.2f} s.  value is an "
                   f"estimate, the more favourable to the CPU of: direct {t_direct:.0f} s per {n}^3 solve (16^3 "
                   f"grown with the exponent) and iterative {t_iter:.0f} s ({iterations} iterations x "
                   f"{fine_launches_per_iteration:.1f} operator applies per iteration x the faster apply)"),
        "measured": {"solve_s_12": t12, "solve_s_16": t16, "exponent": p, "apply9_csr_s_32": t_csr32,
                     "csr_nnz_32": nnz32, f"apply9_element_s_{n}": t_apply},
        "estimates_s": {"direct": t_direct, "iterative": t_iter, f"apply9_csr_s_{n}_grown": t_csr},
        "host_cores_available": len(os.sched_getaffinity(0)),
    }


def cpu_sweep():
    """Longer oracle timings for the record (a few minutes, about 30 GB of host
    memory): direct solves at 12^3 to 24^3, CSR applies at 32^3 and 64^3 and
    matrix-free applies at 64^3 and 128^3 (a 128^3 CSR matrix would hold 2^31
    element entries before summation, about 100 GB to assemble)."""
    rows = {}
    for n, reps in ((12, 3), (16, 3), (20, 1), (24, 1)):
        rows[f"solve_s_{n}"] = cpu_solve_seconds(n, reps)
        print(f"[bench] cpu sweep: solve {n}^3 {rows[f'solve_s_{n}']}", file=sys.stderr, flush=True)
    for n in (64, 128):
        rows[f"apply9_element_s_{n}"] = cpu_apply_seconds(n, 3)[0]
        print(f"[bench] cpu sweep: element apply {n}^3 {rows[f'apply9_element_s_{n}']}", file=sys.stderr, flush=True)
    for n in (32, 64):
        ts, nnz = cpu_apply_seconds(n, 3, csr=True)
        rows[f"apply9_csr_s_{n}"] = ts
        rows[f"csr_nnz_{n}"] = nnz
        print(f"[bench] cpu sweep: CSR apply {n}^3 {ts} (nnz {nnz})", file=sys.stderr, flush=True)
    med = {k: float(np.median(v)) for k, v in rows.items() if k.startswith("solve_s_")}
    for k, v in list(rows.items()):
        if k.startswith("apply9_"):
            med[k] = float(np.median(v))
    solves = {k: v for k, v in med.items() if k.startswith("solve_s_")}
    ns = np.array([int(k.split("_")[-1]) for k in solves])
    ts = np.array(list(solves.values()))
    slope = float(np.polyfit(np.log(ns ** 3.0), np.log(ts), 1)[0])
    return {"study": "CPU oracle timings, one thread", "cpu": _cpu_model(), "host_cores_available":
            len(os.sched_getaffinity(0)), "raw": rows, "median_s": med,
            "solve_exponent_fit_12_to_24": slope}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def solver_study(P, torch, synth, mat, dev, only=None):
    """Outer GMRES iterations, inner conjugate-gradient iterations per block
    map and times of the preconditioner forms (the analogue of the paper's
    Table 1 on one GPU: multigrid instead of algebraic multigrid inside the
    block maps, all nine loads batched; load 0 is the eps^11 load the paper
    reports)."""
    forms = [("SCP-GMRES", P.PHZ_SOLVER_SCP, 0, None), ("SCP-GMRES", P.PHZ_SOLVER_SCP, 1, 1e-8),
             ("SCP-GMRES", P.PHZ_SOLVER_SCP, 1, 1e-4), ("SCP-GMRES", P.PHZ_SOLVER_SCP, 1, 1e-2),
             ("DBP-GMRES", P.PHZ_SOLVER_DBP, 0, None), ("DBP-GMRES", P.PHZ_SOLVER_DBP, 1, 1e-8),
             ("DBP-GMRES", P.PHZ_SOLVER_DBP, 1, 1e-4), ("DBP-GMRES", P.PHZ_SOLVER_DBP, 1, 1e-2),
             ("TriCG", P.PHZ_SOLVER_TRICG, 1, 1e-8), ("TriCG", P.PHZ_SOLVER_TRICG, 1, 1e-4),
             ("TriCG", P.PHZ_SOLVER_TRICG, 1, 1e-2)]
    if only:
        forms = [f for f in forms if f[0] in only]
    rows = []
    for n in (64, 128):
        phi = torch.tensor(synth.paper_levelset(n), device=dev)
        for name, solver, inner, eps in forms:
            opts = dict(precision=P.PHZ_FP64, solver=solver, inner=inner, rtol=1e-8, restart=30, vcycles_a=2,
                        max_iters=600)
            if eps is not None:
                opts["inner_eps"] = eps
            with P.Context(n, mat, stream=torch.cuda.current_stream().cuda_stream, **opts) as ctx:
                ctx.set_levelset(phi)
                ctx.solve()
                ctx.set_levelset(phi)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                status = ctx.solve()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                st = ctx.stats()
            calls = st["inner_calls"]
            rows.append({"n": n, "dofs": 4 * n ** 3, "solver": name,
                         "block_maps": "V-cycles (A 2, potential 1)" if not inner else f"CG to {eps:g}",
                         "status": status, "outer_iters_load0": st["iterations"][0],
                         "cycles_max": max(st["restarts"]) if solver == P.PHZ_SOLVER_TRICG else None,
                         "outer_iters_max": max(st["iterations"]),
                         "cg_iters_per_A_map": st["inner_iters"][0] / calls[0] if calls[0] else None,
                         "cg_iters_per_potential_map": st["inner_iters"][1] / calls[1] if calls[1] else None,
                         "time_s": dt, "setup_ms": st["setup_ms"], "true_residual_max": max(st["true_residual"])})
            print(f"[bench] {rows[-1]}", file=sys.stderr, flush=True)
    return {"study": "preconditioner forms, float64, rtol 1e-8, geometry -prod cos(2 pi x_i) - 0.2, nine loads",
            "rows": rows}


# The paper's optimisation problems: (objective, constraints, what the paper reports for the result).
# bvoigt: its worked example (Sec. 3.1); dh_a/b/c: Eq. (optim prob 2) with the three stiffness targets
# of its Table 3, whose volume target is not printed: it is read as the volume that Table 3 reports.
OPT_PROBLEMS = {
    "bvoigt": ("B_voigt", [("vol", 0.5), ("d_h", 2.9e-10)],
               "converges after about 180 iterations at 100^3; about 9x the base d_h, 43x the base g_h and 7x "
               "the base k_h at about 20% of the base B_Voigt (Sec. 3.1)"),
    "breuss": ("B_reuss", [("vol", 0.5), ("d_h", 2.9e-10)],
               "about 9x the base d_h, 50x the base g_h, 7x the base k_h, at about 11% of the base B_Reuss "
               "(Sec. 3.1)"),
    "dh_a": ("d_h", [("vol", 0.599), ("C_zzzz", 5e9)],
             "Table 3 (a): d_h 3.5e-10, B_Voigt 1.75e10, B_Reuss 4.85e9, g_h 0.197, k_h 0.578"),
    "dh_b": ("d_h", [("vol", 0.586), ("C_zzzz", 2.5e9)],
             "Table 3 (b): d_h 3.89e-10, B_Voigt 1.63e10, B_Reuss 2.45e9, g_h 0.357, k_h 0.584"),
    "dh_c": ("d_h", [("vol", 0.581), ("C_zzzz", 1e9)],
             "Table 3 (c): d_h 4.45e-10, B_Voigt 1.58e10, B_Reuss 9.77e8, g_h 0.889, k_h 0.622"),
}


def optimisation_run(P, torch, synth, n, max_iters, precision, problem="bvoigt", reinit_every=5, smoothing="element",
                     step_control=True):
    """One of the paper's optimisation problems (Sec. 2.3, Sec. 2.6): z-poled PZT-5A, from the level set
    -prod cos(2 pi x_i) - 0.2 reinitialised, reinitialisation every five iterations, the paper's
    stopping rule.  The paper runs them on a 100^3 mesh; the multigrid hierarchy here needs N = m 2^k
    with m <= 10, so the nearest cell is 96^3.  Reports the wall time per iteration and per phase and
    the figures of merit of the result."""
    from paper_2410_03148_amd.optimise import optimise
    objective, constraints, paper = OPT_PROBLEMS[problem]
    mat = synth.material_pzt5a()
    Cb = np.asarray(mat.C).reshape(6, 6)
    base = P.foms(Cb, np.asarray(mat.e).reshape(3, 6), np.asarray(mat.kappa).reshape(3, 3))
    t0 = time.perf_counter()

    def progress(q, J, vals, viol):
        if q % 10 == 0:
            cons = ", ".join(f"{c[0]} {v:.4e}" for c, v in zip(constraints, vals))
            print(f"[bench] optimisation iteration {q}: {objective} {J:.4e}, {cons}, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    opts = dict(precision=precision, rtol=1e-12, restart=12, vcycles_a=2, inner_rtol=1e-4, warm_start=1,
                smoothing=P.PHZ_SMOOTH_QP if smoothing == "qp" else P.PHZ_SMOOTH_ELEMENT)
    with P.Context(n, mat, stream=torch.cuda.current_stream().cuda_stream, **opts) as ctx:
        out = optimise(ctx, mat, synth.paper_levelset(n), objective, constraints, max_iters=max_iters,
                       reinit_every=reinit_every, step_control=step_control, callback=progress)
        st = ctx.stats()
    CH, eH, kH = out["effective"]
    wall = time.perf_counter() - t0
    it = out["iterations"]
    f = P.foms(CH, eH, kH)
    f["C_zzzz"] = float(CH[2, 2])
    f["vol"] = out["constraints"][-1][0]
    steady = out["iter_ms"][1:] or out["iter_ms"]
    return {"study": f"optimisation loop: max {objective} s.t. "
                     + ", ".join(f"{c} = {v:g}" for c, v in constraints)
                     + ", PZT-5A, phi0 = -prod cos(2 pi x_i) - 0.2 reinitialised",
            "problem": problem, "n": n, "reinit_every": reinit_every, "smoothing": smoothing,
            "step_control": step_control, "tau_last": out["tau"][-1] if out["tau"] else None,
            "precision": {P.PHZ_BF16X3_IR: "bf16x3ir", P.PHZ_FP32_IR: "fp32ir", P.PHZ_FP64: "fp64"}[precision],
            "solve": "SCP-GMRES, outer rtol 1e-12, warm start from the last iteration",
            "iterations": it, "converged": out["converged"], "wall_s": wall,
            "ms_per_iteration_mean": float(np.mean(steady)), "ms_per_iteration_median": float(np.median(steady)),
            "phase_ms_per_iteration": out["phase_ms"],
            "last_solve_outer_iterations_max": max(st["iterations"]),
            "final": f,
            "base_material": {k: base[k] for k in ("B_voigt", "B_reuss", "d_h", "g_h", "k_h")},
            "final_over_base": {k: f[k] / base[k] for k in ("B_voigt", "B_reuss", "d_h", "g_h", "k_h")},
            "paper": paper,
            "history_every_5": [[q, out["J"][q], *out["constraints"][q]] for q in range(0, it, 5)]}


def smoothing_study(P, torch, synth, mat):
    """Element smoothing against quadrature-point smoothing (Sec. 2.6) on the random-field workload at
    64^3 and 128^3: solve time, iterations and the relative difference of the tensors, which shrinks
    with h."""
    rows = []
    for n in (64, 128):
        phi = synth.grf_levelset(n, seed=2410, solid_fraction=0.3)
        out = {}
        for name, sm in (("element", P.PHZ_SMOOTH_ELEMENT), ("qp", P.PHZ_SMOOTH_QP)):
            with P.Context(n, mat, stream=torch.cuda.current_stream().cuda_stream, precision=P.PHZ_BF16X3_IR,
                           rtol=1e-10, restart=12, vcycles_a=2, inner_rtol=1e-4, smoothing=sm) as ctx:
                ctx.set_levelset(phi)
                ctx.solve()
                ctx.set_levelset(phi)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.solve()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                st = ctx.stats()
                MH, _ = ctx.effective_nd()
            out[name] = (MH, dt, max(st["iterations"]), st["refinements"])
            print(f"[bench] smoothing {name} {n}^3: {dt:.3f} s, {max(st['iterations'])} iterations", file=sys.stderr,
                  flush=True)
        d = np.abs(out["qp"][0] - out["element"][0]).max() / np.abs(out["element"][0]).max()
        rows.append({"n": n, "solve_s_element": out["element"][1], "solve_s_qp": out["qp"][1],
                     "iters_element": out["element"][2], "iters_qp": out["qp"][2],
                     "refinements": [out["element"][3], out["qp"][3]], "tensor_rel_difference": d})
    return {"study": "element vs quadrature-point smoothing, GRF seed 2410 solid 0.3, split-BF16 form, rtol 1e-10",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--solid-fraction", type=float, default=0.3)
    ap.add_argument("--precision", choices=["bf16x3ir", "fp32ir", "fp64"], default="bf16x3ir")
    ap.add_argument("--restart", type=int, default=12)
    ap.add_argument("--vcycles-a", type=int, default=2)
    ap.add_argument("--no-sequential", action="store_true", help="skip the plain FP64 sequential comparison")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy kernel (y = -x, fp32) over MIB MiB three times, "
                         "to scale hardware byte counters")
    ap.add_argument("--block-kernels", default=None, metavar="K0,K1,K2,K3",
                    help="pin the fine blocks' (full, A, B, S) float kernels, as reported in config.fine_kernels "
                         "(-1 = timed choice); for profiling runs whose timing would change the choice")
    ap.add_argument("--block-tiles", default=None, metavar="T0,T1,T2,T3",
                    help="pin the element-contraction tile per fine block (-1 = timed choice)")
    ap.add_argument("--solver-study-only", default=None, metavar="NAMES",
                    help="comma-separated subset of SCP-GMRES, DBP-GMRES, TriCG for --solver-study")
    ap.add_argument("--solver-study", action="store_true",
                    help="instead of the step benchmark: the solver comparison of Sec. 2.5 (SCP-GMRES and DBP-GMRES, "
                         "fixed V-cycle block maps or conjugate-gradient maps to 1e-8, 1e-4, 1e-2) on the paper's test "
                         "geometry at 64^3 and 128^3, float64, relative tolerance 1e-8; prints one JSON line")
    ap.add_argument("--optimise", type=int, default=0, metavar="ITERS",
                    help="run the paper's optimisation example (at most ITERS iterations) at --opt-n and "
                         "print its timing instead of the solve benchmark")
    ap.add_argument("--smoothing-study", action="store_true",
                    help="compare element and quadrature-point smoothing at 64^3 and 128^3")
    ap.add_argument("--opt-n", type=int, default=96)
    ap.add_argument("--optimise-problem", default="bvoigt", choices=sorted(OPT_PROBLEMS))
    ap.add_argument("--opt-no-step-control", action="store_true",
                    help="keep the objective's full step (no step control)")
    ap.add_argument("--opt-smoothing", default="element", choices=["element", "qp"],
                    help="material smoothing of the optimisation run (element mean or quadrature points)")
    ap.add_argument("--reinit-every", type=int, default=5,
                    help="reinitialise every this many optimisation iterations (the paper: 5)")
    ap.add_argument("--graph", action="store_true",
                    help="run the benchmarked form with every Arnoldi step replayed from a captured HIP graph "
                         "(per-kernel event timing then covers the launches outside the graphs only)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the steps without per-kernel HIP events (no roofline figures)")
    ap.add_argument("--full-kernel-timing", action="store_true",
                    help="bracket every timed kernel class (coarse levels, preconditioner, Arnoldi) with HIP events, "
                         "not only the fine-level operator launches (about 5%% slower steps)")
    ap.add_argument("--cheby-degree", type=int, default=None,
                    help="Chebyshev smoothing degree of the benchmarked form (library option cheby_degree)")
    ap.add_argument("--inner-rtol", type=float, default=None,
                    help="relative target of each float refinement cycle of the benchmarked form")
    ap.add_argument("--reorth-tol", type=float, default=None,
                    help="Arnoldi second-pass rule of the benchmarked form (library option reorth_tol; "
                         "-1 = always two passes)")
    ap.add_argument("--cpu-sweep", action="store_true",
                    help="instead of the step benchmark: longer CPU oracle timings (direct solves at 12^3..24^3, "
                         "element and CSR applies at 64^3 and 128^3); prints one JSON line")
    ap.add_argument("--coarse-kernel", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="pin the coarse levels' float kernel (0 direct, 1 LDS-tiled, 2 LDS-tiled on the compact "
                         "bf16 stencils; 1 and 2 where N %% 16 == 0; -1 = timed choice per level)")
    ap.add_argument("--traffic-summary", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: update profiles/hbm_traffic.json from the output folders of two rocprofv3 --pmc "
                         "runs (FETCH_SIZE, WRITE_SIZE) of this benchmark with --copy-calibration, and print the rows")
    ap.add_argument("--peaks", action="store_true",
                    help="instead of the step benchmark: the GPU's achievable copy, read and write bandwidth and "
                         "dense GEMM rates (bf16, fp32, fp64) from device library kernels; prints one JSON line")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the solve runs on a single MI355X; "
              "multi-GPU sharding is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.cpu_sweep:
        print(json.dumps(cpu_sweep()))
        return

    import torch
    import synth
    import paper_2410_03148_amd as P

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.peaks:
        print(json.dumps(measure_peaks(torch, dev)))
        return
    stream = torch.cuda.current_stream()
    n = args.n
    mat = synth.material_workload()
    phi = synth.grf_levelset(n, seed=2410, solid_fraction=args.solid_fraction)
    phi_d = torch.tensor(phi, device=dev)
    prec = {"bf16x3ir": P.PHZ_BF16X3_IR, "fp32ir": P.PHZ_FP32_IR, "fp64": P.PHZ_FP64}[args.precision]

    # solver settings per form (restart, V-cycles per A-block application and
    # the float cycles' relative target picked by sweeps on this workload; the
    # split-BF16 operators floor a float cycle near 1.5e-5, so its cycles aim
    # at 1e-4); every form stops at a true FP64 residual of 1e-10 per load
    forms = {
        "bf16x3ir": dict(precision=P.PHZ_BF16X3_IR, batched=1, restart=args.restart, vcycles_a=args.vcycles_a,
                         inner_rtol=1e-4 if args.inner_rtol is None else args.inner_rtol),
        "fp32ir": dict(precision=P.PHZ_FP32_IR, batched=1, restart=args.restart, vcycles_a=args.vcycles_a),
        "fp64": dict(precision=P.PHZ_FP64, batched=1, restart=15, vcycles_a=2),
        "fp64_sequential": dict(precision=P.PHZ_FP64, batched=0, restart=30, vcycles_a=2),
    }
    # the same float forms with every Arnoldi step replayed from a captured
    # HIP graph
    forms["bf16x3ir_graph"] = dict(forms["bf16x3ir"], use_graph=1)
    forms["fp32ir_graph"] = dict(forms["fp32ir"], use_graph=1)

    pins = {}
    if args.block_kernels:
        pins["block_kernel"] = [int(v) for v in args.block_kernels.split(",")]
    if args.block_tiles:
        pins["block_tile"] = [int(v) for v in args.block_tiles.split(",")]
    if args.coarse_kernel >= 0:
        pins["coarse_kernel"] = args.coarse_kernel
    if args.reorth_tol is not None:
        pins["reorth_tol"] = args.reorth_tol
    if args.cheby_degree is not None:
        pins["cheby_degree"] = args.cheby_degree

    def make_ctx(form):
        extra = dict(pins) if form == args.precision else {}
        if form == args.precision and args.graph:
            extra["use_graph"] = 1
        return P.Context(n, mat, stream=stream.cuda_stream, rtol=1e-10, **forms[form], **extra)

    grad_d = torch.empty(n ** 3, dtype=torch.float64, device=dev)
    geometry = {"phi": phi_d}

    def step(ctx):
        ctx.set_levelset(geometry["phi"])
        st = ctx.solve()
        Cm, e, k = ctx.effective()
        f, (gC, ge, gk) = P.foms(Cm, e, k, grad_of="d_h")
        ctx.backward(gC, ge, gk, out_rho=grad_d)
        ctx.hj_step(None, cfl=0.5, return_phi=False)
        return st, (Cm, e, k), f

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def run(ctx, warmup, steps, timing=False):
        for i in range(warmup):
            step(ctx)
            log(f"warmup step {i + 1}/{warmup} done")
        torch.cuda.synchronize()
        if timing:
            ctx.kernel_timing(True, fine_only=not args.full_kernel_timing)
        t0 = time.perf_counter()
        for i in range(steps):
            st, tens, f = step(ctx)
            log(f"timed step {i + 1}/{steps} done")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt / steps, st, tens, f

    if args.solver_study:
        only = args.solver_study_only.split(",") if args.solver_study_only else None
        print(json.dumps(solver_study(P, torch, synth, mat, dev, only)))
        return
    if args.smoothing_study:
        print(json.dumps(smoothing_study(P, torch, synth, mat)))
        return
    if args.optimise:
        print(json.dumps(optimisation_run(P, torch, synth, args.opt_n, args.optimise, prec, args.optimise_problem,
                                          args.reinit_every, args.opt_smoothing, not args.opt_no_step_control)))
        return

    if args.copy_calibration:
        cnt = args.copy_calibration * 2 ** 20 // 4
        src = torch.ones(cnt, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 launches, each reads {4 * cnt} B and writes {4 * cnt} B")
        del src, dst

    ctx = make_ctx(args.precision)
    ms, status, tens, f = run(ctx, args.warmup, args.steps, timing=not args.no_kernel_timing)
    stats = ctx.stats()
    ktimes = ctx.kernel_times()
    ctx.kernel_timing(False)
    # the gradient pass on its own (part of every step above): d_h's density
    # sensitivities of a fresh solve (each step's HJ update moved the geometry)
    ctx.set_levelset(phi_d)
    ctx.solve()
    Cm_, e_, k_ = ctx.effective()
    _, (gC_, ge_, gk_) = P.foms(Cm_, e_, k_, grad_of="d_h")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        ctx.backward(gC_, ge_, gk_, out_rho=grad_d)
    torch.cuda.synchronize()
    backward_ms = (time.perf_counter() - t0) / 5 * 1e3
    ctx.close()

    def operator_bench(form, prec_code, apply_code, reps=50):
        """Median of `reps` full-operator applies (9 columns) after 5 warm-ups."""
        c = make_ctx(form)
        c.set_levelset(phi_d)
        dt = torch.float64 if apply_code == P.PHZ_FP64 else torch.float32
        xb = torch.randn((4, 9, n ** 3), dtype=dt, device=dev)
        yb = torch.empty_like(xb)
        for _ in range(5):
            c.apply(P.OP_FULL, 9, apply_code, xb.data_ptr(), yb.data_ptr())
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            c.apply(P.OP_FULL, 9, apply_code, xb.data_ptr(), yb.data_ptr())
            b.record(stream)
        torch.cuda.synchronize()
        t = float(np.median([a.elapsed_time(b) for a, b in evs])) * 1e-3
        kind = c.stats()["fine_kernel"][0] if apply_code == P.PHZ_FP32_IR else None
        c.close()
        w = 8 if apply_code == P.PHZ_FP64 else 4
        nbytes = (4 * 9 + 1 + 4 * 9) * w * n ** 3
        return {"median_ms": t * 1e3, "GB/s": nbytes / t / 1e9, "hbm_frac": nbytes / t / 8e12,
                "algorithmic_bytes": nbytes, "kernel": {None: "gather_f64" if w == 8 else "elem_bf16x3",
                                                        0: "gather_f32", 1: "tiled_gather_f32",
                                                        2: "elem_bf16x3"}[kind]}

    op_bench = {}
    if not args.no_compare:
        op_bench["fp64"] = operator_bench("fp64", P.PHZ_FP64, P.PHZ_FP64)
        op_bench["fp32"] = operator_bench("fp32ir", P.PHZ_FP32_IR, P.PHZ_FP32_IR)
        op_bench["bf16x3"] = operator_bench("bf16x3ir", P.PHZ_BF16X3_IR, P.PHZ_BF16X3_IR)
        log("operator benchmark done")

    result = {
        "metric": "128\u00b3 9-load homogenisation solves/s, mixed vs FP64 at \u22641e-6 rel err; op GB/s",
        "value": 1.0 / ms,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3ir": "bf16x3", "fp32ir": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic GRF level set (seed 2410, corr 0.1, solid {args.solid_fraction}), "
                               f"PZT-like base, 9 loads batched, GMRES({forms[args.precision]['restart']})+SCP/GMG "
                               f"({forms[args.precision]['vcycles_a']} V-cycles per A-block solve), rtol 1e-10",
                   "n": n, "dofs": 4 * n ** 3, "loads": 9,
                   "precision": args.precision, "status": status,
                   "iterations_max": max(stats["iterations"]), "refinements": stats["refinements"],
                   "true_residual_max": max(stats["true_residual"]),
                   "setup_ms": stats["setup_ms"], "solve_ms": stats["solve_ms"],
                   "fine_kernels": stats["fine_kernel"], "mfma_tiles_full_A_B_S": stats["elem_tile"],
                   "coarse_kernels_A_S": [stats["coarse_kernel"][1:8], stats["coarse_kernel"][9:16]],
                   "split_products_operator_precond": ([3, 1] if args.precision == "bf16x3ir" else None),
                   "final_precision": stats["final_precision"], "fallbacks": stats["fallbacks"],
                   "reorth_passes_per_load_step": stats["reorth_passes"] / max(sum(stats["iterations"]), 1)},
    }

    # dominant single kernel from the live event timing of the timed steps
    def roofline_of(name):
        cnt, tot = ktimes[name]
        avg_s = tot / cnt * 1e-3
        fl, by, p = per_node(name)
        flops = fl * n ** 3
        nbytes = by * n ** 3
        ai = fl / by
        # published MI355X peaks: fp64 78.6, fp32 vector 157.3, dense bf16 MFMA 2500 TFLOP/s
        peak_tf = {"f64": 78.6, "f32": 157.3}.get(p, 2500.0)
        ridge = peak_tf * 1e12 / 8e12
        tile = stats["elem_tile"][list(OPS).index(name.split("_")[1])] if name.startswith("elem_") else None
        traffic = measured_traffic(name, tile)
        if ai > ridge:
            return {"bound": "mfma" if name.startswith("elem_") else "alu", "achieved": flops / avg_s / 1e12,
                    "peak": peak_tf, "unit": "TFLOP/s", "frac": flops / avg_s / 1e12 / peak_tf, "traffic": traffic,
                    "kernel": name, "avg_ms": avg_s * 1e3, "algorithmic_bytes": nbytes, "algorithmic_flops": flops}
        return {"bound": "hbm", "achieved": nbytes / avg_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                "frac": nbytes / avg_s / 8e12, "traffic": traffic, "kernel": name, "avg_ms": avg_s * 1e3,
                "algorithmic_bytes": nbytes, "algorithmic_flops": flops}

    single = {k: v for k, v in ktimes.items() if k.startswith(("fine_", "tiled_", "elem_"))}
    if single:
        order = sorted(single, key=lambda k: -single[k][1])
        result["roofline"] = roofline_of(order[0])
        # the A block's plain and Chebyshev element kernels take about the same
        # total time per step, so either may lead: a runner-up within 5% is
        # reported beside it
        if len(order) > 1 and single[order[1]][1] >= 0.95 * single[order[0]][1]:
            result["roofline_runner_up"] = roofline_of(order[1])
        result["kernel_ms_per_step"] = {k: v[1] / args.steps for k, v in sorted(ktimes.items())}
        # the outer operator apply (all four fields, nine loads) as achieved
        # algorithmic HBM bandwidth
        ops = {k: v for k, v in ktimes.items() if k.startswith(("fine_full_k9", "tiled_full_k9", "elem_full_k9"))}
        if ops:
            name = max(ops, key=lambda k: ops[k][1])
            cnt, tot = ops[name]
            avg_s = tot / cnt * 1e-3
            fl, by, _ = per_node(name)
            result["operator"] = {"kernel": name, "avg_ms": avg_s * 1e3, "GB/s": by * n ** 3 / avg_s / 1e9,
                                  "hbm_frac": by * n ** 3 / avg_s / 8e12, "TFLOP/s": fl * n ** 3 / avg_s / 1e12}
    if op_bench:
        # y = calA x on all nine columns, 50 timed applies each, median
        result.setdefault("operator", {})["apply_median"] = op_bench
    result["backward_ms"] = backward_ms

    def compare_form(form, ref_tens, ref_ms, steps):
        c64 = make_ctx(form)
        ms64, st64, t64, f64 = run(c64, 1, steps)
        s64 = c64.stats()
        c64.close()
        errs = {nm: float(np.linalg.norm(a - b) / np.linalg.norm(b)) for nm, a, b in zip(("C", "e", "kappa"), ref_tens, t64)}
        return {"solves_per_s": 1.0 / ms64, "speedup_of_mixed": ms64 / ref_ms, "status": st64,
                "iterations_max": max(s64["iterations"]), "refinements": s64["refinements"],
                "true_residual_max": max(s64["true_residual"]), "restart": forms[form]["restart"],
                "final_precision": s64["final_precision"], "fallbacks": s64["fallbacks"],
                "use_graph": forms[form].get("use_graph", 0),
                "rel_err_of_mixed": errs, "max_rel_err_of_mixed": max(errs.values()), "tensors": t64}

    if not args.no_compare and prec != P.PHZ_FP64:
        cmp = {}
        for form in ("fp32ir", "fp64", "fp64_sequential", args.precision + "_graph"):
            if form == args.precision or form not in forms:
                continue
            if form == "fp64_sequential" and args.no_sequential:
                continue
            cmp[form] = compare_form(form, tens, ms, 1 if form == "fp64_sequential" else 2)
            cmp[form].pop("tensors")
            log(f"{form} comparison done")
        # the other solid fraction of the workload: the default form against
        # FP64 batched on that cell
        other = 0.7 if abs(args.solid_fraction - 0.3) < 1e-12 else 0.3
        geometry["phi"] = torch.tensor(synth.grf_levelset(n, seed=2410, solid_fraction=other), device=dev)
        mixed = compare_form(args.precision, tens, ms, 2)
        ref64 = compare_form("fp64", mixed["tensors"], 1.0 / mixed["solves_per_s"], 2)
        geometry["phi"] = phi_d
        for d in (mixed, ref64):
            d.pop("tensors")
        cmp[f"solid_{other}"] = {"solves_per_s": mixed["solves_per_s"], "iterations_max": mixed["iterations_max"],
                                 "refinements": mixed["refinements"], "true_residual_max": mixed["true_residual_max"],
                                 "status": mixed["status"], "fp64_solves_per_s": ref64["solves_per_s"],
                                 "fp64_iterations_max": ref64["iterations_max"],
                                 "speedup_of_mixed_over_fp64": ref64["speedup_of_mixed"],
                                 "rel_err_of_mixed": ref64["rel_err_of_mixed"],
                                 "max_rel_err_of_mixed": ref64["max_rel_err_of_mixed"]}
        log(f"solid fraction {other} comparison done")
        result["compare"] = cmp

    if not args.no_cpu:
        log("cpu oracle baseline (12^3 and 16^3 solves, median of 3; one full-size operator apply)")
        fine_launches = sum(v[0] for k, v in ktimes.items() if k.startswith(("fine_", "tiled_", "elem_"))) / args.steps
        iters = max(stats["iterations"])
        result["cpu_baseline"] = cpu_baseline(n, iters, fine_launches / max(iters, 1))
    print(json.dumps(result))


if __name__ == "__main__":
    main()
