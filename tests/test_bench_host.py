"""Host logic of bench.py that needs no GPU: the mapping of profiled kernel
names to timing labels and the HBM-traffic summary built from two counter
runs (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy kernel)."""
import csv
import importlib.util
import json
import os
import shutil

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_labels(bench):
    # element kernels keep mangled names in the counter files
    mangled = "_ZN3phz12_GLOBAL__N_111k_elem_mfmaILi3ELi3ELi9ELi1ELb1ELi16ELi4ELi4EEEvjPKfPKDv8_DF16bS3_NS_6OpArgsIfEE"
    assert bench._traffic_label(mangled, 0) == ("elem_A_k9_bf16x1_cheby", 1)
    full = "_ZN3phz12_GLOBAL__N_111k_elem_mfmaILi4ELi4ELi9ELi3ELb0ELi8ELi8ELi4EEEvjPKf"
    assert bench._traffic_label(full, 0) == ("elem_full_k9_bf16x3", 0)
    plain = "phz::(anonymous namespace)::k_elem_mfma<1, 3, 9, 1, false, 16, 8, 2>(unsigned int)"
    assert bench._traffic_label(plain, 0) == ("elem_B_k9_bf16x1", 2)
    st = "void phz::(anonymous namespace)::k_stencil_tiled<1, false, false, true>(unsigned int, float const*)"
    assert bench._traffic_label(st, 32 ** 3) == ("coarse_tiledbf_S_f32@32", None)
    assert bench._traffic_label("void phz::(anonymous namespace)::k_fine_tiled<1, 1, 9, true>(unsigned)", 1) == \
        ("tiled_S_k9_f32_cheby", None)
    assert bench._traffic_label("void k_fine_apply<double, 1, 1, 1, false, true>(unsigned)", 1) == \
        ("fine_S_k1_f64", None)
    # kernels the record does not list, including the float stencil form
    assert bench._traffic_label("void k_stencil_tiled<3, true, true, false>(unsigned)", 64 ** 3) == (None, None)
    assert bench._traffic_label("void k_arnoldi_dots<float, 12>(unsigned)", 1) == (None, None)


def _write_counters(folder, name, counter, rows):
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, f"{name}_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (kernel, grid, value) in enumerate(rows):
            w.writerow([i, grid, kernel, counter, value])


def test_traffic_summary_scales_by_the_copy_kernel(bench, tmp_path):
    rec_path = tmp_path / "hbm_traffic.json"
    shutil.copy(os.path.join(ROOT, "profiles", "hbm_traffic.json"), rec_path)
    elem = "k_elem_mfma<3, 3, 9, 1, false, 16, 4, 4>(unsigned int)"
    copy = "void at::native::elementwise_kernel<neg_kernel>(int)"
    gib = 1 << 30
    # the copy reads and writes 1 GiB: 1,048,576 KiB; FETCH_SIZE reads half of that, so a fetched KiB
    # counts 2048 B; WRITE_SIZE counts KiB
    _write_counters(tmp_path / "f", "fetch", "FETCH_SIZE",
                    [(copy, gib // 4, 524288.0)] * 3 + [(elem, 2097152, 1000.0), (elem, 2097152, 3000.0)])
    _write_counters(tmp_path / "w", "write", "WRITE_SIZE",
                    [(copy, gib // 4, 1048576.0)] * 3 + [(elem, 2097152, 500.0), (elem, 2097152, 500.0)])
    rows = bench.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(rec_path))
    rec = json.load(open(rec_path))
    assert rec["calibration"]["fetch_bytes_per_kib"] == pytest.approx(2048.0)
    assert rec["calibration"]["write_bytes_per_kib"] == pytest.approx(1024.0)
    k = rec["kernels"]["elem_A_k9_bf16x1"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes"] == 2000 * 2048 and k["write_bytes"] == 500 * 1024
    assert k["bytes_per_launch"] == 2000 * 2048 + 500 * 1024
    assert len(rows) == 1 and rows[0].startswith("| elem_A_k9_bf16x1 |")
    # labels the runs did not count keep their earlier figures
    before = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
    assert rec["kernels"]["elem_full_k9_bf16x3"] == before["kernels"]["elem_full_k9_bf16x3"]
