"""Host logic of the benchmark (no GPU): the counter calibration, the
per-kernel and per-step byte accounting, and the staleness rule of the
committed counter records."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def write_counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, (name, grid, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_summary_calibrates_and_splits(tmp_path):
    cb = bench.COPY_BYTES
    # the copy reads each byte at counter factor 0.5 and writes it at 1.0 (KiB)
    fetch = [("__amd_rocclr_copyBuffer", 4096, 0.5 * cb / 1024)] * 3 + [("__amd_rocclr_copyBuffer", 16, 1.0)]
    write = [("__amd_rocclr_copyBuffer", 4096, 1.0 * cb / 1024)] * 3
    kib = lambda b, f: f * b / 1024.0
    # two steps, three CG iterations: the fused update (102.76 MB algorithmic)
    # measured at 1.1x, split 2/3 read, 1/3 written
    upd = bench.ALG_BYTES_PER_CELL["mg_update0"] * 256 * 256 * 64 * 1.1
    for _ in range(3):
        fetch.append(("void uf::k_mg_restrict<true, float>(...)", 262400, kib(upd * 2 / 3, 0.5)))
        write.append(("void uf::k_mg_restrict<true, float>(...)", 262400, kib(upd / 3, 1.0)))
        fetch.append(("void uf::k_cg_Ad<64, float>(...)", 262144, kib(7e7, 0.5)))
        write.append(("void uf::k_cg_Ad<64, float>(...)", 262144, kib(1e6, 1.0)))
    for _ in range(2):
        fetch.append(("void uf::k_advect_fwd<float>(...)", 4325376, kib(9e7, 0.5)))
        write.append(("void uf::k_advect_fwd<float>(...)", 4325376, kib(2e7, 1.0)))
    write_counters(str(tmp_path / "run" / "fetch"), "FETCH_SIZE", fetch)
    write_counters(str(tmp_path / "run" / "write"), "WRITE_SIZE", write)
    out_dir = tmp_path / "out"
    out_dir.mkdir()
    recs, step = bench.traffic_summary(str(tmp_path / "run"), "cmd", out_dir=str(out_dir), name="C1")
    r = recs["mg_update0"]
    assert r["calibration"]["fetch_factor"] == pytest.approx(0.5)
    assert r["calibration"]["write_factor"] == pytest.approx(1.0)
    assert r["calibration"]["copies"] == [3, 3]          # the small runtime copy is left out
    assert r["bytes_per_launch"] == pytest.approx(upd)
    assert r["bytes_per_launch"] / r["alg_bytes_per_launch"] == pytest.approx(1.1)
    assert step["steps"] == 2 and step["cg_iterations"] == 3
    assert step["bytes_fixed_per_step"] == pytest.approx(1.1e8)
    assert step["bytes_per_cg_iteration"] == pytest.approx(upd + 7.1e7)
    saved = json.load(open(out_dir / "traffic_mg_update0_256x256x64.json"))
    assert saved["source_sha256"] == bench.sources_hash("mg_update0")


def test_records_go_stale_with_their_own_kernel_sources_only():
    h_upd = bench.sources_hash("mg_update0")
    assert h_upd == bench.sources_hash("mg_down0")          # same file
    assert h_upd != bench.sources_hash("advect_fwd")
    assert bench.sources_hash() not in (h_upd, bench.sources_hash("advect_fwd"))


def test_algorithmic_bytes_per_step_add_up():
    # seven face and cell kernels, and per iteration A d, the fused update,
    # the level-0 up/smoothing and the coarse levels at 1/7 of level 0
    assert bench.ALG_FIXED_PER_CELL == 196.0
    assert bench.ALG_ITER_PER_CELL == pytest.approx(16 + 24.5 + 8.5 + 13.0 / 7)


def test_cpu_baseline_slab_is_an_eighth_of_the_workload():
    """The oracle's sample: x-slab s of 8 of the workload, the porosity's own
    cells, the configuration otherwise unchanged (FP64)."""
    import numpy as np
    p, phi, cfg = bench.workload("C1")
    ph, c = bench._slab(phi, cfg, 3)
    assert c["nx"] * 8 == cfg["nx"] and c["ny"] == cfg["ny"] and c["nz"] == cfg["nz"] and c["dtype"] == "f64"
    assert np.array_equal(ph, phi[3 * c["nx"]:4 * c["nx"]])
    assert c["wind_dir_deg"] == cfg["wind_dir_deg"] and c["bc"] == cfg["bc"]


def test_every_profiled_kernel_has_bytes_and_sources():
    """Each kernel name the profiler summaries map to has an algorithmic byte
    count and source files (so its counter record can go stale), and the
    marching split moves the fused update's bytes: residual update plus the
    iterate update on the second stream."""
    names = {n for _, n in bench.PROFILE_NAMES}
    for n in names:
        assert n in bench.ALG_BYTES_PER_CELL, n
        assert n in bench.KERNEL_FILES, n
    assert bench.profile_name("void uf::k_mg_update_march<true, float>(...)") == "mg_rupd0"
    assert bench.profile_name("void uf::k_cg_xupd<float>(...)") == "cg_xupd"
    assert bench.profile_name("void uf::k_mg_restrict<true, float>(...)") == "mg_update0"
    b = bench.ALG_BYTES_PER_CELL
    assert b["mg_rupd0"] + b["cg_xupd"] == pytest.approx(b["mg_update0"])


@pytest.mark.skipif(not os.path.exists(os.path.join(ROOT, "paper_2204_01117_amd", "libuf.so")),
                    reason="libuf.so not built")
def test_timer_names_follow_the_header_enum():
    """The binding's kernel-timer names are indexed by the UF_TK_* ids of
    include/uf.h."""
    import re
    import paper_2204_01117_amd as U
    src = open(os.path.join(ROOT, "include", "uf.h")).read()
    ids = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"UF_TK_(\w+) = (\d+)", src))
    assert len(U.TIMED_KERNELS) == ids["COUNT"]
    assert U.TIMED_KERNELS[ids["MG_RUPD0"]] == "mg_rupd0"
    assert U.TIMED_KERNELS[ids["MG_UPDATE0"]] == "mg_update0"
    assert U.TIMED_KERNELS[ids["CG_AD"]] == "cg_Ad"
