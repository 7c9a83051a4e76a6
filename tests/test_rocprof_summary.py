"""The counter summaries behind profiles/ (paper_1910_08448_amd/rocprof_summary.py), on small
synthetic rocprofv3 counter files: the copy-probe scaling of FETCH_SIZE / WRITE_SIZE, the choice
of the inference sweep the run swept with (the compacted path's two colour kernels together),
and the VALU issue rows."""
import csv
import os

import pytest

from paper_1910_08448_amd import rocprof_summary as R

FUSED = "void mpr::k_sweep<float, float, 1, false, false>(mpr::SweepArgs)"
FUSED_ACC = "void mpr::k_sweep<float, float, 2, false, false>(mpr::SweepArgs)"
SPARSE0 = "_ZN3mpr8k_sparseIDF16_fLi1ELb0ELi0EEEvNS_10SparseArgsE"
SPARSE1 = "_ZN3mpr8k_sparseIDF16_fLi1ELb0ELi1EEEvNS_10SparseArgsE"
COPY = "__amd_rocclr_copyBuffer"


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (name, ctr, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name,
                        "Grid_Size": 1 << 20 if name == COPY else 4096, "Counter_Name": ctr,
                        "Counter_Value": val})


def test_traffic_scales_by_the_copy_probe_and_keeps_the_swept_path(tmp_path):
    # a 1 MiB copy: FETCH_SIZE reads 512 KiB (factor 2), WRITE_SIZE 1024 KiB (factor 1); the
    # run swept with the fused kernel (three dispatches), an autotuner candidate ran once
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    _write(f, [(COPY, "FETCH_SIZE", 512), (FUSED, "FETCH_SIZE", 100), (FUSED, "FETCH_SIZE", 110),
               (FUSED, "FETCH_SIZE", 120), (SPARSE0, "FETCH_SIZE", 7), (COPY, "FETCH_SIZE", 9)])
    _write(w, [(COPY, "WRITE_SIZE", 1024), (FUSED, "WRITE_SIZE", 30), (FUSED, "WRITE_SIZE", 30),
               (FUSED, "WRITE_SIZE", 30), (SPARSE0, "WRITE_SIZE", 5)])
    t = R.traffic(f, w, 1)
    assert t["fetch"]["kernels"] == ["fused"] and t["fetch"]["dispatches"] == 3
    assert t["fetch"]["factor"] == pytest.approx(2.0) and t["write"]["factor"] == pytest.approx(1.0)
    assert t["fetch"]["kib_per_sweep"] == pytest.approx(110.0)
    assert t["bytes_per_launch"] == pytest.approx(110.0 * 1024 * 2.0 + 30.0 * 1024)


def test_traffic_of_the_compacted_path_adds_its_two_colour_kernels(tmp_path):
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    rows_f, rows_w = [(COPY, "FETCH_SIZE", 512), (FUSED, "FETCH_SIZE", 999)], [(COPY, "WRITE_SIZE", 1024)]
    for _ in range(3):
        rows_f += [(SPARSE0, "FETCH_SIZE", 50), (SPARSE1, "FETCH_SIZE", 40)]
        rows_w += [(SPARSE0, "WRITE_SIZE", 20), (SPARSE1, "WRITE_SIZE", 10)]
    _write(f, rows_f)
    _write(w, rows_w)
    t = R.traffic(f, w, 1)
    assert t["fetch"]["kernels"] == ["sparse0", "sparse1"]
    assert t["fetch"]["kib_per_sweep"] == pytest.approx(90.0)
    assert t["write"]["kib_per_sweep"] == pytest.approx(30.0)
    assert t["bytes_per_launch"] == pytest.approx(90.0 * 1024 * 2.0 + 30.0 * 1024)


def test_traffic_refuses_a_run_without_its_copy_probe(tmp_path):
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    _write(f, [(FUSED, "FETCH_SIZE", 100)])
    _write(w, [(COPY, "WRITE_SIZE", 1024), (FUSED, "WRITE_SIZE", 30)])
    with pytest.raises(SystemExit):
        R.traffic(f, w, 1)


def test_valu_rows(tmp_path):
    """Issue units per quad-cycle per SIMD = SQ_ACTIVE_INST_VALU / (1024 SIMDs x GRBM_GUI_ACTIVE /
    8 XCDs / 4); lane-units per update = SQ_ACTIVE_INST_VALU x 64 / updates; the compacted path's
    row adds its two colour kernels."""
    d = str(tmp_path / "v")
    quads = 1000.0
    grbm = quads * 4 * 8
    rows = []
    for name, act, act2, trans in ((FUSED, 1.2e6, 0.3e6, 1e4), (SPARSE0, 0.6e6, 0.1e6, 2e3),
                                   (SPARSE1, 0.5e6, 0.1e6, 3e3)):
        rows += [(name, "SQ_INSTS_VALU", act * 0.9), (name, "SQ_ACTIVE_INST_VALU", act),
                 (name, "SQ_ACTIVE_INST_VALU2", act2), (name, "SQ_INSTS_VALU_TRANS_F32", trans),
                 (name, "GRBM_GUI_ACTIVE", grbm)]
    rows += [(FUSED_ACC, "SQ_ACTIVE_INST_VALU", 1.0), (FUSED_ACC, "GRBM_GUI_ACTIVE", grbm)]
    _write(d, rows)
    out = R.valu(d, 64000)
    lines = {l.split("|")[1].strip(): [c.strip() for c in l.split("|")[2:-1]] for l in out.splitlines()[2:]}
    fused = lines["fused"]
    assert float(fused[2]) == pytest.approx(1.2e6 / (1024 * quads), abs=1e-3)     # issue rate
    assert float(fused[6]) == pytest.approx(1.2e6 * 64 / 64000, rel=1e-3)          # lane-units / update
    assert float(fused[7]) == pytest.approx(1e4 * 64 / 64000, rel=1e-2)            # transcendentals
    both = lines["sparse0 + sparse1 (one sweep)"]
    assert float(both[6]) == pytest.approx(1.1e6 * 64 / 64000, rel=1e-3)
    assert float(both[2]) == pytest.approx(1.1e6 / (1024 * 2 * quads), abs=1e-3)
    assert any(k.startswith("other sweep variant") for k in lines)
