"""Host logic of bench.py (no GPU): the one-GPU contract, the reduction of
rocprofv3 CSV output to the text summaries kept under profiles/, and the
per-launch HBM traffic read back from them (scaled by the calibration
kernel, withheld when the summary was taken on other kernel sources)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

NEG = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(at::TensorIteratorBase&)>(int)"
BIN = "void vsr::k_bin(vsr::BinArgs)"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def _write_csvs(tmp_path, fetch_kib, write_kib, valu, valu2, lds, grbm):
    kt = tmp_path / "kt"
    kt.mkdir()
    (kt / "run_kernel_stats.csv").write_text(
        "Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs,StdDev\n"
        f'"{BIN}",4,400000,100000,60.0,90000,110000,1\n')
    pmc = tmp_path / "pmc"
    pmc.mkdir()
    calib_kib = bench.CALIB_BYTES / 1024
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value",
            f'1,"{NEG}",FETCH_SIZE,{0.5 * calib_kib}', f'1,"{NEG}",WRITE_SIZE,{calib_kib}']
    for d in (2, 3):  # two dispatches of the binner, averaged
        rows += [f'{d},"{BIN}",FETCH_SIZE,{fetch_kib[d - 2]}', f'{d},"{BIN}",WRITE_SIZE,{write_kib}',
                 f'{d},"{BIN}",SQ_ACTIVE_INST_VALU,{valu}', f'{d},"{BIN}",SQ_ACTIVE_INST_VALU2,{valu2}',
                 f'{d},"{BIN}",GRBM_GUI_ACTIVE,{grbm}']
    (pmc / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
    # a second counter run of the same program: GRBM_GUI_ACTIVE again (the
    # two runs' values are averaged, not added) beside the LDS counter
    pmc2 = pmc / "second"
    pmc2.mkdir()
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for d in (2, 3):
        rows += [f'{d},"{BIN}",SQ_LDS_IDX_ACTIVE,{lds}', f'{d},"{BIN}",GRBM_GUI_ACTIVE,{grbm}']
    (pmc2 / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
    return kt, pmc


def test_summary_and_traffic(tmp_path, capsys, monkeypatch):
    kt, pmc = _write_csvs(tmp_path, fetch_kib=(900.0, 1100.0), write_kib=200.0, valu=6.4e6, valu2=0.4e6,
                          lds=3.2e6, grbm=1.0e6)
    bench.summarize([str(kt), str(pmc)])
    out = capsys.readouterr().out
    lines = out.splitlines()
    assert lines[0] == f"source {bench.source_hash()}"
    stat = [ln for ln in lines if ln.startswith("stat vsr::k_bin")]
    assert len(stat) == 1 and stat[0].split()[2:4] == ["4", "400.0"] and stat[0].split()[4] == "100.00"
    calib = [ln for ln in lines if ln.startswith("calib")][0].split()
    assert calib[calib.index("fetch_factor") + 1] == "0.5000" and calib[calib.index("write_factor") + 1] == "1.0000"
    kern = [ln for ln in lines if ln.startswith("kernel vsr::k_bin")][0].split()
    vals = dict(zip(kern[2::2], kern[3::2]))
    assert vals["dispatches"] == "2" and float(vals["fetch_kib"]) == 1000.0 and float(vals["write_kib"]) == 200.0
    # SIMD quad-cycles with VALU issue (6.4e6 - 0.4e6 dual) over 256 CUs x
    # 1e6 / 8 busy cycles per XCD; LDS cycles over the same
    assert float(vals["valu_busy"]) == pytest.approx(6.0e6 / (256 * 1.0e6 / 8), abs=1e-3)
    assert float(vals["lds_busy"]) == pytest.approx(3.2e6 / (256 * 1.0e6 / 8), abs=1e-3)
    assert float(vals["GRBM_GUI_ACTIVE"]) == pytest.approx(1.0e6)

    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_1080p_1m.txt").write_text("# header\n" + out)
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    t = bench.traffic_from_profiles("k_bin")
    assert t["fetch_bytes"] == pytest.approx(1000.0 * 1024 / 0.5)
    assert t["write_bytes"] == pytest.approx(200.0 * 1024 / 1.0)
    assert t["bytes"] == pytest.approx(t["fetch_bytes"] + t["write_bytes"])
    assert bench.traffic_from_profiles("k_raster<false>") is None  # not profiled

    # counters taken on other kernel sources are not reported
    (prof / "traffic_1080p_1m.txt").write_text(out.replace(bench.source_hash(), "0" * 16))
    assert bench.traffic_from_profiles("k_bin") is None
    os.remove(prof / "traffic_1080p_1m.txt")
    assert bench.traffic_from_profiles("k_bin") is None


def test_roofline_kernels_are_named_as_profiled():
    """Every kernel whose traffic the bench looks up by a literal name, and
    the benchmark batch's binner and rasterizer, are spelled as the committed
    traffic summary spells them (template arguments without spaces), so a
    roofline's traffic is null only when the profile is stale."""
    import re
    src = open(os.path.join(os.path.dirname(bench.__file__), "bench.py")).read()
    asked = set(re.findall(r'traffic_from_profiles\("([^"]+)"', src))
    asked |= {"k_submit_bin_block16", "k_submit_raster16"}
    path = os.path.join(bench.PROFILES, "traffic_1080p_1m.txt")
    rows = {ln.split()[1] for ln in open(path) if ln.startswith("kernel ")}
    missing = sorted(k for k in asked if "vsr::" + k not in rows)
    assert asked and not missing, missing
