"""Host logic of bench.py that turns rocprofv3 counter files into the
per-launch HBM traffic records (no GPU): which kernels get a record for a
two-call run and for a fused run, the copy-kernel scaling, and the source
digest that invalidates a record once the kernel changes."""
import argparse
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, counter, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def calibration(tmp_path):
    # a copy that FETCH_SIZE reads as half its bytes and WRITE_SIZE as all of them
    kib = bench.COPY_BYTES // 1024
    cf, cw = tmp_path / "cf.csv", tmp_path / "cw.csv"
    write_counters(cf, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", kib // 2)] * 3)
    write_counters(cw, [("__amd_rocclr_copyBuffer", "WRITE_SIZE", kib)] * 3)
    return str(cf), str(cw)


ARGS = argparse.Namespace(kernel="mfma16", bpl=64, workload="unit")
FUSED = "void ddhf::k_ndft_comb<4, 3, true>(int const*, unsigned int const*, float const*)"
NDFT = "void ddhf::k_ndft_mfma16<4, 0>(int const*, unsigned int const*, float const*)"
COMB = "void ddhf::k_comb_fast<4, 3>(float const*, int, ddhf::CombArgs, int, int)"
OTHER = "ddhf::k_radix_scatter(unsigned int const*, unsigned int const*)"


def test_fused_run_writes_only_the_fused_record(tmp_path):
    cf, cw = calibration(tmp_path)
    pf, pw = tmp_path / "pf.csv", tmp_path / "pw.csv"
    write_counters(pf, [(FUSED, "FETCH_SIZE", 100), (FUSED, "FETCH_SIZE", 300),
                        (OTHER, "FETCH_SIZE", 7)])
    write_counters(pw, [(FUSED, "WRITE_SIZE", 50), (FUSED, "WRITE_SIZE", 50)])
    out = tmp_path / "profiles"
    out.mkdir()
    bench.traffic_summary(ARGS, str(pf), str(pw), cf, cw, out_dir=str(out))
    assert sorted(os.listdir(out)) == ["traffic_ndft_comb_mfma16_unit.json"]
    rec = json.load(open(out / "traffic_ndft_comb_mfma16_unit.json"))
    # means per dispatch: 200 KiB fetched (x 2 by the calibration), 50 KiB written
    assert rec["bytes_per_launch"] == pytest.approx(200 * 1024 * 2 + 50 * 1024)
    assert rec["dispatches"] == [2, 2]
    digest = bench.kernel_source_digest(bench.TRAFFIC_SOURCES["comb"])
    assert rec["source_digest"] == digest
    assert bench.load_traffic("ndft_comb_mfma16_unit", digest, str(out)) == rec["bytes_per_launch"]
    # a changed kernel source invalidates the record
    assert bench.load_traffic("ndft_comb_mfma16_unit", "0" * 16, str(out)) is None
    assert bench.load_traffic("ndft_comb_mfma16_other", digest, str(out)) is None


def test_two_call_run_writes_the_ndft_and_comb_records(tmp_path):
    cf, cw = calibration(tmp_path)
    pf, pw = tmp_path / "pf.csv", tmp_path / "pw.csv"
    write_counters(pf, [(NDFT, "FETCH_SIZE", 10), (COMB, "FETCH_SIZE", 1000)])
    write_counters(pw, [(NDFT, "WRITE_SIZE", 5000), (COMB, "WRITE_SIZE", 30)])
    out = tmp_path / "profiles"
    out.mkdir()
    bench.traffic_summary(ARGS, str(pf), str(pw), cf, cw, out_dir=str(out))
    assert sorted(os.listdir(out)) == ["traffic_comb_fast_unit.json",
                                       "traffic_ndft_mfma16_64_unit.json"]
    nd = json.load(open(out / "traffic_ndft_mfma16_64_unit.json"))
    assert nd["bytes_per_launch"] == pytest.approx(10 * 1024 * 2 + 5000 * 1024)
    assert nd["source_digest"] == bench.kernel_source_digest(bench.TRAFFIC_SOURCES["ndft"])


def test_fp32_fused_form_is_not_mistaken_for_the_split_fp16_one(tmp_path):
    cf, cw = calibration(tmp_path)
    pf, pw = tmp_path / "pf.csv", tmp_path / "pw.csv"
    fp32 = FUSED.replace("true>", "false>")
    write_counters(pf, [(fp32, "FETCH_SIZE", 100)])
    write_counters(pw, [(fp32, "WRITE_SIZE", 100)])
    out = tmp_path / "profiles"
    out.mkdir()
    with pytest.raises(SystemExit):   # mfma16 names the split-FP16 form only
        bench.traffic_summary(ARGS, str(pf), str(pw), cf, cw, out_dir=str(out))
    args32 = argparse.Namespace(kernel="mfma", bpl=64, workload="unit")
    bench.traffic_summary(args32, str(pf), str(pw), cf, cw, out_dir=str(out))
    assert sorted(os.listdir(out)) == ["traffic_ndft_comb_mfma_unit.json"]


def test_no_matching_kernel_is_an_error(tmp_path):
    cf, cw = calibration(tmp_path)
    pf, pw = tmp_path / "pf.csv", tmp_path / "pw.csv"
    write_counters(pf, [(OTHER, "FETCH_SIZE", 1)])
    write_counters(pw, [(OTHER, "WRITE_SIZE", 1)])
    with pytest.raises(SystemExit):
        bench.traffic_summary(ARGS, str(pf), str(pw), cf, cw, out_dir=str(tmp_path))
