"""bench.py's accounting on the host: the per-pair work matches the figures the
measurement plan prints (FLOPs per pair with the fixed 2K encoder rows, crop
bytes with and without the contact store), and a kernel entry turns synthetic
launch times into rates and roofline fractions as stated."""

import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from paper_2304_09439_amd import inputs as I  # noqa: E402


@pytest.mark.parametrize("K,widths,n_points,mflop,crop_b", [
    (64, I.SMALL_WIDTHS, 1024, 2.462, 27_760),     # C0
    (128, I.SCALE_WIDTHS, 2048, 18.227, 55_408),   # C1-C3
    (128, I.SCALE_WIDTHS, 4096, 18.227, 104_560),  # C4 (4096 points per shape)
])
def test_per_pair_work_matches_the_plan(K, widths, n_points, mflop, crop_b):
    w = bench.per_pair_work(K, widths, n_points)
    assert (w["enc_flops"] + w["head_flops"]) / 1e6 == pytest.approx(mflop, abs=5e-4)
    assert w["crop_bytes"] + w["contact_bytes"] == crop_b   # the contact store is charged to the head
    assert w["row_flops"] * 2 * K == w["enc_flops"]


def test_kernel_entries_rates_and_fractions():
    w = bench.per_pair_work(128, I.SCALE_WIDTHS, 2048)
    P, steps = 16384, 20
    kt = {"crop": (steps, 0.1 * steps), "encoder_head_bf16": (steps, 0.2 * steps)}
    valid, tiles = P * 2 * 90, P * 2 * 96   # 90 member rows per object, in 96 rows of tiles
    k = bench.kernel_entries(kt, w, P, "scale", steps, "bf16", full_scan=False, rows=(valid, tiles))
    enc = k["encoder_head_bf16"]
    t = 0.2e-3
    method = valid * w["row_flops"] + w["head_flops"] * P
    assert enc["achieved"] == pytest.approx(method / t / 1e12, rel=1e-4)
    assert enc["frac"] == pytest.approx(enc["achieved"] / 2500.0, rel=1e-3)
    fixed = (w["enc_flops"] + w["head_flops"]) * P
    assert enc["fixed_2K_TFLOPs"] == pytest.approx(fixed / t / 1e12, rel=1e-4)
    assert enc["tiles_run_TFLOPs"] == pytest.approx((tiles * w["row_flops"] + w["head_flops"] * P) / t / 1e12,
                                                    rel=1e-4)
    assert enc["frac"] < enc["tiles_run_frac"] < enc["fixed_2K_frac"]
    crop = k["crop"]
    assert crop["bound"] == "hbm"
    assert crop["hbm_bytes_per_pair"] == 2 * 32 + 8 + 8 + 2 * 128 * 16
    assert crop["achieved"] == pytest.approx(crop["hbm_bytes_per_pair"] * P / 0.1e-3 / 1e9, rel=1e-4)
    assert crop["frac"] == pytest.approx(crop["achieved"] / 8000.0, rel=1e-3) and crop["frac"] < 1
    assert crop["scan_GBps"] == pytest.approx(w["crop_bytes"] * P / 0.1e-3 / 1e9, rel=1e-4)
    # the one-workgroup-per-CU kernel of the split schedule is charged the same work at the same peak
    kl = bench.kernel_entries({"crop": (steps, 0.1 * steps), "encoder_head_bf16_lds": (steps, 0.2 * steps)}, w, P,
                              "scale", steps, "bf16", full_scan=False, rows=(valid, tiles))
    lds = kl["encoder_head_bf16_lds"]
    assert lds["bound"] == "mfma" and lds["peak"] == 2500.0
    assert lds["achieved"] == pytest.approx(enc["achieved"], rel=1e-6)
    k32 = bench.kernel_entries({"crop": (1, 0.1), "head_fp32": (1, 0.3)}, w, P, "scale", 1, "fp32")
    assert k32["crop"]["hbm_bytes_per_pair"] == 2 * 32 + 8 + 8 + 2 * 128 * 32
    assert k32["head_fp32"]["achieved"] == pytest.approx(w["head_flops"] * P / 0.3e-3 / 1e12, rel=1e-4)


def test_encoder_rows_counts_valid_and_tile_rows():
    import numpy as np
    counts = np.array([[0, 5], [200, 33], [-1, -1], [128, 64]], np.int32)
    assert bench.encoder_rows(counts, 128) == (0 + 5 + 128 + 33 + 128 + 64, 0 + 32 + 128 + 64 + 128 + 64)


def test_mixed_precision_kernel_peak():
    """The FP8-encoder / BF16-head kernel is charged its encoder FLOPs at the FP8 peak and its head FLOPs at
    the BF16 peak: its peak is the rate at which that work would take its time at those peaks."""
    w = bench.per_pair_work(128, I.SCALE_WIDTHS, 2048)
    P = 1000
    rows = (P * 2 * 100, P * 2 * 128)
    k = bench.kernel_entries({"encoder_fp8_head_bf16": (1, 0.5)}, w, P, "scale", 1, "fp8_encoder", rows=rows)
    e = k["encoder_fp8_head_bf16"]
    enc, head = rows[0] * w["row_flops"], w["head_flops"] * P
    peak = (enc + head) / (enc / 5000.0 + head / 2500.0)
    assert e["peak"] == pytest.approx(peak, abs=0.1) and 2500 < e["peak"] < 5000
    assert e["frac"] == pytest.approx((enc + head) / 0.5e-3 / 1e12 / peak, abs=1e-4)
    assert "peak_basis" in e
    same = bench.kernel_entries({"encoder_head_fp8": (1, 0.5)}, w, P, "scale", 1, "fp8", rows=rows)
    assert same["encoder_head_fp8"]["peak"] == 5000.0 and "peak_basis" not in same["encoder_head_fp8"]


def test_sq_summary_from_counter_csv(tmp_path, capsys):
    """--summarize-sq: means per dispatch over two passes, the vector-issue bound and the matrix-core busy
    fraction derived as stated."""
    import argparse
    header = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value,Start_Timestamp,End_Timestamp\n"
    p1, p2 = tmp_path / "p1", tmp_path / "p2"
    p1.mkdir()
    p2.mkdir()
    rows1 = [f'{d},"void locc::crop_kernel<4, 2>(x)",SQ_VALU_MFMA_BUSY_CYCLES,{v},1000,{1000 + 50000}\n'
             for d, v in ((1, 1000.0), (2, 3000.0))]
    rows1 += ["3,other_kernel,SQ_VALU_MFMA_BUSY_CYCLES,99,0,1\n"]
    rows2 = [f'{d},"void locc::crop_kernel<4, 2>(x)",{c},{v},0,1\n'
             for d, c, v in ((1, "SQ_INSTS_VALU", 1e6), (2, "SQ_INSTS_VALU", 3e6), (1, "SQ_INSTS_MFMA", 10.0),
                             (2, "SQ_INSTS_MFMA", 30.0))]
    (p1 / "a_counter_collection.csv").write_text(header + "".join(rows1))
    (p2 / "b_counter_collection.csv").write_text(header + "".join(rows2))
    args = argparse.Namespace(summarize_sq=[str(p1), str(p2)], kernel="crop_bf16", kernel_match="crop_kernel<4, 2>")
    bench.summarize_sq(args)
    out = dict(line.split()[:2] for line in capsys.readouterr().out.splitlines() if len(line.split()) >= 2)
    assert float(out["SQ_INSTS_VALU"]) == 2e6 and float(out["SQ_INSTS_MFMA"]) == 20
    assert float(out["valu_issue_bound_ns"]) == pytest.approx(2e6 * 4 / (1024 * 2.4), abs=1)
    assert float(out["mfma_busy_frac"]) == pytest.approx(2000.0 / (1024 * 2.4 * 50000), abs=1e-3)
    assert float(out["valu_per_mfma"]) == pytest.approx(1e5)
    assert out["source_sha256"] == bench.source_hash("crop_bf16")
