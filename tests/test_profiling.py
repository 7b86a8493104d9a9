"""Host checks of the counter summaries (no GPU): the copy calibration of the
HBM traffic records uses the copy kernel's dispatches only."""
import csv

from paper_1810_03099_amd import profiling

HDR = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        w.writerows(rows)
    return str(path)


def test_copy_calibration_ignores_the_fill(tmp_path):
    fill = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>>(int)"
    copy = "__amd_rocclr_copyBuffer"
    # a 256 MiB copy whose FETCH_SIZE reads half of the bytes moved; the fill before it reads nothing
    rows = [[1, fill, "FETCH_SIZE", 16.8]] + [[d, copy, "FETCH_SIZE", 131072.0] for d in range(2, 7)]
    cf = _csv(tmp_path / "cf.csv", rows)
    mean, n = profiling.counter_mean(cf, "FETCH_SIZE", profiling.is_copy)
    assert n == 5 and mean == 131072.0
    assert not profiling.is_copy(fill) and profiling.is_copy(copy)


def test_traffic_record_scales_by_the_copy(tmp_path, monkeypatch):
    copy = "__amd_rocclr_copyBuffer"
    kern = "void (anonymous namespace)::k_compare_f32r(float const*, int)"
    cf = _csv(tmp_path / "cf.csv", [[d, copy, "FETCH_SIZE", 131072.0] for d in range(3)])
    cw = _csv(tmp_path / "cw.csv", [[d, copy, "WRITE_SIZE", 262144.0] for d in range(3)])
    kf = _csv(tmp_path / "kf.csv", [[d, kern, "FETCH_SIZE", 1000.0] for d in range(4)])
    kw = _csv(tmp_path / "kw.csv", [[d, kern, "WRITE_SIZE", 500.0] for d in range(4)])
    monkeypatch.setattr(profiling, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))

    class A:
        key, kernel, source = "k", "k_compare_f32r", "paper_1810_03099_amd/csrc/allpairs.h"
        fetch, write, copy_fetch, copy_write = kf, kw, cf, cw
        copy_bytes, command = 256 * 1024 * 1024, "cmd"

    rec = profiling.traffic(A)
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["bytes_per_launch"] == (1000.0 * 2.0 + 500.0) * 1024.0
    assert rec["dispatches"] == [4, 4]
