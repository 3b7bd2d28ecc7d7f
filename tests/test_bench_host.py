"""Host-side analysis in bench.py that the committed profiles rest on, on
synthetic rocprofv3 CSV files: the step-kernel gap analysis and the HBM
traffic from calibrated FETCH_SIZE / WRITE_SIZE counters."""
import csv
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _trace(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_kernel_trace.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writerows(rows)


def test_step_gaps_serial_launches(tmp_path):
    # ten 100 us step kernels with 20 us gaps, and an unrelated kernel that
    # must be ignored; skip=0 keeps every launch
    rows, t = [], 0
    for i in range(10):
        rows.append(["void fnr::k_render_step<1, 8, false>(fnr::RenderArgs)", t, t + 100_000])
        t += 120_000
    rows.append(["void fnr::k_render<0, 8, false>(fnr::RenderArgs)", 0, 5_000_000])
    _trace(str(tmp_path), rows)
    out = bench.step_gaps(str(tmp_path), skip=0.0)
    # window = 9 * 120 + 100 = 1180 us, gaps 9 * 20 = 180 us
    assert "window 1.2 ms, busy 0.847 of it" in out
    assert "mean duration 100.0 us, mean gap 20.0 us, total gap 0.2 ms" in out
    assert "10 launches, the last 10 analysed" in out


def test_step_gaps_overlapping_streams(tmp_path):
    # two streams: A runs 0-100, 150-250; B runs 50-180 (overlaps both):
    # the union is 0-250 with no idle time
    rows = [["k_render_step<1, 8, false>", 0, 100_000],
            ["k_render_step<3, 8, false>", 50_000, 180_000],
            ["k_render_step<1, 8, false>", 150_000, 250_000]]
    _trace(str(tmp_path), rows)
    out = bench.step_gaps(str(tmp_path), skip=0.0)
    assert "busy 1.000 of it" in out
    assert "total gap 0.0 ms" in out
    # a gap after the latest end seen so far, not after the previous launch's
    rows.append(["k_render_step<3, 8, false>", 300_000, 350_000])
    _trace(str(tmp_path), rows)
    out = bench.step_gaps(str(tmp_path), skip=0.0)
    assert "mean gap 16.7 us" in out  # gaps 0, 0, 50 us over three intervals


def _counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, name, v in rows:
            w.writerow([d, name, counter, v])


def test_pmc_traffic_calibration(tmp_path):
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(x)"
    ren = "void fnr::k_render_locc<0, 8, false>(fnr::RenderArgs)"
    f, w = str(tmp_path / "fetch"), str(tmp_path / "write")
    # the calibration kernel reads 1 GiB but FETCH_SIZE shows half of it
    # (factor 2); counter rows split over two per-XCD records per dispatch
    _counters(f, "FETCH_SIZE", [(1, neg, 262144.0), (1, neg, 262144.0), (2, neg, 524288.0),
                                (3, ren, 1000.0), (3, ren, 500.0)])
    _counters(w, "WRITE_SIZE", [(1, neg, 1048576.0), (2, ren, 200.0)])
    out = bench.pmc_traffic(f, w)
    assert out["fetch"]["calib_factor"] == pytest.approx(2.0)
    assert out["fetch"]["kib_per_dispatch"] == pytest.approx(1500.0)
    assert out["fetch"]["bytes"] == pytest.approx(1500.0 * 1024 * 2)
    assert out["write"]["calib_factor"] == pytest.approx(1.0)
    assert out["hbm_bytes_per_launch"] == round(1500 * 1024 * 2 + 200 * 1024)
    # missing calibration kernel: refused
    _counters(w, "WRITE_SIZE", [(2, ren, 200.0)])
    with pytest.raises(SystemExit):
        bench.pmc_traffic(f, w)


def test_pmc_traffic_l2_hit_rate(tmp_path):
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(x)"
    ren = "void fnr::k_render_locc<0, 8, false>(fnr::RenderArgs)"
    f, w, t = str(tmp_path / "fetch"), str(tmp_path / "write"), str(tmp_path / "tcc")
    _counters(f, "FETCH_SIZE", [(1, neg, 524288.0), (3, ren, 1000.0)])
    _counters(w, "WRITE_SIZE", [(1, neg, 1048576.0), (2, ren, 200.0)])
    os.makedirs(t, exist_ok=True)
    with open(os.path.join(t, "run_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writerows([(4, ren, "TCC_HIT_sum", 30.0), (4, ren, "TCC_MISS_sum", 90.0),
                      (5, neg, "TCC_HIT_sum", 1.0), (5, neg, "TCC_MISS_sum", 1.0)])
    out = bench.pmc_traffic(f, w, t)
    assert out["l2_hit_rate"] == pytest.approx(0.25)
    assert (out["tcc_hit"], out["tcc_miss"]) == (30.0, 90.0)


class _V:
    def __init__(self, H, W):
        self.H, self.W = H, W


def test_launch_units_scale_to_every_view_of_the_launch():
    """The oracle's per-ray averages over its sampled pixels are scaled to the
    rays of the whole launch, whatever number of views the oracle finished."""
    totals = dict(rays=1000, hit=700, occ_samples=28_000, pixels=2 * 640_000)
    views = [_V(800, 800)] * 40
    u = bench.launch_units(totals, views)
    assert u["rays"] == 40 * 640_000
    assert u["hit_rays"] == pytest.approx(0.7 * 40 * 640_000)
    assert u["occ_samples"] == pytest.approx(28 * 40 * 640_000)
    b = bench.alg_bytes(u, 100, 8)
    assert b["records"] == pytest.approx(u["occ_samples"] * 100)
    assert b["beta"] == pytest.approx(u["hit_rays"] * 128)
    assert b["writes"] == pytest.approx(u["rays"] * 16)
    assert b["total"] == pytest.approx(b["records"] + b["beta"] + b["writes"])
    # uneven views: rays counted per view
    u2 = bench.launch_units(dict(rays=10, hit=5, occ_samples=40, pixels=0),
                            [_V(256, 256), _V(720, 1280)])
    assert u2["rays"] == 256 * 256 + 720 * 1280
    assert u2["occ_samples"] == pytest.approx(4 * u2["rays"])


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and 1 <= h["usable_cpus"] <= h["nproc"]
    assert isinstance(h["cpu_model"], str) and h["cpu_model"]
    assert bench.oracle_threads() >= 1


def test_linebench_library_exports_and_checks_arguments():
    """The line-gather measurement library loads and exports its entry point;
    argument errors are caught before any device call (no GPU needed)."""
    import ctypes
    lb = ctypes.CDLL(os.path.join(bench.ROOT, "paper_2103_10380_amd", "liblinebench.so"))
    f = lb.fnr_line_gather
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    assert f(None, 1 << 20, 1 << 16, 0, 1, 1, 0, None, None) == -1        # null buffers
    fake = ctypes.c_void_p(16)
    assert f(fake, 1 << 20, 100, 0, 1, 1, 0, fake, None) == -1            # region not lines
    assert f(fake, 1 << 20, 1 << 21, 0, 1, 1, 0, fake, None) == -1        # region > buffer
    assert f(fake, 1 << 20, 1 << 16, 3, 1, 1, 0, fake, None) == -1        # unknown mode
    assert f(fake, 1 << 20, 1 << 16, 0, 0, 1, 0, fake, None) == -1        # no blocks
