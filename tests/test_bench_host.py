"""Host-side logic of bench.py (no GPU): the kernel-name to pass mapping used
by the rocprofv3 summaries, the HBM-traffic lookup guarded by the hash of
the kernel sources, and the two summaries themselves on small synthetic
rocprofv3 CSV files (gated-off dispatches set apart, counter calibration)."""
import csv

import bench

KERNELS = {
    "void pk::prec_f32::k_x_res<256, false, true>(pk::XFwdArgs)": "x_r2c_residual_f32",
    "void pk::prec_f32::k_x_res<256, false, false>(pk::XFwdArgs)": "x_r2c_residual_f32",
    "void pk::prec_f32::k_x_res<256, true, false>(pk::XFwdArgs)": "x_r2c_residual_walls_f32",
    "void pk::prec_f64::k_x_div<256, false>(pk::XFwdArgs)": "x_r2c_divergence_f64",
    "void pk::prec_f64::k_x_fwd<256, false>(pk::XFwdArgs)": "x_r2c_f64",
    "void pk::prec_f32::k_x_fwd<48, true>(pk::XFwdArgs)": "x_r2c_walls_f32",
    "void pk::prec_f32::k_x_inv<256, true, false, true>(pk::XInvArgs)": "x_c2r_accumulate_f32",
    "void pk::prec_f32::k_x_inv<256, true, true, false>(pk::XInvArgs)":
        "x_c2r_accumulate_walls_f32",
    "void pk::prec_f32::k_x_inv<256, false, false, true>(pk::XInvArgs)": "x_c2r_f32",
    "void pk::prec_f64::k_x_inv<256, false, true, false>(pk::XInvArgs)": "x_c2r_walls_f64",
    "void pk::prec_f32::k_y<512, false, 2>(pk::YArgs)": "y_fwd_f32",
    "void pk::prec_f64::k_y<512, true, 0>(pk::YArgs)": "y_inv_f64",
    "void pk::prec_f64::k_yw<512, false>(pk::YArgs)": "y_fwd_walls_f64",
    "void pk::prec_f32::k_yw<96, true>(pk::YArgs)": "y_inv_walls_f32",
    "void pk::prec_f64::k_z_walls<16, 16, 256>(pk::ZArgs, int, int)": "z_walls_f64",
    "void pk::prec_f32::k_z_walls_r<8, 16, 512>(pk::ZArgs, int)": "z_walls_f32",
    "void pk::prec_f32::k_z_per<64>(pk::ZArgs, int)": "z_periodic_f32",
    "void pk::k_residual_check<256>(pk::XFwdArgs)": "residual_check_f64",
    "pk::k_sum_partials(double const*, int, double*, pk::ProbPtrs const*, int, int, int)":
        "sum_partials",
    "void pk::k_correct<256>(pk::CorrArgs)": "correct_f64",
    "pk::k_widen(float const*, double*, unsigned long)": None,
    "__amd_rocclr_copyBuffer": None,
}


def test_pass_of_kernel():
    for name, label in KERNELS.items():
        assert bench.pass_of_kernel(name) == label, name


def test_read_traffic_guarded_by_source_hash(tmp_path, monkeypatch):
    p = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(p))
    p.write_text(f"# comment\nsource_hash = {bench.kernel_hash()}\n"
                 "hbm_bytes[x_r2c_f32] = 1234   # read 1000 write 234\n")
    assert bench.read_traffic("x_r2c_f32") == 1234.0
    assert bench.read_traffic("y_fwd_f32") is None  # pass not in the file
    p.write_text("source_hash = 0123456789abcdef\nhbm_bytes[x_r2c_f32] = 1234\n")
    assert bench.read_traffic("x_r2c_f32") is None  # kernels changed since
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(tmp_path / "missing.txt"))
    assert bench.read_traffic("x_r2c_f32") is None


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_kernels_sets_gated_dispatches_apart(tmp_path):
    res = "void pk::prec_f32::k_x_res<256, false, true>(pk::XFwdArgs)"
    chk = "void pk::k_residual_check<256>(pk::XFwdArgs)"
    rows, t = [], 0
    for name, us in ((res, 100), (res, 4), (res, 110), (res, 120), (res, 4), (chk, 50)):
        rows.append((name, t, t + us * 1000))
        t += us * 1000 + 10
    trace = tmp_path / "trace.csv"
    _write_csv(trace, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = tmp_path / "kernels.txt"
    bench.summarize_kernels(str(trace), str(out), ["cmd"])
    line = next(ln for ln in out.read_text().splitlines() if ln.startswith("x_r2c_residual_f32"))
    f = line.split()
    assert f[1:7] == ["5", "2", "110.00", "100.00", "120.00", f[6]]
    assert abs(float(f[6]) - 100.0 * 338 / 388) < 0.01  # share of all kernel time


def test_summarize_counters_scales_by_the_calibration(tmp_path):
    gib = bench.COPY_BYTES
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>"
    xf = "void pk::prec_f32::k_x_fwd<256, false>(pk::XFwdArgs)"
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the calibration kernel reads its bytes twice in FETCH_SIZE, once in WRITE_SIZE
    _write_csv(tmp_path / "cf.csv", hdr, [(neg, "FETCH_SIZE", 2 * gib / 1024)] * 3)
    _write_csv(tmp_path / "cw.csv", hdr, [(neg, "WRITE_SIZE", gib / 1024)] * 3)
    # three working dispatches and one gated-off dispatch that read almost nothing
    _write_csv(tmp_path / "f.csv", hdr, [(xf, "FETCH_SIZE", v) for v in (1000, 1200, 1100, 5)])
    _write_csv(tmp_path / "w.csv", hdr, [(xf, "WRITE_SIZE", v) for v in (500, 500, 1)])
    out = tmp_path / "traffic.txt"
    bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                             str(tmp_path / "cf.csv"), str(tmp_path / "cw.csv"), str(out), [])
    kv = {}
    for ln in out.read_text().splitlines():
        ln = ln.split("#", 1)[0].strip()
        if "=" in ln:
            k, v = ln.split("=", 1)
            kv[k.strip()] = v.strip()
    assert float(kv["fetch_scale"]) == 0.5 and float(kv["write_scale"]) == 1.0
    assert kv["source_hash"] == bench.kernel_hash()
    # median of the working dispatches: fetch 1100 KiB x 0.5, write 500 KiB x 1
    assert float(kv["hbm_bytes[x_r2c_f32]"]) == 1100 * 1024 * 0.5 + 500 * 1024
