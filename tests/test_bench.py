"""Host logic of bench.py (CPU): the reduction of the two rocprofv3 counter
passes to HBM bytes per dispatch, the roofline object of the dominant kernel,
and the one-GPU guard.  No GPU is touched."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_csv(path, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, name, counter, value in rows:
            f.write(f'{d},"{name}",{counter},{value}\n')


def test_pmc_summary_calibrates_by_the_copy_and_counts_only_the_step_after_it(tmp_path, capsys):
    """FETCH_SIZE and WRITE_SIZE are scaled so that the largest copy dispatch
    reads and writes exactly COPY_BYTES; dispatches before the copy (the
    warm-up step) are left out; radix forms of an NTT pass are merged and
    counter instances of one dispatch summed."""
    kib = bench.COPY_BYTES / 1024
    fetch = [(1, "k_kip(fk::KipArgs)", "FETCH_SIZE", 999999.0),                 # warm-up: ignored
             (2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 4),             # reads count half
             (3, "k_ntt_fwd_cols(fk::NttArgs)", "FETCH_SIZE", 100.0),
             (4, "k_ntt_fwd_cols16(fk::NttArgs)", "FETCH_SIZE", 150.0),
             (4, "k_ntt_fwd_cols16(fk::NttArgs)", "FETCH_SIZE", 50.0),          # second instance
             (5, "k_kip(fk::KipArgs)", "FETCH_SIZE", 400.0)]
    write = [(1, "k_kip(fk::KipArgs)", "WRITE_SIZE", 999999.0),
             (2, "__amd_rocclr_copyBuffer", "WRITE_SIZE", kib / 2),
             (3, "k_ntt_fwd_cols(fk::NttArgs)", "WRITE_SIZE", 80.0),
             (4, "k_ntt_fwd_cols16(fk::NttArgs)", "WRITE_SIZE", 120.0),
             (5, "k_kip(fk::KipArgs)", "WRITE_SIZE", 10.0)]
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(f, fetch)
    _write_csv(w, write)
    bench.pmc_summary(str(f), str(w))
    out = capsys.readouterr().out
    res = json.loads(out.strip().splitlines()[-1])["hbm_GB_per_dispatch"]
    ff, fw = 4.0, 2.0     # COPY_BYTES / (counter value of the copy)
    ntt = ((100 * ff + 80 * fw) + (200 * ff + 120 * fw)) / 2 * 1024 / 1e9
    kip = (400 * ff + 10 * fw) * 1024 / 1e9
    assert set(res) == {"ntt_fwd_cols", "kip"}
    assert res["ntt_fwd_cols"] == pytest.approx(round(ntt, 4))
    assert res["kip"] == pytest.approx(round(kip, 4))


def test_roofline_takes_the_kernel_with_the_most_time_and_its_measured_traffic():
    kernels = {
        "kip": {"ms_per_step": 10.0, "achieved_GBs": 4000.0, "avg_launch_us": 100.0, "launches": 100,
                "bytes_per_launch": 4e8, "frac_copy_ceiling": 4000.0 / bench.COPY_CEILING_GBS},
        "ntt_fwd_cols": {"ms_per_step": 20.0, "achieved_GBs": 5000.0, "avg_launch_us": 400.0, "launches": 50,
                         "bytes_per_launch": 2e9, "frac_copy_ceiling": 5000.0 / bench.COPY_CEILING_GBS,
                         "modmul_per_s": 1.2e12, "frac_modmul_peak": 1.2e12 / bench.MODMUL_PEAK},
    }
    r = bench.roofline(kernels, "mobilenet")
    assert r["kernel"] == "ntt_fwd_cols" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["peak"] == bench.HBM_PEAK_GBS and r["frac"] == pytest.approx(5000.0 / 8000.0, abs=1e-4)
    assert r["traffic"] == bench.TRAFFIC[("mobilenet", "ntt_fwd_cols")]
    assert r["alu"]["peak"] == bench.MODMUL_PEAK and r["alu"]["frac"] == pytest.approx(1.2e12 / bench.MODMUL_PEAK)
    # a kernel whose counters were not taken for this workload reports no traffic
    assert bench.roofline({"kip": kernels["kip"]}, "mobilenet")["traffic"] is None


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
