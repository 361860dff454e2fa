"""Host-side logic of bench.py that needs no GPU: the multi-GPU refusal, the
byte models, and the rocprofv3 CSV summaries (on small hand-made files)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_update_bytes_model():
    # (4 nu + 14) vectors of 8 bytes per unknown: the window MAXPYs (4 nu reads),
    # u, w, m, n, r, x reads and p, s, q, z, x, r, u, w writes
    assert bench.window_update_bytes("pipefcg", 30, 1000) == (4 * 30 + 14) * 8 * 1000
    assert bench.iteration_bytes("pipefcg", 30, 5, 10) > bench.iteration_bytes("fcg", 30, 5, 10)


def test_traffic_guard(monkeypatch):
    # the stored counter reading is reported only for the kernel body it was taken on
    t = bench.update_traffic_bytes()
    assert t is None or t == pytest.approx(17.99e9, rel=1e-3)
    monkeypatch.setitem(bench.UPDATE_TRAFFIC, "body_sha1", "0" * 16)
    assert bench.update_traffic_bytes() is None


def _write(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(f'"{h}"' for h in header) + "\n")
        for r in rows:
            f.write(",".join(f'"{v}"' if isinstance(v, str) else str(v) for v in r) + "\n")


def test_trace_summary_steady_state(tmp_path):
    header = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = []
    t = 0
    for d in range(1, 11):        # ramp: 5 short dispatches, then 5 long ones
        dur = 1000 if d <= 5 else 3000
        rows.append(["KERNEL_DISPATCH", d, "pfk::k_pipefcg_update(long long, double*)", t, t + dur])
        t += dur + 10
    rows.append(["KERNEL_DISPATCH", 11, "void pfk::k_pcg_a<double, pfk::GridT<double, double> >(int)", t, t + 500])
    p = tmp_path / "trace.csv"
    _write(p, header, rows)
    out = bench.trace_summary(str(p), "k_pipefcg_update", 5)
    assert "k_pipefcg_update" in out and "k_pcg_a<double, GridT<double, double> >" in out
    assert "5 dispatches, mean 0.0030 ms" in out


def test_pmc_summary_means(tmp_path):
    header = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = [[1, "pfk::k_pipefcg_update(long long)", "FETCH_SIZE", 100.0],
            [2, "pfk::k_pipefcg_update(long long)", "FETCH_SIZE", 300.0],
            [3, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 50.0]]
    p = tmp_path / "pmc.csv"
    _write(p, header, rows)
    out = bench.pmc_summary(str(p))
    line = next(l for l in out.splitlines() if l.startswith("k_pipefcg_update"))
    assert line.split()[-2:] == ["2", "200.0"]


def test_cpu_baseline_steady_state_sample():
    # the oracle timing reaches the full window before it times, and reports
    # per-thread-count rates scaled to the 256^3 unit
    r = bench.cpu_baseline("pipefcg", n=16, steady=2)
    assert r["kind"] == "oracle" and r["unit"] == "outer_iters/s"
    assert r["cores"] >= 1 and r["host"]["nproc"] >= 1
    rates = r["it_per_s_16cube"]
    assert len(rates) == 2 and all(v > 0 for v in rates.values())
    assert r["value"] == pytest.approx(max(rates.values()) * 16 ** 3 / 256 ** 3, rel=1e-3)
    assert "31..32" in r["sample"]


def test_compact_line_is_short():
    cmp = {"fcg": {"it_per_s": 300.0}, "pipelined_over_unpipelined": 0.64,
           "algorithmic_GBps_whole_iteration": {"pipefcg": 5000.0, "fcg": 5400.0},
           "serving": {"burst": {"converged_solves_per_s": 25.0, "p50_ms": 1.0, "p99_ms": 2.0, "converged": 10,
                                 "requests": 10, "not_converged_sample": [{"n": 1}] * 50},
                       "poisson": {"0.5x": {"converged_solves_per_s": 12.0, "p50_ms": 1.0, "p99_ms": 3.0,
                                            "converged": 10, "not_converged_sample": [{"n": 1}] * 50}}}}
    c = bench.compact_compare(cmp, "fcg")
    assert "not_converged_sample" not in str(c)
    assert c["serving"]["0.5x"][0] == 12.0


def test_batch_member_tiling():
    # the tile width that pads an n x n plane least (64 x 8 or 32 x 16 tiles)
    assert bench.least_padding_tile(32) == 32 and bench.least_padding_tile(96) == 32
    assert bench.least_padding_tile(64) == 64 and bench.least_padding_tile(128) == 64
    assert bench.least_padding_tile(80) == 32 and bench.least_padding_tile(40) == 64

    class FakeOp:
        def set_tiling(self, tx, target, vb):
            self.args = (tx, target, vb)

    # the stencil target makes the z-range into chunks of about zc planes:
    # tiles per plane times ceil(n / zc)
    A = FakeOp()
    bench.batch_member_tiling(A, 96, 32, 512, 32)
    assert A.args == (32, 3 * 6 * 3, 512)
    bench.batch_member_tiling(A, 40, 64, 100, 16)
    assert A.args == (64, 1 * 5 * 3, 100)
