"""Host-side pieces of bench.py: the one-GPU guard, the traffic summary
reader (kernel-source hash gate) and the operation model."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2 and "one GPU" in out.stderr


def _write_profile(path, sha, warmup=1, steps=2):
    with open(path, "w") as f:
        f.write("# rocprofv3 FETCH_SIZE / WRITE_SIZE of plits_kernel<8>\n")
        f.write(f"# kernel_sources_sha256: {sha}\n# warmup: {warmup}\n# steps: {steps}\n")
        f.write("# fetch_factor: 2.0\n# write_factor: 1.0\n")
        f.write("# dispatch generation fetch_kib write_kib\n")
        for g in range(1, warmup + steps + 1):
            f.write(f"{g} {g} {100.0 * g} {10.0 * g}\n")


def test_traffic_reader_scales_and_checks_the_kernel_hash(tmp_path, monkeypatch):
    prof = tmp_path / "p.txt"
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    _write_profile(prof, bench.plits_sources_sha256())
    # timed launches 2 and 3: (200*2 + 20) and (300*2 + 30) KiB
    want = ((200 * 2 + 20) + (300 * 2 + 30)) * 1024.0 / 2
    assert bench.plits_traffic(1, 2, "n50") == pytest.approx(want)
    assert bench.plits_traffic(1, 3, "n50") is None      # other run shape
    assert bench.plits_traffic(1, 2, "n70_70") is None   # other workload
    _write_profile(prof, "0" * 64)
    assert bench.plits_traffic(1, 2, "n50") is None      # kernel changed since


def test_operation_model_counts():
    # iters, moves, idle, cands, elig, nupd, snaps, repairs, cupd
    cnt = [10, 9, 1, 100, 20, 36, 2, 0, 36]
    n, nv = 10, 60
    per_iter = 2 * 2 + 7 * 11 + 10
    per_move = 8 + 3 * 12
    want = 100 * 10 + 20 * 10 + 10 * per_iter + 9 * per_move + 2 * 15
    assert bench.plits_alg_ops(cnt, n, nv) == want


def test_algorithmic_bytes_follow_the_move_definition():
    # iters, moves, idle, cands, elig, nupd, snaps, repairs, cupd
    cnt = [10, 9, 1, 100, 20, 36, 2, 0, 36]
    nv = 60
    # candidates: conflict + tabu entry read (2 + 2 bytes); neighbour updates:
    # one 2-byte conflict entry read and written; scan |V|/8 per iteration;
    # colour (1) and tabu entry (2) per move; |V| per snapshot
    want = 100 * 4 + 36 * 4 + 10 * 8 + 9 * 3 + 2 * 60
    assert bench.plits_alg_bytes(cnt, nv) == want


def test_fifo_replay_of_solo_service_times():
    # arrivals 0, 1, 1.5, 10; service 2, 2, 1, 1: the second waits for the
    # first, the third for the second, the fourth finds the server idle
    start, finish = bench.fifo_latencies([0.0, 1.0, 1.5, 10.0], [2.0, 2.0, 1.0, 1.0])
    assert start == [0.0, 2.0, 4.0, 10.0]
    assert finish == [2.0, 4.0, 5.0, 11.0]


def test_served_stream_rescales_with_the_rate():
    from paper_2103_10453_amd import instances as gen
    a = gen.workload_served(5, 10.0)
    b = gen.workload_served(5, 40.0)
    for x, y in zip(a, b):
        assert (x["grid"] == y["grid"]).all() and x["seed"] == y["seed"]
        assert x["arrival"] == pytest.approx(4.0 * y["arrival"])
