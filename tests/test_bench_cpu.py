"""Host-side logic of the measurement path: bench.py's refusal of more than
one GPU, the profile lookups it reports from, profsum's counter arithmetic
on a small synthetic rocprofv3 database, and the binding's refusal of
device buffers that a kernel would overrun."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2502_15539_amd import profsum  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workload_table_names_every_runner():
    kinds = {w[1] for w in bench.WORKLOADS.values()}
    assert kinds == {"u64", "cached", "bytes", "multi", "serve"}
    assert bench.WORKLOADS["u64_1e9"][0] == 10**9


def test_valu_peak_from_unit_counts():
    # 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction
    assert bench.VALU_PEAK_GINSTS == pytest.approx(614.4)
    # x 64 lanes x 2 (FMA) x 2 (dual issue) = the published fp32 vector peak
    assert bench.VALU_PEAK_GINSTS * 64 * 2 * 2 / 1000 == pytest.approx(157.3, rel=1e-3)


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// header\nint f(int x) { return x + 1; }  // trailing\n/* block\n comment */\n")
    monkeypatch.setattr(profsum, "HERE", str(tmp_path))
    monkeypatch.setattr(profsum, "KERNEL_SOURCES", ["k.hip"])
    h0 = profsum.kernel_source_hash()
    src.write_text("// another header\n\nint f(int x) { return x + 1; }\n")
    assert profsum.kernel_source_hash() == h0
    src.write_text("int f(int x) { return x + 2; }\n")
    assert profsum.kernel_source_hash() != h0


def _fake_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_counts_read_requests_by_size(tmp_path):
    # two dispatches: 1.0e9 and 1.1e9 128-byte line requests, a few 64- and
    # 32-byte ones, 8e9 bytes written; reads addressed to memory beside them
    reads = tmp_path / "r.db"
    write = tmp_path / "w.db"
    k = "ptrhash::query_pipelined<1, unsigned long>(...)"
    _fake_db(reads, [(k, "TCC_EA0_RDREQ_128B_sum", 1.0e9), (k, "TCC_EA0_RDREQ_128B_sum", 1.1e9),
                     (k, "TCC_EA0_RDREQ_64B_sum", 1e6), (k, "TCC_EA0_RDREQ_64B_sum", 1e6),
                     (k, "TCC_EA0_RDREQ_32B_sum", 2e6), (k, "TCC_EA0_RDREQ_32B_sum", 2e6),
                     (k, "TCC_EA0_RDREQ_DRAM_32B_sum", 4.2e9), (k, "TCC_EA0_RDREQ_DRAM_32B_sum", 4.2e9),
                     ("ptrhash::bench_copy_k<1>(...)", "TCC_EA0_RDREQ_128B_sum", 62.5e6)])
    _fake_db(write, [("ptrhash::bench_copy_k<1>(...)", "WRITE_SIZE", 8e9 / 1024), (k, "WRITE_SIZE", 8e9 / 1024)])
    out = tmp_path / "t.json"
    args = type("A", (), {"reads": str(reads), "write": str(write), "kernel": "query_pipelined<1, unsigned long>",
                          "out": str(out)})
    res = profsum.traffic(args)
    assert res["read_bytes"] == pytest.approx(1.05e9 * 128 + 1e6 * 64 + 2e6 * 32)  # mean of the two dispatches
    assert res["write_bytes"] == pytest.approx(8e9)
    assert res["traffic_bytes_per_launch"] == pytest.approx(res["read_bytes"] + 8e9)
    assert res["memory_read_bytes"] == pytest.approx(32 * 4.2e9)
    assert "L2" in res["level"]
    assert json.load(open(out))["kernel_source_sha256"] == profsum.kernel_source_hash()


def test_profile_lookups_report_only_matching_profiles(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("w", 10.0, 10**6) == (None, None)
    roof = bench.profiled_valu("w", 10.0, "query_pipelined<8, unsigned int>")
    assert roof["bound"] == "alu" and roof["achieved"] is None

    good = profsum.kernel_source_hash()
    json.dump({"traffic_bytes_per_launch": 1e9, "read_bytes": 9e8, "write_bytes": 1e8, "level": "L2",
               "kernel_source_sha256": good}, open(tmp_path / "profiles" / "traffic_w.json", "w"))
    b, info = bench.profiled_traffic("w", 10.0, 10**6)
    assert b == 1e9 and info["traffic_GBps"] == pytest.approx(100.0)
    json.dump({"traffic_bytes_per_launch": 1e9, "kernel_source_sha256": "stale"},
              open(tmp_path / "profiles" / "traffic_w.json", "w"))
    assert bench.profiled_traffic("w", 10.0, 10**6)[0] is None

    json.dump({"kernel": "query_pipelined<8, unsigned int>", "valu_insts_per_launch": 6.144e9, "valu_busy_pct": 90.0,
               "valu_utilization_pct": 70.0, "kernel_source_sha256": good},
              open(tmp_path / "profiles" / "valu_w.json", "w"))
    roof = bench.profiled_valu("w", 10.0, "query_pipelined<8, unsigned int>")
    assert roof["achieved"] == pytest.approx(614.4) and roof["frac"] == pytest.approx(1.0)
    roof = bench.profiled_valu("w", 10.0, "query_pipelined<4, unsigned int>")  # another shape: not comparable
    assert roof["achieved"] is None and roof["profiled_kernel"] == "query_pipelined<8, unsigned int>"


class _FakeDeviceTensor:
    """Stands in for a cuda tensor: the binding's checks read only these."""

    def __init__(self, n, itemsize, contiguous=True, cuda=True):
        self.is_cuda = cuda
        self._n, self._size, self._contig = n, itemsize, contiguous

    def is_contiguous(self):
        return self._contig

    def element_size(self):
        return self._size

    def numel(self):
        return self._n

    def data_ptr(self):
        return 4096


def test_binding_refuses_buffers_a_kernel_would_overrun():
    from paper_2502_15539_amd import ptrhash as P

    ok = P._device_tensor(_FakeDeviceTensor(10, 8), "keys", 8, 10)
    assert ok.value == 4096
    for t, msg in [(_FakeDeviceTensor(10, 8, cuda=False), "device"),
                   (_FakeDeviceTensor(10, 8, contiguous=False), "contiguous"),
                   (_FakeDeviceTensor(10, 4), "8-byte"),
                   (_FakeDeviceTensor(9, 8), "10 are needed")]:
        with pytest.raises(ValueError, match=msg):
            P._device_tensor(t, "keys", 8, 10)


def test_overlap_of_dispatches(tmp_path):
    db = tmp_path / "k.db"
    con = sqlite3.connect(db)
    con.execute('create table kernels (name text, start integer, "end" integer)')
    k = "ptrhash::query_multi<4>(...)"
    con.executemany("insert into kernels values (?, ?, ?)",
                    [(k, 0, 10), (k, 5, 15), (k, 15, 20), ("other", 0, 100), (k, 30, 40)])
    con.commit()
    con.close()
    spans = profsum.dispatch_spans(str(db), "query_multi")
    assert sorted(spans) == [(0, 10), (5, 15), (15, 20), (30, 40)]
    st = profsum.overlap_stats(spans)
    assert st["dispatches"] == 4 and st["max_concurrent"] == 2  # 15 ends as 15 starts: no third
    assert st["mean_concurrent"] == pytest.approx(35 / 30)
    assert st["share_of_busy_time_with_2_or_more"] == pytest.approx(5 / 30)


def test_timed_steps_are_the_last_before_the_rooflines():
    q = "void ptrhash::query_pipelined<1, unsigned long>(unsigned long const*, ...)"
    rows = [(q, 0, 30e6), (q, 40e6, 60e6)] + [(q, 100e6 + i * 20e6, 100e6 + i * 20e6 + 18e6) for i in range(5)]
    rows += [("void ptrhash::bench_gather_k<2>(...)", 300e6, 320e6), (q, 400e6, 450e6)]
    st = profsum.timed_steps(rows, "ptrhash::query_pipelined<1, unsigned long>", "bench_gather", 3)
    assert st["dispatches"] == 3 and st["avg_ms"] == pytest.approx(18.0)
    assert st["first_to_last_ms_per_step"] == pytest.approx((198e6 - 140e6) / 1e6 / 3)
    with pytest.raises(SystemExit):
        profsum.timed_steps(rows, "ptrhash::query_pipelined<1, unsigned long>", "bench_gather", 9)


def test_traffic_fetch_size_cross_check(tmp_path):
    k = "ptrhash::query_pipelined<1, unsigned long>(...)"
    reads, write, fetch = tmp_path / "r.db", tmp_path / "w.db", tmp_path / "f.db"
    _fake_db(reads, [(k, "TCC_EA0_RDREQ_128B_sum", 1e9)])
    _fake_db(write, [(k, "WRITE_SIZE", 8e9 / 1024)])
    _fake_db(fetch, [("ptrhash::bench_copy_k<1>(...)", "FETCH_SIZE", 4e9 / 1024), (k, "FETCH_SIZE", 64e9 / 1024)])
    args = type("A", (), {"reads": str(reads), "write": str(write), "kernel": "query_pipelined<1, unsigned long>",
                          "out": str(tmp_path / "t.json"), "fetch": str(fetch), "copy": "bench_copy_k<1>",
                          "copy_bytes": 8e9})
    res = profsum.traffic(args)
    assert res["fetch_size_check"]["scale"] == pytest.approx(2.0)
    assert res["fetch_size_check"]["fetch_bytes_scaled"] == pytest.approx(res["read_bytes"])
