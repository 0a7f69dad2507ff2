"""bench.py host logic that needs no GPU: the traffic figure is taken from
the committed counter summary only when it was measured on the same engine
source and Delta; rocprofv3 databases are summarised per kernel."""
import os
import sqlite3

import bench


def test_traffic_matches_engine_and_delta(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text("traffic_bytes_per_launch: 12345\ndelta: 512\nengine_code_sha256_16: " + bench.engine_hash() + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.read_traffic(512) == 12345.0
    assert bench.read_traffic(1024) is None
    fb = tmp_path / "traffic_b.txt"
    fb.write_text("traffic_bytes_per_launch: 777\ndelta: 1024\nbatch: 8\nengine_code_sha256_16: "
                  + bench.engine_hash() + "\n")
    monkeypatch.setattr(bench, "BATCH_TRAFFIC_FILE", str(fb))
    assert bench.read_traffic(1024, 8) == 777.0
    assert bench.read_traffic(1024, 16) is None and bench.read_traffic(512, 8) is None
    f.write_text("traffic_bytes_per_launch: 12345\ndelta: 512\nengine_code_sha256_16: 0000000000000000\n")
    assert bench.read_traffic(512) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic(512) is None


def test_engine_hash_ignores_comments_only():
    src = 'int a; // note\n  int  b; /* block\n note */ f("x  // y");\n'
    h = bench.engine_hash(src)
    assert bench.engine_hash('int a; int b; f("x  // y");') == h
    assert bench.engine_hash('int a;\n/* other words */ int b; f("x  // y"); // tail') == h
    assert bench.engine_hash('int a; int c; f("x  // y");') != h
    assert bench.engine_hash('int a; int b; f("x // y");') != h
    assert bench.engine_hash('int a; intb; f("x  // y");') != h


def test_committed_profile_is_current():
    """The committed traffic summaries were taken on the committed engine:
    the headline's batched launch of 8 queries at Delta 256, and one query
    per launch at Delta 512."""
    assert os.path.exists(bench.TRAFFIC_FILE) and os.path.exists(bench.BATCH_TRAFFIC_FILE)
    assert bench.read_traffic(256, 8) is not None
    assert bench.read_traffic(512) is not None


def test_kernel_profiles_are_current():
    """The committed kernel traces and counter summaries that stand for the
    current engine were taken on it (a code change without retaking them
    fails here); the older stall counters say which code they were taken on."""
    current = ["k_persistent_road4096_traffic.txt", "kernels_road4096_d512_fused.txt",
               "k_persistent_road4096_batch8_traffic.txt", "kernels_road4096_batch8_d256.txt",
               "k_persistent_road4096_batch8_counters.txt",
               "kernels_road4096_blocks_d2048.txt", "k_persistent_road4096_bins_counters.txt",
               "kernels_kcore_rmat24_lazy.txt", "kernels_sssp_rmat24_d32_unfused.txt",
               "kernels_sssp_rmat24_split_d64_kept_counters.txt"]
    h = bench.engine_hash()
    pdir = os.path.join(os.path.dirname(bench.TRAFFIC_FILE))
    for name in current:
        text = open(os.path.join(pdir, name)).read()
        assert "engine_code_sha256_16: " + h in text, name
    for name in ("k_persistent_road4096_stalls.txt",):
        assert "engine_code_sha256_16: " in open(os.path.join(pdir, name)).read(), name


def test_summarize_rocpd(tmp_path, capsys):
    db = tmp_path / "r.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration integer)")
    con.executemany("insert into kernels values (?, ?)", [("k_a", 100), ("k_a", 300), ("k_b", 50)])
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)",
                    [("k_a", "FETCH_SIZE", 10.0), ("k_a", "FETCH_SIZE", 30.0), ("k_a", "WRITE_SIZE", 5.0)])
    con.commit()
    con.close()
    assert bench.summarize_rocpd(str(db), None) == 0
    out = capsys.readouterr().out.splitlines()
    assert out[1].split()[:3] == ["k_a", "2", "200"]
    assert bench.summarize_rocpd(str(db), "FETCH_SIZE") == 0
    out = capsys.readouterr().out.splitlines()
    assert out[1].split()[:3] == ["k_a", "2", "20.00"]
