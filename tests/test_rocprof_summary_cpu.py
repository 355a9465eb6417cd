"""The rocprofv3 summariser on synthetic profiler output: per-launch HBM
bytes scaled by the streaming copy's counter reading, the counter record
keyed by tile shape and grid, and the generic counter table."""
import csv
import json
import sqlite3
import subprocess
import sys

ROOT = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
SPMM = "void mb::k_spmm<mb::BpShape<4, 128, 1, 2, 4, 0> >(int const*)"
COPY = "mb::k_stream_copy(double*)"


def _files(tmp):
    db = tmp / "t.db"
    con = sqlite3.connect(db)
    c = con.cursor()
    c.execute("create table rocpd_info_kernel_symbol_x (id int, display_name text)")
    c.execute("create table rocpd_kernel_dispatch_x (id int, kernel_id int, start int, end int, "
              "grid_size_x int, workgroup_size_x int)")
    c.execute("insert into rocpd_info_kernel_symbol_x values (1, ?), (2, ?)", (SPMM, COPY))
    rows = [(i, 1, 0, 70000, 1536 * 256, 256) for i in range(4)]
    rows += [(10 + i, 1, 0, 90000, 512 * 256, 256) for i in range(2)]
    rows += [(20, 1, 0, 1000, 1536 * 256, 256)]          # an early exit: left out
    rows += [(30, 2, 0, 400000, 8192 * 256, 256)]
    c.executemany("insert into rocpd_kernel_dispatch_x values (?,?,?,?,?,?)", rows)
    con.commit()
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name",
           "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    paths = {}
    # the copy moves 1 GiB each way; its counter reads half (fetch) and all (write)
    for name, counter, val, copy_val in (("f.csv", "FETCH_SIZE", 100000.0, 524288.0),
                                         ("w.csv", "WRITE_SIZE", 20000.0, 1048576.0)):
        with open(tmp / name, "w", newline="") as fh:
            w = csv.writer(fh)
            w.writerow(hdr)
            for d in range(4):
                w.writerow([d, SPMM, 1536 * 256, 256, counter, val, 0, 70000])
            for d in range(2):
                w.writerow([10 + d, SPMM, 512 * 256, 256, counter, val / 2, 0, 90000])
            w.writerow([20, SPMM, 1536 * 256, 256, counter, 1.0, 0, 1000])
            w.writerow([30, COPY, 8192 * 256, 256, counter, copy_val, 0, 400000])
        paths[counter] = tmp / name
    return db, paths["FETCH_SIZE"], paths["WRITE_SIZE"]


def run(*args):
    r = subprocess.run([sys.executable, "-m", "paper_2608_07327_amd.rocprof_summary", *args],
                       cwd=ROOT, capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_record_is_keyed_by_shape_and_grid_and_scaled_by_the_copy(tmp_path):
    db, f, w = _files(tmp_path)
    rec_path = tmp_path / "rec.json"
    out = run(str(db), str(f), str(w), "--record", str(rec_path), "--sources",
              "k_sparse.hip,dev_common.hpp")
    assert "factor 2.000" in out and "factor 1.000" in out
    rec = json.load(open(rec_path))
    assert set(rec["per_shape"]) == {"4,128,1,2,4,0@1536", "4,128,1,2,4,0@512"}
    e = rec["per_shape"]["4,128,1,2,4,0@1536"]
    # 100000 KiB x 2 (fetch factor) and 20000 KiB x 1 (write factor)
    assert e["fetch_bytes"] == 100000 * 1024 * 2 and e["write_bytes"] == 20000 * 1024
    assert e["launches"] == 4 and e["avg_us"] == 70.0
    e2 = rec["per_shape"]["4,128,1,2,4,0@512"]
    assert e2["fetch_bytes"] == 50000 * 1024 * 2 and e2["avg_us"] == 90.0
    assert len(rec["kernel_hash"]) == 16
    assert rec["hashed_sources"] == ["paper_2608_07327_amd/csrc/k_sparse.hip",
                                     "paper_2608_07327_amd/csrc/dev_common.hpp"]


def test_counter_table_averages_busy_launches_per_grid(tmp_path):
    _, f, w = _files(tmp_path)
    out = run("--counters", str(f), str(w), "--filter", "k_spmm")
    rows = [l for l in out.splitlines() if l.startswith("| `k_spmm")]
    assert len(rows) == 2
    r1536 = [r for r in rows if "| 1536 |" in r][0]
    assert "| 1e+05 | 2e+04 |" in r1536      # the early-exit launch is left out
