"""CPU tests of the rocprofv3 summary tool on a small synthetic database
with the tables it reads (kernels; counters_collection)."""
import sqlite3

from paper_1808_10365_amd import rocprof_summary as rs


def _db(path, kernels, counters=()):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer)")
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into kernels values (?, ?, ?)", kernels)
    con.executemany("insert into counters_collection values (?, ?, ?)", counters)
    con.commit()
    con.close()


def test_trace_stats_and_batched_calls(tmp_path):
    d = tmp_path / "tr"
    d.mkdir()
    ns = 1000
    k = []
    t = 0
    # A trial launch (pass A then pass B, no state kernel), then two graph calls.
    for name, dur in [("sk::batch_pass_a_kernel(x)", 100), ("sk::batch_scan_kernel(x)", 10),
                      ("sk::batch_combine_kernel<4, int, true>(x)", 20),
                      ("sk::batch_pass_a_kernel(x)", 200), ("sk::batch_scan_kernel(x)", 10),
                      ("sk::batch_combine_kernel<4, int, true>(x)", 30), ("sk::batch_state_kernel(x)", 4),
                      ("sk::batch_pass_a_kernel(x)", 210), ("sk::batch_scan_kernel(x)", 12),
                      ("sk::batch_combine_kernel<4, int, true>(x)", 30), ("sk::batch_state_kernel(x)", 4)]:
        k.append((name, t, t + dur * ns))
        t += dur * ns + 5 * ns
    _db(str(d / "run_results.db"), k)
    out = rs.trace(str(d), calls=True)
    lines = out.splitlines()
    row = next(l for l in lines if l.startswith("sk::batch_pass_a_kernel"))
    assert row.split()[1] == "3"                       # three pass A dispatches
    assert abs(float(row.split()[2]) - 170.0) < 1e-6  # their mean
    call = next(l for l in lines if "calls of" in l)
    assert call.strip().startswith("2 calls of 4 kernels")   # the trial launch is not a call
    assert "pass A avg 205.00 us" in call
    filt = rs.trace(str(d), include="scan")
    assert "batch_scan_kernel" in filt and "batch_pass_a_kernel" not in filt


def test_counters_scale_by_copy_probe(tmp_path):
    f, w = tmp_path / "f", tmp_path / "w"
    f.mkdir()
    w.mkdir()
    copy = "__amd_rocclr_copyBuffer"
    _db(str(f / "run_results.db"), [], [(copy, "FETCH_SIZE", 512.0), ("kern", "FETCH_SIZE", 100.0),
                                        ("kern", "FETCH_SIZE", 300.0)])
    _db(str(w / "run_results.db"), [], [(copy, "WRITE_SIZE", 1024.0), ("kern", "WRITE_SIZE", 50.0)])
    c = rs.counters(str(f), str(w), 1024 * 1024)
    assert abs(c["fetch_scale"] - 2.0) < 1e-12 and abs(c["write_scale"] - 1.0) < 1e-12
    kv = c["kernels"]["kern"]
    assert kv["dispatches"] == 2 and kv["fetch_kib"] == 200.0 and kv["write_kib"] == 50.0
    text = rs.counters_text(c)
    # 200 KiB x 2 + 50 KiB x 1 = 460800 bytes.
    assert "0.46" in next(l for l in text.splitlines() if l.startswith("kern "))
