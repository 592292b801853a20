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
    # A trial launch (a counter fill, then pass A, scan, combine<2>), then
    # three graph calls (pass A, scan, combine<4>), then a plan kernel.
    seq = [("__amd_rocclr_fillBufferAligned", 2), ("sk::batch_pass_a_kernel(x)", 100), ("sk::batch_scan_kernel(x)", 10),
           ("sk::batch_combine_kernel<2, int, true>(x)", 20)]
    for p in (200, 210, 220):
        seq += [("sk::batch_pass_a_kernel(x)", p), ("sk::batch_scan_kernel(x)", 12),
                ("sk::batch_combine_kernel<4, int, true>(x)", 30)]
    seq.append(("sk::pass_a_deferred_kernel<4, 16, true>(x)", 300))
    for name, dur in seq:
        k.append((name, t, t + dur * ns))
        t += dur * ns + 5 * ns
    _db(str(d / "run_results.db"), k)
    out = rs.trace(str(d), calls=True)
    lines = out.splitlines()
    row = next(l for l in lines if l.startswith("sk::batch_pass_a_kernel"))
    assert row.split()[1] == "4"                       # four pass A dispatches
    assert abs(float(row.split()[2]) - 182.5) < 1e-6  # their mean
    call = [l for l in lines if "calls of" in l]
    assert len(call) == 1                              # the trial launch after the fill is not a call
    assert call[0].strip().startswith("3 calls of 3 kernels")
    assert "pass A avg 210.00 us" in call[0]
    assert "pass B first start to last end avg 47.00 us" in call[0]   # scan start to combine end: 12 + 5 + 30
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
