"""The wavefront-timeline summary (paper_1808_10365_amd.wave_timeline) on a
made-up timeline: no GPU needed."""
import numpy as np

from paper_1808_10365_amd.wave_timeline import summarize, text


def test_summarize_ranks_wavefronts_per_simd():
    # Two workgroups of 8 wavefronts; wavefronts j and j + 4 share SIMD j.
    # The first on each SIMD ends its reads at 200 us, the second at 260 us
    # (100 MHz ticks); XCD = workgroup index.
    rows = []
    for g in range(2):
        for j in range(8):
            start = 1000 + 10 * g
            reads = start + (20000 if j < 4 else 26000)
            rows.append([start, reads, reads + 400, g, 0, j % 4])
    s = summarize(np.array(rows, dtype=np.int64))
    assert s["wavefronts"] == 16
    assert s["start_us"] == (0.0, 0.1)
    first, second = s["reads_done_mean_by_simd_rank"]
    assert abs(first - 200.05) < 1e-9 and abs(second - 260.05) < 1e-9
    med = s["reads_done_median_by_xcd"]
    assert sorted(med) == [0, 1] and abs(med[0] - 230.0) < 1e-9 and abs(med[1] - 230.1) < 1e-9
    assert abs(s["stores_us_median"] - 4.0) < 1e-9
    assert "second 260.1 us" in text("t", s)
