"""Host-side logic of bench.py: the split oracle run that times the CPU
baseline on several threads must reproduce one whole-stream oracle run."""
import numpy as np
import pytest

import bench
import oracle


@pytest.mark.parametrize("L,n_tasks", [(1, 3), (5, 8), (16, 4), (0, 5)])
def test_split_oracle_equals_whole_run(L, n_tasks):
    rng = np.random.default_rng(L * 10 + n_tasks)
    T, F, N, M = 40 * 16, 2, 8, 16
    x = rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)
    tasks = bench.split_oracle_tasks(T, F, M, L, n_tasks)
    # Every (channel, block) owned by exactly one task.
    owned = np.zeros((F, T // M), dtype=int)
    for f, b0, b1, h in tasks:
        owned[f, b0:b1] += 1
        assert 0 <= h <= b0 and b0 - h <= max(L - 1, 0)
    assert np.all(owned == 1)
    _, parts = bench.run_split_oracle(x, M, L, 0.0, 0.0, tasks, threads=3)
    whole = oracle.sk(x, M, L, 0, 5.0, 0.0, 0.0)
    for (f, b0, b1, h), (v, fl) in zip(tasks, parts):
        np.testing.assert_array_equal(v, whole.V[f, b0:b1])
        np.testing.assert_array_equal(fl, whole.flags[f, b0:b1])


def test_pass_a_algorithmic_bytes():
    # Input bytes plus 8 bytes of S1/S2 per (channel, block, input): the CHIME
    # M = 256 call is 2 GiB + 64 MiB, the figure the roofline divides by.
    import synth
    w = synth.chime(seed=3, block_len=256)
    assert bench.pass_a_bytes([w]) == (1 << 31) + (1 << 26)
    small = synth.Workload("pab", 48, 3, 64 * 5, 64, 1, np.full(48, 2.0), [])
    assert bench.pass_a_bytes([w, small]) == (1 << 31) + (1 << 26) + 48 * 3 * 320 + 8 * 3 * 5 * 48
