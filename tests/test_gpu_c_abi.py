"""The library used from plain C: a gcc-built client (tests/c_abi) that
calls only the public header and the HIP runtime's C API, run as a child
process. It checks an exact result (constant power gives V = 0, every block
flagged low) and the shape-error path."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "sk_c_abi_check")


def test_plain_c_client():
    assert os.path.exists(BIN), f"{BIN} is not built; run __graft_entry__.build()"
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0 and "c abi ok" in r.stdout
