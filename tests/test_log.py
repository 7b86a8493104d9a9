"""The library's structured log (MRC_LOG, MRC_LOG_FILE) on the host: calls
that fail their argument checks (no device work) are logged at level 1 with
their status, and nothing is written at level 0. Each case runs in a fresh
process, since the library reads the environment once."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import ctypes as C, sys
sys.path.insert(0, sys.argv[1])
from paper_1810_03099_amd import mrc
L = mrc.lib()
n = C.c_int64()
opts = mrc.MrcCompareOpts(0.9, 0, 0.02, 0)
st1 = L.mrc_compare(None, None, 10, 16, C.byref(opts), None, 0, C.byref(n), None, None)
d = mrc.MrcDocs(0, None, None, 0)
st2 = L.mrc_sign(None, None, C.byref(d), None, None, None)
print(st1, st2)
"""


def _run(tmp_path, level):
    from paper_1810_03099_amd import mrc
    if not os.path.exists(mrc.LIB_PATH):
        pytest.skip("libmrc.so is not built")
    log = tmp_path / "mrc.jsonl"
    env = dict(os.environ, MRC_LOG=str(level), MRC_LOG_FILE=str(log))
    out = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == [str(mrc.MRC_E_INVAL)] * 2
    return [json.loads(x) for x in log.read_text().splitlines()] if log.exists() else []


def test_level_one_logs_failed_calls(tmp_path):
    lines = _run(tmp_path, 1)
    assert [x["call"] for x in lines] == ["mrc_compare", "mrc_sign"]
    for x in lines:
        assert x["event"] == "call" and x["status"] == -1 and x["wall_ms"] >= 0 and "t_ms" in x
    assert lines[0]["n"] == 10 and lines[0]["k"] == 16 and "flagged" not in lines[0]
    assert lines[1]["n_docs"] == 0


def test_level_zero_writes_nothing(tmp_path):
    assert _run(tmp_path, 0) == []
