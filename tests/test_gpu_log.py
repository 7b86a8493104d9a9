"""The structured log on the GPU (MRC_LOG=3 in a fresh process): one line per
call with its status, sizes and counts, the per-kernel device times of the
call (level 2), and the serving batches and totals (level 3)."""
import json
import os
import subprocess
import sys

import pytest

from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, torch
sys.path.insert(0, sys.argv[1])
from paper_1810_03099_amd import mrc
from synth import corpus as synth
c = synth.generate(0, n_docs=600)
off, tok = torch.from_numpy(c.offsets).cuda(), torch.from_numpy(c.tokens).cuda()
ctx = mrc.mrc_ctx_create(0)
model, sig = mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(16))
mrc.mrc_sign(ctx, model, off, tok)
pairs, stats = mrc.mrc_compare(ctx, sig, 0.9, mrc.PREC_BF16)
db = mrc.mrc_db_create(ctx, 1000, 16)
mrc.mrc_db_insert(db, sig)
mrc.mrc_query(ctx, db, model, off[:11].contiguous(), tok, 16, 0.9, mrc.PREC_FP32)
srv = mrc.mrc_serve_start(ctx, db, model, max_batch=8, n_streams=1, topk=4)
tks = [mrc.mrc_serve_submit(srv, c.doc(i)) for i in range(20)]
res = [mrc.mrc_serve_poll(srv, t, wait_ms=60000) for t in tks]
mrc.mrc_serve_stop(srv)
print(int(stats["n_flagged"]), int(stats["n_band"]), sum(r.status == 0 for r in res))
"""


def test_log_levels_two_and_three(tmp_path):
    require_gpu()
    log = tmp_path / "mrc.jsonl"
    env = dict(os.environ, MRC_LOG="3", MRC_LOG_FILE=str(log))
    out = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    flagged, band, served = map(int, out.stdout.split())
    assert served == 20
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    calls = {x["call"]: x for x in lines if x["event"] == "call"}
    for name in ("mrc_build_and_sign", "mrc_compare", "mrc_db_insert", "mrc_query", "mrc_sign"):
        assert name in calls and calls[name]["status"] == 0, name
    cmp_ = calls["mrc_compare"]
    assert cmp_["n"] == 600 and cmp_["k"] == 16 and cmp_["precision"] == 1
    assert cmp_["flagged"] == flagged and cmp_["band_pairs"] == band
    assert "compare_lowp" in cmp_["stages"] and cmp_["stages"]["compare_lowp"]["ms"] > 0
    assert "sign_counts" in calls["mrc_build_and_sign"]["stages"]
    assert calls["mrc_query"]["collect_attempts"] >= 1
    assert calls["mrc_build_and_sign"]["n_docs"] == 600
    batches = [x for x in lines if x["event"] == "serve_batch"]
    assert sum(x["docs"] for x in batches if x["kind"] == "query") == 20
    stop = [x for x in lines if x["event"] == "serve_stop"]
    assert len(stop) == 1 and stop[0]["completed"] == 20 and stop[0]["rejected"] == 0
