"""Host checks of the serving statistics in bench.py (no GPU): whole-run
percentiles, the percentile after the first fifth of the run, the worst
latency and the worst latency of each tenth of the run, on a scripted server
whose latencies are known."""
import numpy as np

import bench


class _Result:
    def __init__(self, t_submit, t_done):
        self.t_submit_ms, self.t_done_ms, self.status = t_submit, t_done, 0


class _ScriptedServer:
    """Request i is submitted at i ms and takes lat(i) ms."""
    REQ_QUERY = 0

    def __init__(self, lat):
        self.lat, self.n = lat, 0

    def mrc_serve_submit_many(self, srv, offs, toks):
        k = len(offs) - 1
        ids = list(range(self.n, self.n + k))
        self.n += k
        return ids

    def mrc_serve_poll(self, srv, tk, wait_ms=0):
        return _Result(float(tk), float(tk) + self.lat(tk))


def _run(n, lat):
    docs = [np.arange(5, dtype=np.int32)] * 3
    return bench.serve_run(_ScriptedServer(lat), None, [0.0] * n, docs)


def test_uniform_latency():
    out = _run(100, lambda i: 1.0)
    assert out["completed"] == 100
    assert out["p50_ms"] == 1.0 and out["p99_ms"] == 1.0 and out["max_ms"] == 1.0
    assert out["p99_after_first_fifth_ms"] == 1.0
    assert out["max_ms_by_tenth"] == [1.0] * 10


def test_stall_at_the_start_and_in_the_middle():
    # requests 0-9 (the first tenth) stalled 8 ms; request 55 stalled 5 ms
    out = _run(100, lambda i: 8.0 if i < 10 else (5.0 if i == 55 else 1.0))
    assert out["max_ms"] == 8.0
    assert out["p99_ms"] == np.percentile([8.0] * 10 + [5.0] + [1.0] * 89, 99)
    # after the first fifth (submitted at >= 19.8 ms): 80 requests, one of them 5 ms
    late = [5.0] + [1.0] * 79
    assert out["p99_after_first_fifth_ms"] == np.percentile(late, 99)
    by = out["max_ms_by_tenth"]
    assert by[0] == 8.0 and by[5] == 5.0
    assert all(by[w] == 1.0 for w in (1, 2, 3, 4, 6, 7, 8, 9))
