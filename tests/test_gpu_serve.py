"""Serving loop on the GPU: continuous batching over several streams.

Each query's result (top-16 ids and scores, hit count) must be identical
when the query runs alone and when it is submitted concurrently with others,
so that it lands in mixed batches overlapping on the device. Inserts get
consecutive ids and are found by later queries. A tiny memory cap makes the
admission control refuse requests (forced from the host; no device fault)."""
import threading

import numpy as np
import pytest
import torch

from synth import corpus as synth
from tests.gpu_util import device_docs, flush, require_gpu

pytestmark = pytest.mark.gpu
TAU = 0.9


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


@pytest.fixture(scope="module")
def env(lib):
    ctx = lib.mrc_ctx_create(0)
    dbc = synth.generate(1, n_docs=3000)
    o, t = device_docs(dbc)
    model = lib.mrc_build_vocab_idf(ctx, o, t, dbc.vocab, lib.ref_spec(64))
    db = lib.mrc_db_create(ctx, 5000, 64)
    lib.mrc_db_insert_docs(db, model, o, t)
    qc = synth.generate_queries(synth.CONFIGS[1], 240, seed=5, median=300, sigma=1.2, hi=9000, near_of=dbc,
                                near_frac=0.4)
    return dict(ctx=ctx, dbc=dbc, model=model, db=db, qc=qc)


def alone(lib, env, doc, prec):
    o, t = device_docs([doc])
    ids, sc, hits = lib.mrc_query(env["ctx"], env["db"], env["model"], o, t, 16, TAU, prec)
    return ids.cpu().numpy()[0], sc.cpu().numpy()[0], int(hits.cpu().numpy()[0])


@pytest.mark.parametrize("prec,form", [("fp32", "grid"), ("bf16", "grid"), ("fp8", "grid"), ("fp8", "persistent"),
                                       ("fp32", "persistent")])
def test_alone_equals_mixed(lib, env, prec, form):
    p = {"fp32": lib.PREC_FP32, "bf16": lib.PREC_BF16, "fp8": lib.PREC_FP8}[prec]
    qc = env["qc"]
    docs = [qc.doc(i) for i in range(qc.n_docs)]
    ref = [alone(lib, env, d, lib.PREC_FP32) for d in docs]
    # (servers started after this take the context's collection form)
    lib.mrc_ctx_set_scan(env["ctx"], lib.SCAN_PERSISTENT if form == "persistent" else lib.SCAN_GRID)
    try:
        srv = lib.mrc_serve_start(env["ctx"], env["db"], env["model"], max_batch=32, n_streams=3, topk=16, tau=TAU,
                                  precision=p, max_wait_us=300)
    finally:
        lib.mrc_ctx_set_scan(env["ctx"], lib.SCAN_GRID)
    results = {}
    lock = threading.Lock()

    def client(idx):
        tickets = [(i, lib.mrc_serve_submit(srv, docs[i])) for i in idx]
        for i, tk in tickets:
            r = lib.mrc_serve_poll(srv, tk, wait_ms=60000)
            assert r is not None and r.status == 0
            with lock:
                results[i] = r

    rng = np.random.default_rng(3)
    order = rng.permutation(len(docs))
    th = [threading.Thread(target=client, args=(order[w::4],)) for w in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    lib.mrc_serve_stop(srv)
    assert len(results) == len(docs)
    lat = []
    for i, (ids, sc, hits) in enumerate(ref):
        r = results[i]
        n = r.n_top
        got_ids = np.array([r.top[p].id for p in range(n)])
        got_s = np.array([r.top[p].s for p in range(n)], np.float32)
        valid = ids >= 0
        np.testing.assert_array_equal(got_ids, ids[valid])
        np.testing.assert_array_equal(got_s.view(np.uint32), sc[valid].view(np.uint32))
        assert r.n_hits == hits
        lat.append(r.t_done_ms - r.t_submit_ms)
    flush(f"  {prec} {form}: {len(docs)} queries mixed == alone; latency p50 {np.percentile(lat, 50):.2f} ms "
          f"p99 {np.percentile(lat, 99):.2f} ms")


def test_inserts_then_queries(lib, env):
    ctx = env["ctx"]
    db = lib.mrc_db_create(ctx, 1000, 64)
    srv = lib.mrc_serve_start(ctx, db, env["model"], max_batch=16, n_streams=2, topk=4, tau=TAU)
    dbc = env["dbc"]
    docs = [dbc.doc(i) for i in range(100)]
    tickets = [lib.mrc_serve_submit(srv, d, lib.REQ_INSERT) for d in docs]
    ids = []
    for tk in tickets:
        r = lib.mrc_serve_poll(srv, tk, wait_ms=60000)
        assert r.status == 0 and r.kind == lib.REQ_INSERT
        ids.append(r.id)
    assert sorted(ids) == list(range(100))
    # every inserted document finds itself (score 1, first place unless an identical copy has a lower id)
    qt = [lib.mrc_serve_submit(srv, docs[i]) for i in range(0, 100, 9)]
    for k, tk in zip(range(0, 100, 9), qt):
        r = lib.mrc_serve_poll(srv, tk, wait_ms=60000)
        assert r.status == 0
        top_ids = [r.top[p].id for p in range(r.n_top)]
        assert ids[k] in top_ids and r.n_hits >= 1
    lib.mrc_serve_stop(srv)


def test_admission_refuses_over_cap(lib, env):
    srv = lib.mrc_serve_start(env["ctx"], env["db"], env["model"], hbm_frac=1e-9, n_streams=1)
    tk = lib.mrc_serve_submit(srv, env["qc"].doc(0))
    r = lib.mrc_serve_poll(srv, tk, wait_ms=30000)
    assert r.status == lib.MRC_E_NOMEM
    with pytest.raises(lib.MrcError):
        lib.mrc_serve_submit(srv, np.array([env["dbc"].vocab + 5], np.int32))
    lib.mrc_serve_stop(srv)


def test_submit_many_equals_alone(lib, env):
    # all queries in one CSR call: each result equals the query run alone
    qc = env["qc"]
    srv = lib.mrc_serve_start(env["ctx"], env["db"], env["model"], max_batch=64, n_streams=2, topk=16, tau=TAU,
                              precision=lib.PREC_BF16, max_wait_us=300)
    tickets = lib.mrc_serve_submit_many(srv, qc.offsets, qc.tokens)
    assert len(tickets) == qc.n_docs and tickets == sorted(tickets)
    for i, tk in enumerate(tickets):
        r = lib.mrc_serve_poll(srv, tk, wait_ms=60000)
        assert r is not None and r.status == 0 and r.kind == lib.REQ_QUERY
        ids, sc, hits = alone(lib, env, qc.doc(i), lib.PREC_FP32)
        valid = ids >= 0
        np.testing.assert_array_equal(np.array([r.top[p].id for p in range(r.n_top)]), ids[valid])
        np.testing.assert_array_equal(np.array([r.top[p].s for p in range(r.n_top)], np.float32).view(np.uint32),
                                      sc[valid].view(np.uint32))
        assert r.n_hits == hits
    # a token id outside the vocabulary anywhere rejects the whole call (host check)
    bad_tok = qc.tokens[: int(qc.offsets[3])].copy()
    bad_tok[-1] = env["dbc"].vocab
    with pytest.raises(lib.MrcError):
        lib.mrc_serve_submit_many(srv, qc.offsets[:4], bad_tok)
    lib.mrc_serve_stop(srv)
    flush(f"  submit_many: {qc.n_docs} queries in one call == alone")


@pytest.mark.parametrize("order", ["ctx_first", "db_first"])
def test_handles_destroyed_in_any_order(lib, order):
    # a context destroyed before its model and database, and a database and
    # model destroyed while a server uses them, are freed only when the last
    # holder goes; the server keeps answering meanwhile
    c = synth.generate(0, n_docs=300)
    o, t = device_docs(c)
    ctx = lib.mrc_ctx_create(0)
    m = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(16))
    db = lib.mrc_db_create(ctx, 400, 16)
    lib.mrc_db_insert_docs(db, m, o, t)
    srv = lib.mrc_serve_start(ctx, db, m, max_batch=8, n_streams=1, topk=4, tau=TAU)
    if order == "ctx_first":
        ctx.close()
    db.close()
    m.close()
    r = lib.mrc_serve_poll(srv, lib.mrc_serve_submit(srv, c.doc(3)), wait_ms=60000)
    assert r is not None and r.status == 0 and r.n_hits >= 1 and r.top[0].s >= 0.999
    lib.mrc_serve_stop(srv)
    if order == "db_first":
        ctx.close()
