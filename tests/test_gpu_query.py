"""GPU parity of the resident database and batched queries.

FP32 query results (top-16 ids and scores, hit counts) must equal, bit for
bit, the exact top lists computed with the oracle's FP32 chain on the same
unit vectors (score descending, id ascending); BF16 and FP8 queries must
return exactly the FP32 results. Against the FP64 oracle, each top-16 score
lies within the query's largest rounding bound (tests/fp_bounds.py), and a hit
count may differ only by rows whose float64 score lies within their bound of
tau."""
import numpy as np
import pytest
import torch

from oracle import mrc as om
from synth import corpus as synth
from tests.fp_bounds import matrix_bound
from tests.gpu_util import device_docs, flush, require_gpu

pytestmark = pytest.mark.gpu
TAU = 0.9


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.mrc_ctx_create(0)


def chain_topk(qunit, dbunit, topk, tau):
    nq, ndb = qunit.shape[0], dbunit.shape[0]
    ii = np.repeat(np.arange(nq), ndb)
    jj = np.tile(np.arange(ndb), nq)
    both = np.concatenate([qunit, dbunit]).astype(np.float32)
    s = om.score32_pairs(both, ii, jj + nq).reshape(nq, ndb)
    ids = np.full((nq, topk), -1, np.int64)
    sc = np.zeros((nq, topk), np.float32)
    for q in range(nq):
        o = np.lexsort((np.arange(ndb), -s[q].astype(np.float64)))[:topk]
        ids[q, :o.size] = o
        sc[q, :o.size] = s[q, o]
    return ids, sc, (s >= np.float32(tau)).sum(axis=1)


@pytest.fixture(scope="module")
def setup(lib, ctx):
    spec = synth.CONFIGS[1]
    dbc = synth.generate(1, n_docs=3000)
    qc = synth.generate_queries(spec, 150, seed=77, median=300, sigma=1.2, hi=6000, near_of=dbc, near_frac=0.4)
    o, t = device_docs(dbc)
    model = lib.mrc_build_vocab_idf(ctx, o, t, dbc.vocab, lib.ref_spec(64))
    db = lib.mrc_db_create(ctx, 4000, 64)
    first = lib.mrc_db_insert_docs(db, model, o, t)
    assert first == 0 and lib.mrc_db_size(db) == (3000, 64)
    sig_db = lib.mrc_sign(ctx, model, o, t)
    qo, qt = device_docs(qc)
    sig_q = lib.mrc_sign(ctx, model, qo, qt)
    dbunit = lib.mrc_normalise(ctx, sig_db)["unit"].cpu().numpy()
    qunit = lib.mrc_normalise(ctx, sig_q)["unit"].cpu().numpy()
    return dict(dbc=dbc, qc=qc, model=model, db=db, qo=qo, qt=qt, dbunit=dbunit, qunit=qunit)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_query_equals_exact_chain(lib, ctx, setup, prec):
    p = {"fp32": lib.PREC_FP32, "bf16": lib.PREC_BF16, "fp8": lib.PREC_FP8}[prec]
    ids, sc, hits = lib.mrc_query(ctx, setup["db"], setup["model"], setup["qo"], setup["qt"], 16, TAU, p)
    ids, sc, hits = ids.cpu().numpy(), sc.cpu().numpy(), hits.cpu().numpy()
    wids, wsc, whits = chain_topk(setup["qunit"], setup["dbunit"], 16, TAU)
    np.testing.assert_array_equal(ids, wids)
    np.testing.assert_array_equal(sc.view(np.uint32), wsc.view(np.uint32))
    np.testing.assert_array_equal(hits, whits)
    flush(f"  {prec}: mean hits {hits.mean():.2f}, queries with a hit {int((hits > 0).sum())}")


@pytest.mark.parametrize("form", ["grid", "persistent"])
@pytest.mark.parametrize("nq", [10, 40, 200])
def test_query_prefix_threshold_exact(lib, nq, form):
    # 20,000 rows: the first pass sees a 16,384-row prefix, whose 16th best is
    # only a lower bound; batches of 10, 40 and 200 queries run the collection
    # with 1, 2 and 4 query groups per wavefront
    # (both collection forms: grid-strided and persistent work items)
    ctx = lib.mrc_ctx_create(0)
    lib.mrc_ctx_set_scan(ctx, lib.SCAN_PERSISTENT if form == "persistent" else lib.SCAN_GRID)
    dbc = synth.generate(1)
    qc = synth.generate_queries(synth.CONFIGS[1], nq, seed=101 + nq, median=300, sigma=1.2, hi=6000, near_of=dbc,
                                near_frac=0.4)
    o, t = device_docs(dbc)
    model = lib.mrc_build_vocab_idf(ctx, o, t, dbc.vocab, lib.ref_spec(64))
    db = lib.mrc_db_create(ctx, dbc.n_docs, 64, precisions=(lib.PREC_BF16, lib.PREC_FP8))
    lib.mrc_db_insert_docs(db, model, o, t)
    qo, qt = device_docs(qc)
    dbunit = lib.mrc_normalise(ctx, lib.mrc_sign(ctx, model, o, t))["unit"].cpu().numpy()
    qunit = lib.mrc_normalise(ctx, lib.mrc_sign(ctx, model, qo, qt))["unit"].cpu().numpy()
    wids, wsc, whits = chain_topk(qunit, dbunit, 16, TAU)
    for p in (lib.PREC_FP32, lib.PREC_BF16, lib.PREC_FP8):
        ids, sc, hits = lib.mrc_query(ctx, db, model, qo, qt, 16, TAU, p)
        np.testing.assert_array_equal(ids.cpu().numpy(), wids)
        np.testing.assert_array_equal(sc.cpu().numpy().view(np.uint32), wsc.view(np.uint32))
        np.testing.assert_array_equal(hits.cpu().numpy(), whits)
    flush(f"  nq={nq} {form}: 20,000 rows, prefix threshold, all precisions == exact chain; mean hits "
          f"{whits.mean():.2f}")


@pytest.mark.parametrize("form", ["grid", "persistent"])
@pytest.mark.parametrize("k", [100, 512])
def test_query_k_shapes(lib, k, form):
    # k = 100: partial 16-component blocks in every layout; k = 512: the
    # largest query length (32 FP32 chunks, 16 BF16, 4 FP8)
    ctx = lib.mrc_ctx_create(0)
    lib.mrc_ctx_set_scan(ctx, lib.SCAN_PERSISTENT if form == "persistent" else lib.SCAN_GRID)
    dbc = synth.generate(2, n_docs=2500)
    qc = synth.generate_queries(synth.CONFIGS[2], 70, seed=9 + k, median=400, sigma=1.2, hi=6000, near_of=dbc,
                                near_frac=0.4)
    o, t = device_docs(dbc)
    model = lib.mrc_build_vocab_idf(ctx, o, t, dbc.vocab, lib.ref_spec(k))
    db = lib.mrc_db_create(ctx, dbc.n_docs, k)
    lib.mrc_db_insert_docs(db, model, o, t)
    qo, qt = device_docs(qc)
    dbunit = lib.mrc_normalise(ctx, lib.mrc_sign(ctx, model, o, t))["unit"].cpu().numpy()
    qunit = lib.mrc_normalise(ctx, lib.mrc_sign(ctx, model, qo, qt))["unit"].cpu().numpy()
    wids, wsc, whits = chain_topk(qunit, dbunit, 16, TAU)
    for p in (lib.PREC_FP32, lib.PREC_BF16, lib.PREC_FP8):
        ids, sc, hits = lib.mrc_query(ctx, db, model, qo, qt, 16, TAU, p)
        np.testing.assert_array_equal(ids.cpu().numpy(), wids)
        np.testing.assert_array_equal(sc.cpu().numpy().view(np.uint32), wsc.view(np.uint32))
        np.testing.assert_array_equal(hits.cpu().numpy(), whits)


def test_query_k_above_limit_rejected(lib, ctx):
    dbc = synth.generate(2, n_docs=300)
    o, t = device_docs(dbc)
    model = lib.mrc_build_vocab_idf(ctx, o, t, dbc.vocab, lib.ref_spec(600))
    db = lib.mrc_db_create(ctx, 400, 600)
    lib.mrc_db_insert_docs(db, model, o, t)
    with pytest.raises(lib.MrcError) as e:
        lib.mrc_query(ctx, db, model, o, t, 16, TAU)
    assert e.value.status == lib.MRC_E_INVAL


def test_query_vs_fp64_oracle(lib, ctx, setup):
    dbc, qc = setup["dbc"], setup["qc"]
    omodel = om.build_model(dbc.offsets, dbc.tokens, dbc.vocab, om.RefSpec(k=64))
    sdb = om.normalise(om.sign(dbc.offsets, dbc.tokens, omodel)[0])
    sq = om.normalise(om.sign(qc.offsets, qc.tokens, omodel)[0])
    oids, osc, ohits = om.query_topk(sdb, sq, 16, TAU)
    ids, sc, hits = lib.mrc_query(ctx, setup["db"], setup["model"], setup["qo"], setup["qt"], 16, TAU)
    sc, hits = sc.cpu().numpy().astype(np.float64), hits.cpu().numpy()
    bound = matrix_bound(setup["qunit"], sq, setup["dbunit"], sdb)
    # the k-th largest of two score lists that differ row by row by at most b
    # differ by at most b
    assert np.all(np.abs(sc - osc) <= bound.max(axis=1)[:, None])
    s64 = sq @ sdb.T
    near = np.abs(s64 - TAU) <= bound
    lo = ohits - (near & (s64 >= TAU)).sum(axis=1)      # near-tie hits the GPU may drop
    hi = ohits + (near & (s64 < TAU)).sum(axis=1)       # near-tie rows the GPU may add
    assert np.all((hits >= lo) & (hits <= hi)), np.nonzero((hits < lo) | (hits > hi))[0][:5]
    flush(f"  hits equal the fp64 oracle's for {int((hits == ohits).sum())} of {hits.size} queries; "
          f"near-tie rows {int(near.sum())}")


def test_query_edge_cases(lib, ctx, setup):
    m = setup["model"]
    small = lib.mrc_db_create(ctx, 10, 64)
    dbc = setup["dbc"].subset(range(5))
    o, t = device_docs(dbc)
    lib.mrc_db_insert_docs(small, m, o, t)
    qc = synth.from_docs([np.zeros(0, np.int32), dbc.doc(2)], dbc.vocab)
    qo, qt = device_docs(qc)
    for p in (lib.PREC_FP32, lib.PREC_BF16, lib.PREC_FP8):
        ids, sc, hits = lib.mrc_query(ctx, small, m, qo, qt, 16, TAU, p)
        ids = ids.cpu().numpy()
        assert ids[0, :5].tolist() == [0, 1, 2, 3, 4] and np.all(ids[0, 5:] == -1)   # zero query: ties by id
        assert ids[1, 0] == 2 and np.all(ids[1, 5:] == -1)
        assert hits.cpu().numpy()[1] >= 1
    with pytest.raises(lib.MrcError) as e:
        lib.mrc_db_insert_docs(small, m, *device_docs(setup["dbc"].subset(range(6))))
    assert e.value.status == lib.MRC_E_OVERFLOW


def test_db_save_load_roundtrip(lib, ctx, setup, tmp_path):
    p = tmp_path / "db.bin"
    lib.mrc_db_save(setup["db"], p)
    db2 = lib.mrc_db_load(ctx, p)
    assert lib.mrc_db_size(db2) == (3000, 64)
    for prec in (lib.PREC_FP32, lib.PREC_BF16):
        a = lib.mrc_query(ctx, setup["db"], setup["model"], setup["qo"], setup["qt"], 16, TAU, prec)
        b = lib.mrc_query(ctx, db2, setup["model"], setup["qo"], setup["qt"], 16, TAU, prec)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    raw = bytearray(p.read_bytes())
    raw[40] ^= 4
    p.write_bytes(bytes(raw))
    with pytest.raises(lib.MrcError):
        lib.mrc_db_load(ctx, p)


def test_query_rejects_malformed_input(lib, ctx, setup):
    """A query batch with an out-of-vocabulary token id, decreasing offsets or
    an end offset past its token buffer is rejected (MRC_E_INVAL), also on a
    context that has answered queries before (its scratch holds the last
    batch's signatures); the context stays usable."""
    m, db = setup["model"], setup["db"]
    qc = setup["qc"].subset(range(6))
    qo, qt = device_docs(qc)
    lib.mrc_query(ctx, db, m, setup["qo"], setup["qt"], 16, TAU)
    bad = qt.clone()
    bad[3] = qc.vocab
    cases = [("token id = vocab", qo, bad)]
    boff = qo.clone()
    boff[2] = boff[3] + 1
    cases.append(("decreasing offsets", boff, qt))
    boff = qo.clone()
    boff[-1] = qt.numel() + 1
    cases.append(("end offset past the tokens", boff, qt))
    for name, o, t in cases:
        for p in (lib.PREC_FP32, lib.PREC_BF16, lib.PREC_FP8):
            with pytest.raises(lib.MrcError) as e:
                lib.mrc_query(ctx, db, m, o, t, 16, TAU, p)
            assert e.value.status == lib.MRC_E_INVAL, name
    ids, sc, hits = lib.mrc_query(ctx, db, m, qo, qt, 16, TAU)
    wids, wsc, whits = chain_topk(setup["qunit"][:6], setup["dbunit"], 16, TAU)
    np.testing.assert_array_equal(ids.cpu().numpy(), wids)
    np.testing.assert_array_equal(hits.cpu().numpy(), whits)


@pytest.mark.parametrize("form", ["grid", "persistent"])
def test_query_candidate_capacity_grows(lib, form):
    """More than 2,048 rows at or above tau for one query: the collection's
    first per-query capacity (2,048 candidates on a fresh context) overflows,
    the call grows it and runs again, and the results still equal the exact
    chain's. The database holds 2,600 near copies of one document (1-3% of its
    tokens replaced) and 600 other documents; the model comes from an ordinary
    3,000-document corpus (built from the database itself, the copied terms
    would be the most frequent ones, which the default selection drops)."""
    c0 = synth.generate(1, n_docs=3000)
    rng = np.random.default_rng(2024)
    base = c0.doc(int(np.argmax(c0.lengths())))          # the longest document (about 2,000 tokens)
    docs = [c0.doc(i) for i in range(600)]
    for _ in range(2600):
        d = base.copy()
        pos = rng.choice(d.size, max(1, int(rng.uniform(0.01, 0.03) * d.size)), replace=False)
        d[pos] = rng.integers(0, c0.vocab, pos.size)
        docs.append(d)
    order = rng.permutation(len(docs))
    dbc = synth.from_docs([docs[i] for i in order], c0.vocab)
    qc = synth.from_docs([base, docs[700], docs[5]], c0.vocab)
    for prec in (lib.PREC_FP8, lib.PREC_BF16, lib.PREC_FP32):
        fresh = lib.mrc_ctx_create(0)
        lib.mrc_ctx_set_scan(fresh, lib.SCAN_PERSISTENT if form == "persistent" else lib.SCAN_GRID)
        model = lib.mrc_build_vocab_idf(fresh, *device_docs(c0), c0.vocab, lib.ref_spec(64))
        o, t = device_docs(dbc)
        db = lib.mrc_db_create(fresh, dbc.n_docs, 64)
        lib.mrc_db_insert_docs(db, model, o, t)
        qo, qt = device_docs(qc)
        dbunit = lib.mrc_normalise(fresh, lib.mrc_sign(fresh, model, o, t))["unit"].cpu().numpy()
        qunit = lib.mrc_normalise(fresh, lib.mrc_sign(fresh, model, qo, qt))["unit"].cpu().numpy()
        wids, wsc, whits = chain_topk(qunit, dbunit, 16, TAU)
        assert whits[0] > 2048 and whits[1] > 2048
        ids, sc, hits = lib.mrc_query(fresh, db, model, qo, qt, 16, TAU, prec)
        np.testing.assert_array_equal(ids.cpu().numpy(), wids)
        np.testing.assert_array_equal(sc.cpu().numpy().view(np.uint32), wsc.view(np.uint32))
        np.testing.assert_array_equal(hits.cpu().numpy(), whits)
        flush(f"  precision {prec}: hits {hits.cpu().numpy().tolist()} (first capacity 2048)")
        del db, model
        fresh.close()
