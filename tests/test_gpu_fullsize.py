"""GPU parity at the full benchmark sizes, in the bench's launch configuration
(mrc_build_and_sign, then mrc_compare over the whole corpus).

Full-size outputs are checked where the oracle can follow them:
  * signatures of sampled documents against the float64 oracle (model of the
    whole corpus), to 1e-5 absolute;
  * every flagged pair's score equals the float32 chain over the GPU's unit
    signatures bit for bit, and randomly sampled pairs are flagged exactly when
    their chain score is >= tau;
  * the flagged set against the float64 oracle's decisions (all pairs of the
    20,000-document corpus; all pairs of a 5,000-document subsample of the
    200,000-document one), except pairs whose float64 score lies within its
    rounding bound of tau (tests/fp_bounds.py);
  * the BF16 and FP8 forms flag exactly the FP32 set."""
import numpy as np
import pytest
import torch

from oracle import mrc as om
from synth import corpus as synth
from tests.fp_bounds import pair_bound
from tests.gpu_util import flush, require_gpu

pytestmark = pytest.mark.gpu
TAU = 0.9
SIG_TOL = 1e-5


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.mrc_ctx_create(0)


def _build(lib, ctx, cfg):
    c = synth.generate(cfg)
    k = synth.CONFIGS[cfg].k
    off = torch.from_numpy(c.offsets).cuda()
    tok = torch.from_numpy(c.tokens).cuda()
    sig = torch.empty((c.n_docs, k), dtype=torch.float32, device="cuda")
    model, _ = lib.mrc_build_and_sign(ctx, off, tok, c.vocab, lib.ref_spec(k), sig_out=sig)
    return c, k, model, sig


def _check_signatures(c, k, sig, m, rows):
    sub = c.subset(rows)
    osig, _ = om.sign(sub.offsets, sub.tokens, m)
    got = sig[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    err = np.abs(got - osig).max()
    assert err <= SIG_TOL, err
    return err


def _check_chain(lib, ctx, sig, gi, gj, gs, n, rng, n_sample):
    unit = lib.mrc_normalise(ctx, sig)["unit"].cpu().numpy()
    ref = om.score32_pairs(unit, gi, gj)
    np.testing.assert_array_equal(gs.view(np.uint32), ref.view(np.uint32))
    i = rng.integers(0, n, n_sample)
    j = rng.integers(0, n, n_sample)
    keep = i != j
    i, j = np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])
    s = om.score32_pairs(unit, i, j)
    flagged = set(zip(gi.tolist(), gj.tolist()))
    got = np.array([(a, b) in flagged for a, b in zip(i.tolist(), j.tolist())])
    np.testing.assert_array_equal(got, s >= np.float32(TAU))
    return int(got.sum())


def _check_vs_fp64(unit, shat, gset, oi, oj, restrict=None):
    """Decisions against the float64 oracle: a pair may differ only if its
    float64 score lies within the pair's rounding bound of tau. `unit` holds
    the GPU's float32 unit rows for the oracle's rows `shat`."""
    oset = set(zip(oi.tolist(), oj.tolist()))
    if restrict is not None:
        gset = {(a, b) for a, b in gset if a < restrict and b < restrict}
    diff = sorted((gset - oset) | (oset - gset))
    if diff:
        di = np.array([p[0] for p in diff])
        dj = np.array([p[1] for p in diff])
        s64 = om.pair_scores(shat, di, dj)
        b = pair_bound(unit, shat, di, dj)
        assert np.all(np.abs(s64 - TAU) <= b), (s64 - TAU)[np.abs(s64 - TAU) > b][:5]
    return len(gset & oset), len(diff)


def test_plain_full_20k_k64(lib, ctx):
    c, k, model, sig = _build(lib, ctx, 1)
    n = c.n_docs
    flush(f"  plain_full n={n} k={k} tokens={c.tokens.size}")
    m = om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=k))
    info = lib.mrc_model_info(model)
    assert (info["n_listed"], info["lo"], info["hi"]) == (m.order.size, m.lo, m.hi)
    np.testing.assert_array_equal(lib.mrc_model_get(model)["df"], m.df)
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(n, 300, replace=False))
    err = _check_signatures(c, k, sig, m, rows)
    pairs, st = lib.mrc_compare(ctx, sig, TAU, lib.PREC_FP32, capacity=8 * 1024 * 1024)
    gi, gj, gs, _ = lib.pairs_to_numpy(pairs)
    assert st["n_flagged"] == gi.size and np.all(gi < gj)
    hits = _check_chain(lib, ctx, sig, gi, gj, gs, n, rng, 400_000)
    # float64 oracle over all pairs of the corpus
    osig, _ = om.sign(c.offsets, c.tokens, m)
    shat = om.normalise(osig)
    oi, oj, _ = om.compare_pairs(shat, TAU)
    gset = set(zip(gi.tolist(), gj.tolist()))
    unit = lib.mrc_normalise(ctx, sig)["unit"].cpu().numpy()
    common, ties = _check_vs_fp64(unit, shat, gset, oi, oj)
    for name, p in [("bf16", lib.PREC_BF16), ("fp8", lib.PREC_FP8)]:
        pl, _ = lib.mrc_compare(ctx, sig, TAU, p, 0.02, capacity=8 * 1024 * 1024)
        li, lj, _, _ = lib.pairs_to_numpy(pl)
        assert set(zip(li.tolist(), lj.tolist())) == gset, name
    flush(f"    sig max err {err:.2e}; flagged {gi.size}; sampled hits {hits}; fp64 common {common}, "
          f"near-tie differences {ties}")


def test_precision_200k_k256_sampled(lib, ctx):
    c, k, model, sig = _build(lib, ctx, 2)
    n = c.n_docs
    flush(f"  precision n={n} k={k} tokens={c.tokens.size}")
    m = om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=k))
    rng = np.random.default_rng(6)
    rows = np.sort(rng.choice(n, 300, replace=False))
    err = _check_signatures(c, k, sig, m, rows)
    pairs, st = lib.mrc_compare(ctx, sig, TAU, lib.PREC_FP32, capacity=16 * 1024 * 1024)
    gi, gj, gs, _ = lib.pairs_to_numpy(pairs)
    assert st["n_flagged"] == gi.size and np.all(gi < gj)
    hits = _check_chain(lib, ctx, sig, gi, gj, gs, n, rng, 400_000)
    gset = set(zip(gi.tolist(), gj.tolist()))
    for name, p in [("bf16", lib.PREC_BF16), ("fp8", lib.PREC_FP8)]:
        pl, _ = lib.mrc_compare(ctx, sig, TAU, p, 0.02, capacity=16 * 1024 * 1024)
        li, lj, _, _ = lib.pairs_to_numpy(pl)
        assert set(zip(li.tolist(), lj.tolist())) == gset, name
    # float64 oracle decisions on all pairs of the first 5,000 documents
    sub = c.subset(np.arange(5000))
    osig, _ = om.sign(sub.offsets, sub.tokens, m)
    shat = om.normalise(osig)
    oi, oj, _ = om.compare_pairs(shat, TAU)
    unit = lib.mrc_normalise(ctx, sig[:5000].contiguous())["unit"].cpu().numpy()
    common, ties = _check_vs_fp64(unit, shat, gset, oi, oj, restrict=5000)
    flush(f"    sig max err {err:.2e}; flagged {gi.size}; sampled hits {hits}; subsample fp64 common {common}, "
          f"near-tie differences {ties}")


def _chain_topk_rows(both, qrows, n_db, topk, tau):
    """Exact top lists of the listed query rows of `both` (its first n_db rows
    are the database) by the oracle's float32 chain over every database row
    (score descending, id ascending) and their counts of rows >= tau. Queries
    are scored in threads: each chain call is a foreign call that releases the
    interpreter lock."""
    from concurrent.futures import ThreadPoolExecutor
    db_ids = np.arange(n_db, dtype=np.int64)

    def one(qr):
        s = om.score32_pairs(both, np.full(n_db, qr, np.int64), db_ids)
        t = np.partition(s, n_db - topk)[n_db - topk]          # the topk-th largest score
        cand = np.nonzero(s >= t)[0]
        o = cand[np.lexsort((cand, -s[cand].astype(np.float64)))][:topk]
        return o, s[o], int((s >= np.float32(tau)).sum())

    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(one, qrows))


def test_serving_1m_k128_query_batch_sampled(lib, ctx):
    """The serving database at full size: 1,000,000 signed documents (k = 128,
    FP32 + BF16 copies) and one 4,096-query mrc_query batch, as the serving
    loop issues it. For 64 sampled queries the top-16 ids, scores (bit for bit)
    and hit counts equal the oracle's float32 chain over all 1,000,000 rows, at
    both precisions."""
    cs = synth.CONFIGS[3]
    flush("  generating the 1,000,000-document corpus")
    c = synth.generate(3)
    k = cs.k
    off = torch.from_numpy(c.offsets).cuda()
    tok = torch.from_numpy(c.tokens).cuda()
    sig = torch.empty((c.n_docs, k), dtype=torch.float32, device="cuda")
    model, _ = lib.mrc_build_and_sign(ctx, off, tok, c.vocab, lib.ref_spec(k), sig_out=sig)
    db = lib.mrc_db_create(ctx, c.n_docs, k, precisions=(lib.PREC_BF16,))
    assert lib.mrc_db_insert(db, sig) == 0
    del off, tok
    qc = synth.generate_queries(cs, 4096, seed=31, median=400, sigma=1.2, hi=20000, near_of=c, near_frac=0.2)
    qo = torch.from_numpy(qc.offsets).cuda()
    qt = torch.from_numpy(qc.tokens).cuda()
    flush(f"  database {c.n_docs} x k={k}; 4096 queries, {qc.tokens.size} tokens")
    dbunit = lib.mrc_normalise(ctx, sig)["unit"].cpu().numpy()
    qunit = lib.mrc_normalise(ctx, lib.mrc_sign(ctx, model, qo, qt))["unit"].cpu().numpy()
    del sig
    rng = np.random.default_rng(12)
    near = np.nonzero(qc.source >= 0)[0]
    qs = np.sort(np.concatenate([rng.choice(near, 16, replace=False),
                                 rng.choice(np.setdiff1d(np.arange(4096), near), 48, replace=False)]))
    both = np.concatenate([dbunit, qunit[qs]])
    want = _chain_topk_rows(both, c.n_docs + np.arange(qs.size), c.n_docs, 16, TAU)
    flush(f"  oracle chain done; sampled hits {[w[2] for w in want][:16]}")
    for p in (lib.PREC_FP32, lib.PREC_BF16):
        ids, sc, hits = lib.mrc_query(ctx, db, model, qo, qt, 16, TAU, p)
        ids, sc, hits = ids.cpu().numpy(), sc.cpu().numpy(), hits.cpu().numpy()
        for r, q in enumerate(qs):
            wid, wsc, wh = want[r]
            np.testing.assert_array_equal(ids[q], wid)
            np.testing.assert_array_equal(sc[q].view(np.uint32), wsc.view(np.uint32))
            assert hits[q] == wh, (p, q)
        assert np.all(ids[:, 0] >= 0)
        flush(f"    precision {p}: 64 sampled queries equal the chain over 1,000,000 rows")
