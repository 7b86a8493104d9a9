"""GPU parity of the comparators: MD5 term hashes, Simhash-64 words and
Hamming pairs (integers, bit-exact against the oracle), and exact cosine."""
import numpy as np
import pytest
import torch

from oracle import comparators as oc
from oracle import mrc as om
from synth import corpus as synth
from tests.gpu_util import device_docs, flush, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.mrc_ctx_create(0)


def _model(lib, ctx, c, k=16):
    o, t = device_docs(c)
    return lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(k, mode=lib.SEL_ALL)), o, t


def test_md5_term_hashes_bit_exact(lib, ctx):
    c = synth.generate(1, n_docs=300)
    gm, _, _ = _model(lib, ctx, c)
    got = lib.mrc_term_hashes(ctx, gm).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, oc.md5_term_hashes(c.vocab))


@pytest.mark.parametrize("cfg,n_docs", [(0, None), (1, 2500)])
def test_simhash_bit_exact(lib, ctx, cfg, n_docs):
    c = synth.generate(cfg, n_docs=n_docs)
    gm, o, t = _model(lib, ctx, c)
    got = lib.mrc_simhash(ctx, gm, o, t).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, oc.simhash64(c.offsets, c.tokens, c.vocab))


def test_simhash_edge_documents(lib, ctx):
    rng = np.random.default_rng(2)
    V = 5000
    docs = [np.zeros(0, np.int32), np.array([V - 1]), np.array([3, 9]), np.full(50_000, 11), rng.integers(0, V, 9000),
            rng.integers(0, V, 65), rng.integers(0, V, 64), rng.integers(0, V, 63)]
    c = synth.from_docs(docs, V)
    gm, o, t = _model(lib, ctx, c, k=4)
    got = lib.mrc_simhash(ctx, gm, o, t).cpu().numpy().view(np.uint64)
    h = oc.md5_term_hashes(V)
    np.testing.assert_array_equal(got, oc.simhash64(c.offsets, c.tokens, V, h))
    assert got[0] == 0 and got[1] == h[V - 1] and got[2] == (h[3] & h[9])


@pytest.mark.parametrize("n,max_dist", [(2000, 3), (5000, 6), (1, 3), (2, 3), (257, 0)])
def test_hamming_pairs_exact(lib, ctx, n, max_dist):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 2 ** 63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    for a in range(0, n - 1, 7):     # planted near copies
        flip = rng.integers(0, 64, int(rng.integers(0, 5)))
        m = np.uint64(0)
        for f in flip:
            m |= np.uint64(1) << np.uint64(int(f))
        x[a + 1] = x[a] ^ m
    got = lib.mrc_hamming_pairs(ctx, torch.from_numpy(x.view(np.int64)).cuda(), max_dist)
    gi, gj, gd, _ = lib.pairs_to_numpy(got)
    oi, oj, od = oc.hamming_pairs(x, max_dist)
    assert set(zip(gi.tolist(), gj.tolist(), gd.astype(np.int64).tolist())) == \
        set(zip(oi.tolist(), oj.tolist(), od.tolist()))


def test_simhash_hamming_on_corpus(lib, ctx):
    c = synth.generate(0)
    gm, o, t = _model(lib, ctx, c)
    sim = lib.mrc_simhash(ctx, gm, o, t)
    got = lib.mrc_hamming_pairs(ctx, sim, 3)
    gi, gj, gd, _ = lib.pairs_to_numpy(got)
    osim = oc.simhash64(c.offsets, c.tokens, c.vocab)
    oi, oj, od = oc.hamming_pairs(osim, 3)
    assert set(zip(gi.tolist(), gj.tolist())) == set(zip(oi.tolist(), oj.tolist()))
    flush(f"  simhash pairs <= 3: {gi.size}")


@pytest.mark.parametrize("cfg,n_docs,tau", [(0, None, 0.9), (1, 3000, 0.9), (1, 1500, 0.5), (0, 300, 0.2)])
def test_exact_cosine_matches_oracle(lib, ctx, cfg, n_docs, tau):
    """GPU FP32 exact cosine vs the FP64 oracle: same pair set except pairs
    within 1e-5 of tau, scores within 1e-5."""
    c = synth.generate(cfg, n_docs=n_docs)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(16))
    got = lib.mrc_exact_cosine(ctx, gm, o, t, tau)
    gi, gj, gs, _ = lib.pairs_to_numpy(got)
    omodel = om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=16))
    oi, oj, os_ = oc.exact_cosine_pairs(c.offsets, c.tokens, omodel, tau)
    g = set(zip(gi.tolist(), gj.tolist()))
    w = set(zip(oi.tolist(), oj.tolist()))
    diff = g ^ w
    if diff:
        di = np.array([p[0] for p in diff])
        dj = np.array([p[1] for p in diff])
        s64 = oc.exact_cosine_scores(c.offsets, c.tokens, omodel, di, dj)
        assert np.all(np.abs(s64 - tau) <= 1e-5), "pair sets differ away from the threshold"
    s64 = oc.exact_cosine_scores(c.offsets, c.tokens, omodel, gi, gj)
    assert np.abs(gs - s64).max() <= 1e-5
    flush(f"  exact cosine n={c.n_docs} tau={tau}: {gi.size} pairs, {len(diff)} near-tie differences")


@pytest.mark.parametrize("V", [3000, 40000])
def test_exact_cosine_edge_documents(lib, ctx, V):
    """Duplicates, permutations, empty and one-token documents, and documents
    above 8,192 tokens (a direct LDS count array for V <= 32,768, global tables
    above); the whole flagged set against the oracle at a lower threshold."""
    rng = np.random.default_rng(8)
    base = rng.integers(0, V, 300)
    long_doc = rng.integers(0, V, 9000)
    docs = [np.zeros(0, np.int32), base, base.copy(), rng.permutation(base), np.array([5]), np.array([5]),
            rng.integers(0, V, 6000), rng.integers(0, V, 50), long_doc, rng.permutation(long_doc),
            np.concatenate([long_doc, rng.integers(0, V, 3000)])]
    c = synth.from_docs(docs, V)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, V, lib.ref_spec(4))
    got = lib.mrc_exact_cosine(ctx, gm, o, t, 0.999)
    gi, gj, gs, _ = lib.pairs_to_numpy(got)
    pairs = set(zip(gi.tolist(), gj.tolist()))
    assert {(1, 2), (1, 3), (2, 3), (4, 5), (8, 9)} <= pairs
    assert not any(0 in p for p in pairs)            # empty document pairs with nothing
    # every pair at tau = 0.2 (the long documents with each other and the rest) against the oracle
    omodel = om.build_model(c.offsets, c.tokens, V, om.RefSpec(k=4))
    got = lib.mrc_exact_cosine(ctx, gm, o, t, 0.2)
    gi, gj, gs, _ = lib.pairs_to_numpy(got)
    oi, oj, _ = oc.exact_cosine_pairs(c.offsets, c.tokens, omodel, 0.2)
    assert set(zip(gi.tolist(), gj.tolist())) == set(zip(oi.tolist(), oj.tolist()))
    # FP32 accumulation over the terms a pair shares: |error| <= ~2 n u (u = 2^-24) for n shared
    # terms (the long documents share thousands), plus the 1e-5 budget of short documents
    terms = [set(np.asarray(d).tolist()) for d in docs]
    shared = np.array([len(terms[i] & terms[j]) for i, j in zip(gi.tolist(), gj.tolist())])
    s64 = oc.exact_cosine_scores(c.offsets, c.tokens, omodel, gi, gj)
    assert np.all(np.abs(gs - s64) <= 1e-5 + 2.0 * shared * 2.0 ** -24)
