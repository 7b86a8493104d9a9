"""Pins of the CPU oracle against things other than itself (no GPU needed).

Each test fixes the oracle to a definition, a closed form, a library routine of
the textbook operation, brute force on tiny inputs, or an invariant the paper
states, chosen so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them.
"""
import hashlib
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute, comparators as cmpo, mrc
from synth import corpus as synth


def _tiny_corpus(rng, n_docs, vocab, max_len):
    docs = []
    for _ in range(n_docs):
        L = int(rng.integers(0, max_len + 1))
        docs.append(rng.integers(0, vocab, L).astype(np.int32))
    return synth.from_docs(docs, vocab)


def _select_fn(spec):
    return lambda n: mrc.selection_bounds(n, spec)


# --------------------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(60))
def test_oracle_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    vocab = int(rng.integers(4, 64))
    c = _tiny_corpus(rng, int(rng.integers(1, 30)), vocab, 25)
    docs = [c.doc(d) for d in range(c.n_docs)]
    df_listed = len({int(t) for t in c.tokens})
    if df_listed == 0:
        return
    k = int(rng.integers(1, df_listed + 1))
    mode = int(rng.integers(0, 4))
    spec = mrc.RefSpec(k=k, mode=mode, lo=0, hi=-1, m=df_listed,
                       drop_top_ppm=int(rng.integers(0, 300_000)),
                       idf_mode=int(rng.integers(0, 2)), ref_weight=int(rng.integers(0, 2)))
    try:
        lo, hi = mrc.selection_bounds(df_listed, spec)
    except ValueError:
        return
    mdl = mrc.build_model(c.offsets, c.tokens, vocab, spec)
    b = brute.model(docs, vocab, k, _select_fn(spec), idf_smooth=spec.idf_mode == mrc.IDF_SMOOTH,
                    ref_idf=spec.ref_weight == mrc.REF_IDF)
    assert mdl.df.tolist() == b["df"]
    np.testing.assert_allclose(mdl.idf, b["idf"], rtol=0, atol=1e-13)
    assert mdl.order.tolist() == b["list"]
    for j, p in enumerate(b["parts"]):
        assert sorted(np.nonzero(mdl.part_of == j)[0].tolist()) == sorted(p)
    np.testing.assert_allclose(mdl.rnorm, b["rnorm"], rtol=1e-13)
    sig, norm = mrc.sign(c.offsets, c.tokens, mdl)
    for d, doc in enumerate(docs):
        s, n = brute.signature(doc, b)
        np.testing.assert_allclose(sig[d], s, rtol=0, atol=1e-12)
        assert abs(norm[d] - n) <= 1e-12 * max(1.0, n)
    # signature comparison = Eq. (1) on the signatures
    shat = mrc.normalise(sig)
    S = mrc.mrc_scores(shat, shat)
    for i in range(len(docs)):
        for j in range(len(docs)):
            assert abs(S[i, j] - brute.cosine(sig[i], sig[j])) <= 1e-12
    # exact cosine comparator
    tau = 0.3
    ei, ej, es = cmpo.exact_cosine_pairs(c.offsets, c.tokens, mdl, tau)
    want = [(i, j) for i in range(len(docs)) for j in range(i + 1, len(docs))
            if brute.tfidf_cosine(docs[i], docs[j], b["idf"]) >= tau]
    got = list(zip(ei.tolist(), ej.tolist()))
    # exclude pairs within rounding distance of the threshold from the set check
    near = {(i, j) for i in range(len(docs)) for j in range(i + 1, len(docs))
            if abs(brute.tfidf_cosine(docs[i], docs[j], b["idf"]) - tau) < 1e-12}
    assert set(got) - near == set(want) - near
    for i, j, s in zip(ei, ej, es):
        assert abs(s - brute.tfidf_cosine(docs[i], docs[j], b["idf"])) <= 1e-12


@pytest.mark.parametrize("seed", range(10))
def test_compare_pairs_matches_brute_all_pairs(seed):
    rng = np.random.default_rng(100 + seed)
    n, k = 40, 8
    sig = rng.random((n, k)) ** 3
    sig[rng.random(n) < 0.1] = 0.0
    sig[5] = sig[3] * 2.5                      # a scaled copy: MRC exactly 1 in exact arithmetic
    shat = mrc.normalise(sig)
    i, j, s = mrc.compare_pairs(shat, 0.9, block=7)
    want = {(a, b) for a in range(n) for b in range(a + 1, n) if brute.cosine(sig[a], sig[b]) >= 0.9}
    assert set(zip(i.tolist(), j.tolist())) == want
    assert (3, 5) in want
    assert np.all(i < j)


def test_pair_scores_match_brute_cosine():
    """MRC(i, j) of listed pairs (Eq. (1) on the signatures) against the
    pure-Python cosine of the raw signatures: ordered pairs in both directions,
    i == j, zero rows and a scaled copy."""
    rng = np.random.default_rng(7)
    n, k = 30, 6
    sig = rng.random((n, k)) ** 2
    sig[[6, 11]] = 0.0
    sig[4] = sig[1] * 3.0
    shat = mrc.normalise(sig)
    i = rng.integers(0, n, 300)
    j = rng.integers(0, n, 300)
    i[:6] = [1, 4, 2, 6, 6, 0]
    j[:6] = [4, 1, 2, 3, 11, 29]
    got = mrc.pair_scores(shat, i, j)
    for a, b, g in zip(i.tolist(), j.tolist(), got):
        assert abs(g - brute.cosine(sig[a], sig[b])) <= 1e-12
    assert abs(got[0] - 1.0) <= 1e-15 and abs(got[2] - 1.0) <= 1e-15   # scaled copy, self
    assert got[3] == 0.0 and got[4] == 0.0                                # zero rows
    np.testing.assert_array_equal(mrc.pair_scores(shat, j, i), got)       # symmetric


# --------------------------------------------------------------------------- general references

@pytest.mark.parametrize("seed", range(20))
def test_sign_matrix_matches_brute_force(seed):
    """Dense reference columns with arbitrary weights (negative ones, shared
    terms, a zero column) against the pure-Python Eq. (1) between the dense
    TF-IDF vector and each column."""
    rng = np.random.default_rng(500 + seed)
    vocab = int(rng.integers(4, 40))
    c = _tiny_corpus(rng, int(rng.integers(1, 20)), vocab, 20)
    docs = [c.doc(d) for d in range(c.n_docs)]
    listed = len({int(t) for t in c.tokens})
    if listed == 0:
        return
    spec = mrc.RefSpec(k=1, mode=mrc.SEL_ALL, idf_mode=int(rng.integers(0, 2)))
    mdl = mrc.build_model(c.offsets, c.tokens, vocab, spec)
    k = int(rng.integers(1, 9))
    R = rng.standard_normal((vocab, k)) * (rng.random((vocab, k)) < 0.5)
    R[:, 0] = 0.0 if k > 1 and seed % 3 == 0 else R[:, 0]
    sig, norm = mrc.sign_matrix(c.offsets, c.tokens, mdl, R)
    b = brute.model(docs, vocab, 1, lambda n: (0, n), idf_smooth=spec.idf_mode == mrc.IDF_SMOOTH)
    for d, doc in enumerate(docs):
        tf = brute.counts(doc)
        w = [tf.get(t, 0) * b["idf"][t] for t in range(vocab)]
        for j in range(k):
            assert abs(sig[d, j] - brute.cosine(w, R[:, j].tolist())) <= 1e-12
        assert abs(norm[d] - math.sqrt(sum(x * x for x in w))) <= 1e-12 * max(1.0, norm[d])


@pytest.mark.parametrize("ref_weight", [0, 1])
def test_sign_matrix_of_the_parts_is_the_mrc_signature(ref_weight):
    """With the model's own parts as columns (indicator or idf weights), the
    general signature is Section 4's signature."""
    c = synth.generate(0, n_docs=300)
    for spec in (mrc.RefSpec(k=16, ref_weight=ref_weight),
                 mrc.RefSpec(k=7, mode=mrc.SEL_REGION, lo=10, hi=500, ref_weight=ref_weight)):
        mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, spec)
        a, na = mrc.sign(c.offsets, c.tokens, mdl)
        b, nb = mrc.sign_matrix(c.offsets, c.tokens, mdl, mrc.reference_matrix(mdl))
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-13)
        np.testing.assert_array_equal(na, nb)


def test_sign_matrix_closed_forms():
    """Columns that are documents' own TF-IDF vectors give the exact cosine
    (sklearn); a column that is the union of two disjoint parts combines their
    indicator signatures as (s_a sqrt|P_a| + s_b sqrt|P_b|) / sqrt(|P_a| + |P_b|);
    a column of one term gives that term's share of the unit TF-IDF vector."""
    from sklearn.feature_extraction.text import TfidfTransformer
    from sklearn.metrics.pairwise import cosine_similarity
    import scipy.sparse as sp
    c = synth.generate(0, n_docs=250)
    mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, mrc.RefSpec(k=16))
    doc, term, tf = mrc.term_counts(c.offsets, c.tokens, c.vocab)
    TF = sp.csr_matrix((tf, (doc, term)), shape=(c.n_docs, c.vocab))
    W = TfidfTransformer(norm=None, smooth_idf=True).fit_transform(TF)
    cols = [3, 17, 100, 249]
    R = np.asarray(W[cols].todense()).T
    sig, _ = mrc.sign_matrix(c.offsets, c.tokens, mdl, R)
    np.testing.assert_allclose(sig, cosine_similarity(W, W[cols]), rtol=0, atol=1e-12)
    # union of parts 2 and 5
    P = mrc.reference_matrix(mdl)
    s_ind, _ = mrc.sign(c.offsets, c.tokens, mdl)
    na, nb = (mdl.part_of == 2).sum(), (mdl.part_of == 5).sum()
    su, _ = mrc.sign_matrix(c.offsets, c.tokens, mdl, (P[:, 2] + P[:, 5])[:, None])
    want = (s_ind[:, 2] * math.sqrt(na) + s_ind[:, 5] * math.sqrt(nb)) / math.sqrt(na + nb)
    np.testing.assert_allclose(su[:, 0], want, rtol=0, atol=1e-13)
    # one term per column
    t = int(mdl.order[40])
    e = np.zeros((c.vocab, 1))
    e[t, 0] = 2.5
    s1, norm = mrc.sign_matrix(c.offsets, c.tokens, mdl, e)
    d2, t2, w2, _ = mrc.tfidf(c.offsets, c.tokens, mdl)
    want = np.zeros(c.n_docs)
    want[d2[t2 == t]] = w2[t2 == t] / norm[d2[t2 == t]]
    np.testing.assert_allclose(s1[:, 0], want, rtol=0, atol=1e-14)


# --------------------------------------------------------------------------- library routines

def test_exact_cosine_scores_match_sklearn_at_listed_pairs():
    """exact_cosine_scores (Eq. (1) on the TF-IDF vectors, and on raw counts
    with idf NONE) at listed pairs against sklearn's cosine_similarity of the
    same vectors."""
    from sklearn.feature_extraction.text import TfidfTransformer
    from sklearn.metrics.pairwise import cosine_similarity
    import scipy.sparse as sp
    c = synth.generate(0, n_docs=300)
    doc, term, tf = mrc.term_counts(c.offsets, c.tokens, c.vocab)
    TF = sp.csr_matrix((tf, (doc, term)), shape=(c.n_docs, c.vocab))
    rng = np.random.default_rng(3)
    i = rng.integers(0, c.n_docs, 2000)
    j = rng.integers(0, c.n_docs, 2000)
    dup = np.nonzero(c.source >= 0)[0]
    i = np.concatenate([i, dup, np.arange(5)])
    j = np.concatenate([j, c.source[dup], np.arange(5)])
    for idf_mode, W in [(mrc.IDF_SMOOTH, TfidfTransformer(norm=None, smooth_idf=True).fit_transform(TF)),
                        (mrc.IDF_NONE, TF.astype(np.float64))]:
        mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, mrc.RefSpec(k=16, idf_mode=idf_mode))
        G = cosine_similarity(W)
        got = cmpo.exact_cosine_scores(c.offsets, c.tokens, mdl, i, j)
        np.testing.assert_allclose(got, G[i, j], rtol=0, atol=1e-12)
        np.testing.assert_allclose(got[-5:], 1.0, atol=1e-12)
        assert np.all(got[2000:2000 + dup.size] > 0.5)      # near duplicates and copies



def test_smooth_idf_and_tfidf_match_sklearn():
    from sklearn.feature_extraction.text import TfidfTransformer
    import scipy.sparse as sp
    c = synth.generate(0, n_docs=300)
    spec = mrc.RefSpec(k=16)
    mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, spec)
    doc, term, tf = mrc.term_counts(c.offsets, c.tokens, c.vocab)
    TF = sp.csr_matrix((tf, (doc, term)), shape=(c.n_docs, c.vocab))
    tr = TfidfTransformer(norm=None, smooth_idf=True, sublinear_tf=False).fit(TF)
    np.testing.assert_allclose(mdl.idf, tr.idf_, rtol=1e-14)
    W = tr.transform(TF).tocsr()
    d2, t2, w2, norm = mrc.tfidf(c.offsets, c.tokens, mdl)
    np.testing.assert_allclose(np.asarray(W[d2, t2]).ravel(), w2, rtol=1e-14)
    np.testing.assert_allclose(np.sqrt(np.asarray(W.multiply(W).sum(axis=1)).ravel()), norm, rtol=1e-13)


def test_exact_cosine_matches_sklearn_cosine_similarity():
    from sklearn.feature_extraction.text import TfidfTransformer
    from sklearn.metrics.pairwise import cosine_similarity
    import scipy.sparse as sp
    c = synth.generate(0, n_docs=400)
    mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, mrc.RefSpec(k=16))
    doc, term, tf = mrc.term_counts(c.offsets, c.tokens, c.vocab)
    TF = sp.csr_matrix((tf, (doc, term)), shape=(c.n_docs, c.vocab))
    W = TfidfTransformer(norm=None, smooth_idf=True).fit_transform(TF)
    G = cosine_similarity(W)
    tau = 0.5
    i, j, s = cmpo.exact_cosine_pairs(c.offsets, c.tokens, mdl, tau, block=128)
    np.testing.assert_allclose(s, G[i, j], atol=1e-12)
    ii, jj = np.nonzero(np.triu(G, 1) >= tau)
    assert set(zip(i.tolist(), j.tolist())) == set(zip(ii.tolist(), jj.tolist()))
    assert len(i) > 10          # the corpus holds near duplicates


# --------------------------------------------------------------------------- closed forms

def test_one_term_per_part_reduces_mrc_to_exact_cosine():
    """ALL selection, k = V' (each listed term its own part), indicator weights:
    every |r_j| = 1 and sig_d is w_d / |w_d| with its entries permuted, so the
    signature cosine equals the exact cosine (the limit in which the paper sees
    the error fall to zero as parts grow)."""
    from sklearn.metrics.pairwise import cosine_similarity
    rng = np.random.default_rng(7)
    c = _tiny_corpus(rng, 60, 300, 80)
    Vp = len(np.unique(c.tokens))
    mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, mrc.RefSpec(k=Vp, mode=mrc.SEL_ALL))
    sig, _ = mrc.sign(c.offsets, c.tokens, mdl)
    shat = mrc.normalise(sig)
    W = cmpo.tfidf_matrix(c.offsets, c.tokens, mdl)
    np.testing.assert_allclose(mrc.mrc_scores(shat, shat), cosine_similarity(W), atol=1e-12)
    np.testing.assert_allclose(mdl.rnorm, 1.0)


def test_single_part_closed_form():
    """k = 1: sig_d = sum of w_dt over the selection / (|w_d| sqrt(m)), and every
    pair of non-zero signatures scores exactly 1."""
    c = synth.generate(0, n_docs=120)
    spec = mrc.RefSpec(k=1)
    mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, spec)
    sig, norm = mrc.sign(c.offsets, c.tokens, mdl)
    m = mdl.hi - mdl.lo
    sel = set(mdl.order[mdl.lo:mdl.hi].tolist())
    for d in range(0, c.n_docs, 7):
        toks = c.doc(d)
        w = {}
        for t in toks:
            w[int(t)] = w.get(int(t), 0.0) + mdl.idf[int(t)]
        nw = math.sqrt(sum(v * v for v in w.values()))
        want = sum(v for t, v in w.items() if t in sel) / (nw * math.sqrt(m))
        assert abs(sig[d, 0] - want) <= 1e-12
    shat = mrc.normalise(sig)
    nz = np.nonzero(sig[:, 0] > 0)[0]
    S = mrc.mrc_scores(shat[nz], shat[nz])
    np.testing.assert_allclose(S, 1.0, atol=1e-15)


def test_hand_worked_example():
    """Three documents over terms {0..5}, raw counts (idf NONE), ALL selection.
    df = [2,3,1,1,1,0] -> sorted list by (df desc, id asc) = [1, 0, 2, 3, 4].
    k = 2 -> parts {1,0,2} and {3,4}, |r| = (sqrt 3, sqrt 2).
    doc0 = 0 0 1 2   tf {0:2, 1:1, 2:1}, |w| = sqrt 6
        sig = (2+1+1)/(sqrt6 sqrt3), 0
    doc1 = 1 3 3 4   tf {1:1, 3:2, 4:1}, |w| = sqrt 6
        sig = 1/(sqrt6 sqrt3), (2+1)/(sqrt6 sqrt2)
    doc2 = 0 1       tf {0:1, 1:1}, |w| = sqrt 2
        sig = 2/(sqrt2 sqrt3), 0
    MRC(0,2) = 1 (both signatures lie on the first axis);
    MRC(0,1) = a / sqrt(a^2 + b^2) with a = 1/sqrt18, b = 3/sqrt12."""
    docs = [[0, 0, 1, 2], [1, 3, 3, 4], [0, 1]]
    c = synth.from_docs([np.array(d) for d in docs], 6)
    spec = mrc.RefSpec(k=2, mode=mrc.SEL_ALL, idf_mode=mrc.IDF_NONE)
    mdl = mrc.build_model(c.offsets, c.tokens, 6, spec)
    assert mdl.df.tolist() == [2, 3, 1, 1, 1, 0]
    assert mdl.order.tolist() == [1, 0, 2, 3, 4]
    assert mdl.part_of.tolist() == [0, 0, 0, 1, 1, -1]
    sig, norm = mrc.sign(c.offsets, c.tokens, mdl)
    s6, s3, s2 = math.sqrt(6), math.sqrt(3), math.sqrt(2)
    want = np.array([[4 / (s6 * s3), 0.0], [1 / (s6 * s3), 3 / (s6 * s2)], [2 / (s2 * s3), 0.0]])
    np.testing.assert_allclose(sig, want, atol=1e-15)
    np.testing.assert_allclose(norm, [s6, s6, s2], atol=1e-15)
    S = mrc.mrc_scores(mrc.normalise(sig), mrc.normalise(sig))
    a, b = 1 / math.sqrt(18), 3 / math.sqrt(12)
    assert abs(S[0, 2] - 1.0) < 1e-15
    assert abs(S[0, 1] - a / math.sqrt(a * a + b * b)) < 1e-15


def test_partition_sizes():
    for m in range(1, 60):
        for k in range(1, m + 1):
            s = mrc.partition_sizes(m, k)
            assert s.sum() == m and s.max() - s.min() <= 1
            assert np.all(np.diff(s) <= 0)          # the larger parts come first
    assert mrc.partition_sizes(10, 3).tolist() == [4, 3, 3]


def test_selection_bounds():
    S = mrc.RefSpec
    assert mrc.selection_bounds(8000, S(k=4, mode=mrc.SEL_REGION, lo=6000, hi=8000)) == (6000, 8000)
    assert mrc.selection_bounds(8000, S(k=4, mode=mrc.SEL_REGION, lo=6000, hi=-1)) == (6000, 8000)
    assert mrc.selection_bounds(8000, S(k=60, mode=mrc.SEL_RAREST, m=1500)) == (6500, 8000)
    assert mrc.selection_bounds(8000, S(k=8, mode=mrc.SEL_ALL)) == (0, 8000)
    # ceil(V' * 5%) computed in exact integers
    assert mrc.selection_bounds(20, S(k=2))[0] == 1
    assert mrc.selection_bounds(21, S(k=2))[0] == 2
    assert mrc.selection_bounds(130858, S(k=64))[0] == 6543
    with pytest.raises(ValueError):
        mrc.selection_bounds(10, S(k=11, mode=mrc.SEL_ALL))
    with pytest.raises(ValueError):
        mrc.selection_bounds(10, S(k=2, mode=mrc.SEL_RAREST, m=11))


# --------------------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def small():
    c = synth.generate(0, n_docs=500)
    mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, mrc.RefSpec(k=16))
    sig, norm = mrc.sign(c.offsets, c.tokens, mdl)
    return c, mdl, sig, norm


def test_self_similarity_symmetry_range(small):
    c, mdl, sig, _ = small
    shat = mrc.normalise(sig)
    S = mrc.mrc_scores(shat, shat)
    nz = np.abs(sig).sum(axis=1) > 0
    np.testing.assert_allclose(np.diag(S)[nz], 1.0, atol=1e-12)
    np.testing.assert_array_equal(S, S.T)
    assert S.min() >= -1e-15 and S.max() <= 1 + 1e-12
    assert sig.min() >= 0 and sig.max() <= 1 + 1e-12          # Section 3: cosine in [0, 1]
    W = cmpo.tfidf_matrix(c.offsets, c.tokens, mdl)
    G = (W @ W.T).toarray()
    nzw = np.asarray(W.sum(axis=1)).ravel() > 0
    np.testing.assert_allclose(np.diag(G)[nzw], 1.0, atol=1e-12)


def test_bag_of_words_and_repetition_invariance(small):
    """Section 3: cosine does not depend on word order. Repeating every token of
    a document c times scales w_d and leaves its cosines unchanged."""
    c, mdl, sig, _ = small
    rng = np.random.default_rng(3)
    docs = [rng.permutation(c.doc(d)) for d in range(c.n_docs)]
    c2 = synth.from_docs(docs, c.vocab)
    sig2, _ = mrc.sign(c2.offsets, c2.tokens, mdl)
    np.testing.assert_array_equal(sig, sig2)
    docs3 = [np.repeat(c.doc(d), 3) for d in range(c.n_docs)]
    c3 = synth.from_docs(docs3, c.vocab)
    sig3, _ = mrc.sign(c3.offsets, c3.tokens, mdl)
    np.testing.assert_allclose(sig, sig3, atol=1e-13)
    h = cmpo.md5_term_hashes(c.vocab)
    np.testing.assert_array_equal(cmpo.simhash64(c.offsets, c.tokens, c.vocab, h),
                                  cmpo.simhash64(c2.offsets, c2.tokens, c.vocab, h))


def test_exact_duplicates_identical(small):
    c, mdl, sig, _ = small
    dup = np.nonzero(c.kind == 1)[0]
    assert dup.size == 0            # config 1 has near duplicates only
    c2 = synth.generate(1, n_docs=400)
    mdl2 = mrc.build_model(c2.offsets, c2.tokens, c2.vocab, mrc.RefSpec(k=64))
    sig2, _ = mrc.sign(c2.offsets, c2.tokens, mdl2)
    shat = mrc.normalise(sig2)
    h = cmpo.simhash64(c2.offsets, c2.tokens, c2.vocab)
    exact = np.nonzero(c2.kind == 1)[0]
    assert exact.size > 0
    for d in exact:
        s = c2.source[d]
        np.testing.assert_array_equal(sig2[d], sig2[s])
        assert abs(shat[d] @ shat[s] - 1.0) < 1e-12
        assert cmpo.hamming(h[d], h[s]) == 0


def test_more_parts_track_cosine_better():
    """Soft trend the paper reports (Section 4): the error of MRC against exact
    cosine falls as the number of parts grows at a fixed reference. Checked
    coarsely (k = 2 worse than k = 64 worse than one term per part)."""
    c = synth.generate(0, n_docs=200)
    maes = []
    for k in (2, 64, None):
        mdl0 = mrc.build_model(c.offsets, c.tokens, c.vocab, mrc.RefSpec(k=1, mode=mrc.SEL_ALL))
        Vp = mdl0.order.size
        spec = mrc.RefSpec(k=Vp if k is None else k, mode=mrc.SEL_ALL)
        mdl = mrc.build_model(c.offsets, c.tokens, c.vocab, spec)
        sig, _ = mrc.sign(c.offsets, c.tokens, mdl)
        shat = mrc.normalise(sig)
        W = cmpo.tfidf_matrix(c.offsets, c.tokens, mdl)
        G = (W @ W.T).toarray()
        iu = np.triu_indices(c.n_docs, 1)
        maes.append(cmpo.mae_variance(mrc.mrc_scores(shat, shat)[iu], G[iu])[0])
    assert maes[0] > maes[1] > maes[2]
    assert maes[2] < 1e-12


# --------------------------------------------------------------------------- quantisers

def _f32_probe_values(rng):
    vals = [0.0, 1.0, 0.5, 2.0 ** -6, 2.0 ** -7, 2.0 ** -9, 2.0 ** -10, 448.0, 447.99, 440.0, 464.0 - 1e-4,
            1 + 2 ** -8, 1 + 2 ** -7 + 2 ** -8, 3 * 2 ** -10, 2.0 ** -133]
    grid = np.float32(np.linspace(0, 448, 200_001))
    return np.concatenate([np.float32(vals), grid, np.float32(rng.random(50_000) * 448),
                           np.float32(2.0 ** rng.uniform(-20, 8.8, 50_000))])


def test_bf16_quantiser_matches_torch():
    import torch
    rng = np.random.default_rng(11)
    x = _f32_probe_values(rng)
    x = np.concatenate([x, -x, np.float32(rng.standard_normal(10_000))])
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(mrc.bf16_codes(x), want)
    np.testing.assert_array_equal(mrc.bf16_value(want),
                                  torch.from_numpy(x).to(torch.bfloat16).float().numpy())


def test_fp8_quantiser_matches_torch():
    import torch
    rng = np.random.default_rng(12)
    x = _f32_probe_values(rng)
    x = x[x <= 448.0]
    x = np.concatenate([x, -x[x > 0]])
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(mrc.fp8_e4m3fn_codes(x), want)
    allc = np.arange(256, dtype=np.uint8)
    tv = torch.from_numpy(allc).view(torch.float8_e4m3fn).float().numpy()
    ov = mrc.fp8_e4m3fn_value(allc)
    np.testing.assert_array_equal(np.isnan(tv), np.isnan(ov))
    np.testing.assert_array_equal(tv[~np.isnan(tv)], ov[~np.isnan(ov)])


def _exact_f32(fr: Fraction) -> Fraction:
    """Round an exact rational to the nearest float32 (ties to even), by value."""
    if fr == 0:
        return Fraction(0)
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - 23)
    q = a / ulp
    fl = math.floor(q)
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * fl * ulp


@pytest.mark.parametrize("seed", range(8))
def test_fma_chain_matches_exact_rounding(seed):
    """Each step of the plain FP32 chain is one correctly rounded a*b + acc."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 40))
    a = np.float32(rng.random((2, k)) * (1.0 if seed % 2 else 1e-3))
    acc = Fraction(0)
    for c in range(k):
        acc = _exact_f32(Fraction(float(a[0, c])) * Fraction(float(a[1, c])) + acc)
    got = mrc.score32_pairs(a, [0], [1])[0]
    assert Fraction(float(got)) == acc
    # symmetric by construction
    assert mrc.score32_pairs(a, [1], [0])[0] == got


def test_fp32_rounding_bound_covers_the_chain():
    """The bound the GPU parity tests use to excuse near-ties (tests/fp_bounds.py)
    covers the float32 chain of rounded unit vectors against the float64 score,
    on random rows and on rows built to cancel (large products of both signs)."""
    from tests.fp_bounds import pair_bound
    rng = np.random.default_rng(12)
    for k in (7, 64, 256):
        x = rng.random((200, k)) ** 3
        x[100:] = rng.standard_normal((100, k)) * np.exp(rng.standard_normal((100, k)) * 4)
        shat = mrc.normalise(x)
        u32 = shat.astype(np.float32)
        i = rng.integers(0, 200, 3000)
        j = rng.integers(0, 200, 3000)
        c = mrc.score32_pairs(u32, i, j).astype(np.float64)
        s64 = mrc.pair_scores(shat, i, j)
        b = pair_bound(u32, shat, i, j)
        assert np.all(np.abs(c - s64) <= b)
        assert b.max() < 1e-4 and np.median(b) < 1e-5


def test_lowp_band_covers_quantisation_error():
    rng = np.random.default_rng(5)
    for k in (64, 128, 256):
        s = np.abs(rng.standard_normal((300, k))) ** 2
        s[:, : k // 3] *= 0.01
        shat = np.float32(mrc.normalise(s))
        ii = rng.integers(0, 300, 4000)
        jj = rng.integers(0, 300, 4000)
        s32 = mrc.score32_pairs(shat, ii, jj).astype(np.float64)
        # bf16
        qb = mrc.bf16_value(mrc.bf16_codes(shat)).astype(np.float64)
        eb = mrc.row_quant_error(shat, qb)
        assert eb.max() <= 2.0 ** -8 * 1.0001
        lp = np.einsum("pc,pc->p", qb[ii], qb[jj])
        assert np.all(np.abs(lp - s32) <= mrc.lowp_band(eb[ii], eb[jj], k, nominal=0.0))
        assert mrc.lowp_band(eb[ii], eb[jj], k).max() == 0.02
        # fp8 with per-row scale
        codes, scale = mrc.fp8_quantise_rows(shat)
        # power-of-two scales just covering each row: max|s| / scale lies in
        # (224, 448], so the largest code (its rounding) lies in [224, 448]
        nz = scale > 0
        assert np.all(np.frexp(scale[nz].astype(np.float64))[0] == 0.5)
        top = np.abs(mrc.fp8_e4m3fn_value(codes)).max(axis=1)
        assert np.all((top[nz] >= 224.0) & (top[nz] <= 448.0))
        q8 = mrc.fp8_dequantise_rows(codes, scale)
        e8 = mrc.row_quant_error(shat, q8)
        lp8 = np.einsum("pc,pc->p", q8[ii], q8[jj])
        assert np.all(np.abs(lp8 - s32) <= mrc.lowp_band(e8[ii], e8[jj], k, nominal=0.0))


# --------------------------------------------------------------------------- simhash

def test_md5_reference_vectors():
    """RFC 1321 Appendix A.5 test suite values for the hash the Simhash table uses."""
    assert hashlib.md5(b"").hexdigest() == "d41d8cd98f00b204e9800998ecf8427e"
    assert hashlib.md5(b"abc").hexdigest() == "900150983cd24fb0d6963f7d28e17f72"
    assert hashlib.md5(b"message digest").hexdigest() == "f96b697d7cb7938d525a2f31aaf161d0"


def test_simhash_rules():
    vocab = 64
    h = cmpo.md5_term_hashes(vocab)
    assert h[0] == int.from_bytes(hashlib.md5(b"\0\0\0\0").digest()[:8], "little")
    docs = [[5], [5, 5, 5], [3, 9], [], [3, 9, 9]]
    c = synth.from_docs([np.array(d, dtype=np.int32) for d in docs], vocab)
    sim = cmpo.simhash64(c.offsets, c.tokens, vocab, h)
    assert sim[0] == h[5] and sim[1] == h[5]          # one term: the simhash is its hash
    assert sim[2] == (int(h[3]) & int(h[9]))           # a 0 column sum gives bit 0
    assert sim[3] == 0
    assert sim[4] == h[9]                              # 9 twice outvotes 3 once
    for d, doc in enumerate(docs):
        assert int(sim[d]) == brute.simhash(doc, h)


def test_hamming_and_pairs():
    rng = np.random.default_rng(9)
    x = rng.integers(0, 2 ** 63, 300, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 300, dtype=np.uint64)
    x[10] = x[3] ^ np.uint64(0b1011)
    x[20] = x[3]
    for a, b in [(0, 1), (3, 10), (3, 20), (7, 7)]:
        assert cmpo.hamming(x[a], x[b]) == brute.hamming(x[a], x[b])
    i, j, d = cmpo.hamming_pairs(x, 3, block=37)
    want = {(a, b) for a in range(300) for b in range(a + 1, 300) if brute.hamming(x[a], x[b]) <= 3}
    assert set(zip(i.tolist(), j.tolist())) == want
    assert (3, 10) in want and (3, 20) in want


# --------------------------------------------------------------------------- query and metrics

def test_query_topk_tie_break_and_hits():
    db = np.array([[1, 0], [0, 1], [1, 0], [1, 1], [1, 0]], float)
    q = np.array([[1, 0], [0, 0]], float)
    ids, sc, hits = mrc.query_topk(mrc.normalise(db), mrc.normalise(q), 4, 0.9)
    assert ids[0].tolist() == [0, 2, 4, 3]             # equal scores: ascending id
    np.testing.assert_allclose(sc[0], [1, 1, 1, math.sqrt(0.5)])
    assert hits.tolist() == [3, 0]
    assert ids[1].tolist() == [0, 1, 2, 3]             # zero query: every score 0


def test_mae_variance_closed_form():
    approx = [0.5, 0.7, 1.0]
    truth = [0.4, 0.9, 1.0]
    mae, var = cmpo.mae_variance(approx, truth)
    assert abs(mae - (0.1 + 0.2 + 0.0) / 3) < 1e-15
    e = [0.1, -0.2, 0.0]
    m = sum(e) / 3
    assert abs(var - sum((x - m) ** 2 for x in e) / 3) < 1e-15
    r, p = cmpo.recall_precision([0, 1], [2, 3], [0, 5], [2, 6])
    assert r == 0.5 and p == 0.5
    # Eq. (2) as printed: the signed pair sum over the number of documents
    # (errors of opposite sign cancel, unlike the MAE)
    assert abs(cmpo.mae_paper_literal(approx, truth, 3) - (0.1 - 0.2 + 0.0) / 3) < 1e-15
    assert abs(cmpo.mae_paper_literal(approx, truth, 10) - (0.1 - 0.2) / 10) < 1e-15
    assert cmpo.mae_paper_literal([0.3], [0.3], 2) == 0.0


def test_simhash_similarity_closed_form():
    np.testing.assert_array_equal(cmpo.simhash_similarity([0, 3, 32, 64]), [1.0, 61 / 64, 0.5, 0.0])
    x = np.array([0x0123456789ABCDEF], np.uint64)
    assert cmpo.simhash_similarity(cmpo.hamming(x, x))[0] == 1.0
    assert cmpo.simhash_similarity(cmpo.hamming(x, ~x))[0] == 0.0
    y = x ^ np.uint64(0b10110)
    assert cmpo.simhash_similarity(cmpo.hamming(x, y))[0] == 1.0 - 3 / 64
