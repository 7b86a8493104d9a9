"""GPU parity of the model build and signing against the CPU oracle.

Integers (df, the sorted list, parts) bit-exact; idf bit-exact against the
oracle's float64 idf rounded to float32; signatures within 1e-5 absolute of the
float64 oracle (the stated tolerance for FP32 signatures)."""
import numpy as np
import pytest

from oracle import mrc as om
from synth import corpus as synth
from tests.gpu_util import device_docs, flush, require_gpu

pytestmark = pytest.mark.gpu

SIG_TOL = 1e-5


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.mrc_ctx_create(0)


def _spec_pair(lib, k, mode=om.SEL_DROP_TOP, **kw):
    o = om.RefSpec(k=k, mode=mode, **kw)
    g = lib.ref_spec(k, mode=mode, lo=o.lo, hi=o.hi, m=o.m, drop_top_ppm=o.drop_top_ppm,
                     idf_mode=o.idf_mode, ref_weight=o.ref_weight)
    return o, g


def _check_model(lib, gm, om_model, vocab):
    got = lib.mrc_model_get(gm)
    np.testing.assert_array_equal(got["df"].astype(np.int64), om_model.df)
    Vp = om_model.order.size
    assert got["n_listed"] == Vp
    assert (got["lo"], got["hi"]) == (om_model.lo, om_model.hi)
    np.testing.assert_array_equal(got["term_at"][:Vp], om_model.order)
    tail = np.sort(np.nonzero(om_model.df == 0)[0])
    np.testing.assert_array_equal(got["term_at"][Vp:], tail)            # df = 0 terms, ascending id
    np.testing.assert_array_equal(got["rank_of"][got["term_at"]], np.arange(vocab))
    np.testing.assert_array_equal(got["part_of"], om_model.part_of)
    np.testing.assert_array_equal(got["idf"], om_model.idf.astype(np.float32))
    np.testing.assert_allclose(got["rnorm"], om_model.rnorm, rtol=1e-6)


def _run(lib, ctx, c, k, mode=om.SEL_DROP_TOP, **kw):
    ospec, gspec = _spec_pair(lib, k, mode, **kw)
    o, t = device_docs(c)
    flush(f"  build+sign n={c.n_docs} V={c.vocab} k={k} mode={mode} {kw}")
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    sig, norm = lib.mrc_sign(ctx, gm, o, t, with_norm=True)
    omodel = om.build_model(c.offsets, c.tokens, c.vocab, ospec)
    osig, onorm = om.sign(c.offsets, c.tokens, omodel)
    return gm, omodel, sig.cpu().numpy(), norm.cpu().numpy(), osig, onorm


@pytest.mark.parametrize("cfg,n_docs,k", [(0, None, 16), (1, 3000, 64), (2, 1500, 256)])
def test_build_and_sign_match_oracle(lib, ctx, cfg, n_docs, k):
    c = synth.generate(cfg, n_docs=n_docs)
    gm, omodel, sig, norm, osig, onorm = _run(lib, ctx, c, k)
    _check_model(lib, gm, omodel, c.vocab)
    assert np.abs(sig - osig).max() <= SIG_TOL
    np.testing.assert_allclose(norm, onorm, rtol=2e-6)


def test_rebuild_reuses_tables_without_stale_values(lib, ctx):
    # a destroyed model's device block is kept for the next build of the same
    # size: a model built into it must equal the oracle's, and one of another
    # size must still build correctly after it
    a = synth.generate(0, n_docs=1500, seed=11)
    b = synth.generate(0, n_docs=900, seed=12)
    for c in (a, b, a):
        gm, omodel, sig, _, osig, _ = _run(lib, ctx, c, 16)
        _check_model(lib, gm, omodel, c.vocab)
        assert np.abs(sig - osig).max() <= SIG_TOL
        gm.close()
    c = synth.generate(1, n_docs=700)
    gm, omodel, sig, _, osig, _ = _run(lib, ctx, c, 64)
    _check_model(lib, gm, omodel, c.vocab)
    assert np.abs(sig - osig).max() <= SIG_TOL


@pytest.mark.parametrize("mode,kw", [
    (om.SEL_ALL, {}),
    (om.SEL_REGION, {"lo": 100, "hi": 2100}),
    (om.SEL_RAREST, {"m": 1500}),
    (om.SEL_DROP_TOP, {"idf_mode": om.IDF_NONE}),
    (om.SEL_DROP_TOP, {"ref_weight": om.REF_IDF}),
])
def test_reference_modes(lib, ctx, mode, kw):
    c = synth.generate(0, n_docs=700)
    gm, omodel, sig, norm, osig, onorm = _run(lib, ctx, c, 30, mode, **kw)
    _check_model(lib, gm, omodel, c.vocab)
    assert np.abs(sig - osig).max() <= SIG_TOL


@pytest.mark.parametrize("V", [4096, 65536])
def test_edge_documents(lib, ctx, V):
    """Empty documents, one-token documents, the largest id, documents on both
    sides of every length-class boundary (LDS wavefront up to 512 tokens; LDS
    workgroup tables of 4096, 8192 and 16384 slots up to 2048, 4096 and 8192;
    beyond: a direct LDS count array when V <= 32768, global tables above),
    50,000 repeats of one id."""
    rng = np.random.default_rng(4)
    docs = [np.zeros(0, np.int32), np.array([V - 1], np.int32), np.array([0], np.int32)]
    for L in (1, 63, 64, 65, 511, 512, 513, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 9999, 10001, 30000):
        docs.append(rng.zipf(1.3, L).astype(np.int64) % V)
    docs.append(np.full(50_000, 7, np.int32))
    docs.append(np.arange(V, dtype=np.int32))
    docs += [rng.integers(0, V, int(rng.integers(0, 300))) for _ in range(200)]
    c = synth.from_docs(docs, V)
    gm, omodel, sig, norm, osig, onorm = _run(lib, ctx, c, 8, om.SEL_ALL)
    _check_model(lib, gm, omodel, V)
    assert np.abs(sig - osig).max() <= SIG_TOL
    np.testing.assert_allclose(norm, onorm, rtol=2e-6)
    assert np.all(sig[0] == 0) and norm[0] == 0


def _edge_corpus(V=4096):
    rng = np.random.default_rng(4)
    docs = [np.zeros(0, np.int32), np.array([V - 1], np.int32), np.array([0], np.int32)]
    for L in (1, 63, 64, 65, 511, 512, 513, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 9999, 10001, 30000):
        docs.append(rng.zipf(1.3, L).astype(np.int64) % V)
    docs.append(np.full(50_000, 7, np.int32))
    docs += [rng.integers(0, V, int(rng.integers(0, 300))) for _ in range(200)]
    return synth.from_docs(docs, V)


@pytest.mark.parametrize("which", ["small", "full3000", "edge", "edge_bigv"])
def test_build_and_sign_equals_build_then_sign(lib, ctx, which):
    """The fused call signs the model corpus from the build's count lists; it
    must give the same model and the same signature and norm bits."""
    if which.startswith("edge"):
        c, k, mode = _edge_corpus(4096 if which == "edge" else 65536), 8, om.SEL_ALL
    else:
        c = synth.generate(0) if which == "small" else synth.generate(1, n_docs=3000)
        k, mode = (16, om.SEL_DROP_TOP) if which == "small" else (64, om.SEL_DROP_TOP)
    _, gspec = _spec_pair(lib, k, mode)
    o, t = device_docs(c)
    flush(f"  fused build+sign {which} n={c.n_docs}")
    gm, sig, norm = lib.mrc_build_and_sign(ctx, o, t, c.vocab, gspec, with_norm=True)
    gm2 = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    sig2, norm2 = lib.mrc_sign(ctx, gm2, o, t, with_norm=True)
    a, b = lib.mrc_model_get(gm), lib.mrc_model_get(gm2)
    for key in ("df", "idf", "term_at", "rank_of", "part_of", "rnorm"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(sig.cpu().numpy(), sig2.cpu().numpy())
    np.testing.assert_array_equal(norm.cpu().numpy(), norm2.cpu().numpy())
    omodel = om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=k, mode=mode))
    osig, _ = om.sign(c.offsets, c.tokens, omodel)
    assert np.abs(sig.cpu().numpy() - osig).max() <= SIG_TOL


def test_build_and_sign_large_corpus(lib, ctx):
    """From 65,536 documents on, the fused call signs through the form that
    keeps the most frequent terms' information in LDS: the same model and the
    same signature and norm bits as building, then signing separately."""
    c = synth.generate(1, n_docs=70000)
    _, gspec = _spec_pair(lib, 64, om.SEL_DROP_TOP)
    o, t = device_docs(c)
    flush(f"  fused build+sign n={c.n_docs}")
    gm, sig, norm = lib.mrc_build_and_sign(ctx, o, t, c.vocab, gspec, with_norm=True)
    gm2 = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    sig2, norm2 = lib.mrc_sign(ctx, gm2, o, t, with_norm=True)
    a, b = lib.mrc_model_get(gm), lib.mrc_model_get(gm2)
    for key in ("df", "idf", "term_at", "rank_of", "part_of", "rnorm"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(sig.cpu().numpy(), sig2.cpu().numpy())
    np.testing.assert_array_equal(norm.cpu().numpy(), norm2.cpu().numpy())


def test_norm_is_exact_sum_rounded_once(lib, ctx):
    """|w_d| is the square root of the exact sum of (tf * idf32)^2, rounded to
    float64 once, square-rooted in float64, then rounded to float32; checked
    against exact rational arithmetic on the GPU model's own float32 idf."""
    import math
    from fractions import Fraction
    c = _edge_corpus()
    _, gspec = _spec_pair(lib, 8, om.SEL_ALL)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    _, norm = lib.mrc_sign(ctx, gm, o, t, with_norm=True)
    norm = norm.cpu().numpy()
    idf = lib.mrc_model_get(gm)["idf"]
    for d in range(c.n_docs):
        ids, tf = np.unique(c.doc(d), return_counts=True)
        exact = sum(Fraction(int(f)) ** 2 * Fraction(float(idf[i])) ** 2 for i, f in zip(ids, tf))
        want = np.float32(math.sqrt(float(exact))) if exact else np.float32(0)
        assert norm[d] == want, (d, norm[d], want)


def test_large_vocabulary_df(lib, ctx):
    """A vocabulary past the LDS histogram slices (df by atomics) and one just
    inside them: df bit-exact, signatures within tolerance."""
    rng = np.random.default_rng(9)
    for V in (8 * 65536, 8 * 65536 + 1000):
        docs = [rng.integers(0, V, int(rng.integers(1, 700))) for _ in range(600)]
        docs.append(np.array([V - 1], np.int32))
        c = synth.from_docs(docs, V)
        gm, omodel, sig, norm, osig, onorm = _run(lib, ctx, c, 32, om.SEL_ALL)
        _check_model(lib, gm, omodel, V)
        assert np.abs(sig - osig).max() <= SIG_TOL


def test_sign_is_deterministic_and_batch_independent(lib, ctx):
    c = synth.generate(1, n_docs=2000)
    _, gspec = _spec_pair(lib, 64)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    a = lib.mrc_sign(ctx, gm, o, t).cpu().numpy()
    b = lib.mrc_sign(ctx, gm, o, t).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    rng = np.random.default_rng(1)
    perm = rng.permutation(c.n_docs)[:500]
    sub = c.subset(perm)
    o2, t2 = device_docs(sub)
    s2 = lib.mrc_sign(ctx, gm, o2, t2).cpu().numpy()
    np.testing.assert_array_equal(s2, a[perm])          # alone vs in a different mix
    one = c.subset([perm[0]])
    o3, t3 = device_docs(one)
    np.testing.assert_array_equal(lib.mrc_sign(ctx, gm, o3, t3).cpu().numpy()[0], a[perm[0]])


def test_invalid_inputs_raise(lib, ctx):
    import torch
    c = synth.generate(0, n_docs=50)
    _, gspec = _spec_pair(lib, 16)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    bad = t.clone()
    bad[5] = c.vocab
    with pytest.raises(lib.MrcError) as e:
        lib.mrc_sign(ctx, gm, o, bad)
    assert e.value.status == lib.MRC_E_INVAL
    bad[5] = -3
    with pytest.raises(lib.MrcError):
        lib.mrc_build_vocab_idf(ctx, o, bad, c.vocab, gspec)
    boff = o.clone()
    boff[3] = boff[4] + 1          # decreasing offsets
    with pytest.raises(lib.MrcError):
        lib.mrc_sign(ctx, gm, boff, t)
    boff = o.clone()
    boff[-1] = t.numel() + 1       # past the token buffer: rejected before any token is read
    with pytest.raises(lib.MrcError):
        lib.mrc_sign(ctx, gm, boff, t)
    boff = o.clone()
    boff[0] = 1
    with pytest.raises(lib.MrcError):
        lib.mrc_build_vocab_idf(ctx, boff, t, c.vocab, gspec)
    with pytest.raises(lib.MrcError):                     # more parts than selected terms
        lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(16, mode=lib.SEL_RAREST, m=10))
    # a document longer than 2^22 tokens
    long_o = torch.tensor([0, 5, 5 + (1 << 22) + 1], dtype=torch.int64, device="cuda")
    long_t = torch.zeros((1 << 22) + 6, dtype=torch.int32, device="cuda")
    with pytest.raises(lib.MrcError) as e:
        lib.mrc_sign(ctx, gm, long_o, long_t)
    assert "2^22" in str(e.value)
    with pytest.raises(lib.MrcError):
        lib.mrc_build_and_sign(ctx, long_o, long_t, c.vocab, gspec)
    # the context stays usable after input errors
    sig = lib.mrc_sign(ctx, gm, o, t)
    assert torch.isfinite(sig).all()


def test_model_save_load_roundtrip(lib, ctx, tmp_path):
    c = synth.generate(0, n_docs=300)
    _, gspec = _spec_pair(lib, 16)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    p = tmp_path / "m.bin"
    lib.mrc_model_save(gm, p)
    gm2 = lib.mrc_model_load(ctx, p)
    a, b = lib.mrc_model_get(gm), lib.mrc_model_get(gm2)
    for key in ("df", "idf", "term_at", "rank_of", "part_of", "rnorm"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(lib.mrc_sign(ctx, gm, o, t).cpu().numpy(),
                                  lib.mrc_sign(ctx, gm2, o, t).cpu().numpy())
    raw = bytearray(p.read_bytes())
    raw[100] ^= 1
    p.write_bytes(bytes(raw))
    with pytest.raises(lib.MrcError):
        lib.mrc_model_load(ctx, p)
