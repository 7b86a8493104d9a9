"""GPU parity of signing against general reference matrices (Section 4's
construction with Section 6's weighted vector-space models) against the CPU
oracle: signatures within 1e-5 absolute of the float64 oracle, norms equal to
mrc_sign's (the same exact sum), the model's parts as columns equal to
mrc_sign's signature within float rounding."""
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


def _model(lib, ctx, c, k=16):
    o, t = device_docs(c)
    ospec = om.RefSpec(k=k)
    gspec = lib.ref_spec(k, mode=ospec.mode, lo=ospec.lo, hi=ospec.hi, m=ospec.m,
                         drop_top_ppm=ospec.drop_top_ppm, idf_mode=ospec.idf_mode, ref_weight=ospec.ref_weight)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    return gm, om.build_model(c.offsets, c.tokens, c.vocab, ospec), o, t


def _random_R(rng, V, k, kind):
    if kind == "dense":
        return rng.random((V, k))
    if kind == "sparse_overlap":
        # each column weights ~2% of the terms; columns share terms; a few negative weights
        R = np.where(rng.random((V, k)) < 0.02, rng.random((V, k)) * 3.0, 0.0)
        R[rng.random((V, k)) < 0.002] = -0.5
        return R
    if kind == "with_zero_column":
        R = rng.random((V, k))
        R[:, k // 2] = 0.0
        return R
    raise ValueError(kind)


@pytest.mark.parametrize("k,kind", [(1, "dense"), (64, "dense"), (65, "sparse_overlap"),
                                    (200, "with_zero_column"), (256, "sparse_overlap"), (1024, "dense")])
def test_sign_matrix_matches_oracle(lib, ctx, k, kind):
    import torch
    n_docs = 300 if k >= 512 else 1200
    c = synth.generate(0, n_docs=n_docs)
    gm, omodel, o, t = _model(lib, ctx, c)
    rng = np.random.default_rng(1000 + k)
    R = _random_R(rng, c.vocab, k, kind).astype(np.float32)
    flush(f"  sign_matrix n={c.n_docs} V={c.vocab} k={k} {kind}")
    sig, norm = lib.mrc_sign_matrix(ctx, gm, o, t, torch.from_numpy(R).cuda(), with_norm=True)
    osig, onorm = om.sign_matrix(c.offsets, c.tokens, omodel, R.astype(np.float64))
    sig = sig.cpu().numpy()
    assert np.abs(sig - osig).max() <= SIG_TOL
    _, ref_norm = lib.mrc_sign(ctx, gm, o, t, with_norm=True)
    np.testing.assert_array_equal(norm.cpu().numpy(), ref_norm.cpu().numpy())
    np.testing.assert_allclose(norm.cpu().numpy(), onorm, rtol=2e-6)
    if kind == "with_zero_column":
        assert np.all(sig[:, k // 2] == 0)


@pytest.mark.parametrize("ref_weight", [om.REF_ONE, om.REF_IDF])
def test_parts_as_columns_give_the_mrc_signature(lib, ctx, ref_weight):
    import torch
    c = synth.generate(0, n_docs=1500)
    o, t = device_docs(c)
    ospec = om.RefSpec(k=32, ref_weight=ref_weight)
    gspec = lib.ref_spec(32, mode=ospec.mode, drop_top_ppm=ospec.drop_top_ppm, idf_mode=ospec.idf_mode,
                         ref_weight=ref_weight)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, gspec)
    omodel = om.build_model(c.offsets, c.tokens, c.vocab, ospec)
    R = om.reference_matrix(omodel).astype(np.float32)
    flush(f"  sign_matrix parts-as-columns ref_weight={ref_weight}")
    got = lib.mrc_sign_matrix(ctx, gm, o, t, torch.from_numpy(R).cuda()).cpu().numpy()
    want = lib.mrc_sign(ctx, gm, o, t).cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=4e-7)
    osig, _ = om.sign(c.offsets, c.tokens, omodel)
    assert np.abs(got - osig).max() <= SIG_TOL


def test_sign_matrix_edge_documents(lib, ctx):
    """Empty and one-token documents, documents across every length class of
    the count pass, 50,000 repeats of one id, every id once; a hot set that
    covers the whole listed vocabulary."""
    import torch
    rng = np.random.default_rng(7)
    V = 4096
    docs = [np.zeros(0, np.int32), np.array([V - 1], np.int32), np.array([0], np.int32)]
    for L in (63, 64, 65, 511, 512, 513, 2048, 2049, 4097, 8193, 10001, 30000):
        docs.append(rng.zipf(1.3, L).astype(np.int64) % V)
    docs.append(np.full(50_000, 7, np.int32))
    docs.append(np.arange(V, dtype=np.int32))
    docs += [rng.integers(0, V, int(rng.integers(0, 300))) for _ in range(100)]
    c = synth.from_docs(docs, V)
    gm, omodel, o, t = _model(lib, ctx, c, k=8)
    for k in (3, 100):
        R = rng.random((V, k)).astype(np.float32)
        flush(f"  sign_matrix edge docs k={k}")
        sig = lib.mrc_sign_matrix(ctx, gm, o, t, torch.from_numpy(R).cuda()).cpu().numpy()
        osig, _ = om.sign_matrix(c.offsets, c.tokens, omodel, R.astype(np.float64))
        assert np.abs(sig - osig).max() <= SIG_TOL
        assert np.all(sig[0] == 0)


def test_sign_matrix_invalid_inputs(lib, ctx):
    import torch
    c = synth.generate(0, n_docs=50)
    gm, _, o, t = _model(lib, ctx, c)
    R = torch.rand((c.vocab, 8), device="cuda")
    with pytest.raises(ValueError):
        lib.mrc_sign_matrix(ctx, gm, o, t, R[:-1].contiguous())
    with pytest.raises(lib.MrcError) as e:
        lib.mrc_sign_matrix(ctx, gm, o, t, torch.rand((c.vocab, 1025), device="cuda"))
    assert e.value.status == lib.MRC_E_INVAL
    bad = t.clone()
    bad[3] = c.vocab
    with pytest.raises(lib.MrcError) as e:
        lib.mrc_sign_matrix(ctx, gm, o, bad, R)
    assert e.value.status == lib.MRC_E_INVAL
    boff = o.clone()
    boff[3] = boff[4] + 1
    with pytest.raises(lib.MrcError):
        lib.mrc_sign_matrix(ctx, gm, boff, t, R)
    sig = lib.mrc_sign_matrix(ctx, gm, o, t, R)
    assert torch.isfinite(sig).all()
