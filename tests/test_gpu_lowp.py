"""GPU parity of the BF16 and FP8 comparison forms.

Decisions must equal the FP32 plain path exactly. Rescored pairs carry the
FP32 chain score bit for bit; every low-precision score must equal the
dot product of the oracle-dequantised codes within FP32 accumulation error
(this also checks the matrix-core operand formats), and must lie within the
proven band of the FP32 score."""
import numpy as np
import pytest

from oracle import mrc as om
from synth import corpus as synth
from tests.gpu_util import device_docs, flush, require_gpu

pytestmark = pytest.mark.gpu
TAU = 0.9


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.mrc_ctx_create(0)


def _signed(lib, ctx, cfg, n_docs, k):
    c = synth.generate(cfg, n_docs=n_docs)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(k))
    return c, lib.mrc_sign(ctx, gm, o, t)


def _pairset(lib, pairs):
    i, j, s, f = lib.pairs_to_numpy(pairs)
    return i, j, s, f


@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
@pytest.mark.parametrize("cfg,n_docs,k", [(0, None, 16), (1, 3000, 64), (2, 2500, 256), (1, 700, 100)])
def test_lowp_decisions_equal_fp32(lib, ctx, prec_name, cfg, n_docs, k):
    prec = {"bf16": lib.PREC_BF16, "fp8": lib.PREC_FP8}[prec_name]
    c, sig = _signed(lib, ctx, cfg, n_docs, k)
    flush(f"  {prec_name} n={c.n_docs} k={k}")
    p32, _ = lib.mrc_compare(ctx, sig, TAU, lib.PREC_FP32)
    plp, st = lib.mrc_compare(ctx, sig, TAU, prec, 0.02)
    i32, j32, s32, _ = _pairset(lib, p32)
    il, jl, sl, fl = _pairset(lib, plp)
    assert set(zip(il.tolist(), jl.tolist())) == set(zip(i32.tolist(), j32.tolist()))
    assert st["n_flagged"] == il.size
    q = lib.mrc_normalise(ctx, sig, unit=True, bf16=True, fp8=True, err=True)
    unit = q["unit"].cpu().numpy()
    ref32 = om.score32_pairs(unit, il, jl)
    resc = (fl & 1) == 1
    np.testing.assert_array_equal(sl[resc].view(np.uint32), ref32[resc].view(np.uint32))
    # certain pairs: low-precision score equals the exact dot of the dequantised codes
    if prec_name == "bf16":
        deq = om.bf16_value(q["bf16"].cpu().numpy().view(np.uint16)).astype(np.float64)
        e = om.row_quant_error(unit, deq)
    else:
        deq = om.fp8_dequantise_rows(q["fp8"].cpu().numpy(), q["scale"].cpu().numpy())
        e = om.row_quant_error(unit, deq)
    cert = ~resc
    dot = np.einsum("pc,pc->p", deq[il[cert]], deq[jl[cert]])
    # accumulation slack of the matrix cores (FP8: shorter internal significand, measured)
    acc = 3 * k * 2.0 ** -24 if prec_name == "bf16" else max(3 * k * 2.0 ** -24, 2.0 ** -10)
    scale_ij = (1 + e[il[cert]]) * (1 + e[jl[cert]])
    assert np.all(np.abs(sl[cert] - dot) <= acc * scale_ij + 2.0 ** -20)
    band = om.lowp_band(e[il], e[jl], k) + acc * (1 + e[il]) * (1 + e[jl])
    assert np.all(np.abs(sl[cert].astype(np.float64) - ref32[cert]) <= band[cert])
    assert np.all(sl[cert] >= TAU)
    flush(f"    flagged={il.size} rescored={st['n_band']} nominal={st['n_band_nominal']} "
          f"flips_outside_nominal={st['n_flip_outside_nominal']} max_err={st['max_abs_err']:.4g}")
    if prec_name == "bf16":
        assert st["n_flip_outside_nominal"] == 0     # the proven BF16 bound is inside the nominal band


@pytest.mark.parametrize("cfg,n_docs,k", [(1, 3000, 64), (2, 2500, 256)])
def test_fp8_decisions_across_tau(lib, ctx, cfg, n_docs, k):
    """FP8 candidates pass each 32x32 block's own threshold (from its rows'
    largest errors): at every tau, and down into the bulk of unrelated pairs'
    scores, the flagged set still equals the FP32 path's and every rescored
    score is the FP32 chain."""
    c, sig = _signed(lib, ctx, cfg, n_docs, k)
    q = lib.mrc_normalise(ctx, sig, unit=True)
    unit = q["unit"].cpu().numpy()
    n = c.n_docs
    for tau in (0.7, 0.8, 0.85, 0.95):
        flush(f"  fp8 n={n} k={k} tau={tau}")
        p32, _ = lib.mrc_compare(ctx, sig, tau, lib.PREC_FP32)
        p8, st = lib.mrc_compare(ctx, sig, tau, lib.PREC_FP8, 0.02)
        i32, j32, _, _ = _pairset(lib, p32)
        i8, j8, s8, f8 = _pairset(lib, p8)
        np.testing.assert_array_equal(np.sort(i8 * n + j8), np.sort(i32 * n + j32))
        resc = (f8 & 1) == 1
        ref32 = om.score32_pairs(unit, i8[resc], j8[resc])
        np.testing.assert_array_equal(s8[resc].view(np.uint32), ref32.view(np.uint32))
        flush(f"    flagged={i8.size} rescored={st['n_band']}")


@pytest.mark.parametrize("prec_name", ["fp8", "bf16"])
def test_lowp_decisions_with_mixed_row_errors(lib, ctx, prec_name):
    """Rows whose low-precision errors differ widely (half of them with a few
    large components over many tiny ones), in clusters of near-duplicates so
    that many pairs lie near every tau: the candidate thresholds (FP8: each
    32x32 block's own) still keep every pair the FP32 path flags."""
    prec = {"bf16": lib.PREC_BF16, "fp8": lib.PREC_FP8}[prec_name]
    import torch
    rng = np.random.default_rng(7)
    n, k = 3000, 128
    base = rng.random((n // 10, k)) ** 3
    spiky = rng.random(n // 10) < 0.5
    base[spiky] = rng.random((int(spiky.sum()), k)) ** 12 * 1e-3
    for r in np.nonzero(spiky)[0]:
        base[r, rng.choice(k, 4, replace=False)] += rng.random(4) + 0.5
    sig = np.repeat(base, 10, axis=0) + rng.normal(0, 0.03, (n, k)) ** 2
    perm = rng.permutation(n)
    sig = np.ascontiguousarray(sig[perm], dtype=np.float32)
    dsig = torch.from_numpy(sig).cuda()
    q = lib.mrc_normalise(ctx, dsig, unit=True, fp8=True, err=True)
    e8 = q["err"].cpu().numpy()[1]
    flush(f"  FP8 row errors: min {e8.min():.4f} median {np.median(e8):.4f} max {e8.max():.4f}")
    assert e8.max() > 4 * e8.min()
    unit = q["unit"].cpu().numpy()
    # the dense rows' pairs score about 0.55-0.65, the near-duplicates' about 0.97-1
    for tau in (0.55, 0.6, 0.65, 0.97, 0.99):
        p32, _ = lib.mrc_compare(ctx, dsig, tau, lib.PREC_FP32)
        p8, st = lib.mrc_compare(ctx, dsig, tau, prec, 0.02)
        i32, j32, _, _ = _pairset(lib, p32)
        i8, j8, s8, f8 = _pairset(lib, p8)
        flush(f"    {prec_name} tau={tau}: flagged {i32.size}, rescored {st['n_band']}")
        np.testing.assert_array_equal(np.sort(i8 * n + j8), np.sort(i32 * n + j32))
        resc = (f8 & 1) == 1
        ref32 = om.score32_pairs(unit, i8[resc], j8[resc])
        np.testing.assert_array_equal(s8[resc].view(np.uint32), ref32.view(np.uint32))


def test_lowp_overflow_and_tiny(lib, ctx):
    import torch
    c, sig = _signed(lib, ctx, 0, None, 16)
    for prec in (lib.PREC_BF16, lib.PREC_FP8):
        full, _ = lib.mrc_compare(ctx, sig, TAU, prec)
        small, _ = lib.mrc_compare(ctx, sig, TAU, prec, capacity=3)     # the binding retries on overflow
        assert set(zip(*lib.pairs_to_numpy(small)[:2])) == set(zip(*lib.pairs_to_numpy(full)[:2]))
        for m in (0, 1, 2, 65):
            p, _ = lib.mrc_compare(ctx, sig[:m].contiguous(), TAU, prec)
            p32, _ = lib.mrc_compare(ctx, sig[:m].contiguous(), TAU, lib.PREC_FP32)
            assert set(zip(*lib.pairs_to_numpy(p)[:2])) == set(zip(*lib.pairs_to_numpy(p32)[:2]))
        z = torch.zeros((5, 16), device="cuda")
        z[1] = sig[0]
        z[4] = sig[0] * 7.0
        p, _ = lib.mrc_compare(ctx, z, TAU, prec)
        assert set(zip(*lib.pairs_to_numpy(p)[:2])) == {(1, 4)}


def test_lowp_error_vs_fp64_oracle(lib, ctx):
    """Reported quantity: max / mean error of the low-precision scores against
    the float64 oracle on flagged pairs (precision-form subsample)."""
    c, sig = _signed(lib, ctx, 2, 3000, 256)
    osig = om.sign(c.offsets, c.tokens, om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=256)))[0]
    shat = om.normalise(osig)
    for prec in (lib.PREC_BF16, lib.PREC_FP8):
        p, st = lib.mrc_compare(ctx, sig, 0.5, prec)
        i, j, s, f = lib.pairs_to_numpy(p)
        s64 = om.pair_scores(shat, i, j)
        err = np.abs(s.astype(np.float64) - s64)
        flush(f"  prec={prec} pairs={i.size} max_err={err.max():.4g} mean_err={err.mean():.4g}")
        assert err.max() <= (0.02 if prec == lib.PREC_BF16 else 0.15)
