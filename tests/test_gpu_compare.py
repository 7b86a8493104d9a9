"""GPU parity of the all-pairs signature comparison.

FP32 plain path: every score is the fixed float32 multiply-add chain over the
unit signatures, so the GPU's flagged set must equal, pair for pair, the set
the oracle's C chain flags on the same unit signatures, with bit-identical
scores. Against the float64 oracle every score lies within its rounding bound
(tests/fp_bounds.py: the chain's own rounding plus the float32 unit vectors'
distance from the float64 ones), and the decisions agree except for pairs
whose float64 score lies within that bound of tau (counted, not failed)."""
import ctypes

import numpy as np
import pytest

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


def _signed(lib, ctx, cfg, n_docs, k):
    c = synth.generate(cfg, n_docs=n_docs)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(k))
    sig = lib.mrc_sign(ctx, gm, o, t)
    return c, sig


def all_pairs_score32(unit):
    """Every pair i < j through the oracle's C chain (small n only)."""
    n = unit.shape[0]
    iu, ju = np.triu_indices(n, 1)
    return iu, ju, om.score32_pairs(unit, iu, ju)


@pytest.mark.parametrize("cfg,n_docs,k", [(0, None, 16), (1, 3000, 64), (1, 1000, 64), (2, 600, 256)])
def test_fp32_decisions_equal_the_chain_and_the_oracle(lib, ctx, cfg, n_docs, k):
    c, sig = _signed(lib, ctx, cfg, n_docs, k)
    n = c.n_docs
    flush(f"  compare fp32 n={n} k={k}")
    pairs, stats = lib.mrc_compare(ctx, sig, TAU, lib.PREC_FP32)
    gi, gj, gs, gf = lib.pairs_to_numpy(pairs)
    assert stats["n_flagged"] == gi.size and stats["n_pairs_compared"] == n * (n - 1) // 2
    assert np.all(gi < gj)
    unit = lib.mrc_normalise(ctx, sig)["unit"].cpu().numpy()
    iu, ju, s32 = all_pairs_score32(unit)
    want = s32 >= np.float32(TAU)
    got = set(zip(gi.tolist(), gj.tolist()))
    assert got == set(zip(iu[want].tolist(), ju[want].tolist()))
    # bit-identical scores
    order = np.lexsort((gj, gi))
    ref = om.score32_pairs(unit, gi[order], gj[order])
    np.testing.assert_array_equal(gs[order].view(np.uint32), ref.view(np.uint32))
    # against the float64 oracle
    osig = om.sign(c.offsets, c.tokens, om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=k)))[0]
    shat = om.normalise(osig)
    s64 = (shat @ shat.T)[iu, ju]
    bound = matrix_bound(unit, shat, unit, shat)[iu, ju]
    err = np.abs(s32.astype(np.float64) - s64)
    assert np.all(err <= bound), (err.max(), bound[np.argmax(err - bound)])
    far = np.abs(s64 - TAU) > bound
    assert np.array_equal(want[far], (s64 >= TAU)[far])
    flush(f"    flagged={gi.size} max |fp32 - fp64| {err.max():.2e} (largest bound {bound.max():.2e}); "
          f"near-ties excluded={int((~far).sum())}")


@pytest.mark.parametrize("mode,k", [("all", 8), ("frequent_half", 512), ("rare_half", 1024), ("rarest", 1024),
                                    ("drop_top", 32)])
def test_fp32_decisions_across_selections_and_k(lib, ctx, mode, k):
    """The selection x k shapes of the sweep: the comparison's flagged set and
    its bare count (no output buffer) equal the chain's set on the same unit
    signatures, from 8 parts (most pairs flagged) to 1,024 parts."""
    import torch
    c = synth.generate(1, n_docs=400)
    o, t = device_docs(c)
    listed = lib.mrc_model_info(lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(8, mode=lib.SEL_ALL)))[
        "n_listed"]
    kw = {"all": dict(mode=lib.SEL_ALL), "drop_top": dict(mode=lib.SEL_DROP_TOP),
          "frequent_half": dict(mode=lib.SEL_REGION, lo=0, hi=listed // 2),
          "rare_half": dict(mode=lib.SEL_REGION, lo=listed // 2, hi=listed),
          "rarest": dict(mode=lib.SEL_RAREST, m=listed // 10)}[mode]
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(k, **kw))
    sig = lib.mrc_sign(ctx, gm, o, t)
    flush(f"  compare fp32 selection={mode} k={k} listed={listed}")
    pairs, stats = lib.mrc_compare(ctx, sig, TAU, lib.PREC_FP32)
    gi, gj, gs, _ = lib.pairs_to_numpy(pairs)
    unit = lib.mrc_normalise(ctx, sig)["unit"].cpu().numpy()
    iu, ju, s32 = all_pairs_score32(unit)
    want = s32 >= np.float32(TAU)
    assert set(zip(gi.tolist(), gj.tolist())) == set(zip(iu[want].tolist(), ju[want].tolist()))
    order = np.lexsort((gj, gi))
    np.testing.assert_array_equal(gs[order].view(np.uint32), om.score32_pairs(unit, gi[order], gj[order]).view(np.uint32))
    n = ctypes.c_int64()
    opts = lib.MrcCompareOpts(TAU, lib.PREC_FP32, 0.02, 0)
    st = lib.lib().mrc_compare(ctx, ctypes.c_void_p(sig.data_ptr()), sig.shape[0], sig.shape[1], ctypes.byref(opts),
                               None, 0, ctypes.byref(n), None,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == (lib.MRC_E_OVERFLOW if gi.size else lib.MRC_OK) and n.value == gi.size
    flush(f"    flagged={gi.size} of {iu.size}")


@pytest.mark.parametrize("k,tau", [(16, -2.0), (64, -2.0), (64, 0.5), (100, -2.0), (600, 0.0)])
def test_fp32_dense_output(lib, ctx, k, tau):
    """Thresholds that flag most or all pairs: the flag walk's dense paths
    (tiles with more flagged pairs than a wavefront's stage holds write
    straight to the output) still emit each flagged pair once, with the chain
    score, for every tile kernel (k = 16, 64, 100, 600)."""
    c, sig = _signed(lib, ctx, 1, 1500, k)
    n = c.n_docs
    q = lib.mrc_normalise(ctx, sig, unit=True)
    unit = q["unit"].cpu().numpy()
    iu, ju, s32 = all_pairs_score32(unit)
    want = s32 >= np.float32(tau)
    flush(f"  k={k} tau={tau}: {int(want.sum())} of {iu.size} pairs")
    pairs, stats = lib.mrc_compare(ctx, sig, tau, lib.PREC_FP32, capacity=int(want.sum()) + 16)
    gi, gj, gs, _ = lib.pairs_to_numpy(pairs)
    assert gi.size == int(want.sum()) == stats["n_flagged"]
    key = gi * n + gj
    order = np.argsort(key)
    np.testing.assert_array_equal(key[order], (iu * n + ju)[want])
    np.testing.assert_array_equal(gs[order].view(np.uint32), s32[want].view(np.uint32))


def test_fp32_overflow_protocol_and_tiny_inputs(lib, ctx):
    import torch
    c, sig = _signed(lib, ctx, 0, None, 16)
    pairs, _ = lib.mrc_compare(ctx, sig, TAU)
    total = pairs.shape[0]
    assert total > 10
    # explicit small capacity: the C call reports OVERFLOW with the exact count
    buf = torch.empty((5, 4), dtype=torch.int32, device="cuda")
    n = ctypes.c_int64()
    opts = lib.MrcCompareOpts(TAU, lib.PREC_FP32, 0.02, 0)
    st = lib.lib().mrc_compare(ctx, ctypes.c_void_p(sig.data_ptr()), sig.shape[0], sig.shape[1], ctypes.byref(opts),
                               ctypes.c_void_p(buf.data_ptr()), 5, ctypes.byref(n), None,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == lib.MRC_E_OVERFLOW and n.value == total
    for m in (0, 1, 2, 3, 129):
        p, s = lib.mrc_compare(ctx, sig[:m].contiguous(), TAU)
        want = {(i, j) for i, j in zip(*lib.pairs_to_numpy(pairs)[:2]) if j < m}
        assert set(zip(*lib.pairs_to_numpy(p)[:2])) == want
    # zero signatures never pair; identical rows score 1
    z = torch.zeros((4, 16), device="cuda")
    z[2] = sig[0]
    z[3] = sig[0] * 3.0
    p, _ = lib.mrc_compare(ctx, z, TAU)
    assert set(zip(*lib.pairs_to_numpy(p)[:2])) == {(2, 3)}


def test_score_pairs_matches_chain(lib, ctx):
    import torch
    c, sig = _signed(lib, ctx, 1, 500, 64)
    unit = lib.mrc_normalise(ctx, sig)["unit"]
    rng = np.random.default_rng(0)
    ii = rng.integers(0, 500, 10_000).astype(np.int32)
    jj = rng.integers(0, 500, 10_000).astype(np.int32)
    out = lib.mrc_score_pairs(ctx, unit, torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()).cpu().numpy()
    ref = om.score32_pairs(unit.cpu().numpy(), ii, jj)
    np.testing.assert_array_equal(out.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("cfg,n,k", [(2, 800, 256), (1, 500, 20), (2, 300, 300), (2, 200, 1024), (1, 300, 18)])
def test_quantisers_match_oracle(lib, ctx, cfg, n, k):
    # k a multiple of 4: 4, 8, ..., 64 lanes per row and 1-4 float4 groups per
    # lane; k = 18: one component per lane
    c, sig = _signed(lib, ctx, cfg, n, k)
    q = lib.mrc_normalise(ctx, sig, unit=True, bf16=True, fp8=True, err=True)
    unit = q["unit"].cpu().numpy()
    osig = om.sign(c.offsets, c.tokens, om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=k)))[0]
    assert np.abs(unit - om.normalise(osig)).max() <= 1e-5
    np.testing.assert_array_equal(q["bf16"].cpu().numpy().view(np.uint16), om.bf16_codes(unit))
    codes, scale = om.fp8_quantise_rows(unit)
    np.testing.assert_array_equal(q["scale"].cpu().numpy(), scale)
    np.testing.assert_array_equal(q["fp8"].cpu().numpy(), codes)
    err = q["err"].cpu().numpy()
    eb = om.row_quant_error(unit, om.bf16_value(om.bf16_codes(unit)))
    e8 = om.row_quant_error(unit, om.fp8_dequantise_rows(codes, scale))
    assert np.all(err[0] >= eb) and np.all(err[0] <= eb * (1 + 1e-6) + 1e-30)
    assert np.all(err[1] >= e8) and np.all(err[1] <= e8 * (1 + 1e-6) + 1e-30)


def test_normalise_alignment_independent(lib, ctx):
    # the same rows from a 16-byte aligned and a 4-byte aligned buffer give the same bits
    import torch
    c, sig = _signed(lib, ctx, 1, 300, 64)
    buf = torch.zeros(sig.numel() + 1, dtype=torch.float32, device=sig.device)
    mis = buf[1:].view(sig.shape)
    mis.copy_(sig)
    assert mis.data_ptr() % 16 != 0
    a = lib.mrc_normalise(ctx, sig, unit=True, bf16=True, fp8=True, err=True)
    b = lib.mrc_normalise(ctx, mis, unit=True, bf16=True, fp8=True, err=True)
    for key in ("unit", "bf16", "fp8", "scale", "err"):
        np.testing.assert_array_equal(a[key].cpu().numpy().view(np.uint8), b[key].cpu().numpy().view(np.uint8))
