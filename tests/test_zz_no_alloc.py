"""The no-allocation FP32 comparison (mrc_compare_f32_noalloc, scratch in a
fixed device array of the library) against mrc_compare at MRC_PREC_FP32:
the same pairs with bit-identical scores, on two calls in a row (the second
with a smaller input, so stale contents of the array would show), through
the C ABI; the context's device memory does not grow; sizes beyond the array
and the two-call protocol."""
import ctypes as C

import numpy as np
import pytest

from synth import corpus as synth
from tests.gpu_util import device_docs, flush, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


def _sigs(lib, ctx, n_docs, k, seed):
    c = synth.generate(1, n_docs=n_docs, seed=seed)
    o, t = device_docs(c)
    gm = lib.mrc_build_vocab_idf(ctx, o, t, c.vocab, lib.ref_spec(k))
    return lib.mrc_sign(ctx, gm, o, t)


def _pair_set(pairs):
    a = pairs.cpu().numpy()
    return {(int(i), int(j)): int(s) for i, j, s in zip(a[:, 0], a[:, 1], a[:, 2])}


def _noalloc_raw(lib, ctx, sig, tau, cap):
    """One call through the raw C symbol (ctypes); returns (status, n_found, pairs)."""
    import torch
    n, k = sig.shape
    buf = torch.zeros((max(cap, 1), 4), dtype=torch.int32, device="cuda")
    nf = C.c_int64(-1)
    fn = lib.lib().mrc_compare_f32_noalloc
    st = fn(ctx, C.c_void_p(sig.data_ptr()), C.c_int64(n), C.c_int32(k), C.c_float(tau),
            C.c_void_p(buf.data_ptr()) if cap > 0 else None, C.c_int64(cap), C.byref(nf), None)
    return st, nf.value, buf[: min(cap, max(nf.value, 0))]


@pytest.mark.parametrize("k", [64, 200])
def test_noalloc_equals_compare_on_two_calls(lib, k):
    ctx = lib.mrc_ctx_create(0)
    big = _sigs(lib, ctx, 6000, k, seed=11)
    small = _sigs(lib, ctx, 2500, k, seed=12)
    for name, sig in (("first, 6000 rows", big), ("second, 2500 rows", small)):
        flush(f"  noalloc k={k} {name}")
        want, _ = lib.mrc_compare(ctx, sig, 0.9, lib.PREC_FP32)
        used0, _ = lib.mrc_ctx_memory(ctx)
        st, nf, got = _noalloc_raw(lib, ctx, sig, 0.9, want.shape[0] + 1024)
        used1, _ = lib.mrc_ctx_memory(ctx)
        assert st == lib.MRC_OK, lib.lib().mrc_last_error().decode()
        assert used1 == used0
        assert nf == want.shape[0]
        assert _pair_set(got) == _pair_set(want)


def test_noalloc_overflow_and_limits(lib):
    import torch
    ctx = lib.mrc_ctx_create(0)
    sig = _sigs(lib, ctx, 3000, 64, seed=13)
    want, _ = lib.mrc_compare(ctx, sig, 0.9, lib.PREC_FP32)
    assert want.shape[0] > 10
    flush("  noalloc two-call protocol")
    st, nf, got = _noalloc_raw(lib, ctx, sig, 0.9, 10)
    assert st == lib.MRC_E_OVERFLOW and nf == want.shape[0]
    assert set(_pair_set(got).items()) <= set(_pair_set(want).items())
    n_found, over = lib.mrc_compare_f32_noalloc(ctx, sig, 0.9, torch.zeros((0, 4), dtype=torch.int32,
                                                                         device="cuda"))
    assert over and n_found == want.shape[0]
    # one row past the fixed array (k = 256: 256 columns, 32 MiB = 32,768 rows)
    k = 256
    rows = lib.NOALLOC_MAX_UNIT_BYTES // (k * 4)
    assert rows == 32768
    s = torch.rand((rows + 1, k), device="cuda")
    flush(f"  noalloc rejects n={rows + 1} k={k}")
    st, _, _ = _noalloc_raw(lib, ctx, s, 0.9, 0)
    assert st == lib.MRC_E_INVAL
    assert "fixed scratch array" in lib.lib().mrc_last_error().decode()
    # trivial sizes
    for n in (0, 1):
        st, nf, _ = _noalloc_raw(lib, ctx, torch.rand((max(n, 1), 8), device="cuda")[:n], 0.9, 4)
        assert st == lib.MRC_OK and nf == 0
    # the context stays usable and the array is cleared per call
    st, nf, got = _noalloc_raw(lib, ctx, sig, 0.9, want.shape[0])
    assert st == lib.MRC_OK and _pair_set(got) == _pair_set(want)
