"""GPU parity of the character 3-gram front end (mrc_trigrams) against the
oracle: offsets and ids bit-exact (integer work), on synthetic text, on random
bytes of every value with ragged lengths (0, 1, 2 and 3 bytes included), on
enough documents for several offset blocks and a multi-round block scan, and
on one long document; the two-call protocol, empty input and malformed offsets;
and the ids feeding the model and signature calls."""
import ctypes

import numpy as np
import pytest

from oracle import mrc as om
from oracle import trigram as ot
from synth.text import generate_text
from tests.gpu_util import flush, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return require_gpu()


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.mrc_ctx_create(0)


def _run(lib, ctx, text, off, capacity=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(text, np.uint8)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda()
    tok_off, ids = lib.mrc_trigrams(ctx, t, o, capacity=capacity)
    torch.cuda.synchronize()
    return tok_off.cpu().numpy(), ids.cpu().numpy()


def _check(lib, ctx, text, off, label):
    flush(f"  trigrams {label}: {off.size - 1} docs, {text.size} bytes")
    got_off, got = _run(lib, ctx, text, off)
    want_off, want = ot.trigram_csr(text, off)
    np.testing.assert_array_equal(got_off, want_off)
    np.testing.assert_array_equal(got, want)


def test_synthetic_text(lib, ctx):
    text, off = generate_text(2000, seed=7)
    _check(lib, ctx, text, off, "synthetic")


@pytest.mark.parametrize("seed", [0, 1])
def test_random_bytes_ragged(lib, ctx, seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 700, 3000)
    lens[:8] = [0, 1, 2, 3, 0, 4, 2, 1]
    lens[-3:] = [1, 0, 2]
    text = rng.integers(0, 256, int(lens.sum()), dtype=np.uint8)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    _check(lib, ctx, text, off, f"random bytes seed {seed}")


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_text_pointer_not_word_aligned(lib, ctx, shift):
    """The caller's text may start at any byte address: the map reads whole
    aligned words only where they lie inside the buffer."""
    import torch
    rng = np.random.default_rng(20 + shift)
    lens = rng.integers(0, 300, 500)
    lens[:4] = [5, 0, 3, 1]
    text = rng.integers(0, 256, int(lens.sum()), dtype=np.uint8)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pad = torch.from_numpy(np.concatenate([np.full(shift, 65, np.uint8), text, np.full(7, 66, np.uint8)])).cuda()
    t = pad[shift:shift + text.size]
    assert t.is_contiguous() and t.data_ptr() % 4 == shift % 4
    flush(f"  trigrams text at byte offset {shift}")
    tok_off, ids = lib.mrc_trigrams(ctx, t, torch.from_numpy(off).cuda())
    want_off, want = ot.trigram_csr(text, off)
    np.testing.assert_array_equal(tok_off.cpu().numpy(), want_off)
    np.testing.assert_array_equal(ids.cpu().numpy(), want)


def test_many_documents_and_one_long(lib, ctx):
    rng = np.random.default_rng(11)
    # 600,000 documents: 293 offset blocks of 2,048, more than one round of the block scan
    lens = rng.integers(0, 7, 600_000)
    text = rng.integers(0, 256, int(lens.sum()), dtype=np.uint8)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    _check(lib, ctx, text, off, "600k short documents")
    long = rng.integers(0, 256, 3_000_001, dtype=np.uint8)
    _check(lib, ctx, long, np.array([0, 1, long.size], np.int64), "one 3 MB document")


def test_protocol_empty_and_malformed(lib, ctx):
    import torch
    text, off = generate_text(50, seed=3)
    want_off, want = ot.trigram_csr(text, off)
    t = torch.from_numpy(text).cuda()
    o = torch.from_numpy(off).cuda()
    tok_off = torch.empty(off.size, dtype=torch.int64, device="cuda")
    n = ctypes.c_int64()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.lib().mrc_trigrams(ctx, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(o.data_ptr()), off.size - 1,
                                text.size, ctypes.c_void_p(tok_off.data_ptr()), None, 0, ctypes.byref(n), s)
    assert st == lib.MRC_E_OVERFLOW and n.value == want.size
    np.testing.assert_array_equal(tok_off.cpu().numpy(), want_off)
    # capacity exactly the total
    got_off, got = _run(lib, ctx, text, off, capacity=int(want.size))
    np.testing.assert_array_equal(got, want)
    # no documents
    got_off, got = _run(lib, ctx, np.zeros(0, np.uint8), np.zeros(1, np.int64))
    assert got_off.tolist() == [0] and got.size == 0
    # malformed offsets: decreasing, a last offset that is not the byte count, a first that is not 0
    for bad in ([0, 5, 3, 10], [0, 3, 9], [1, 3, 10]):
        b = torch.tensor(bad, dtype=torch.int64, device="cuda")
        tt = torch.zeros(10, dtype=torch.uint8, device="cuda")
        with pytest.raises(lib.MrcError):
            lib.mrc_trigrams(ctx, tt, b)


def test_ids_feed_the_method(lib, ctx):
    text, off = generate_text(400, seed=9)
    tok_off, ids = _run(lib, ctx, text, off)
    import torch
    o = torch.from_numpy(tok_off).cuda()
    t = torch.from_numpy(ids).cuda()
    k = 32
    model, sig = lib.mrc_build_and_sign(ctx, o, t, lib.TRIGRAM_VOCAB, lib.ref_spec(k))
    want_off, want = ot.trigram_csr(text, off)
    osig = om.sign(want_off, want, om.build_model(want_off, want, ot.VOCAB, om.RefSpec(k=k)))[0]
    assert np.abs(sig.cpu().numpy().astype(np.float64) - osig).max() <= 1e-5
    flush(f"    signed {off.size - 1} documents over {np.unique(ids).size} distinct 3-grams")
