"""Pins of the character 3-gram oracle (CPU only).

Worked examples computed by hand from the stated reading (letters case-folded
to 0-25, every other byte the separator 26, id = 729 s0 + 27 s1 + s2), closed
forms for the counts, invariances, and the vectorised form against the
per-byte loops on random text with every byte value."""
import numpy as np
import pytest

from oracle import trigram as ot
from synth.text import generate_text


def test_worked_examples():
    # 'a','b','c' = 0, 1, 2
    assert ot.doc_trigrams(b"abc") == [0 * 729 + 1 * 27 + 2]
    # "The" = t(19) h(7) e(4) -> 19*729 + 7*27 + 4 = 13851 + 189 + 4
    assert ot.doc_trigrams(b"The") == [14044]
    # "a b": a, separator, b
    assert ot.doc_trigrams(b"a b") == [0 * 729 + 26 * 27 + 1]
    # "zzzz": two windows of z(25)
    assert ot.doc_trigrams(b"zzzz") == [25 * 729 + 25 * 27 + 25] * 2
    # three separators of any kind give the last id
    assert ot.doc_trigrams(b" 7\xff") == [ot.VOCAB - 1]


def test_counts_and_range():
    for L in range(0, 8):
        ids = ot.doc_trigrams(bytes(range(97, 97 + L)))
        assert len(ids) == max(L - 2, 0)
    rng = np.random.default_rng(3)
    doc = rng.integers(0, 256, 5000, dtype=np.uint8).tobytes()
    ids = ot.doc_trigrams(doc)
    assert len(ids) == 4998 and min(ids) >= 0 and max(ids) < ot.VOCAB


def test_case_folding_and_separator_invariance():
    assert ot.doc_trigrams(b"Hello, World") == ot.doc_trigrams(b"hELLO; wORLD")
    # every non-letter byte is the same symbol
    seps = [b for b in range(256) if not (65 <= b <= 90 or 97 <= b <= 122)]
    assert len(seps) == 256 - 52
    assert {ot.symbol(b) for b in seps} == {ot.SEPARATOR}
    assert sorted(ot.symbol(b) for b in range(65, 91)) == list(range(26))
    # a window's id decodes back to its three symbols
    for w in (b"qZ.", b"..a", b"M\x00k"):
        (i,) = ot.doc_trigrams(w)
        assert (i // 729, (i // 27) % 27, i % 27) == tuple(ot.symbol(b) for b in w)


def test_windows_never_cross_documents():
    text = b"abcXYZ"
    off, ids = ot.trigram_csr(np.frombuffer(text, np.uint8), [0, 3, 6])
    assert off.tolist() == [0, 1, 2]
    assert ids.tolist() == ot.doc_trigrams(b"abc") + ot.doc_trigrams(b"XYZ")


@pytest.mark.parametrize("seed", [0, 1])
def test_vectorised_equals_loops(seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 40, 300)
    lens[:5] = [0, 1, 2, 3, 0]
    text = rng.integers(0, 256, int(lens.sum()), dtype=np.uint8)
    off = np.concatenate([[0], np.cumsum(lens)])
    tok_off, ids = ot.trigram_csr(text, off)
    want = []
    for d in range(lens.size):
        got = ids[tok_off[d]:tok_off[d + 1]].tolist()
        w = ot.doc_trigrams(text[off[d]:off[d + 1]].tobytes())
        assert got == w
        want += w
    assert ids.tolist() == want


def test_synthetic_text_shape():
    text, off = generate_text(500, seed=5)
    assert off[0] == 0 and off[-1] == text.size and np.all(np.diff(off) >= 0)
    lens = np.diff(off)
    assert 1000 < np.median(lens) < 5000
    tok_off, ids = ot.trigram_csr(text, off)
    assert ids.size == np.maximum(lens - 2, 0).sum()
    # a natural-text-like id distribution: many distinct ids, a heavy head
    u, c = np.unique(ids, return_counts=True)
    assert u.size > 5000 and c.max() > 50 * np.median(c)
