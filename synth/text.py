"""Seeded synthetic raw text (bytes) for the character 3-gram front end.

Stands in for the paper's newsgroup text: words of 1-12 letters drawn from a
Zipf-ranked vocabulary of random letter strings, with capitalised words,
digits, punctuation, line breaks and a few bytes above 0x7F; document lengths
lognormal in words. Draws bytes only: no 3-gram or any other arithmetic of the
method.
"""
from __future__ import annotations

import numpy as np

SEPARATORS = np.frombuffer(b"       ,.\n;-", dtype=np.uint8)


def generate_text(n_docs: int, seed: int = 1810, median_words: float = 300.0, sigma: float = 0.8,
                  n_words: int = 50_000, max_words: int = 20_000):
    """Returns (text uint8 [n_bytes], offsets int64 [n_docs + 1])."""
    rng = np.random.default_rng(seed)
    # the vocabulary: random letter strings, lengths 1-12
    wl = rng.integers(1, 13, n_words)
    wstart = np.zeros(n_words + 1, dtype=np.int64)
    np.cumsum(wl, out=wstart[1:])
    letters = rng.integers(ord("a"), ord("z") + 1, int(wstart[-1])).astype(np.uint8)
    # a few words carry a digit or a byte above 0x7F
    odd = rng.random(n_words) < 0.02
    letters[wstart[:-1][odd]] = rng.choice(np.frombuffer(b"0123456789\xc3\xa9", dtype=np.uint8), int(odd.sum()))
    # words per document
    nw = np.clip(np.rint(rng.lognormal(np.log(median_words), sigma, n_docs)), 0, max_words).astype(np.int64)
    nw[rng.random(n_docs) < 0.01] = 0  # some empty documents
    total = int(nw.sum())
    # Zipf ranks over the vocabulary
    ranks = np.minimum(rng.zipf(1.2, total) - 1, n_words - 1)
    word = rng.permutation(n_words)[ranks]
    lens = wl[word] + 1                                 # word + one separator
    pos = np.zeros(total + 1, dtype=np.int64)
    np.cumsum(lens, out=pos[1:])
    text = np.empty(int(pos[-1]), dtype=np.uint8)
    # copy each word's letters: index arithmetic over a flat gather
    within = np.arange(int(pos[-1]), dtype=np.int64) - np.repeat(pos[:-1], lens)
    src_word = np.repeat(word, lens)
    is_sep = within == np.repeat(lens - 1, lens)
    src = wstart[src_word] + np.minimum(within, wl[src_word] - 1)
    text[:] = letters[src]
    text[is_sep] = SEPARATORS[rng.integers(0, SEPARATORS.size, int(is_sep.sum()))]
    # capitalise about one word in ten
    cap = rng.random(total) < 0.1
    first = pos[:-1][cap]
    up = (text[first] >= ord("a")) & (text[first] <= ord("z"))
    text[first[up]] -= 32
    doc_end_word = np.cumsum(nw)
    offsets = np.zeros(n_docs + 1, dtype=np.int64)
    offsets[1:] = pos[doc_end_word]
    return text, offsets
