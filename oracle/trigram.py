"""Character 3-gram front end: the oracle (TEST INFRASTRUCTURE ONLY).

Sections 3-4 treat a document, and the reference, as a vector of character
3-gram counts; the paper does not fix the alphabet. Reading taken here: the 26
ASCII letters, case-folded, are symbols 0-25 and every other byte (space,
digit, punctuation, control, any byte >= 0x80) is one separator symbol 26.
Every window of three consecutive bytes of a document is one 3-gram, with id
27^2 s0 + 27 s1 + s2 in [0, 27^3); a document of L bytes gives max(L - 2, 0)
ids in text order. Runs of separators are not collapsed.

`doc_trigrams` is the plain per-byte definition (pure Python, small inputs);
`trigram_csr` is the same definition over a whole byte buffer with NumPy, for
sizes the loops cannot reach. The tests pin the second to the first, and the
first to worked examples, closed forms and invariances.
"""
from __future__ import annotations

import numpy as np

ALPHABET = 27
SEPARATOR = 26
VOCAB = ALPHABET ** 3


def symbol(byte: int) -> int:
    """Symbol of one byte: 'a'/'A' .. 'z'/'Z' -> 0..25, anything else -> 26."""
    if 65 <= byte <= 90:
        return byte - 65
    if 97 <= byte <= 122:
        return byte - 97
    return SEPARATOR


def doc_trigrams(doc: bytes) -> list[int]:
    """Ids of every window of three consecutive bytes, in order."""
    out = []
    for i in range(len(doc) - 2):
        s0, s1, s2 = symbol(doc[i]), symbol(doc[i + 1]), symbol(doc[i + 2])
        out.append(s0 * ALPHABET * ALPHABET + s1 * ALPHABET + s2)
    return out


def trigram_csr(text, offsets):
    """(token offsets int64 [n+1], ids int32) of every document of a byte CSR."""
    t = np.frombuffer(bytes(text), dtype=np.uint8) if not isinstance(text, np.ndarray) else text
    off = np.asarray(offsets, dtype=np.int64)
    n = off.size - 1
    lens = np.diff(off)
    counts = np.maximum(lens - 2, 0)
    tok_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=tok_off[1:])
    table = np.array([symbol(b) for b in range(256)], dtype=np.int32)
    sym = table[t]
    if t.size < 3:
        return tok_off, np.zeros(0, dtype=np.int32)
    ids = sym[:-2] * (ALPHABET * ALPHABET) + sym[1:-1] * ALPHABET + sym[2:]
    # window starting at byte p belongs to its document when p + 2 < the document's end
    doc_of = np.repeat(np.arange(n, dtype=np.int64), lens)
    starts = np.arange(t.size - 2, dtype=np.int64)
    keep = starts + 2 < off[1:][doc_of[: t.size - 2]]
    out = ids[keep].astype(np.int32)
    assert out.size == tok_off[-1]
    return tok_off, out
