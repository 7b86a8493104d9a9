"""Pure-Python loops over tiny corpora (test infrastructure only).

An independent second statement of the method with dicts, sets and math
functions only, used to check `oracle.mrc` term by term. Same readings as
`oracle.mrc` (see its module docstring).
"""
from __future__ import annotations

import math


def counts(doc):
    tf = {}
    for t in doc:
        tf[int(t)] = tf.get(int(t), 0) + 1
    return tf


def model(docs, vocab, k, select, idf_smooth=True, ref_idf=False):
    """`select(n_listed)` returns (lo, hi). Returns a dict with df, idf, list,
    parts (list of term lists) and reference norms."""
    N = len(docs)
    df = [0] * vocab
    for d in docs:
        for t in set(int(x) for x in d):
            df[t] += 1
    idf = [(math.log((1 + N) / (1 + df[t])) + 1) if idf_smooth else 1.0 for t in range(vocab)]
    listed = sorted([t for t in range(vocab) if df[t] > 0], key=lambda t: (-df[t], t))
    lo, hi = select(len(listed))
    chosen = listed[lo:hi]
    m = len(chosen)
    q, r = m // k, m % k
    parts, pos = [], 0
    for j in range(k):
        size = q + (1 if j < r else 0)
        parts.append(chosen[pos:pos + size])
        pos += size
    rho = {}
    for p in parts:
        for t in p:
            rho[t] = idf[t] if ref_idf else 1.0
    rnorm = [math.sqrt(sum(rho[t] ** 2 for t in p)) for p in parts]
    return {"df": df, "idf": idf, "list": listed, "parts": parts, "rho": rho, "rnorm": rnorm}


def signature(doc, mdl):
    tf = counts(doc)
    w = {t: c * mdl["idf"][t] for t, c in tf.items()}
    norm = math.sqrt(sum(v * v for v in w.values()))
    sig = []
    for p, rn in zip(mdl["parts"], mdl["rnorm"]):
        num = sum(w.get(t, 0.0) * mdl["rho"][t] for t in p)
        sig.append(num / (norm * rn) if norm > 0 and rn > 0 else 0.0)
    return sig, norm


def cosine(a, b):
    """Eq. (1) on two dense lists."""
    dot = sum(x * y for x, y in zip(a, b))
    na = math.sqrt(sum(x * x for x in a))
    nb = math.sqrt(sum(y * y for y in b))
    return dot / (na * nb) if na > 0 and nb > 0 else 0.0


def tfidf_cosine(d1, d2, idf):
    w1 = {t: c * idf[t] for t, c in counts(d1).items()}
    w2 = {t: c * idf[t] for t, c in counts(d2).items()}
    dot = sum(v * w2.get(t, 0.0) for t, v in w1.items())
    n1 = math.sqrt(sum(v * v for v in w1.values()))
    n2 = math.sqrt(sum(v * v for v in w2.values()))
    return dot / (n1 * n2) if n1 > 0 and n2 > 0 else 0.0


def simhash(doc, hashes):
    cols = [0] * 64
    for t in doc:
        h = int(hashes[int(t)])
        for b in range(64):
            cols[b] += 1 if (h >> b) & 1 else -1
    out = 0
    for b in range(64):
        if cols[b] > 0:
            out |= 1 << b
    return out


def hamming(x, y):
    return bin(int(x) ^ int(y)).count("1")
