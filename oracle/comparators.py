"""Oracle comparators and evaluation metrics (test infrastructure only).

* exact cosine (Eq. (1)) on the TF-IDF vectors: the ground truth the paper
  compares against (Section 5, every document compared with every other);
* Simhash-64 and Hamming distance (Section 3);
* MAE and variance of Eqs. (2)-(3), and recall / precision of a flagged pair set.
"""
from __future__ import annotations

import hashlib

import numpy as np
import scipy.sparse as sp

from . import mrc


# --------------------------------------------------------------------------- exact cosine

def tfidf_matrix(offsets, tokens, model: mrc.Model):
    """Rows w_d / |w_d| as a sparse matrix (zero rows for empty documents)."""
    doc, term, w, norm = mrc.tfidf(offsets, tokens, model)
    n = int(len(offsets) - 1)
    scale = np.divide(1.0, norm, out=np.zeros_like(norm), where=norm > 0)
    return sp.csr_matrix((w * scale[doc], (doc, term)), shape=(n, model.vocab))


def exact_cosine_pairs(offsets, tokens, model: mrc.Model, tau: float, block: int = 2048):
    """All pairs i < j with cosine(w_i, w_j) >= tau (Eq. (1)). Returns (i, j, s)
    sorted by (i, j). Row blocks only bound memory."""
    W = tfidf_matrix(offsets, tokens, model)
    WT = W.T.tocsc()
    n = W.shape[0]
    oi, oj, os_ = [], [], []
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        G = (W[r0:r1] @ WT).toarray()
        ii, jj = np.nonzero(G >= tau)
        keep = jj > ii + r0
        oi.append(ii[keep] + r0)
        oj.append(jj[keep])
        os_.append(G[ii[keep], jj[keep]])
    if not oi:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    return np.concatenate(oi), np.concatenate(oj), np.concatenate(os_)


def exact_cosine_scores(offsets, tokens, model: mrc.Model, i, j):
    W = tfidf_matrix(offsets, tokens, model)
    i = np.asarray(i)
    j = np.asarray(j)
    return np.asarray(W[i].multiply(W[j]).sum(axis=1)).ravel()


# --------------------------------------------------------------------------- simhash

def md5_term_hashes(vocab: int):
    """h(t) = the first 8 bytes, read little-endian, of MD5 over t as a 4-byte
    little-endian integer (the paper hashes tokens with MD5 or SHA1 into N bits;
    the token encoding and bit order are this reading)."""
    out = np.empty(vocab, dtype=np.uint64)
    for t in range(vocab):
        d = hashlib.md5(int(t).to_bytes(4, "little")).digest()
        out[t] = int.from_bytes(d[:8], "little")
    return out


def simhash64(offsets, tokens, vocab: int, hashes=None):
    """Simhash (Section 3): every token occurrence adds +1 to bit column b when
    bit b of its hash is 1 and -1 when it is 0; bit b of the result is 1 when
    the column sum is greater than 0, else 0."""
    if hashes is None:
        hashes = md5_term_hashes(vocab)
    doc, term, tf = mrc.term_counts(offsets, tokens, vocab)
    n = int(len(offsets) - 1)
    bits = ((hashes[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.int64)
    pm = 2 * bits - 1                                               # V x 64 of +-1
    TF = sp.csr_matrix((tf, (doc, term)), shape=(n, vocab), dtype=np.int64)
    acc = np.asarray(TF @ pm)                                       # exact integers
    out = np.zeros(n, dtype=np.uint64)
    for b in range(64):
        out |= (acc[:, b] > 0).astype(np.uint64) << np.uint64(b)
    return out


def hamming(x, y):
    """Number of differing bits between 64-bit words."""
    return np.bitwise_count(np.bitwise_xor(np.asarray(x, np.uint64), np.asarray(y, np.uint64))).astype(np.int64)


def hamming_pairs(sim, max_dist: int, block: int = 4096):
    """All pairs i < j with Hamming(sim_i, sim_j) <= max_dist, sorted by (i, j)."""
    sim = np.asarray(sim, np.uint64)
    n = sim.shape[0]
    oi, oj, od = [], [], []
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        h = hamming(sim[r0:r1, None], sim[None, :])
        ii, jj = np.nonzero(h <= max_dist)
        keep = jj > ii + r0
        oi.append(ii[keep] + r0)
        oj.append(jj[keep])
        od.append(h[ii[keep], jj[keep]])
    if not oi:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(oi), np.concatenate(oj), np.concatenate(od)


# --------------------------------------------------------------------------- metrics

def mae_variance(approx, truth):
    """Eqs. (2)-(3) as read: MAE = mean over pairs of |M - cos|; variance =
    mean over pairs of (e - mean(e))^2 with e = M - cos. The printed Eq. (2)
    has no absolute value and divides a pair sum by the number of documents;
    `paper_literal` returns that form for the record."""
    a = np.asarray(approx, np.float64)
    t = np.asarray(truth, np.float64)
    e = a - t
    if e.size == 0:
        return 0.0, 0.0
    return float(np.abs(e).mean()), float(((e - e.mean()) ** 2).mean())


def mae_paper_literal(approx, truth, n_docs: int):
    e = np.asarray(approx, np.float64) - np.asarray(truth, np.float64)
    return float(e.sum() / n_docs)


def simhash_similarity(dist):
    """Similarity of two Simhash words for the error metrics: 1 - H / 64."""
    return 1.0 - np.asarray(dist, np.float64) / 64.0


def recall_precision(found_i, found_j, true_i, true_j):
    """Recall and precision of a flagged pair set against a ground-truth set."""
    f = set(zip(np.asarray(found_i).tolist(), np.asarray(found_j).tolist()))
    t = set(zip(np.asarray(true_i).tolist(), np.asarray(true_j).tolist()))
    tp = len(f & t)
    recall = tp / len(t) if t else 1.0
    precision = tp / len(f) if f else 1.0
    return recall, precision
