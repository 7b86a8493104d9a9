"""FP64 oracle of the Multi-reference Cosine method (test infrastructure only).

Follows the paper step by step:

  Section 3      a document is a vector of term counts (the paper counts
                 character 3-grams; here a term is an integer id) and two
                 vectors are compared by the cosine of Eq. (1)
  Section 4      a reference is a frequency-sorted list of terms with the
                 zero-frequency entries removed, optionally restricted to a
                 frequency region or to the rarest terms, and split into k
                 equal parts; a document's signature is its cosine against
                 each part
  Section 6      weighted vector-space models (future work): realised as TF-IDF

Readings where the paper is silent (each one is listed in the design notes):

* term frequency of the reference list = document frequency over the model
  corpus, frozen after the model is built;
* idf SMOOTH = ln((1 + N) / (1 + df)) + 1, or NONE (weight = raw count, the
  paper's own unweighted vectors);
* ties in the frequency-sorted list are broken by ascending term id;
* parts are contiguous runs of the list; when m is not a multiple of k the
  first m mod k parts hold one extra term;
* a reference part is the indicator vector of its terms (ONE) or carries the
  terms' idf (IDF);
* the signature-vs-signature similarity that Eq. (2) calls multi reference
  cosine is the cosine of Eq. (1) applied to the two signatures; it is 0 when
  either signature is zero;
* a pair i < j is a (near-)duplicate when that similarity is >= tau.

Everything below is plain NumPy in float64 (integers exact). It imports nothing
from the HIP product.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

IDF_SMOOTH, IDF_NONE = 0, 1
SEL_ALL, SEL_REGION, SEL_RAREST, SEL_DROP_TOP = 0, 1, 2, 3
REF_ONE, REF_IDF = 0, 1


@dataclass(frozen=True)
class RefSpec:
    """How the reference is chosen and split (Section 4).

    mode ALL      every term of the sorted list (the "all 3-grams" reference)
    mode REGION   positions lo .. hi-1 of the sorted list (hi < 0 means the end)
    mode RAREST   the last m positions (the paper's rarest / single-document terms)
    mode DROP_TOP positions ceil(V' * drop_top_ppm / 1e6) .. V'-1, i.e. the list
                  without its most frequent share
    """
    k: int
    mode: int = SEL_DROP_TOP
    lo: int = 0
    hi: int = -1
    m: int = 0
    drop_top_ppm: int = 50_000
    idf_mode: int = IDF_SMOOTH
    ref_weight: int = REF_ONE


@dataclass
class Model:
    n_docs: int
    vocab: int
    df: np.ndarray          # int64 [V]
    idf: np.ndarray         # float64 [V]
    order: np.ndarray       # int64 [V']  term ids, sorted list (df desc, id asc), df > 0 only
    lo: int                 # selected positions [lo, hi) of `order`
    hi: int
    k: int
    part_of: np.ndarray     # int64 [V]  reference part of each term, -1 if not selected
    rho: np.ndarray         # float64 [V]  reference weight of each term (0 if not selected)
    rnorm: np.ndarray       # float64 [k]  |r_j|
    spec: RefSpec


# --------------------------------------------------------------------------- counts

def term_counts(offsets, tokens, vocab: int):
    """tf[d][t] = number of occurrences of term t in document d (Section 3, the
    counting of all N-grams of a document into an M-dimensional vector).

    Returns (doc, term, tf) for the distinct (document, term) pairs, sorted by
    document then term id."""
    offsets = np.asarray(offsets, dtype=np.int64)
    tokens = np.asarray(tokens, dtype=np.int64)
    if tokens.size and (tokens.min() < 0 or tokens.max() >= vocab):
        raise ValueError("token id outside [0, vocab)")
    n = offsets.shape[0] - 1
    doc_of_token = np.repeat(np.arange(n, dtype=np.int64), np.diff(offsets))
    keys = doc_of_token * vocab + tokens
    uniq, tf = np.unique(keys, return_counts=True)
    return uniq // vocab, uniq % vocab, tf.astype(np.int64)


def document_frequency(term, vocab: int):
    """df[t] = number of documents of the model corpus that contain t. This is
    the reading of the paper's corpus frequency of a 3-gram (Section 4)."""
    return np.bincount(np.asarray(term, dtype=np.int64), minlength=vocab).astype(np.int64)


def idf_weights(df, n_docs: int, idf_mode: int):
    """Inverse document frequency. The paper proposes weighted vector space
    models as future work (Section 6) without a formula; SMOOTH is
    ln((1+N)/(1+df)) + 1, NONE keeps the paper's raw counts."""
    df = np.asarray(df, dtype=np.float64)
    if idf_mode == IDF_NONE:
        return np.ones_like(df)
    if idf_mode != IDF_SMOOTH:
        raise ValueError("unknown idf mode")
    return np.log((1.0 + n_docs) / (1.0 + df)) + 1.0


# --------------------------------------------------------------------------- reference

def sorted_term_list(df):
    """Terms with non-zero frequency, sorted by frequency descending (Section 4:
    the zero-frequency 3-grams are removed and the list is sorted descending);
    ties by ascending id."""
    df = np.asarray(df, dtype=np.int64)
    ids = np.nonzero(df > 0)[0]
    order = np.lexsort((ids, -df[ids]))
    return ids[order]


def selection_bounds(n_listed: int, spec: RefSpec):
    """Positions [lo, hi) of the sorted list that form the reference (Section 4:
    all terms; a frequency region such as 6000-8000; the rarest terms)."""
    Vp = int(n_listed)
    if spec.mode == SEL_ALL:
        lo, hi = 0, Vp
    elif spec.mode == SEL_REGION:
        lo = int(spec.lo)
        hi = Vp if spec.hi < 0 else min(int(spec.hi), Vp)
    elif spec.mode == SEL_RAREST:
        lo, hi = Vp - int(spec.m), Vp
    elif spec.mode == SEL_DROP_TOP:
        lo = -((-Vp * int(spec.drop_top_ppm)) // 1_000_000)      # ceil, exact integers
        hi = Vp
    else:
        raise ValueError("unknown selection mode")
    if lo < 0 or hi > Vp or hi - lo < int(spec.k) or spec.k < 1:
        raise ValueError("reference selection holds fewer terms than parts")
    return lo, hi


def partition_sizes(m: int, k: int):
    """Split m listed terms into k contiguous parts of equal length (Section 4);
    the first m mod k parts get one extra term."""
    q, r = divmod(int(m), int(k))
    return np.array([q + (1 if j < r else 0) for j in range(k)], dtype=np.int64)


def build_model(offsets, tokens, vocab: int, spec: RefSpec) -> Model:
    """Counts, df, idf, the sorted list, the selection and its k parts."""
    n = int(len(offsets) - 1)
    _, term, _ = term_counts(offsets, tokens, vocab)
    df = document_frequency(term, vocab)
    idf = idf_weights(df, n, spec.idf_mode)
    order = sorted_term_list(df)
    lo, hi = selection_bounds(order.shape[0], spec)
    sizes = partition_sizes(hi - lo, spec.k)
    part_of = np.full(vocab, -1, dtype=np.int64)
    part_of[order[lo:hi]] = np.repeat(np.arange(spec.k, dtype=np.int64), sizes)
    rho = np.zeros(vocab, dtype=np.float64)
    sel = part_of >= 0
    rho[sel] = 1.0 if spec.ref_weight == REF_ONE else idf[sel]
    if spec.ref_weight not in (REF_ONE, REF_IDF):
        raise ValueError("unknown reference weight")
    rnorm = np.sqrt(np.bincount(part_of[sel], weights=rho[sel] ** 2, minlength=spec.k))
    return Model(n, vocab, df, idf, order, lo, hi, int(spec.k), part_of, rho, rnorm, spec)


# --------------------------------------------------------------------------- signing

def tfidf(offsets, tokens, model: Model):
    """w[d][t] = tf * idf and |w_d| = sqrt(sum_t w^2) (Eq. (1)'s vector norm).
    Returns (doc, term, w, norm[N])."""
    doc, term, tf = term_counts(offsets, tokens, model.vocab)
    w = tf.astype(np.float64) * model.idf[term]
    n = int(len(offsets) - 1)
    norm = np.sqrt(np.bincount(doc, weights=w * w, minlength=n))
    return doc, term, w, norm


def sign(offsets, tokens, model: Model):
    """MRC signature (Section 4): sig[d][j] = cosine(w_d, r_j)
    = (sum over terms t of part j of w_dt * rho_t) / (|w_d| * |r_j|),
    0 for an empty document. Returns (sig [N][k], norm [N])."""
    doc, term, w, norm = tfidf(offsets, tokens, model)
    n = int(len(offsets) - 1)
    part = model.part_of[term]
    sel = part >= 0
    num = np.zeros((n, model.k), dtype=np.float64)
    np.add.at(num, (doc[sel], part[sel]), w[sel] * model.rho[term[sel]])
    den = norm[:, None] * model.rnorm[None, :]
    sig = np.divide(num, den, out=np.zeros_like(num), where=den > 0)
    return sig, norm


# --------------------------------------------------------------------------- general references

def reference_matrix(model: Model):
    """The k reference vectors of a model as the columns of a dense V x k
    matrix: R[t, part_of[t]] = rho_t (Section 4's parts; every term in at most
    one column)."""
    R = np.zeros((model.vocab, model.k), dtype=np.float64)
    sel = np.nonzero(model.part_of >= 0)[0]
    R[sel, model.part_of[sel]] = model.rho[sel]
    return R


def sign_matrix(offsets, tokens, model: Model, R):
    """Signature against k general reference vectors, the columns of a V x k
    matrix R whose entries may weight their terms and whose columns may share
    terms (Section 4's construction with Section 6's weighted vector-space
    models): sig[d][j] = w_d . r_j / (|w_d| |r_j|), Eq. (1) between the
    document's TF-IDF vector (the model's idf) and column j; 0 when either norm
    is 0. The model's own parts play no role. Returns (sig [N][k], norm [N])."""
    import scipy.sparse as sp
    R = np.asarray(R, dtype=np.float64)
    if R.ndim != 2 or R.shape[0] != model.vocab:
        raise ValueError("R must be vocab x k")
    doc, term, w, norm = tfidf(offsets, tokens, model)
    n = int(len(offsets) - 1)
    W = sp.csr_matrix((w, (doc, term)), shape=(n, model.vocab))
    num = np.asarray(W @ R)
    rnorm = np.sqrt((R * R).sum(axis=0))
    den = norm[:, None] * rnorm[None, :]
    sig = np.divide(num, den, out=np.zeros_like(num), where=den > 0)
    return sig, norm


# --------------------------------------------------------------------------- comparison

def normalise(sig):
    """Unit-length signatures; a zero signature stays zero. Cosine between two
    signatures (Eq. (1) on the signatures) is then their dot product."""
    sig = np.asarray(sig, dtype=np.float64)
    nrm = np.sqrt((sig * sig).sum(axis=1))
    return np.divide(sig, nrm[:, None], out=np.zeros_like(sig), where=nrm[:, None] > 0)


def mrc_scores(shat_a, shat_b):
    """multi reference cosine(D_i, D_j) for every i of block a and j of block b."""
    return np.asarray(shat_a, np.float64) @ np.asarray(shat_b, np.float64).T


def compare_pairs(shat, tau: float, block: int = 2048):
    """All pairs i < j with MRC(i, j) >= tau. Returns (i, j, s) sorted by (i, j).
    Rows are taken a block at a time only to bound memory; every score is the
    same dot product."""
    shat = np.asarray(shat, np.float64)
    n = shat.shape[0]
    out_i, out_j, out_s = [], [], []
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        s = mrc_scores(shat[r0:r1], shat)
        ii, jj = np.nonzero(s >= tau)
        keep = jj > ii + r0
        out_i.append(ii[keep] + r0)
        out_j.append(jj[keep])
        out_s.append(s[ii[keep], jj[keep]])
    if not out_i:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    return np.concatenate(out_i), np.concatenate(out_j), np.concatenate(out_s)


def pair_scores(shat, i, j):
    """MRC(i, j) for listed pairs (used to score sampled pairs at full size)."""
    shat = np.asarray(shat, np.float64)
    return np.einsum("pc,pc->p", shat[np.asarray(i)], shat[np.asarray(j)])


def query_topk(shat_db, shat_q, topk: int, tau: float):
    """For each query, the topk database rows by MRC (score descending, id
    ascending) and the number of rows with MRC >= tau. Section 1's use: compare
    each new page with all the other pages through their signatures."""
    s = mrc_scores(shat_q, shat_db)
    nq, ndb = s.shape
    ids = np.zeros((nq, topk), np.int64) - 1
    sc = np.zeros((nq, topk))
    ar = np.arange(ndb, dtype=np.int64)
    for q in range(nq):
        o = np.lexsort((ar, -s[q]))[:topk]
        ids[q, :o.size] = o
        sc[q, :o.size] = s[q, o]
    hits = (s >= tau).sum(axis=1).astype(np.int64)
    return ids, sc, hits


# --------------------------------------------------------------------------- quantisers

def bf16_codes(x32):
    """Round-to-nearest-even float32 -> bfloat16 (the upper 16 bits after
    rounding). Finite inputs only."""
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def bf16_value(codes):
    return (np.asarray(codes, np.uint16).astype(np.uint32) << 16).view(np.float32)


_E4M3_VALUES = None


def fp8_e4m3fn_value(codes):
    """Decode OCP float8 e4m3fn: 1 sign, 4 exponent (bias 7), 3 mantissa bits,
    subnormals at exponent 0, no infinities, S.1111.111 is NaN."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    f = c & 7
    mag = np.where(e == 0, f / 8.0 * 2.0 ** -6, (1.0 + f / 8.0) * 2.0 ** (e - 7))
    mag = np.where((e == 15) & (f == 7), np.nan, mag)
    return s * mag


def fp8_e4m3fn_codes(x32):
    """Round-to-nearest-even float32 -> float8 e4m3fn for |x| <= 448 (the
    largest finite value). Chooses, among the representable values, the one
    nearest to x, ties to the even code; computed exactly in float64."""
    global _E4M3_VALUES
    if _E4M3_VALUES is None:
        _E4M3_VALUES = fp8_e4m3fn_value(np.arange(0, 127, dtype=np.uint8))   # +0 .. 448
    x = np.asarray(x32, dtype=np.float32).astype(np.float64)
    a = np.abs(x)
    if np.any(a > 464.0) or np.any(~np.isfinite(a)):
        raise ValueError("value outside the finite e4m3fn range")
    vals = _E4M3_VALUES
    hi = np.searchsorted(vals, a, side="left")            # first value >= a
    hi = np.minimum(hi, vals.size - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = a - vals[lo]
    dhi = vals[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a == vals[hi], hi, code)
    code = np.where(a > 448.0, 126, code)                 # (448, 464] rounds to 448
    return (code | np.where(np.signbit(x), 0x80, 0)).astype(np.uint8)


def fp8_quantise_rows(shat32):
    """Per-row FP8 form: scale_i = the smallest power of two >= max_c |s_ic| / 448
    (the quotient taken in float32), q_ic = RNE_e4m3fn(s_ic / scale_i) (float32
    division, exact for a power of two), zero rows get scale 0 and zero codes.
    A power-of-two scale is what the matrix cores can apply as an E8M0 operand
    scale; the paper defines no FP8 form (this is the candidate filter's code).
    Returns (codes uint8 [N][k], scale float32 [N])."""
    x = np.asarray(shat32, dtype=np.float32)
    mx = np.abs(x).max(axis=1) if x.shape[1] else np.zeros(x.shape[0], np.float32)
    q = (mx / np.float32(448.0)).astype(np.float32)
    m, e = np.frexp(q.astype(np.float64))                 # q = m 2^e, m in [0.5, 1)
    scale = np.where(m == 0.5, q.astype(np.float64), np.ldexp(1.0, e)).astype(np.float32)
    scale = np.where(q > 0, scale, np.float32(0.0)).astype(np.float32)
    safe = np.where(scale > 0, scale, np.float32(1.0)).astype(np.float32)
    y = (x / safe[:, None]).astype(np.float32)
    codes = fp8_e4m3fn_codes(y)
    codes[scale == 0] = 0
    return codes, scale


def fp8_dequantise_rows(codes, scale):
    return fp8_e4m3fn_value(codes) * np.asarray(scale, np.float64)[:, None]


def row_quant_error(shat32, deq):
    """eps_i = || s_i - deq(q_i) ||_2 in float64."""
    d = np.asarray(shat32, np.float64) - np.asarray(deq, np.float64)
    return np.sqrt((d * d).sum(axis=1))


def lowp_band(eps_i, eps_j, k: int, nominal: float = 0.02):
    """Per-pair rescoring band for a low-precision score (the reading for the
    FP8 form): with a_i = deq(q_i) = s_i + e_i and |e_i| = eps_i, |s| <= 1,
    |a_i . a_j - s_i . s_j| <= eps_i + eps_j + eps_i*eps_j, plus float32
    accumulation of the low-precision sum and of the plain chain (each at most
    k * 2^-24 times |a_i||a_j| <= (1+eps_i)(1+eps_j)) and two scale roundings.
    The band is the larger of that bound and the nominal +-0.02."""
    e1 = np.asarray(eps_i, np.float64)
    e2 = np.asarray(eps_j, np.float64)
    acc = k * 2.0 ** -24
    bound = e1 + e2 + e1 * e2 + acc * (1 + e1) * (1 + e2) + acc + 2.0 ** -21
    return np.maximum(nominal, bound)


# --------------------------------------------------------------------------- FP32 chain

_FMA_LIB = None


def _fma_lib():
    global _FMA_LIB
    if _FMA_LIB is None:
        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "_fma_chain.so")
        if not os.path.exists(so):
            build_fma_chain()
        lib = ctypes.CDLL(so)
        lib.oracle_score32_pairs.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_score32_pairs.restype = None
        lib.oracle_score32.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib.oracle_score32.restype = ctypes.c_float
        _FMA_LIB = lib
    return _FMA_LIB


def build_fma_chain():
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "fma_chain.c")
    so = os.path.join(here, "_fma_chain.so")
    tmp = so + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", src, "-o", tmp, "-lm"])
    os.replace(tmp, so)
    return so


def score32_pairs(shat32, i, j):
    """The plain FP32 score of each listed pair: acc = 0; for c = 0..k-1:
    acc = fmaf(s_ic, s_jc, acc) (one correctly rounded multiply-add per term,
    ascending c). This fixed chain is the definition the FP32 path follows."""
    x = np.ascontiguousarray(shat32, dtype=np.float32)
    ii = np.ascontiguousarray(i, dtype=np.int64)
    jj = np.ascontiguousarray(j, dtype=np.int64)
    out = np.zeros(ii.shape[0], dtype=np.float32)
    _fma_lib().oracle_score32_pairs(x.ctypes.data, x.shape[1], ii.ctypes.data,
                                    jj.ctypes.data, ii.shape[0], out.ctypes.data)
    return out
