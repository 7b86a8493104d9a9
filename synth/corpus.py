"""Synthetic near-duplicate corpora with the shape of the paper's workload.

The paper evaluates on NEWS20 (about 18,828 newsgroup documents, Section 5) with
character 3-grams as terms. That dataset is not available here, and none of its
items are reproduced. Instead every corpus is drawn from a seeded generator of
integer term ids whose statistics mimic natural text:

* term ranks follow a global Zipf law, P(rank r) proportional to r**-s, truncated
  to the vocabulary, drawn by inverse-CDF sampling (rank r maps to id r-1);
* 20 topics, each a seeded permutation of the ids; every document picks one topic
  uniformly and each of its tokens comes from the topic's Zipf (rank r maps to
  perm[r-1]) with probability `topic_weight`, else from the global Zipf;
* document lengths are lognormal, L = clip(round(exp(ln(median) + sigma*z)));
* a share of documents are exact copies of an original, and a share are near
  duplicates: a uniform edit rate e in [e_lo, e_hi], max(1, round(e*L)) distinct
  positions, each replaced (p=0.5, by a fresh draw from the source's topic
  mixture) or deleted (p=0.5);
* document order is shuffled afterwards; `source[d]` keeps the index of the
  original each copy came from (-1 for originals).

Seeds are 181003099 + the 0-based position of the configuration in `CONFIGS`.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 181003099


@dataclass(frozen=True)
class CorpusSpec:
    name: str
    n_docs: int
    vocab: int
    median_len: float
    sigma: float
    len_lo: int
    len_hi: int
    exact_frac: float
    near_frac: float
    edit_lo: float
    edit_hi: float
    k: int
    zipf_s: float = 1.1
    n_topics: int = 20
    topic_weight: float = 0.5
    tau: float = 0.9


# The five workload shapes. Index in this tuple = seed offset.
CONFIGS = (
    CorpusSpec("plain_small", 2_000, 16_384, 200, 0.8, 20, 2_000, 0.00, 0.10, 0.01, 0.10, 16),
    CorpusSpec("plain_full", 20_000, 131_072, 300, 0.8, 20, 2_000, 0.05, 0.10, 0.01, 0.15, 64),
    CorpusSpec("precision", 200_000, 262_144, 400, 0.8, 20, 2_000, 0.05, 0.10, 0.01, 0.15, 256),
    CorpusSpec("serving_db", 1_000_000, 262_144, 400, 0.8, 20, 2_000, 0.05, 0.10, 0.01, 0.15, 128),
    CorpusSpec("serving_fp8_db", 4_000_000, 262_144, 400, 0.8, 20, 2_000, 0.05, 0.10, 0.01, 0.15, 256),
)


def config_seed(index: int) -> int:
    return BASE_SEED + int(index)


@dataclass
class Corpus:
    """A batch of documents as a token CSR: doc d owns tokens[offsets[d]:offsets[d+1]]."""
    offsets: np.ndarray            # int64 [N+1]
    tokens: np.ndarray             # int32 [T]
    vocab: int
    source: np.ndarray             # int64 [N]; -1 for originals
    kind: np.ndarray               # int8 [N]; 0 original, 1 exact copy, 2 near duplicate
    spec: CorpusSpec | None = None
    extra: dict = field(default_factory=dict)

    @property
    def n_docs(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def doc(self, d: int) -> np.ndarray:
        return self.tokens[self.offsets[d]:self.offsets[d + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def subset(self, idx) -> "Corpus":
        idx = np.asarray(idx, dtype=np.int64)
        docs = [self.doc(int(d)) for d in idx]
        return from_docs(docs, self.vocab, spec=self.spec)


def from_docs(docs, vocab: int, spec: CorpusSpec | None = None) -> Corpus:
    lens = np.array([len(d) for d in docs], dtype=np.int64)
    offsets = np.zeros(len(docs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    tokens = (np.concatenate([np.asarray(d, dtype=np.int32) for d in docs])
              if len(docs) and offsets[-1] > 0 else np.zeros(0, dtype=np.int32))
    n = len(docs)
    return Corpus(offsets, tokens.astype(np.int32), vocab,
                  np.full(n, -1, np.int64), np.zeros(n, np.int8), spec)


class _Sampler:
    """Global + per-topic Zipf token draws over ids 0..V-1."""

    def __init__(self, rng: np.random.Generator, vocab: int, s: float, n_topics: int,
                 topic_weight: float):
        ranks = np.arange(1, vocab + 1, dtype=np.float64)
        p = ranks ** (-s)
        self.cdf = np.cumsum(p)
        self.vocab = vocab
        self.topic_weight = topic_weight
        self.perms = np.stack([rng.permutation(vocab).astype(np.int32) for _ in range(n_topics)])

    def draw(self, rng: np.random.Generator, topics: np.ndarray) -> np.ndarray:
        """One token per entry of `topics` (the topic of the document it belongs to)."""
        n = topics.shape[0]
        u = rng.random(n)
        use_topic = rng.random(n) < self.topic_weight

        def part(sl):
            r0 = np.searchsorted(self.cdf, u[sl] * self.cdf[-1], side="right")
            np.minimum(r0, self.vocab - 1, out=r0)      # rank r0+1 -> index r0
            out = r0.astype(np.int32)
            m = use_topic[sl]
            out[m] = self.perms[topics[sl][m], r0[m]]
            return out

        if n < (1 << 22):
            return part(slice(None))
        # large draws: the same per-element steps over slices in threads (NumPy
        # releases the GIL inside them)
        from concurrent.futures import ThreadPoolExecutor
        step = -(-n // 64)
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            return np.concatenate(list(ex.map(part, [slice(i, min(n, i + step)) for i in range(0, n, step)])))


def _lengths(rng, n, median, sigma, lo, hi):
    z = rng.standard_normal(n)
    return np.clip(np.rint(np.exp(np.log(median) + sigma * z)), lo, hi).astype(np.int64)


def generate(spec_or_index, n_docs: int | None = None, seed: int | None = None) -> Corpus:
    """Draw a corpus. `spec_or_index` is a CorpusSpec or an index into CONFIGS.

    `n_docs` overrides the document count (keeping every other statistic), which
    the tests use for reduced-size cases.
    """
    if isinstance(spec_or_index, int):
        spec = CONFIGS[spec_or_index]
        if seed is None:
            seed = config_seed(spec_or_index)
    else:
        spec = spec_or_index
        if seed is None:
            seed = BASE_SEED
    N = spec.n_docs if n_docs is None else int(n_docs)
    rng = np.random.default_rng(np.random.PCG64(seed))
    sampler = _Sampler(rng, spec.vocab, spec.zipf_s, spec.n_topics, spec.topic_weight)

    n_exact = int(round(spec.exact_frac * N))
    n_near = int(round(spec.near_frac * N))
    n_orig = N - n_exact - n_near
    if n_orig <= 0:
        raise ValueError("corpus needs at least one original document")

    # originals, drawn in one vectorised pass
    o_topic = rng.integers(0, spec.n_topics, n_orig)
    o_len = _lengths(rng, n_orig, spec.median_len, spec.sigma, spec.len_lo, spec.len_hi)
    o_off = np.zeros(n_orig + 1, np.int64)
    np.cumsum(o_len, out=o_off[1:])
    o_tok = sampler.draw(rng, np.repeat(o_topic, o_len))

    docs_tok = [None] * N
    topic = np.empty(N, np.int64)
    source = np.full(N, -1, np.int64)
    kind = np.zeros(N, np.int8)
    for d in range(n_orig):
        docs_tok[d] = o_tok[o_off[d]:o_off[d + 1]]
        topic[d] = o_topic[d]

    # exact copies
    ex_src = rng.integers(0, n_orig, n_exact)
    for i, s in enumerate(ex_src):
        d = n_orig + i
        docs_tok[d] = docs_tok[s].copy()
        topic[d] = topic[s]
        source[d] = s
        kind[d] = 1

    # near duplicates
    nr_src = rng.integers(0, n_orig, n_near)
    for i, s in enumerate(nr_src):
        d = n_orig + n_exact + i
        base = docs_tok[s]
        L = base.shape[0]
        e = rng.uniform(spec.edit_lo, spec.edit_hi)
        n_edit = min(L, max(1, int(round(e * L))))
        pos = rng.choice(L, n_edit, replace=False)
        replace = rng.random(n_edit) < 0.5
        new = base.copy()
        rp = pos[replace]
        if rp.size:
            new[rp] = sampler.draw(rng, np.full(rp.size, topic[s], np.int64))
        keep = np.ones(L, bool)
        keep[pos[~replace]] = False
        docs_tok[d] = new[keep]
        topic[d] = topic[s]
        source[d] = s
        kind[d] = 2

    # shuffle document order; remap sources to shuffled indices
    perm = rng.permutation(N)           # new position p holds old doc perm[p]
    inv = np.empty(N, np.int64)
    inv[perm] = np.arange(N)
    docs_tok = [docs_tok[o] for o in perm]
    src_old = source[perm]
    source_new = np.where(src_old >= 0, inv[np.maximum(src_old, 0)], -1)
    c = from_docs(docs_tok, spec.vocab, spec)
    c.source = source_new.astype(np.int64)
    c.kind = kind[perm]
    c.extra["topic"] = topic[perm]
    c.extra["seed"] = seed
    return c


def generate_queries(spec: CorpusSpec, n: int, seed: int, median: float = 400.0,
                     sigma: float = 1.2, lo: int = 20, hi: int = 20_000,
                     near_of: Corpus | None = None, near_frac: float = 0.2) -> Corpus:
    """Query documents for the serving workloads (lognormal lengths, a share of
    them near duplicates of documents in `near_of`)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    sampler = _Sampler(rng, spec.vocab, spec.zipf_s, spec.n_topics, spec.topic_weight)
    lens = _lengths(rng, n, median, sigma, lo, hi)
    topics = rng.integers(0, spec.n_topics, n)
    docs = []
    source = np.full(n, -1, np.int64)
    for q in range(n):
        if near_of is not None and rng.random() < near_frac:
            s = int(rng.integers(0, near_of.n_docs))
            base = near_of.doc(s)
            L = base.shape[0]
            if L == 0:
                docs.append(base.copy())
                continue
            n_edit = min(L, max(1, int(round(rng.uniform(0.01, 0.10) * L))))
            pos = rng.choice(L, n_edit, replace=False)
            new = base.copy()
            new[pos] = sampler.draw(rng, np.full(n_edit, topics[q], np.int64))
            docs.append(new)
            source[q] = s
        else:
            docs.append(sampler.draw(rng, np.full(int(lens[q]), topics[q], np.int64)))
    c = from_docs(docs, spec.vocab, spec)
    c.source = source
    c.kind = (source >= 0).astype(np.int8) * 2
    return c
