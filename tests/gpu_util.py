"""Helpers for the GPU tests: device copies of synthetic corpora and a shared
library context. Holds none of the method's arithmetic."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_03099_amd import mrc
    if not os.path.exists(mrc.LIB_PATH):
        # with a GPU present the product must be there: fail loudly, never fall back
        raise RuntimeError(f"{mrc.LIB_PATH} missing: the HIP library must be built before GPU tests")
    return mrc


def device_docs(corpus_or_docs, vocab=None):
    import torch
    if hasattr(corpus_or_docs, "offsets"):
        off, tok = corpus_or_docs.offsets, corpus_or_docs.tokens
    else:
        docs = corpus_or_docs
        lens = np.array([len(d) for d in docs], np.int64)
        off = np.zeros(len(docs) + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        tok = np.concatenate([np.asarray(d, np.int32) for d in docs]) if off[-1] else np.zeros(0, np.int32)
    o = torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(tok, np.int32)).cuda()
    if t.numel() == 0:
        t = torch.zeros(1, dtype=torch.int32, device="cuda")
    return o, t


def flush(msg):
    print(msg, flush=True)
