"""Thin Python binding of libmrc (the C ABI in include/mrc.h).

Argument marshalling only: every step of the method runs in the HIP library.
Torch tensors supply device memory and the HIP stream (torch's current stream
unless one is given). The functions keep the C names.

If libmrc.so has not been built, importing works but the first call raises
MrcUnavailable: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

try:
    import torch
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrc.so")

MRC_OK, MRC_E_INVAL, MRC_E_NOMEM, MRC_E_OVERFLOW, MRC_E_HIP, MRC_E_BUSY, MRC_E_STATE = 0, -1, -2, -3, -4, -5, -6
SEL_ALL, SEL_REGION, SEL_RAREST, SEL_DROP_TOP = 0, 1, 2, 3
IDF_SMOOTH, IDF_NONE = 0, 1
REF_ONE, REF_IDF = 0, 1
PREC_FP32, PREC_BF16, PREC_FP8 = 0, 1, 2
SCAN_GRID, SCAN_PERSISTENT = 0, 1
REQ_QUERY, REQ_INSERT = 0, 1

# names of the exported C functions (checked against include/mrc.h by the tests)
EXPORTS = (
    "mrc_ctx_create", "mrc_ctx_destroy", "mrc_ctx_memory", "mrc_ctx_set_timing", "mrc_ctx_set_scan", "mrc_ctx_kernel_time",
    "mrc_last_error", "mrc_build_vocab_idf", "mrc_build_and_sign", "mrc_model_destroy", "mrc_model_info", "mrc_model_get",
    "mrc_model_save", "mrc_model_load", "mrc_sign", "mrc_sign_matrix", "mrc_compare", "mrc_compare_f32_noalloc", "mrc_normalise", "mrc_score_pairs",
    "mrc_trigrams", "mrc_simhash", "mrc_term_hashes", "mrc_hamming_pairs", "mrc_exact_cosine", "mrc_db_create",
    "mrc_db_destroy", "mrc_db_insert", "mrc_db_insert_docs", "mrc_db_size", "mrc_db_save", "mrc_db_load",
    "mrc_query", "mrc_serve_start", "mrc_serve_submit", "mrc_serve_submit_many", "mrc_serve_poll", "mrc_serve_stop",
)


class MrcUnavailable(RuntimeError):
    pass


class MrcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class MrcDocs(C.Structure):
    _fields_ = [("n_docs", C.c_int64), ("offsets", C.c_void_p), ("tokens", C.c_void_p), ("n_tokens", C.c_int64)]


class MrcRefSpec(C.Structure):
    _fields_ = [("k", C.c_int32), ("mode", C.c_int32), ("lo", C.c_int64), ("hi", C.c_int64),
                ("m", C.c_int64), ("drop_top_ppm", C.c_int64), ("idf_mode", C.c_int32),
                ("ref_weight", C.c_int32)]


class MrcCompareOpts(C.Structure):
    _fields_ = [("tau", C.c_float), ("precision", C.c_int32), ("band", C.c_float), ("reserved", C.c_int32)]


class MrcCompareStats(C.Structure):
    _fields_ = [("n_pairs_compared", C.c_int64), ("n_flagged", C.c_int64), ("n_band", C.c_int64),
                ("n_band_nominal", C.c_int64), ("n_flip_outside_nominal", C.c_int64),
                ("max_abs_err", C.c_float), ("mean_abs_err", C.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MrcHit(C.Structure):
    _fields_ = [("id", C.c_int64), ("s", C.c_float), ("flags", C.c_int32)]


class MrcServeOpts(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("n_streams", C.c_int32), ("topk", C.c_int32), ("tau", C.c_float),
                ("precision", C.c_int32), ("max_queue", C.c_int32), ("hbm_frac", C.c_double),
                ("max_batch_tokens", C.c_int64), ("max_wait_us", C.c_int32)]


class MrcResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("kind", C.c_int32), ("id", C.c_int64), ("n_hits", C.c_int32),
                ("n_top", C.c_int32), ("top", MrcHit * 64), ("t_submit_ms", C.c_double),
                ("t_start_ms", C.c_double), ("t_done_ms", C.c_double)]


PAIR_DTYPE = np.dtype([("i", np.int32), ("j", np.int32), ("s", np.float32), ("flags", np.int32)])
HIT_DTYPE = np.dtype([("id", np.int64), ("s", np.float32), ("flags", np.int32)])

_lib = None
_lock = threading.Lock()

_P = C.c_void_p
_SIGS = {
    "mrc_ctx_create": [C.POINTER(_P), C.c_int32, C.c_size_t],
    "mrc_ctx_destroy": [_P],
    "mrc_ctx_memory": [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
    "mrc_ctx_set_timing": [_P, C.c_int32],
    "mrc_ctx_set_scan": [_P, C.c_int32],
    "mrc_ctx_kernel_time": [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32],
    "mrc_build_vocab_idf": [_P, C.POINTER(MrcDocs), C.c_int32, C.POINTER(MrcRefSpec), C.POINTER(_P), _P],
    "mrc_build_and_sign": [_P, C.POINTER(MrcDocs), C.c_int32, C.POINTER(MrcRefSpec), C.POINTER(_P), _P, _P, _P],
    "mrc_model_destroy": [_P],
    "mrc_model_info": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                       C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "mrc_model_get": [_P, _P, _P, _P, _P, _P, _P],
    "mrc_model_save": [_P, C.c_char_p],
    "mrc_model_load": [_P, C.c_char_p, C.POINTER(_P)],
    "mrc_sign": [_P, _P, C.POINTER(MrcDocs), _P, _P, _P],
    "mrc_sign_matrix": [_P, _P, C.POINTER(MrcDocs), _P, C.c_int32, _P, _P, _P],
    "mrc_compare": [_P, _P, C.c_int64, C.c_int32, C.POINTER(MrcCompareOpts), _P, C.c_int64,
                    C.POINTER(C.c_int64), C.POINTER(MrcCompareStats), _P],
    "mrc_compare_f32_noalloc": [_P, _P, C.c_int64, C.c_int32, C.c_float, _P, C.c_int64, C.POINTER(C.c_int64), _P],
    "mrc_normalise": [_P, _P, C.c_int64, C.c_int32, _P, _P, _P, _P, _P, _P],
    "mrc_score_pairs": [_P, _P, C.c_int64, C.c_int32, _P, _P, C.c_int64, _P, _P],
    "mrc_trigrams": [_P, _P, _P, C.c_int64, C.c_int64, _P, _P, C.c_int64, C.POINTER(C.c_int64), _P],
    "mrc_simhash": [_P, _P, C.POINTER(MrcDocs), _P, _P],
    "mrc_term_hashes": [_P, _P, _P, _P],
    "mrc_hamming_pairs": [_P, _P, C.c_int64, C.c_int32, _P, C.c_int64, C.POINTER(C.c_int64), _P],
    "mrc_exact_cosine": [_P, _P, C.POINTER(MrcDocs), C.c_float, _P, C.c_int64, C.POINTER(C.c_int64), _P],
    "mrc_db_create": [_P, C.c_int64, C.c_int32, C.c_uint32, C.POINTER(_P)],
    "mrc_db_destroy": [_P],
    "mrc_db_insert": [_P, _P, C.c_int64, C.POINTER(C.c_int64), _P],
    "mrc_db_insert_docs": [_P, _P, C.POINTER(MrcDocs), C.POINTER(C.c_int64), _P],
    "mrc_db_size": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)],
    "mrc_db_save": [_P, C.c_char_p],
    "mrc_db_load": [_P, C.c_char_p, C.c_uint32, C.POINTER(_P)],
    "mrc_query": [_P, _P, _P, C.POINTER(MrcDocs), C.c_int32, C.c_float, C.c_int32, _P, _P, _P],
    "mrc_serve_start": [_P, _P, _P, C.POINTER(MrcServeOpts), C.POINTER(_P)],
    "mrc_serve_submit": [_P, _P, C.c_int64, C.c_int32, C.POINTER(C.c_uint64)],
    "mrc_serve_submit_many": [_P, _P, _P, C.c_int64, C.c_int32, _P, C.POINTER(C.c_int64)],
    "mrc_serve_poll": [_P, C.c_uint64, C.POINTER(MrcResult), C.c_int32],
    "mrc_serve_stop": [_P],
}


def lib():
    """Load libmrc.so (once). Raises MrcUnavailable when it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise MrcUnavailable(f"{LIB_PATH} is not built; run python -m paper_1810_03099_amd.build")
            L = C.CDLL(LIB_PATH)
            for name, args in _SIGS.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = C.c_int32
            L.mrc_last_error.argtypes = []
            L.mrc_last_error.restype = C.c_char_p
            _lib = L
    return _lib


def _check(status, fn):
    if status != MRC_OK:
        msg = lib().mrc_last_error().decode(errors="replace")
        raise MrcError(status, f"{fn}: {msg}")


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _docs(offsets, tokens):
    n = int(offsets.numel()) - 1
    d = MrcDocs(n, _dptr(offsets, torch.int64, "offsets"), _dptr(tokens, torch.int32, "tokens"),
                int(tokens.numel()))
    return d, (offsets, tokens)


class _Handle:
    _destroy = None

    def __init__(self, ptr, owner=None):
        self.ptr = ptr
        self.owner = owner

    def close(self):
        if self.ptr is not None and self.ptr.value:
            getattr(lib(), self._destroy)(self.ptr)
        self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return self.ptr


class Ctx(_Handle):
    _destroy = "mrc_ctx_destroy"


class Model(_Handle):
    _destroy = "mrc_model_destroy"

    def info(self):
        return mrc_model_info(self)


class Db(_Handle):
    _destroy = "mrc_db_destroy"


class Server(_Handle):
    _destroy = "mrc_serve_stop"


def ref_spec(k, mode=SEL_DROP_TOP, lo=0, hi=-1, m=0, drop_top_ppm=50_000, idf_mode=IDF_SMOOTH,
             ref_weight=REF_ONE):
    return MrcRefSpec(int(k), int(mode), int(lo), int(hi), int(m), int(drop_top_ppm), int(idf_mode),
                      int(ref_weight))


# ------------------------------------------------------------------ context

def mrc_ctx_create(device=0, hbm_budget_bytes=0):
    p = C.c_void_p()
    _check(lib().mrc_ctx_create(C.byref(p), int(device), int(hbm_budget_bytes)), "mrc_ctx_create")
    return Ctx(p)


def mrc_ctx_memory(ctx):
    u, b = C.c_size_t(), C.c_size_t()
    _check(lib().mrc_ctx_memory(ctx, C.byref(u), C.byref(b)), "mrc_ctx_memory")
    return u.value, b.value


def mrc_ctx_set_timing(ctx, enabled=True):
    _check(lib().mrc_ctx_set_timing(ctx, 1 if enabled else 0), "mrc_ctx_set_timing")


def mrc_ctx_set_scan(ctx, form):
    """Query collection form: SCAN_GRID (default) or SCAN_PERSISTENT."""
    _check(lib().mrc_ctx_set_scan(ctx, int(form)), "mrc_ctx_set_scan")


def mrc_ctx_kernel_time(ctx, kernel, reset=False):
    ms, n = C.c_double(), C.c_int64()
    _check(lib().mrc_ctx_kernel_time(ctx, kernel.encode(), C.byref(ms), C.byref(n), 1 if reset else 0),
           "mrc_ctx_kernel_time")
    return ms.value, n.value


# ------------------------------------------------------------------ model

def mrc_build_vocab_idf(ctx, offsets, tokens, vocab_size, spec, stream=None):
    d, _keep = _docs(offsets, tokens)
    p = C.c_void_p()
    _check(lib().mrc_build_vocab_idf(ctx, C.byref(d), int(vocab_size), C.byref(spec), C.byref(p),
                                     _stream(stream)), "mrc_build_vocab_idf")
    return Model(p, ctx)


def mrc_build_and_sign(ctx, offsets, tokens, vocab_size, spec, sig_out=None, norm_out=None, stream=None,
                       with_norm=False):
    """Model of the corpus and the corpus' signatures in one call. Returns (model, sig[, norm])."""
    d, _keep = _docs(offsets, tokens)
    if sig_out is None:
        sig_out = torch.empty((d.n_docs, spec.k), dtype=torch.float32, device=offsets.device)
    if norm_out is None and with_norm:
        norm_out = torch.empty((d.n_docs,), dtype=torch.float32, device=offsets.device)
    p = C.c_void_p()
    _check(lib().mrc_build_and_sign(ctx, C.byref(d), int(vocab_size), C.byref(spec), C.byref(p),
                                    _dptr(sig_out, torch.float32, "sig_out"), _dptr(norm_out, torch.float32, "norm_out"),
                                    _stream(stream)), "mrc_build_and_sign")
    m = Model(p, ctx)
    return (m, sig_out, norm_out) if with_norm else (m, sig_out)


def mrc_model_info(model):
    n, V, k, nl, lo, hi = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().mrc_model_info(model, C.byref(n), C.byref(V), C.byref(k), C.byref(nl), C.byref(lo),
                                C.byref(hi)), "mrc_model_info")
    return {"n_docs": n.value, "vocab": V.value, "k": k.value, "n_listed": nl.value, "lo": lo.value,
            "hi": hi.value}


def mrc_model_get(model):
    info = mrc_model_info(model)
    V, k = info["vocab"], info["k"]
    df = np.zeros(V, np.uint32)
    idf = np.zeros(V, np.float32)
    term_at = np.zeros(V, np.int32)
    rank_of = np.zeros(V, np.int32)
    part_of = np.zeros(V, np.int32)
    rnorm = np.zeros(k, np.float64)
    _check(lib().mrc_model_get(model, df.ctypes.data, idf.ctypes.data, term_at.ctypes.data, rank_of.ctypes.data,
                               part_of.ctypes.data, rnorm.ctypes.data), "mrc_model_get")
    return {"df": df, "idf": idf, "term_at": term_at, "rank_of": rank_of, "part_of": part_of, "rnorm": rnorm,
            **info}


def mrc_model_save(model, path):
    _check(lib().mrc_model_save(model, str(path).encode()), "mrc_model_save")


def mrc_model_load(ctx, path):
    p = C.c_void_p()
    _check(lib().mrc_model_load(ctx, str(path).encode(), C.byref(p)), "mrc_model_load")
    return Model(p, ctx)


# ------------------------------------------------------------------ signing

def mrc_sign(ctx, model, offsets, tokens, sig_out=None, norm_out=None, stream=None, with_norm=False):
    d, _keep = _docs(offsets, tokens)
    k = mrc_model_info(model)["k"]
    if sig_out is None:
        sig_out = torch.empty((d.n_docs, k), dtype=torch.float32, device=offsets.device)
    if norm_out is None and with_norm:
        norm_out = torch.empty((d.n_docs,), dtype=torch.float32, device=offsets.device)
    _check(lib().mrc_sign(ctx, model, C.byref(d), _dptr(sig_out, torch.float32, "sig_out"),
                          _dptr(norm_out, torch.float32, "norm_out"), _stream(stream)), "mrc_sign")
    return (sig_out, norm_out) if with_norm else sig_out


def mrc_sign_matrix(ctx, model, offsets, tokens, R, sig_out=None, norm_out=None, stream=None, with_norm=False):
    """Signatures against the columns of a dense [V][k] float32 device matrix R."""
    d, _keep = _docs(offsets, tokens)
    if R.dim() != 2 or int(R.shape[0]) != mrc_model_info(model)["vocab"]:
        raise ValueError("R must be a [V][k] matrix, V = the model's vocabulary")
    k = int(R.shape[1])
    if sig_out is None:
        sig_out = torch.empty((d.n_docs, k), dtype=torch.float32, device=offsets.device)
    if norm_out is None and with_norm:
        norm_out = torch.empty((d.n_docs,), dtype=torch.float32, device=offsets.device)
    _check(lib().mrc_sign_matrix(ctx, model, C.byref(d), _dptr(R, torch.float32, "R"), k,
                                 _dptr(sig_out, torch.float32, "sig_out"), _dptr(norm_out, torch.float32, "norm_out"),
                                 _stream(stream)), "mrc_sign_matrix")
    return (sig_out, norm_out) if with_norm else sig_out


# ------------------------------------------------------------------ comparison

def _pairs_call(fn_name, call, capacity, device):
    """Run a pair-emitting call with the two-call protocol."""
    cap = int(capacity)
    while True:
        buf = torch.empty((max(cap, 1), 4), dtype=torch.int32, device=device)
        n = C.c_int64()
        st = call(C.c_void_p(buf.data_ptr()) if cap > 0 else None, cap, C.byref(n))
        if st == MRC_E_OVERFLOW:
            cap = int(n.value)
            continue
        _check(st, fn_name)
        return buf[: n.value]


def mrc_compare(ctx, sig, tau=0.9, precision=PREC_FP32, band=0.02, capacity=None, stream=None):
    """Returns (pairs [n_found, 4] int32 device tensor: i, j, float bits of s, flags; stats dict)."""
    n, k = sig.shape
    opts = MrcCompareOpts(float(tau), int(precision), float(band), 0)
    stats = MrcCompareStats()
    sp = _dptr(sig, torch.float32, "sig")
    s = _stream(stream)

    def call(buf, cap, nfound):
        return lib().mrc_compare(ctx, sp, int(n), int(k), C.byref(opts), buf, cap, nfound, C.byref(stats), s)

    pairs = _pairs_call("mrc_compare", call, capacity if capacity is not None else 4 * n + 1024, sig.device)
    return pairs, stats.as_dict()


NOALLOC_MAX_UNIT_BYTES = 32 << 20


def mrc_compare_f32_noalloc(ctx, sig, tau, pairs_out, stream=None):
    """FP32 all-pairs comparison into the caller's pair buffer (int32 device
    tensor [capacity, 4]); the library allocates nothing. Returns
    (n_found, overflowed): on overflow the first `capacity` pairs are written
    and n_found is the exact count."""
    n, k = sig.shape
    cap = int(pairs_out.shape[0])
    nf = C.c_int64()
    st = lib().mrc_compare_f32_noalloc(ctx, _dptr(sig, torch.float32, "sig"), int(n), int(k), float(tau),
                                       _dptr(pairs_out, torch.int32, "pairs_out") if cap > 0 else None, cap,
                                       C.byref(nf), _stream(stream))
    if st == MRC_E_OVERFLOW:
        return int(nf.value), True
    _check(st, "mrc_compare_f32_noalloc")
    return int(nf.value), False


def pairs_to_numpy(pairs):
    """(i, j, s, flags) numpy arrays from a pair tensor."""
    a = pairs.cpu().numpy()
    return a[:, 0].astype(np.int64), a[:, 1].astype(np.int64), a[:, 2].view(np.float32).copy(), a[:, 3].copy()


def mrc_normalise(ctx, sig, unit=True, bf16=False, fp8=False, err=False, stream=None):
    n, k = sig.shape
    dev = sig.device
    u = torch.empty((n, k), dtype=torch.float32, device=dev) if unit else None
    b = torch.empty((n, k), dtype=torch.int16, device=dev) if bf16 else None
    q = torch.empty((n, k), dtype=torch.uint8, device=dev) if fp8 else None
    sc = torch.empty((n,), dtype=torch.float32, device=dev) if fp8 else None
    e = torch.empty((2, n), dtype=torch.float32, device=dev) if err else None
    _check(lib().mrc_normalise(ctx, _dptr(sig, torch.float32), int(n), int(k), _dptr(u), _dptr(b), _dptr(q),
                               _dptr(sc), _dptr(e), _stream(stream)), "mrc_normalise")
    return {"unit": u, "bf16": b, "fp8": q, "scale": sc, "err": e}


def mrc_score_pairs(ctx, unit, ii, jj, stream=None):
    n, k = unit.shape
    out = torch.empty(ii.shape, dtype=torch.float32, device=unit.device)
    _check(lib().mrc_score_pairs(ctx, _dptr(unit, torch.float32), int(n), int(k), _dptr(ii, torch.int32),
                                 _dptr(jj, torch.int32), int(ii.numel()), _dptr(out), _stream(stream)),
           "mrc_score_pairs")
    return out


# ------------------------------------------------------------------ text front end

TRIGRAM_VOCAB = 27 ** 3


def mrc_trigrams(ctx, text, text_offsets, capacity=None, stream=None):
    """Character 3-gram ids of raw text. text: device uint8 [n_bytes];
    text_offsets: device int64 [n_docs + 1]. Returns (offsets int64 [n_docs + 1],
    ids int32 [total]) on the device, with the two-call protocol handled here."""
    n = int(text_offsets.numel()) - 1
    if n < 0:
        raise MrcError(MRC_E_INVAL, "mrc_trigrams: text_offsets is empty")
    nb = int(text.numel())
    dev = text_offsets.device
    tok_off = torch.empty((n + 1,), dtype=torch.int64, device=dev)
    tp = _dptr(text, torch.uint8, "text") if nb > 0 else None
    op = _dptr(text_offsets, torch.int64, "text_offsets")
    s = _stream(stream)
    cap = int(capacity) if capacity is not None else max(nb, 1)
    while True:
        ids = torch.empty((max(cap, 1),), dtype=torch.int32, device=dev)
        total = C.c_int64()
        st = lib().mrc_trigrams(ctx, tp, op, n, nb, _dptr(tok_off), _dptr(ids) if cap > 0 else None, cap,
                                C.byref(total), s)
        if st == MRC_E_OVERFLOW:
            cap = int(total.value)
            continue
        _check(st, "mrc_trigrams")
        return tok_off, ids[: total.value]


# ------------------------------------------------------------------ comparators

def mrc_term_hashes(ctx, model, stream=None):
    V = mrc_model_info(model)["vocab"]
    out = torch.empty((V,), dtype=torch.int64, device=torch.device("cuda", torch.cuda.current_device()))
    _check(lib().mrc_term_hashes(ctx, model, _dptr(out), _stream(stream)), "mrc_term_hashes")
    return out


def mrc_simhash(ctx, model, offsets, tokens, out=None, stream=None):
    d, _keep = _docs(offsets, tokens)
    if out is None:
        out = torch.empty((d.n_docs,), dtype=torch.int64, device=offsets.device)
    _check(lib().mrc_simhash(ctx, model, C.byref(d), _dptr(out, torch.int64), _stream(stream)), "mrc_simhash")
    return out


def mrc_hamming_pairs(ctx, sim, max_dist=3, capacity=None, stream=None):
    n = int(sim.numel())
    sp = _dptr(sim, torch.int64, "sim")
    s = _stream(stream)

    def call(buf, cap, nfound):
        return lib().mrc_hamming_pairs(ctx, sp, n, int(max_dist), buf, cap, nfound, s)

    return _pairs_call("mrc_hamming_pairs", call, capacity if capacity is not None else 4 * n + 1024, sim.device)


def mrc_exact_cosine(ctx, model, offsets, tokens, tau=0.9, capacity=None, stream=None):
    d, _keep = _docs(offsets, tokens)
    s = _stream(stream)

    def call(buf, cap, nfound):
        return lib().mrc_exact_cosine(ctx, model, C.byref(d), float(tau), buf, cap, nfound, s)

    return _pairs_call("mrc_exact_cosine", call, capacity if capacity is not None else 4 * d.n_docs + 1024,
                       offsets.device)


# ------------------------------------------------------------------ database + query

def mrc_db_create(ctx, capacity, k, precisions=(PREC_BF16, PREC_FP8)):
    mask = 0
    for p in precisions:
        mask |= 1 << int(p)
    p = C.c_void_p()
    _check(lib().mrc_db_create(ctx, int(capacity), int(k), mask, C.byref(p)), "mrc_db_create")
    return Db(p, ctx)


def mrc_db_insert(db, sig, stream=None):
    first = C.c_int64()
    _check(lib().mrc_db_insert(db, _dptr(sig, torch.float32, "sig"), int(sig.shape[0]), C.byref(first),
                               _stream(stream)), "mrc_db_insert")
    return first.value


def mrc_db_insert_docs(db, model, offsets, tokens, stream=None):
    d, _keep = _docs(offsets, tokens)
    first = C.c_int64()
    _check(lib().mrc_db_insert_docs(db, model, C.byref(d), C.byref(first), _stream(stream)),
           "mrc_db_insert_docs")
    return first.value


def mrc_db_size(db):
    n, k = C.c_int64(), C.c_int32()
    _check(lib().mrc_db_size(db, C.byref(n), C.byref(k)), "mrc_db_size")
    return n.value, k.value


def mrc_db_save(db, path):
    _check(lib().mrc_db_save(db, str(path).encode()), "mrc_db_save")


def mrc_db_load(ctx, path, precisions=(PREC_BF16, PREC_FP8)):
    mask = 0
    for p in precisions:
        mask |= 1 << int(p)
    p = C.c_void_p()
    _check(lib().mrc_db_load(ctx, str(path).encode(), mask, C.byref(p)), "mrc_db_load")
    return Db(p, ctx)


def mrc_query(ctx, db, model, offsets, tokens, topk=16, tau=0.9, precision=PREC_FP32, stream=None):
    """Returns (top [nq, topk, 2] as (ids int64 tensor, scores float tensor), n_hits int32 tensor)."""
    d, _keep = _docs(offsets, tokens)
    nq = d.n_docs
    top = torch.empty((nq, topk, 2), dtype=torch.int64, device=offsets.device)
    hits = torch.empty((nq,), dtype=torch.int32, device=offsets.device)
    _check(lib().mrc_query(ctx, db, model, C.byref(d), int(topk), float(tau), int(precision), _dptr(top),
                           _dptr(hits), _stream(stream)), "mrc_query")
    ids = top[:, :, 0]
    raw = top.view(torch.int32).reshape(nq, topk, 4)        # id (2 words), s, flags
    scores = raw[:, :, 2].contiguous().view(torch.float32)
    return ids, scores, hits


# ------------------------------------------------------------------ serving

def mrc_serve_start(ctx, db, model, max_batch=256, n_streams=2, topk=16, tau=0.9, precision=PREC_FP32,
                    max_queue=100_000, hbm_frac=0.8, max_batch_tokens=1 << 22, max_wait_us=200):
    o = MrcServeOpts(int(max_batch), int(n_streams), int(topk), float(tau), int(precision), int(max_queue),
                     float(hbm_frac), int(max_batch_tokens), int(max_wait_us))
    p = C.c_void_p()
    _check(lib().mrc_serve_start(ctx, db, model, C.byref(o), C.byref(p)), "mrc_serve_start")
    return Server(p, (ctx, db, model))


def mrc_serve_submit(srv, tokens: np.ndarray, kind=REQ_QUERY):
    t = np.ascontiguousarray(tokens, dtype=np.int32)
    ticket = C.c_uint64()
    st = lib().mrc_serve_submit(srv, t.ctypes.data if t.size else None, int(t.size), int(kind), C.byref(ticket))
    if st == MRC_E_BUSY:
        return None
    _check(st, "mrc_serve_submit")
    return ticket.value


def mrc_serve_submit_many(srv, offsets: np.ndarray, tokens: np.ndarray, kind=REQ_QUERY):
    """Submit len(offsets) - 1 documents (host CSR arrays) in one call; returns
    the tickets of those queued (fewer than asked when the queue filled)."""
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    t = np.ascontiguousarray(tokens, dtype=np.int32)
    n = max(int(o.size) - 1, 0)
    tickets = np.zeros(max(n, 1), dtype=np.uint64)
    acc = C.c_int64(0)
    st = lib().mrc_serve_submit_many(srv, o.ctypes.data if o.size else None, t.ctypes.data if t.size else None, n,
                                     int(kind), tickets.ctypes.data, C.byref(acc))
    if st != MRC_E_BUSY:
        _check(st, "mrc_serve_submit_many")
    return tickets[:acc.value].tolist()


def mrc_serve_poll(srv, ticket, wait_ms=0):
    r = MrcResult()
    st = lib().mrc_serve_poll(srv, C.c_uint64(ticket), C.byref(r), int(wait_ms))
    if st == MRC_E_BUSY:
        return None
    _check(st, "mrc_serve_poll")
    return r


def mrc_serve_stop(srv):
    srv.close()
