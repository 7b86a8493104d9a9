"""Benchmark of the MRC near-duplicate path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|bf16|fp8]
                [--no-cpu-baseline] [--no-extras]

Workload: the full-scale plain-method corpus (20,000 synthetic documents over a
131,072-term vocabulary, lognormal lengths with median 300, 5% exact and 10%
near duplicates, k = 64 reference parts, tau = 0.9), resident in HBM before the
timed region. One step runs the whole hot path on it: model build (term counts,
df, idf, frequency-sorted list, parts), signing of every document, and the
all-pairs comparison at the chosen precision (with FP32 rescoring for BF16 /
FP8). `value` = signature pairs compared per second over whole steps
(N(N-1)/2 pairs per step).

Extras (same corpus, outside the timed steps): every precision form, the
comparators (exact TF-IDF cosine, Simhash-64 + Hamming), recall / precision
against exact cosine, each form's error against a float64 comparison of the
same signatures, query latency against a database of the corpus, and the sign
pass against HBM bandwidth. Then two legs on the larger workloads
(--no-scale-legs skips them): the precision form (200,000 documents, k = 256:
the comparison kernels at FP32 / BF16 / FP8 against their matrix-core peaks)
and the serving form (a 1,000,000-row k = 128 database: build rate, mrc_query
batches, the serving loop's p50 / p99 under Poisson arrivals at half of its
saturation). Only the CPU-baseline leg runs the FP64 oracle (its timed sample,
and the check of the step's decisions and scores against it).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "fp32_vector_TFLOPs": 157.3,
    "fp32_matrix_TFLOPs": 157.3,
    "bf16_mfma_TFLOPs": 2500.0,
    "fp8_mfma_TFLOPs": 5000.0,
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--workload", default="plain_full", choices=["plain_full", "precision", "serving", "sweep", "text"],
                    help="plain_full: 20k docs, k=64 (default); precision: 200k docs, k=256; "
                         "serving: 1M-signature database, k=128, query stream; sweep: reference "
                         "selection x k on the 20k-document corpus (accuracy and time curves); text: "
                         "raw text to character 3-gram ids (200k documents), then the plain step on them")
    ap.add_argument("--query-only", action="store_true",
                    help="serving workload: build the database and time the mrc_query batches only")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="serving workload: length of each offered-load run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-scale-legs", action="store_true",
                    help="skip the precision-form (200k docs) and serving-form (1M-row database) legs of the extras")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (calibrates HBM byte counters) and exit")
    return ap.parse_args()


def copy_probe(mib):
    import torch
    x = torch.ones(mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 4, "copies": 5, "ms_each": dt * 1e3,
                      "GBps_read_plus_write": 2 * x.numel() * 4 / dt / 1e9}))


def source_digest(rel):
    """Digest of the kernel's source files ("a.hip+b.h": all of them, in order)."""
    h = hashlib.sha256()
    for part in rel.split("+"):
        with open(os.path.join(ROOT, part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter runs, if the kernel's
    source is unchanged since they were taken (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)[kernel]
        if source_digest(t["source"]) != t["source_sha"]:
            return None
        return t["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def timed(mrc, ctx, kernel, fn, reps):
    """Average device time of `kernel` (HIP events on its launch stream) over reps calls."""
    mrc.mrc_ctx_set_timing(ctx, True)
    mrc.mrc_ctx_kernel_time(ctx, kernel, reset=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    wall = (time.perf_counter() - t0) / reps
    ms, n = mrc.mrc_ctx_kernel_time(ctx, kernel, reset=True)
    mrc.mrc_ctx_set_timing(ctx, False)
    return (ms / n if n else None), wall * 1e3, out


def cpu_affinity():
    """The host CPUs this process may run on, as ranges ("0-15")."""
    try:
        cpus = sorted(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return None
    out, lo = [], None
    for x, nxt in zip(cpus, cpus[1:] + [None]):
        lo = x if lo is None else lo
        if nxt != x + 1:
            out.append(f"{lo}-{x}" if x != lo else str(x))
            lo = None
    return ",".join(out)


def cpu_baseline(c, k, tau, sample_note="full workload"):
    """The FP64 oracle on the same workload (one whole step: build, sign, compare)."""
    from oracle import mrc as om
    try:
        from threadpoolctl import threadpool_info
        threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    m = om.build_model(c.offsets, c.tokens, c.vocab, om.RefSpec(k=k))
    sig, _ = om.sign(c.offsets, c.tokens, m)
    shat = om.normalise(sig)
    i, j, s = om.compare_pairs(shat, tau)
    dt = time.perf_counter() - t0
    n = c.n_docs
    pairs = n * (n - 1) / 2
    return {"value": pairs / dt, "unit": "pairs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{sample_note}: {n} docs, one step (build + sign + all-pairs compare), float64 NumPy, "
                      f"{dt:.2f} s", "seconds": dt, "host_cpus": os.cpu_count(), "affinity": cpu_affinity()}, shat, (i, j)


def main():
    a = parse()
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; multi-GPU sharding is designed but not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_1810_03099_amd import mrc
    from synth import corpus as synth

    prec = {"fp32": mrc.PREC_FP32, "bf16": mrc.PREC_BF16, "fp8": mrc.PREC_FP8}[a.precision]
    if a.workload == "serving":
        print(json.dumps(serving(a, mrc, synth, prec)))
        return
    if a.workload == "sweep":
        print(json.dumps(sweep(mrc, synth)))
        return
    if a.workload == "text":
        print(json.dumps(text_front_end(a, mrc)))
        return
    spec_idx = 1 if a.workload == "plain_full" else 2
    cs = synth.CONFIGS[spec_idx]
    k, tau = cs.k, cs.tau
    c = synth.generate(spec_idx)
    n = c.n_docs
    log(f"corpus {cs.name}: {n} docs, {c.tokens.size} tokens")
    torch.cuda.set_device(0)
    off = torch.from_numpy(c.offsets).cuda()
    tok = torch.from_numpy(c.tokens).cuda()
    ctx = mrc.mrc_ctx_create(0)
    sig = torch.empty((n, k), dtype=torch.float32, device="cuda")
    cap = 8 * 1024 * 1024 if a.workload == "plain_full" else 16 * 1024 * 1024
    state = {}

    def step():
        model, _ = mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(k), sig_out=sig)
        pairs, stats = mrc.mrc_compare(ctx, sig, tau, prec, 0.02, capacity=cap)
        state["model"], state["pairs"], state["stats"] = model, pairs, stats

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    # timed steps (kernel timing off, so no events between launches)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {a.steps} steps: {dt * 1e3 / a.steps:.3f} ms/step")
    # per-kernel times (HIP events on the launch stream) over further steps
    kernels = ["df_count", "df_hist", "rank_sort", "sign_counts", "normalise", "compare_f32", "compare_lowp",
               "rescore"]
    mrc.mrc_ctx_set_timing(ctx, True)
    for kname in kernels:
        mrc.mrc_ctx_kernel_time(ctx, kname, reset=True)
    for _ in range(max(5, a.steps // 2)):
        step()
    torch.cuda.synchronize()
    ktimes = {}
    for kname in kernels:
        ms, cnt = mrc.mrc_ctx_kernel_time(ctx, kname)
        if cnt:
            ktimes[kname] = {"avg_ms": ms / cnt, "launches": cnt}
    mrc.mrc_ctx_set_timing(ctx, False)

    ms_step = dt * 1e3 / a.steps
    pairs_per_step = n * (n - 1) / 2
    value = pairs_per_step / (dt / a.steps)
    flops = pairs_per_step * 2 * k
    if prec == mrc.PREC_FP32:
        kname, pk, bound = "compare_f32", PEAKS["fp32_matrix_TFLOPs"], "mfma"
        src = "paper_1810_03099_amd/csrc/compare.hip"
    else:
        kname = "compare_lowp"
        pk = PEAKS["bf16_mfma_TFLOPs"] if prec == mrc.PREC_BF16 else PEAKS["fp8_mfma_TFLOPs"]
        bound, src = "mfma", "paper_1810_03099_amd/csrc/compare.hip"
    avg_s = ktimes[kname]["avg_ms"] / 1e3
    achieved = flops / avg_s / 1e12
    roof = {"kernel": kname, "bound": bound, "achieved": achieved, "peak": pk, "unit": "TFLOP/s",
            "frac": achieved / pk, "traffic": measured_traffic(f"{kname}/{a.precision}/{a.workload}"),
            "algorithmic_flops_per_launch": flops,
            "note": "all-pairs signature contraction N(N-1)/2 x 2k flop per launch over the launch's HIP-event time"}

    # signing a batch of new documents (the hash pass of mrc_sign) on the same corpus
    mrc.mrc_sign(ctx, state["model"], off, tok, sig_out=sig)
    sign_ms, _, _ = timed(mrc, ctx, "sign", lambda: mrc.mrc_sign(ctx, state["model"], off, tok, sig_out=sig), 10)
    out = {
        "metric": "near-dup pairs compared/s & docs signed/s at stated recall; p50/p99 query ms",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[a.precision],
        "data": "synthetic (seeded Zipf/topic/lognormal generator with planted duplicates; stands in for NEWS20)",
        "config": {"workload": f"{cs.name}: {n} docs, vocab {cs.vocab}, k={k}, tau={tau}, reference = frequency-"
                               f"sorted list without its top 5%", "n_docs": n, "vocab": cs.vocab, "k": k,
                   "tau": tau, "tokens": int(c.tokens.size), "precision": a.precision},
        "docs_signed_per_s": n / (sign_ms / 1e3) if sign_ms else None,
        "flagged_pairs": int(state["stats"]["n_flagged"]),
        "kernel_avg_ms": ktimes,
        "roofline": roof,
    }
    shat = None
    if a.workload == "precision":
        if not a.no_cpu_baseline:
            # bounded sample (about 10 s of host work): the oracle's whole step on
            # the first 50,000 documents, reported per pair
            log("cpu baseline (oracle, 50,000-document subsample)")
            cb, _, _ = cpu_baseline(c.subset(np.arange(50000)), k, tau, "50,000-document subsample of the workload")
            out["cpu_baseline"] = cb
        if not a.no_extras:
            out["extras"] = precision_extras(mrc, ctx, c, sig, k, tau, cap)
        print(json.dumps(out))
        return
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cb, shat, (oi, oj) = cpu_baseline(c, k, tau)
        out["cpu_baseline"] = cb
        gi, gj, gs, _ = mrc.pairs_to_numpy(state["pairs"])
        g = set(zip(gi.tolist(), gj.tolist()))
        o = set(zip(oi.tolist(), oj.tolist()))
        out["decisions_vs_fp64_oracle"] = {"gpu_only": len(g - o), "oracle_only": len(o - g), "common": len(g & o)}
        if gi.size:
            # the step's flagged scores against the oracle's float64 scores of the same pairs
            from oracle import mrc as om
            e = np.abs(gs.astype(np.float64) - om.pair_scores(shat, gi, gj))
            out["flagged_scores_vs_fp64_oracle"] = {"max": float(e.max()), "mean": float(e.mean()),
                                                    "pairs": int(e.size)}
    if not a.no_extras:
        out["extras"] = extras(mrc, ctx, c, off, tok, sig, state["model"], k, tau, cap, sign_ms,
                               ktimes.get("sign_counts", {}).get("avg_ms"))
        if not a.no_scale_legs:
            # the precision and serving forms' workloads, measured in the same run
            del off, tok, sig, state
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            out["extras"]["precision_form"] = precision_leg(mrc, synth)
            out["extras"]["serving_form"] = serving_leg(mrc, synth)
    print(json.dumps(out))


def text_front_end(a, mrc):
    """Raw text -> character 3-gram ids (mrc_trigrams) on 200,000 synthetic
    documents (50,000 generated, repeated four times; about 670 MB), against
    HBM bandwidth; then the plain step (model, signatures, FP32 all-pairs at
    k = 64) on the ids of the first 20,000 documents."""
    import torch
    from synth.text import generate_text
    log("text: generating")
    t50, o50 = generate_text(50_000, seed=1810)
    text = np.tile(t50, 4)
    off = np.concatenate([[0]] + [o50[1:] + i * t50.size for i in range(4)]).astype(np.int64)
    n = off.size - 1
    torch.cuda.set_device(0)
    ctx = mrc.mrc_ctx_create(0)
    dt = torch.from_numpy(text).cuda()
    do = torch.from_numpy(off).cuda()
    tok_off, ids = mrc.mrc_trigrams(ctx, dt, do)
    torch.cuda.synchronize()
    n_ids = int(ids.numel())
    cap = n_ids
    for _ in range(a.warmup):
        mrc.mrc_trigrams(ctx, dt, do, capacity=cap)
    torch.cuda.synchronize()
    kms, wall, _ = timed(mrc, ctx, "trigrams", lambda: mrc.mrc_trigrams(ctx, dt, do, capacity=cap), a.steps)
    torch.cuda.synchronize()
    # algorithmic bytes of the map kernel: text read once, ids written once,
    # both offset arrays read once
    by = text.size + 4 * n_ids + 16 * (n + 1)
    achieved = by / (kms / 1e3) / 1e9
    out = {"metric": "raw text bytes to character 3-gram ids per second", "value": text.size / (wall / 1e3),
           "unit": "bytes/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": wall,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
           "data": "synthetic text (Zipf-ranked random-letter words, punctuation, digits, bytes above 0x7F)",
           "config": {"workload": "text_200k", "docs": n, "bytes": int(text.size), "ids": n_ids},
           "roofline": {"kernel": "trigrams", "bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                        "frac": achieved / 8000.0, "traffic": None, "algorithmic_bytes_per_launch": int(by),
                        "note": "text + 4 B per id + 16 B per document over the map kernel's HIP-event time; "
                                "value = bytes per second of whole calls (offsets pass, host check, map)"},
           "kernel_avg_ms": kms}
    # the plain step on the ids of the first 20,000 documents
    m = 20_000
    sub_off = tok_off[: m + 1].contiguous()
    sub_ids = ids[: int(tok_off[m].item())].contiguous()

    def step():
        model, sig = mrc.mrc_build_and_sign(ctx, sub_off, sub_ids, mrc.TRIGRAM_VOCAB, mrc.ref_spec(64))
        pairs, st = mrc.mrc_compare(ctx, sig, 0.9, mrc.PREC_FP32, capacity=8 * 1024 * 1024)
        return st["n_flagged"]

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        flagged = step()
    torch.cuda.synchronize()
    out["plain_step_on_3grams"] = {"docs": m, "vocab": mrc.TRIGRAM_VOCAB, "k": 64,
                                   "ms": (time.perf_counter() - t0) / 5 * 1e3, "flagged": int(flagged)}
    if not a.no_cpu_baseline:
        from oracle import trigram as ot
        log("cpu baseline (oracle, 50,000 documents)")
        t0 = time.perf_counter()
        ot.trigram_csr(t50, o50)
        sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": t50.size / sec, "unit": "bytes/s", "cores": 1, "kind": "oracle",
                               "sample": f"the 50,000 generated documents ({t50.size} bytes), NumPy", "seconds": sec,
                               "affinity": cpu_affinity()}
    return out


SWEEP_KS = (8, 16, 32, 64, 128, 256, 512, 1024)


def count_flagged(mrc, ctx, sig, tau):
    """Number of FP32-flagged pairs, from the two-call protocol's count alone."""
    import ctypes
    import torch
    n, k = sig.shape
    opts = mrc.MrcCompareOpts(float(tau), mrc.PREC_FP32, 0.02, 0)
    found = ctypes.c_int64()
    st = mrc.lib().mrc_compare(ctx, ctypes.c_void_p(sig.data_ptr()), int(n), int(k), ctypes.byref(opts), None, 0,
                               ctypes.byref(found), None,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st not in (mrc.MRC_OK, mrc.MRC_E_OVERFLOW):
        raise RuntimeError("mrc_compare: " + mrc.lib().mrc_last_error().decode(errors="replace"))
    return int(found.value)


def sweep(mrc, synth):
    """Reference selection x k (the paper's experiments over reference regions and
    partition counts, Section 4, Figs. 1-18) on the 20,000-document corpus: for each
    selection and k, the time of model build + signing and of the FP32 all-pairs
    comparison, the flagged count, recall and precision against exact TF-IDF
    cosine at tau, and MAE / variance (Eqs. 2-3, as read: mean |MRC - cos| and
    the variance of MRC - cos) over all pairs of the first 2,000 documents.

    Flagged sets are never materialised: the comparison reports its count, and
    the true positives are the exact-cosine pairs whose MRC score (the same
    float32 chain the comparison decides with) reaches tau."""
    import torch
    cs = synth.CONFIGS[1]
    tau = cs.tau
    c = synth.generate(1)
    n = c.n_docs
    torch.cuda.set_device(0)
    off = torch.from_numpy(c.offsets).cuda()
    tok = torch.from_numpy(c.tokens).cuda()
    sub = c.subset(np.arange(2000))
    so = torch.from_numpy(sub.offsets).cuda()
    st_ = torch.from_numpy(sub.tokens).cuda()
    ctx = mrc.mrc_ctx_create(0)
    log("sweep: exact cosine")
    # idf does not depend on the selection: one model serves the exact comparator
    m0, _ = mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(8, mode=mrc.SEL_ALL))
    v_listed = mrc.mrc_model_info(m0)["n_listed"]
    ep = mrc.mrc_exact_cosine(ctx, m0, off, tok, tau, capacity=4 * 1024 * 1024)
    ei = ep[:, 0].contiguous()
    ej = ep[:, 1].contiguous()
    n_exact = int(ep.shape[0])
    sp = mrc.mrc_exact_cosine(ctx, m0, so, st_, -2.0, capacity=2000 * 1999 // 2 + 16)
    si = sp[:, 0].contiguous()
    sj = sp[:, 1].contiguous()
    scos = sp[:, 2].cpu().numpy().view(np.float32).astype(np.float64)
    del m0
    sels = [("all", dict(mode=mrc.SEL_ALL)),
            ("drop_top_5pct", dict(mode=mrc.SEL_DROP_TOP)),
            ("frequent_half", dict(mode=mrc.SEL_REGION, lo=0, hi=v_listed // 2)),
            ("rare_half", dict(mode=mrc.SEL_REGION, lo=v_listed // 2, hi=v_listed)),
            ("rarest_10pct", dict(mode=mrc.SEL_RAREST, m=v_listed // 10))]
    rows = []
    for name, kw in sels:
        for k in SWEEP_KS:
            spec = mrc.ref_spec(k, **kw)
            sig = torch.empty((n, k), dtype=torch.float32, device="cuda")
            mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, spec, sig_out=sig)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                model, _ = mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, spec, sig_out=sig)
            torch.cuda.synchronize()
            sign_ms = (time.perf_counter() - t0) / 3 * 1e3
            info = mrc.mrc_model_info(model)
            flagged = count_flagged(mrc, ctx, sig, tau)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                count_flagged(mrc, ctx, sig, tau)
            torch.cuda.synchronize()
            cmp_ms = (time.perf_counter() - t0) / 3 * 1e3
            unit = mrc.mrc_normalise(ctx, sig)["unit"]
            tp = int((mrc.mrc_score_pairs(ctx, unit, ei, ej) >= tau).sum().item()) if n_exact else 0
            usub = unit[:2000].contiguous()
            e = mrc.mrc_score_pairs(ctx, usub, si, sj).double().cpu().numpy() - scos
            zero = int((sig.abs().sum(dim=1) == 0).sum().item())
            rows.append({"selection": name, "k": k, "m": int(info["hi"] - info["lo"]), "sign_ms": sign_ms,
                         "compare_ms": cmp_ms, "flagged": flagged,
                         "recall": tp / n_exact if n_exact else 1.0,
                         "precision": tp / flagged if flagged else 1.0,
                         "mae": float(np.abs(e).mean()), "variance": float(((e - e.mean()) ** 2).mean()),
                         "zero_signatures": zero})
            r = rows[-1]
            log(f"sweep {name:14s} k={k:5d} m={r['m']:7d} sign {sign_ms:7.3f} ms  compare {cmp_ms:7.3f} ms  "
                f"flagged {flagged:10d}  recall {r['recall']:.4f}  precision {r['precision']:.4f}  "
                f"mae {r['mae']:.4f}  var {r['variance']:.5f}")
            del model, sig, unit, usub
    return {"workload": "sweep", "data": "synthetic",
            "config": {"workload": cs.name, "docs": n, "vocab": c.vocab, "listed_terms": int(v_listed), "tau": tau,
                       "ks": list(SWEEP_KS), "mae_sample": "all pairs of the first 2,000 documents"},
            "exact_cosine_flagged": n_exact, "rows": rows}


def fp64_unit(sig):
    """Rows of a signature tensor scaled to unit length in float64 (zero rows stay zero)."""
    s = sig.double().cpu().numpy()
    nr = np.linalg.norm(s, axis=1, keepdims=True)
    return np.divide(s, nr, out=np.zeros_like(s), where=nr > 0)


def fp64_pair_scores(sig, gi, gj):
    """Cosine of the signature rows gi and gj, computed in float64 (evaluation only)."""
    u = fp64_unit(sig)
    return np.einsum("ij,ij->i", u[gi], u[gj])


def precision_extras(mrc, ctx, c, sig, k, tau, cap):
    """All three forms on the whole corpus (times, decisions), and their scores
    against a float64 comparison of the same FP32 signatures on a 5,000-document
    subsample (the signatures' own error against the float64 method is what the
    parity tests bound)."""
    import torch
    n = c.n_docs
    pairs_total = n * (n - 1) / 2
    forms, sets = {}, {}
    for name, p, kn in [("fp32", mrc.PREC_FP32, "compare_f32"), ("bf16", mrc.PREC_BF16, "compare_lowp"),
                        ("fp8", mrc.PREC_FP8, "compare_lowp")]:
        mrc.mrc_compare(ctx, sig, tau, p, 0.02, capacity=cap)
        kms, wall, (pairs, st) = timed(mrc, ctx, kn, lambda: mrc.mrc_compare(ctx, sig, tau, p, 0.02, capacity=cap), 3)
        rms = None
        if p != mrc.PREC_FP32:
            rms, _, _ = timed(mrc, ctx, "rescore", lambda: mrc.mrc_compare(ctx, sig, tau, p, 0.02, capacity=cap), 2)
        gi, gj, _, _ = mrc.pairs_to_numpy(pairs)
        sets[name] = set(zip(gi.tolist(), gj.tolist()))
        pk = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}[name]
        forms[name] = {"kernel_ms": kms, "rescore_ms": rms, "call_ms": wall,
                       "pairs_per_s_call": pairs_total / (wall / 1e3), "pairs_per_s_kernel": pairs_total / (kms / 1e3),
                       "mfma_frac": pairs_total * 2 * k / (kms / 1e3) / 1e12 / pk, "flagged": int(gi.size),
                       "rescored": st["n_band"], "rescored_in_nominal_band": st["n_band_nominal"],
                       "flips_a_fixed_0.02_band_would_make": st["n_flip_outside_nominal"]}
        log(f"precision form {name}: kernel {kms:.3f} ms, call {wall:.3f} ms")
    forms["decisions_identical_to_fp32"] = all(sets[x] == sets["fp32"] for x in ("bf16", "fp8"))
    # each form's scores of all pairs of the first 5,000 documents against the
    # float64 comparison of the same signatures
    ssub = sig[:5000].contiguous()
    u = fp64_unit(ssub)
    iu = np.triu_indices(5000, 1)
    ref = (u @ u.T)[iu]
    err = {}
    for name, p in [("fp32", mrc.PREC_FP32), ("bf16", mrc.PREC_BF16), ("fp8", mrc.PREC_FP8)]:
        pairs, _ = mrc.mrc_compare(ctx, ssub, -2.0, p, 0.02, capacity=5000 * 4999 // 2 + 16)
        gi, gj, gs, _ = mrc.pairs_to_numpy(pairs)
        got = np.zeros((5000, 5000))
        got[gi, gj] = gs
        e = np.abs(got[iu] - ref)
        err[name] = {"max": float(e.max()), "mean": float(e.mean()), "pairs": int(e.size)}
    torch.cuda.synchronize()
    return {"forms": forms, "err_vs_fp64_comparison_5000_subsample": err,
            "note": "subsample scores are the form's own scores (no rescoring applies at tau = -2)"}


def extras(mrc, ctx, c, off, tok, sig, model, k, tau, cap, sign_ms, counts_ms):
    import torch
    from synth import corpus as synth
    n = c.n_docs
    pairs_total = n * (n - 1) / 2
    ex = {}
    # precision forms on the same signatures
    forms = {}
    pair_sets = {}
    for name, p, kn in [("fp32", mrc.PREC_FP32, "compare_f32"), ("bf16", mrc.PREC_BF16, "compare_lowp"),
                        ("fp8", mrc.PREC_FP8, "compare_lowp")]:
        mrc.mrc_compare(ctx, sig, tau, p, 0.02, capacity=cap)
        kms, wall, (pairs, st) = timed(mrc, ctx, kn, lambda: mrc.mrc_compare(ctx, sig, tau, p, 0.02, capacity=cap), 5)
        rms = None
        if p != mrc.PREC_FP32:
            rms, _, _ = timed(mrc, ctx, "rescore", lambda: mrc.mrc_compare(ctx, sig, tau, p, 0.02, capacity=cap), 2)
        gi, gj, gs, gf = mrc.pairs_to_numpy(pairs)
        pair_sets[name] = set(zip(gi.tolist(), gj.tolist()))
        f = {"kernel_ms": kms, "rescore_ms": rms, "call_ms": wall, "pairs_per_s_kernel": pairs_total / (kms / 1e3),
             "pairs_per_s_call": pairs_total / (wall / 1e3), "flagged": int(gi.size),
             "rescored": st["n_band"], "rescored_in_nominal_band": st["n_band_nominal"],
             "flips_a_fixed_0.02_band_would_make": st["n_flip_outside_nominal"],
             "max_abs_err_vs_fp32": st["max_abs_err"], "mean_abs_err_vs_fp32": st["mean_abs_err"]}
        pk = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}[name]
        f["mfma_frac"] = pairs_total * 2 * k / (kms / 1e3) / 1e12 / pk
        if gi.size:
            # against a float64 comparison of the same FP32 signatures
            err = np.abs(gs.astype(np.float64) - fp64_pair_scores(sig, gi, gj))
            f["err_vs_fp64_comparison"] = {"max": float(err.max()), "mean": float(err.mean())}
        forms[name] = f
        log(f"form {name}: {kms:.4f} ms")
    forms["decisions_identical_to_fp32"] = all(pair_sets[x] == pair_sets["fp32"] for x in ("bf16", "fp8"))
    ex["forms"] = forms
    # comparators
    log("comparators")
    mrc.mrc_exact_cosine(ctx, model, off, tok, tau, capacity=cap)
    ems, ewall, ep = timed(mrc, ctx, "exact_cosine", lambda: mrc.mrc_exact_cosine(ctx, model, off, tok, tau,
                                                                                  capacity=cap), 2)
    ei, ej, _, _ = mrc.pairs_to_numpy(ep)
    exact = set(zip(ei.tolist(), ej.tolist()))
    mrc.mrc_simhash(ctx, model, off, tok)
    sms, swall, sim = timed(mrc, ctx, "simhash", lambda: mrc.mrc_simhash(ctx, model, off, tok), 5)
    hms, hwall, hp = timed(mrc, ctx, "hamming", lambda: mrc.mrc_hamming_pairs(ctx, sim, 3, capacity=cap), 5)
    hi, hj, _, _ = mrc.pairs_to_numpy(hp)
    simset = set(zip(hi.tolist(), hj.tolist()))

    def rp(found):
        tp = len(found & exact)
        return {"recall": tp / len(exact) if exact else 1.0, "precision": tp / len(found) if found else 1.0,
                "flagged": len(found)}

    ex["comparators"] = {
        "exact_cosine": {"call_ms": ewall, "kernel_ms": ems, "pairs_per_s": pairs_total / (ewall / 1e3),
                         "flagged": len(exact)},
        "simhash64": {"sign_ms": sms, "docs_per_s": n / (sms / 1e3), "hamming_ms": hms,
                      "hamming_pairs_per_s": pairs_total / (hms / 1e3), "flagged_hamming_le_3": len(simset)},
    }
    ex["vs_exact_cosine_at_tau"] = {"mrc_fp32": rp(pair_sets["fp32"]), "simhash_hamming_le_3": rp(simset)}
    # signing against HBM. mrc_sign: tokens in + offsets + signatures out;
    # signing from the build's count lists: 8 B per distinct (doc, term) + offsets + signatures out
    docid = np.repeat(np.arange(n, dtype=np.int64), np.diff(c.offsets))
    nnz = int(np.unique(docid * c.vocab + c.tokens).size)
    ex["sign_roofline"] = {}
    for name, ms, by in [("mrc_sign", sign_ms, c.tokens.size * 4 + (n + 1) * 8 + n * k * 4),
                         ("sign_counts", counts_ms, nnz * 8 + (n + 1) * 8 + n * k * 4)]:
        if ms:
            ex["sign_roofline"][name] = {"bound": "hbm", "algorithmic_bytes": int(by), "avg_ms": ms,
                                         "achieved_GBps": by / (ms / 1e3) / 1e9,
                                         "frac": by / (ms / 1e3) / 1e9 / 8000.0}
    ex["sign_roofline"]["nnz"] = nnz
    # queries against a database of the corpus
    log("queries")
    db = mrc.mrc_db_create(ctx, n + 1024, k)
    mrc.mrc_db_insert(db, sig)
    qc = synth.generate_queries(synth.CONFIGS[1], 512, seed=11, median=300, sigma=1.2, hi=20000, near_of=c,
                                near_frac=0.2)
    qo = torch.from_numpy(qc.offsets).cuda()
    qt = torch.from_numpy(qc.tokens).cuda()
    singles = []
    for i in range(200):
        a, b = int(qc.offsets[i]), int(qc.offsets[i + 1])
        o1 = torch.tensor([0, b - a], dtype=torch.int64, device="cuda")
        t1 = qt[a:b].contiguous() if b > a else torch.zeros(1, dtype=torch.int32, device="cuda")
        singles.append((o1, t1))
    torch.cuda.synchronize()
    q = {}
    for name, p in [("fp32", mrc.PREC_FP32), ("bf16", mrc.PREC_BF16), ("fp8", mrc.PREC_FP8)]:
        lat = []
        for o1, t1 in singles:
            t0 = time.perf_counter()
            mrc.mrc_query(ctx, db, model, o1, t1, 16, tau, p)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
        lat = np.array(lat[10:])
        mrc.mrc_query(ctx, db, model, qo, qt, 16, tau, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            mrc.mrc_query(ctx, db, model, qo, qt, 16, tau, p)
        torch.cuda.synchronize()
        bt = (time.perf_counter() - t0) / 3
        q[name] = {"single_query_p50_ms": float(np.percentile(lat, 50)),
                   "single_query_p99_ms": float(np.percentile(lat, 99)),
                   "batch512_ms": bt * 1e3, "batch512_queries_per_s": 512 / bt}
    q["database_rows"] = n
    ex["query"] = q
    return ex


def precision_leg(mrc, synth, tau=0.9):
    """The precision form's workload (200,000 documents over a 262,144-term
    vocabulary, median 400 tokens, k = 256): model build + signing, then the
    all-pairs comparison kernels at FP32, BF16 and FP8 (+ FP32 rescoring of
    the band), each timed with HIP events on its launch stream and set against
    its form's dense matrix-core peak; decisions across the forms, and each
    form's error against a float64 comparison on a 5,000-document subsample."""
    import torch
    cs = synth.CONFIGS[2]
    k = cs.k
    log(f"precision form: generating {cs.n_docs} docs")
    c = synth.generate(2)
    ctx = mrc.mrc_ctx_create(0)
    off = torch.from_numpy(c.offsets).cuda()
    tok = torch.from_numpy(c.tokens).cuda()
    sig = torch.empty((c.n_docs, k), dtype=torch.float32, device="cuda")
    mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(k), sig_out=sig)
    torch.cuda.synchronize()
    kms, wall, _ = timed(mrc, ctx, "sign_counts", lambda: mrc.mrc_build_and_sign(ctx, off, tok, c.vocab,
                                                                               mrc.ref_spec(k), sig_out=sig), 3)
    out = {"workload": f"precision: {c.n_docs} docs, vocab {cs.vocab}, k={k}, tau={tau}, band 0.02 (FP8: per-pair "
                       f"bound, at least 0.02)", "tokens": int(c.tokens.size),
           "build_and_sign_ms": wall, "docs_signed_per_s": c.n_docs / (wall / 1e3), "sign_counts_ms": kms,
           "algorithmic_flops_per_compare_launch": c.n_docs * (c.n_docs - 1) / 2 * 2 * k}
    del off, tok
    out.update(precision_extras(mrc, ctx, c, sig, k, tau, 16 * 1024 * 1024))
    for name in ("fp32", "bf16", "fp8"):
        f = out["forms"][name]
        f["achieved_TFLOPs"] = out["algorithmic_flops_per_compare_launch"] / (f["kernel_ms"] / 1e3) / 1e12
    del sig, c
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def serving_leg(mrc, synth, tau=0.9, n_queries=4096, seconds=3.0):
    """The serving form's workload, short: a 1,000,000-signature database
    (k = 128, FP32 + BF16 copies) built and signed on the GPU; closed-loop
    mrc_query batches of 1, 256 and 4096 queries (FP32 and BF16); the serving
    loop (2 streams, batches up to 4096) at saturation and under Poisson
    arrivals at half of it, p50 / p99 submit-to-result latency."""
    import torch
    cs = synth.CONFIGS[3]
    k = cs.k
    log(f"serving form: generating the {cs.n_docs}-document database corpus")
    c = synth.generate(3)
    n = c.n_docs
    ctx = mrc.mrc_ctx_create(0)
    off = torch.from_numpy(c.offsets).cuda()
    tok = torch.from_numpy(c.tokens).cuda()
    sig = torch.empty((n, k), dtype=torch.float32, device="cuda")
    model, _ = mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(k), sig_out=sig)
    del model
    torch.cuda.synchronize()
    kms, wall, (model, _) = timed(mrc, ctx, "sign_counts",
                                  lambda: mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(k),
                                                                 sig_out=sig), 3)
    docid = np.repeat(np.arange(n, dtype=np.int64), np.diff(c.offsets))
    nnz = int(np.unique(docid * c.vocab + c.tokens).size)
    del docid
    by = nnz * 8 + (n + 1) * 8 + n * k * 4
    out = {"workload": f"serving: database {n} signatures x k={k} (FP32 + BF16) resident, queries lognormal median "
                       f"400, sigma 1.2, 20-20,000 tokens, 20% near duplicates of database documents; top-16 + "
                       f"tau={tau}",
           "database_build": {"docs": n, "tokens": int(c.tokens.size), "build_and_sign_ms": wall,
                              "docs_signed_per_s": n / (wall / 1e3),
                              "sign_counts": {"bound": "hbm", "avg_ms": kms, "algorithmic_bytes": by, "nnz": nnz,
                                              "achieved_GBps": by / (kms / 1e3) / 1e9,
                                              "frac": by / (kms / 1e3) / 1e9 / PEAKS["hbm_GBps"]}}}
    log(f"serving form: build + sign {wall:.1f} ms, sign_counts {kms:.2f} ms")
    db = mrc.mrc_db_create(ctx, n + 65536, k, precisions=(mrc.PREC_BF16,))
    mrc.mrc_db_insert(db, sig)
    torch.cuda.synchronize()
    del off, tok, sig
    torch.cuda.empty_cache()
    qc = synth.generate_queries(cs, n_queries, seed=31, median=400, sigma=1.2, hi=20000, near_of=c, near_frac=0.2)
    del c
    qo = torch.from_numpy(qc.offsets).cuda()
    qt = torch.from_numpy(qc.tokens).cuda()
    batch = {}
    for pname, p in [("fp32", mrc.PREC_FP32), ("bf16", mrc.PREC_BF16)]:
        rows = {}
        for b in (1, 256, 4096):
            o1 = (qo[:b + 1] - qo[0]).contiguous()
            t1 = qt[int(qc.offsets[0]):int(qc.offsets[b])].contiguous()
            mrc.mrc_query(ctx, db, model, o1, t1, 16, tau, p)
            torch.cuda.synchronize()
            reps = 10 if b < 256 else 3
            t0 = time.perf_counter()
            for _ in range(reps):
                mrc.mrc_query(ctx, db, model, o1, t1, 16, tau, p)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            rows[str(b)] = {"ms": dt * 1e3, "queries_per_s": b / dt, "pairs_per_s": b * n / dt}
        batch[pname] = rows
        log(f"serving form mrc_query {pname}: " + ", ".join(f"b={b} {r['ms']:.2f} ms" for b, r in rows.items()))
    out["query_batches"] = batch
    docs = [qc.doc(i) for i in range(qc.n_docs)]
    loop = {}
    rng = np.random.default_rng(41)
    for pname, p in [("bf16", mrc.PREC_BF16), ("fp32", mrc.PREC_FP32)]:
        srv = mrc.mrc_serve_start(ctx, db, model, max_batch=4096, n_streams=2, topk=16, tau=tau, precision=p,
                                  max_wait_us=500)
        sat = serve_run(mrc, srv, [0.0] * 8192, docs)
        lam = 0.5 * sat["docs_per_s"]
        m = int(min(max(lam * seconds, 200), 40000))
        half = serve_run(mrc, srv, rng.exponential(1.0 / lam, m).tolist(), docs)
        half["offered_docs_per_s"] = lam
        mrc.mrc_serve_stop(srv)
        loop[pname] = {"saturation_queries_per_s": sat["docs_per_s"], "poisson_0.5": half}
        log(f"serving form loop {pname}: saturation {sat['docs_per_s']:.0f}/s; at 0.5 load p50 "
            f"{half['p50_ms']:.2f} ms, p99 {half['p99_ms']:.2f} ms (after the first fifth "
            f"{half['p99_after_first_fifth_ms']:.2f} ms), max {half['max_ms']:.2f} ms, host lag {half['lag_ms']:.2f} ms")
    out["serving_loop"] = loop
    del db, model, qo, qt
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def serving_fp8(mrc, synth, ctx, run, tau):
    """Serving with an FP8 database at scale: 4,000,000 rows x k = 256 (FP8 codes
    + row scales + the FP32 rescoring copy) of 4,000,000 distinct synthetic
    documents, drawn in four chunks of 1,000,000 with distinct seeds: the first
    chunk builds the model, the others are signed against it (frozen) and
    appended as they are made. A 50% insert / 50% query stream of documents of
    20-50,000 tokens (20% of the queries near duplicates of database documents)
    with an 80% admission cap; the same stream against the FP32 plain path on
    the same database."""
    import torch
    spec = synth.CONFIGS[4]
    k = spec.k
    chunk = 1_000_000
    n_chunks = spec.n_docs // chunk
    db = mrc.mrc_db_create(ctx, spec.n_docs + 400_000, k, precisions=(mrc.PREC_FP8,))
    model, qc = None, None
    t_sign = 0.0
    for g in range(n_chunks):
        log(f"FP8-scale database: generating chunk {g + 1} of {n_chunks}")
        cg = synth.generate(4, n_docs=chunk, seed=synth.config_seed(4) + 7919 * g)
        off = torch.from_numpy(cg.offsets).cuda()
        tok = torch.from_numpy(cg.tokens).cuda()
        sig = torch.empty((chunk, k), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if g == 0:
            model, _ = mrc.mrc_build_and_sign(ctx, off, tok, cg.vocab, mrc.ref_spec(k), sig_out=sig)
        else:
            mrc.mrc_sign(ctx, model, off, tok, sig_out=sig)
        mrc.mrc_db_insert(db, sig)
        torch.cuda.synchronize()
        t_sign += time.perf_counter() - t0
        if g == 0:
            qc = synth.generate_queries(spec, 12000, seed=37, median=400, sigma=1.2, hi=50000, near_of=cg,
                                        near_frac=0.2)
        del off, tok, sig, cg
        torch.cuda.empty_cache()
    rows, _ = mrc.mrc_db_size(db)
    log(f"FP8 database: {rows} rows x k={k} ({t_sign:.2f} s of signing + inserting)")
    docs = [qc.doc(i) for i in range(qc.n_docs)]
    res = {"database_rows": rows, "k": k, "hbm_frac": 0.8,
           "database": f"{spec.n_docs} distinct documents in {n_chunks} chunks of {chunk} (distinct seeds); the "
                       "first builds the model, the others are signed with it frozen (FP8 codes + scales + FP32 "
                       "copy)",
           "database_sign_and_insert_s": t_sign,
           "stream": "alternating insert / query, lengths lognormal median 400, sigma 1.2, 20-50,000 tokens, 20% "
                     "of the documents near duplicates of database documents"}
    rng = np.random.default_rng(43)
    # the grid-strided collection for both precisions; FP8 also with the
    # persistent collection (work items from a device counter, as many
    # workgroups as are resident)
    for pname, p, form in [("fp8", mrc.PREC_FP8, mrc.SCAN_GRID), ("fp32", mrc.PREC_FP32, mrc.SCAN_GRID),
                           ("fp8_persistent_scan", mrc.PREC_FP8, mrc.SCAN_PERSISTENT)]:
        mrc.mrc_ctx_set_scan(ctx, form)
        srv = mrc.mrc_serve_start(ctx, db, model, max_batch=4096, n_streams=2, topk=16, tau=tau, precision=p,
                                  max_wait_us=500, hbm_frac=0.8)
        sat = run([0.0] * 8192, srv=srv, docs=docs, mixed=True)
        lam = 0.5 * sat["docs_per_s"]
        half = run(rng.exponential(1.0 / lam, int(min(max(lam * 3.0, 200), 40000))).tolist(), srv=srv, docs=docs,
                   mixed=True)
        half["offered_docs_per_s"] = lam
        mrc.mrc_serve_stop(srv)
        res[pname] = {"saturation": sat, "poisson_0.5": half,
                      "collection": "persistent" if form == mrc.SCAN_PERSISTENT else "grid"}
        log(f"FP8-scale serving {pname}: saturation {sat['docs_per_s']:.0f} docs/s; at 0.5 load query p50 "
            f"{half['query_p50_ms']:.2f} ms, p99 {half['query_p99_ms']:.2f} ms")
    mrc.mrc_ctx_set_scan(ctx, mrc.SCAN_GRID)
    res["database_rows_after"] = mrc.mrc_db_size(db)[0]
    return res


def serve_run(mrc, srv, arrival_gaps, docs, mixed=False):
    """Submit requests at the given arrival gaps (seconds; all zero = everything at
    once): every request already due goes in one submit_many call (one per kind
    when mixed: odd requests insert, even ones query), so the host loop keeps up
    with the schedule (lag_ms = the largest delay of a submission behind its due
    time). Latency is submit-to-result on the server's clock."""
    n_req = len(arrival_gaps)
    sel = [docs[i % len(docs)] for i in range(n_req)]
    offs = np.zeros(n_req + 1, np.int64)
    np.cumsum([d.size for d in sel], out=offs[1:])
    toks = np.concatenate(sel).astype(np.int32)
    tickets = []
    lag = 0.0
    t0 = time.perf_counter()
    due = t0 + np.cumsum(np.asarray(arrival_gaps, np.float64))
    i = 0
    while i < n_req:
        now = time.perf_counter()
        if now < due[i]:
            if due[i] - now > 2e-4:
                time.sleep((due[i] - now) * 0.5)
            continue
        lag = max(lag, now - due[i])
        j = max(int(np.searchsorted(due, now, side="right")), i + 1)
        if not mixed:
            got = mrc.mrc_serve_submit_many(srv, offs[i:j + 1] - offs[i], toks[offs[i]:offs[j]])
            tickets += [(tk, mrc.REQ_QUERY) for tk in got]
            tickets += [(None, mrc.REQ_QUERY)] * (j - i - len(got))
        else:  # odd requests insert, even ones query; one call per kind, the earliest kind first
            for par in (i % 2, 1 - i % 2):
                ks = list(range(i + ((par - i) % 2), j, 2))
                if not ks:
                    continue
                kind = mrc.REQ_INSERT if par else mrc.REQ_QUERY
                o2 = np.zeros(len(ks) + 1, np.int64)
                np.cumsum([sel[x].size for x in ks], out=o2[1:])
                got = mrc.mrc_serve_submit_many(srv, o2, np.concatenate([sel[x] for x in ks]), kind)
                tickets += [(tk, kind) for tk in got]
                tickets += [(None, kind)] * (len(ks) - len(got))
        i = j
    res = [(mrc.mrc_serve_poll(srv, tk, wait_ms=120000), kind) for tk, kind in tickets if tk is not None]
    wall = time.perf_counter() - t0
    ok = [(r, kind) for r, kind in res if r is not None and r.status == 0]
    lat = [r.t_done_ms - r.t_submit_ms for r, _ in ok]
    latq = [r.t_done_ms - r.t_submit_ms for r, kind in ok if kind == mrc.REQ_QUERY]
    first = min(r.t_submit_ms for r, _ in res)
    last = max(r.t_done_ms for r, _ in res)
    # the same percentiles over the requests submitted after the first fifth
    # of the run, and the worst latency: a transient at the start of a run
    # (after the saturation burst) shows as a p99 well above this one
    t_cut = first + 0.2 * (max(r.t_submit_ms for r, _ in ok) - first) if ok else first
    late = [r.t_done_ms - r.t_submit_ms for r, _ in ok if r.t_submit_ms >= t_cut]
    # the worst latency of each tenth of the run by submit time: where a stall fell
    t_last = max((r.t_submit_ms for r, _ in ok), default=first)
    span = max(t_last - first, 1e-9)
    worst = [0.0] * 10
    for r, _ in ok:
        w = min(9, int((r.t_submit_ms - first) / span * 10))
        worst[w] = max(worst[w], r.t_done_ms - r.t_submit_ms)
    out = {"offered": n_req, "admitted": len(res), "completed": len(lat),
           "p50_ms": percentile_ms(lat, 50), "p99_ms": percentile_ms(lat, 99),
           "p99_after_first_fifth_ms": percentile_ms(late, 99), "max_ms": max(lat) if lat else None,
           "max_ms_by_tenth": [round(x, 3) for x in worst],
           "docs_per_s": len(lat) / ((last - first) / 1e3), "wall_s": wall, "lag_ms": lag * 1e3}
    if mixed:
        out["query_p50_ms"] = percentile_ms(latq, 50)
        out["query_p99_ms"] = percentile_ms(latq, 99)
    return out


def percentile_ms(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def serving(a, mrc, synth, prec):
    """Serving form: a 1,000,000-signature database (k = 128, FP32 + BF16 copies)
    resident in HBM, queried by new documents. Reports the database build
    (documents signed per second at that scale), closed-loop batch throughput
    of mrc_query, and the serving loop under Poisson arrivals at fractions of
    its measured saturation rate (p50 / p99 latency from submit to result)."""
    import torch
    spec_idx = 3
    cs = synth.CONFIGS[spec_idx]
    k, tau = cs.k, 0.9
    log(f"generating the database corpus ({cs.n_docs} docs)")
    c = synth.generate(spec_idx)
    n = c.n_docs
    log(f"corpus: {n} docs, {c.tokens.size} tokens")
    torch.cuda.set_device(0)
    ctx = mrc.mrc_ctx_create(0)
    off = torch.from_numpy(c.offsets).cuda()
    tok = torch.from_numpy(c.tokens).cuda()
    sig = torch.empty((n, k), dtype=torch.float32, device="cuda")
    # database build: model + signatures of all documents (the first call warms up)
    model, _ = mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(k), sig_out=sig)
    del model
    torch.cuda.synchronize()
    kms, wall, (model, _) = timed(mrc, ctx, "sign_counts",
                                  lambda: mrc.mrc_build_and_sign(ctx, off, tok, c.vocab, mrc.ref_spec(k),
                                                                 sig_out=sig), 3)
    build = {"docs": n, "tokens": int(c.tokens.size), "build_and_sign_ms": wall,
             "docs_signed_per_s_build_and_sign": n / (wall / 1e3), "sign_counts_kernel_ms": kms}
    log(f"build + sign: {wall:.1f} ms ({n / (wall / 1e3):.3g} docs/s)")
    db = mrc.mrc_db_create(ctx, n + 65536, k, precisions=(mrc.PREC_BF16,))
    mrc.mrc_db_insert(db, sig)
    torch.cuda.synchronize()
    del off, tok, sig
    torch.cuda.empty_cache()
    qc = synth.generate_queries(cs, 12000, seed=31, median=400, sigma=1.2, hi=20000, near_of=c, near_frac=0.2)
    qo = torch.from_numpy(qc.offsets).cuda()
    qt = torch.from_numpy(qc.tokens).cuda()
    docs = [qc.doc(i) for i in range(qc.n_docs)]
    out = {"metric": "near-dup pairs compared/s & docs signed/s at stated recall; p50/p99 query ms",
           "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[a.precision],
           "data": "synthetic (seeded Zipf/topic/lognormal generator; database 1M docs, queries lognormal "
                   "median 400, sigma 1.2, 20-20,000 tokens, 20% near duplicates of database docs)",
           "config": {"workload": f"serving_db: {n} signatures x k={k} resident (FP32 + BF16), top-16 + tau={tau}",
                      "n_db": n, "k": k, "tau": tau, "precision": a.precision},
           "database_build": build}
    # closed-loop batches through mrc_query (queries already on the device)
    batch = {}
    for pname, p in [("fp32", mrc.PREC_FP32), ("bf16", mrc.PREC_BF16)]:
        rows = {}
        for b in (1, 16, 256, 4096):
            o1 = (qo[:b + 1] - qo[0]).contiguous()
            t1 = qt[int(qc.offsets[0]):int(qc.offsets[b])].contiguous()
            mrc.mrc_query(ctx, db, model, o1, t1, 16, tau, p)
            torch.cuda.synchronize()
            reps = 20 if b < 256 else 5
            t0 = time.perf_counter()
            for _ in range(reps):
                mrc.mrc_query(ctx, db, model, o1, t1, 16, tau, p)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            rows[str(b)] = {"ms": dt * 1e3, "docs_per_s": b / dt, "pairs_per_s": b * n / dt}
        batch[pname] = rows
        log(f"mrc_query {pname}: " + ", ".join(f"b={b} {r['ms']:.2f} ms" for b, r in rows.items()))
    out["query_batches"] = batch
    if a.query_only:
        b4 = batch[a.precision if a.precision in batch else "bf16"]["4096"]
        out.update({"value": b4["pairs_per_s"], "unit": "pairs/s", "steps": 5, "warmup": 1, "ms_per_step": b4["ms"],
                    "note": "value = query-row pairs/s of a 4096-query mrc_query batch (closed loop)"})
        return out
    # serving loop: saturation (everything submitted at once), then Poisson arrivals
    srv = mrc.mrc_serve_start(ctx, db, model, max_batch=4096, n_streams=2, topk=16, tau=tau, precision=prec,
                              max_wait_us=500)
    state = {"srv": srv}

    def run(arrival_gaps, srv=None, docs=docs, mixed=False):
        return serve_run(mrc, srv if srv is not None else state["srv"], arrival_gaps, docs, mixed)

    sat = run([0.0] * 32768)
    sat_rate = sat["docs_per_s"]
    log(f"serving saturation: {sat_rate:.0f} docs/s, p50 {sat['p50_ms']:.1f} ms, p99 {sat['p99_ms']:.1f} ms")
    rng = np.random.default_rng(41)
    loads = {}
    for frac in (0.25, 0.5, 0.8, 0.95):
        lam = frac * sat_rate
        m = int(min(max(lam * a.serve_seconds, 200), 60000))
        r = run(rng.exponential(1.0 / lam, m).tolist())
        r["offered_docs_per_s"] = lam
        loads[str(frac)] = r
        log(f"load {frac}: offered {lam:.0f}/s, achieved {r['docs_per_s']:.0f}/s, p50 {r['p50_ms']:.2f} ms, "
            f"p99 {r['p99_ms']:.2f} ms, host lag {r['lag_ms']:.2f} ms")
    mrc.mrc_serve_stop(srv)
    out["serving"] = {"saturation": sat, "poisson": loads, "max_batch": 4096, "n_streams": 2,
                      "precision": a.precision}
    del db, model, qo, qt
    torch.cuda.empty_cache()
    del c
    out["serving_fp8_at_scale"] = serving_fp8(mrc, synth, ctx, run, tau)
    out["value"] = sat_rate * n
    out["unit"] = "pairs/s"
    out["steps"] = 1
    out["warmup"] = 1
    out["ms_per_step"] = 1e3 / sat_rate
    out["p50_query_ms_at_0.5_load"] = loads["0.5"]["p50_ms"]
    out["p99_query_ms_at_0.5_load"] = loads["0.5"]["p99_ms"]
    out["note"] = ("value = serving-loop queries/s at saturation x database rows; ms_per_step = ms per query "
                   "at saturation; latencies are submit-to-result on the host clock")
    return out


if __name__ == "__main__":
    main()
