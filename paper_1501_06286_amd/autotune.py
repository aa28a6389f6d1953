"""Launch-configuration autotuner.

For a plan and a column count t it times the candidate launch tunings of
``qmc_plan_set_tuning`` (sparse or dense outer front, outer radix, chunk of
column pairs per pass, one or two streams, plain or non-temporal stores of X
and of the intermediate)
on the GPU
with HIP events, keeps the fastest, and caches the choice in a JSON file keyed
by the GPU architecture and the plan's shape (rule, L, M, s, t, dtype).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Tuple

CACHE = os.environ.get("QMC_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "qmcfast", "autotune.json"))


def outer_radices(M2: int, qmax: int = 128) -> List[int]:
    """outer_q values worth trying for an outer length M2: the default (0:
    all of M2 in one back pass when M2 <= qmax, else 32 values of w2 per
    back-pass output column), and the other splits: 16 and 32 in registers,
    the LDS back pass's 64 and 128 (up to qmax, the dtype's limit), as far as
    the split allows; for M2 = 3 x 2^j or 5 x 2^j the same with that factor
    kept in the back pass (12, 24, 48, 96 or 10, 20, 40, 80).  A value equal
    to the default is not tried twice."""
    qdef = M2 if M2 <= qmax else max(32, M2 // 64)
    base = ((12, 24, 48, 96) if M2 % 3 == 0 else (10, 20, 40, 80) if M2 % 5 == 0
            else (16, 32, 64, 128))
    return [0] + [q for q in base
                  if M2 > 16 and q < M2 and M2 % q == 0 and M2 // q <= 64 and q <= qmax
                  and q != qdef]


def qmax_of(plan) -> int:
    return 128 if plan.torch_dtype.itemsize == 4 else 64


def candidates(pairs: int, M2: int = 1, qmax: int = 128) -> List[Dict[str, int]]:
    """Sparse front (with item or with bucket twiddles): every chunk, one or
    two streams, plain or non-temporal stores of X.  Dense front (one
    stream): every chunk, both store kinds.
    Each with cached or streaming stores of the intermediate and every outer
    radix of ``outer_radices``.  Bucket twiddles need M2 a power of two (for
    M2 = 3 x 2^j or 5 x 2^j the library runs front 3 as front 1: not tried
    twice)."""
    chunks = [0] + [c for c in (8, 16, 32, 64, 128, 256, 512, 1024) if c < pairs]
    qs = outer_radices(M2, qmax)
    fronts = (1, 3) if M2 & (M2 - 1) == 0 else (1,)
    out = []
    for q in qs:
        for ni in (1, 2):  # cached or streaming stores of the intermediate
            for front in fronts:  # item twiddles, bucket twiddles
                for c in chunks:
                    for streams in ((1, 2) if c else (1,)):
                        for nt in (0, 1):
                            out.append({"chunk_pairs": c, "streams": streams, "nt_store": nt,
                                        "front": front, "outer_q": q, "nt_inter": ni})
            for c in chunks:
                for nt in (0, 1):
                    out.append({"chunk_pairs": c, "streams": 1, "nt_store": nt, "front": 2,
                                "outer_q": q, "nt_inter": ni})
    return out


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


_LIB_SHA = None


def _lib_sha() -> str:
    """Hash of the loaded library file: a tuning timed on other kernels is
    not reused."""
    global _LIB_SHA
    if _LIB_SHA is None:
        import hashlib
        import paper_1501_06286_amd as q
        h = hashlib.sha256()
        with open(q.LIB_PATH, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _LIB_SHA = h.hexdigest()[:16]
    return _LIB_SHA


def cache_key(plan, t: int) -> str:
    i = plan.info()
    return (f"{_arch()}|lib{_lib_sha()}|rule{i['rule']}|L{i['L']}|M{i['M']}|s{i['s']}|t{t}"
            f"|dtype{i['dtype']}")


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def time_config(plan, A, X, cfg: Dict[str, int], reps: int = 3) -> float:
    """Milliseconds per qmc_matmul with the given tuning (events on the caller's stream)."""
    import torch
    import paper_1501_06286_amd as q
    plan.set_tuning(**cfg)
    ws = plan.workspace(A.shape[1], A.device)
    q.matmul(plan, A, out=X, workspace=ws)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        q.matmul(plan, A, out=X, workspace=ws)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def refine(plan, A, X, results, reps: int, top: int = 4, rounds: int = 5) -> Dict[str, int]:
    """The first sweep's few fastest tunings (often within a few percent of
    each other) timed again in turns, several rounds: the one with the least
    median time, so that the choice does not follow one noisy sample; a
    one-stream tuning within 2% of it is preferred."""
    order = sorted(results, key=lambda r: r[1])[:top]
    if len(order) < 2:
        return order[0][0]
    times = [[] for _ in order]
    for _ in range(rounds):
        for i, (cfg, _) in enumerate(order):
            times[i].append(time_config(plan, A, X, cfg, reps))
    med = [sorted(ts)[len(ts) // 2] for ts in times]
    best = min(range(len(order)), key=lambda i: med[i])
    # within 2% of the fastest (about the spread of repeated timings), one
    # stream wins: its passes do not overlap, so their launch times (and the
    # per-kernel rooflines) are their own
    one = [i for i in range(len(order))
           if order[i][0].get("streams", 1) == 1 and med[i] <= 1.02 * med[best]]
    return order[min(one, key=lambda i: med[i]) if one else best][0]


def tune(plan, t: int, reps: int = 3, use_cache: bool = True,
         cands: Optional[List[Dict[str, int]]] = None) -> Tuple[Dict[str, int], List]:
    """Pick and set the fastest tuning for (plan, t).  Returns (best, timings)."""
    import torch
    key = cache_key(plan, t)
    if cands is not None:  # a choice among other candidates is cached apart
        key += "|cands" + hashlib.sha1(json.dumps(cands, sort_keys=True).encode()).hexdigest()[:12]
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["best"]
        plan.set_tuning(**best)
        return best, cache[key].get("timings", [])
    A = torch.randn((plan.s, t), dtype=plan.torch_dtype, device="cuda")
    X = torch.empty((plan.N, t), dtype=plan.torch_dtype, device="cuda")
    results = []
    for cfg in (cands or candidates((t + 1) // 2, plan.info()["M2"], qmax_of(plan))):
        results.append((cfg, time_config(plan, A, X, cfg, reps)))
    best = refine(plan, A, X, results, reps)
    plan.set_tuning(**best)
    if use_cache:
        cache = _load()
        cache[key] = {"best": best, "timings": [[c, round(ms, 4)] for c, ms in results]}
        _store(cache)
    return best, results


def tune_korobov(U, t: int, reps: int = 3, chunks=(0, 16, 32, 64, 128, 256)) -> Tuple[int, List]:
    """Pick and set the fastest blocks-per-run for a union of Korobov rules."""
    import torch
    import paper_1501_06286_amd as q
    A = torch.randn((U.s, t), dtype=U.torch_dtype, device="cuda")
    X = torch.empty((U.N, t), dtype=U.torch_dtype, device="cuda")
    results = []
    for c in chunks:
        if c >= U.K - 1:
            continue
        U.set_chunk(c)
        ws = U.workspace(t, "cuda")
        q.korobov_matmul(U, A, out=X, workspace=ws)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            q.korobov_matmul(U, A, out=X, workspace=ws)
        e1.record()
        e1.synchronize()
        results.append((c, e0.elapsed_time(e1) / reps))
    best = min(results, key=lambda r: r[1])[0]
    U.set_chunk(best)
    return best, results


def tune_batch(plans, As, reps: int = 3, qs=None) -> Tuple[Dict[int, int], List]:
    """Pick the outer radix of a batch's products by timing whole batched runs:
    for each outer length M2 in the batch, every admissible outer_q with the
    other products at the default; the products of one M2 form their own
    launch groups, so the choices are made one M2 at a time.  Sets the
    plans' tunings and returns ({M2: outer_q}, timings)."""
    import torch
    import paper_1501_06286_amd as q

    def run_ms():
        b = q.Batch(plans, As)
        b.run()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.run()
        e1.record()
        e1.synchronize()
        b.close()
        return e0.elapsed_time(e1) / reps

    m2s = sorted({p.info()["M2"] for p in plans})
    best, timings = {}, []
    for p in plans:
        p.set_tuning(**{**p.get_tuning(), "outer_q": 0})
    for m2 in m2s:
        if m2 <= 16:
            continue
        group = [p for p in plans if p.info()["M2"] == m2]
        res = []
        qmax = min(qmax_of(p) for p in group)
        for oq in (qs if qs is not None else outer_radices(m2, qmax)):
            if oq and (oq > m2 or m2 // oq > 64 or oq > qmax):
                continue
            for p in group:
                p.set_tuning(**{**p.get_tuning(), "outer_q": oq})
            res.append((oq, run_ms()))
        choice = min(res, key=lambda r: r[1])[0]
        for p in group:
            p.set_tuning(**{**p.get_tuning(), "outer_q": choice})
        best[m2] = choice
        timings.append((m2, res))
    return best, timings


def tune_batch_chunk(batch, reps: int = 3, chunks_mib=(128, 256, 384, 512, 1024, 0),
                     nts=(0, 2)) -> Tuple[Tuple[int, int], List]:
    """Pick the run size of a batch (intermediates per run, in MiB; 0 = one
    run of all products) and the store kind of its intermediates (automatic
    or streaming) by timing whole runs of the batch; sets the fastest and
    returns ((chunk_bytes, nt_inter), timings)."""
    import torch
    results = []
    for mib in chunks_mib:
        for nt in nts:
            batch.set_chunk(mib << 20, nt)
            batch.run()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                batch.run()
            e1.record()
            e1.synchronize()
            results.append(((mib << 20, nt), e0.elapsed_time(e1) / reps))
    best = min(results, key=lambda r: r[1])[0]
    batch.set_chunk(*best)
    return best, results
