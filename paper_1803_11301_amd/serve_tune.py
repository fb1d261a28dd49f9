"""Settings of the product server chosen by measurement on a request mix.

The server (polymul_server_* in fpmul.h) has three settings that change when
and how products run, never what they are: the number of launch slots, the
product length up to which requests are batched into one launch, and the
largest batch.  tune_server times a list of candidate settings on the
caller's mix of operand lengths.  For each candidate it measures

* the saturated rate X: the whole mix submitted at once, `bursts` times,
  the median rate (one burst alone varies by 10-15% between runs);
* the latency of an open-loop Poisson stream of the same mix arriving at
  rho * X: p50 and p99 from submit to completion as the server sees it.

The choice is the candidate with the highest X whose p99 meets p99_limit_ms
(all of them when no limit is given); if none meets it, the one with the
lowest p99.  Operands are random bits in two device pools, one request's
operands at seeded offsets in them, so the mix costs two pool allocations
and one output buffer.
"""
from __future__ import annotations

import time

DEFAULT_CANDIDATES = (
    # (slots, batch_limit_bits, max_batch)
    (8, 1 << 20, 512),
    (8, 1 << 18, 512),
    (8, 1 << 21, 512),
    (12, 1 << 20, 512),
    (4, 1 << 20, 512),
    (8, 1 << 20, 256),
)


def choose(table, p99_limit_ms=None):
    """The chosen row of `table` (dicts with saturated_per_s and p99_ms): the
    highest saturated rate among the rows within the p99 limit, else the
    lowest p99."""
    if not table:
        raise ValueError("no candidates were measured")
    ok = [r for r in table if p99_limit_ms is None or r["p99_ms"] <= p99_limit_ms]
    if ok:
        return max(ok, key=lambda r: r["saturated_per_s"])
    return min(table, key=lambda r: r["p99_ms"])


def tune_server(ctx, len_a, len_b, candidates=DEFAULT_CANDIDATES, rho: float = 0.8, p99_limit_ms=None,
                bursts: int = 3, hbm_budget: int = 8 << 30, seed: int = 0x5EED0570):
    """Measure each (slots, batch_limit_bits, max_batch) of `candidates` on
    the mix of operand lengths (len_a[k], len_b[k]) and return
    {"choice": row, "table": rows}; each row holds the setting, the
    saturated rate, its bursts, and p50/p99 at rho times it."""
    import numpy as np
    import torch

    from . import fpmul, synth

    la = np.asarray(len_a, dtype=np.int64)
    lb = np.asarray(len_b, dtype=np.int64)
    if la.shape != lb.shape or la.size == 0 or (la <= 0).any() or (lb <= 0).any():
        raise ValueError("len_a and len_b must be equal-length lists of positive lengths")
    if not 0.0 < rho < 1.0:
        raise ValueError("rho must be in (0, 1)")
    n = la.size
    pool_bits = int(max(la.max(), lb.max())) + 64 * 1024
    dev = torch.device("cuda", ctx.device)
    pa = torch.from_numpy(synth.dense_poly(seed, pool_bits).view(np.int64)).to(dev)
    pb = torch.from_numpy(synth.dense_poly(seed + 1, pool_bits).view(np.int64)).to(dev)
    pw = pool_bits // 64
    rng = np.random.default_rng(seed)
    offa = rng.integers(0, pw - (la + 63) // 64 + 1)
    offb = rng.integers(0, pw - (lb + 63) // 64 + 1)
    ow = (la + lb - 1 + 63) // 64
    ooff = np.concatenate([[0], np.cumsum(ow)[:-1]])
    out = torch.empty(int(ow.sum()), dtype=torch.int64, device=dev)
    args = [(pa.data_ptr() + 8 * int(offa[k]), int(la[k]), pb.data_ptr() + 8 * int(offb[k]), int(lb[k]),
             out.data_ptr() + 8 * int(ooff[k])) for k in range(n)]
    gaps = rng.exponential(1.0, n)   # unit-rate inter-arrival times, scaled per candidate
    torch.cuda.synchronize()

    table = []
    for slots, limit, max_batch in candidates:
        srv = fpmul.Server(ctx, hbm_budget=hbm_budget, slots=slots, batch_limit_bits=limit, max_batch=max_batch)
        try:
            rates = []
            for _ in range(bursts):
                t0 = time.perf_counter()
                tks = [srv.submit(*x) for x in args]
                for tk in tks:
                    srv.wait(tk)
                rates.append(n / (time.perf_counter() - t0))
            X = float(np.median(rates))
            due = np.cumsum(gaps / (rho * X))
            tks = []
            t0 = time.perf_counter()
            for k in range(n):
                # sleep through the longer gaps, spin the last 0.1 ms (the
                # launcher threads of the server need the host's cores too)
                while True:
                    left = due[k] - (time.perf_counter() - t0)
                    if left <= 0:
                        break
                    if left > 2e-4:
                        time.sleep(left - 1e-4)
                tks.append(srv.submit(*args[k]))
            done = [srv.wait(tk) for tk in tks]
        finally:
            srv.close()
        lat = np.array([(d - s0) / 1e6 for s0, _, d in done])
        table.append({"slots": slots, "batch_limit_bits": limit, "max_batch": max_batch,
                      "saturated_per_s": round(X, 1), "bursts_per_s": [round(r, 1) for r in rates],
                      "rho": rho, "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3)})
    del pa, pb, out
    return {"choice": choose(table, p99_limit_ms), "table": table, "p99_limit_ms": p99_limit_ms,
            "requests": n}
