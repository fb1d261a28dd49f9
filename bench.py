#!/usr/bin/env python3
"""Benchmark: ms per product of two 2^30-bit polynomials in GF(2)[x] on one MI355X.

One step = one full product (BasisCvt, Encode, Butterfly for both operands,
pointwise products, iButterfly, Decode, iBasisCvt) with the operands already
resident in HBM.  Prints ONE JSON line on stdout; details go to stderr.

    python bench.py [--steps K] [--warmup W] [--workload large|mid|small] [--no-cpu]

The K timed steps run as a user runs them; then the same K steps run again
with a HIP event pair that the library records around every kernel on its
launch stream (polymul_profile_enable), which gives the per-kernel durations
and the roofline (those events add about 0.1 ms per product, reported as
ms_per_step_profiled).  The roofline entry
is for the kernel with the largest total time, priced against HBM at 8 TB/s
with the nominal algorithmic bytes of its stage (each stage streams its input
and output once): BasisCvt 2A+2B, Encode A+B+2N, Butterfly 2N per transform,
pointwise 3N, iButterfly 2N, Decode 2N, iBasisCvt 2N (A, B operand bytes,
N transform bytes).  Fused kernels are priced by the data they transform,
read once and written once (KERNEL_BYTES).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (operand bits, seed, top bit forced, description)
    "small": (1 << 16, 0x5EED0016, False, "single product 2^16 x 2^16 bits, uniform random"),
    "mid": (1 << 24, 0x5EED0024, True, "single product 2^24 x 2^24 bits, uniform random, top bit forced"),
    "large": (1 << 30, 0x5EED0030, False, "single product 2^30 x 2^30 bits, uniform random"),
}

# Algorithmic bytes per launch of each kernel of the large-size schedule: the
# data it transforms read once and written once at natural size (A, B operand
# bytes, N transform bytes).  Fused kernels count each input and output once.
KERNEL_BYTES = {
    "basiscvt_zeta": lambda A, B, N: 2 * A,             # two launches per operand
    "basiscvt_rows": lambda A, B, N: 2 * A,             # one per operand
    "basiscvt_outer_encode": lambda A, B, N: A + N,     # one per operand
    "butterfly_upper": lambda A, B, N: 4 * N,           # A and B together
    "butterfly_bottom": lambda A, B, N: 4 * N,          # A and B together
    "pointwise": lambda A, B, N: 3 * N,                 # read A, B; write C
    "ibutterfly_bottom": lambda A, B, N: 2 * N,
    "ibutterfly_upper": lambda A, B, N: 2 * N,
    "decode_outer": lambda A, B, N: 2 * N,
    "ibasiscvt_rows": lambda A, B, N: 2 * N,
    "ibasiscvt_zeta": lambda A, B, N: 2 * N,
    "ibasiscvt_store": lambda A, B, N: 2 * N,
}


# HBM bytes per launch measured with rocprofv3 (FETCH_SIZE and WRITE_SIZE
# passes, each scaled by what the counter reads for a plain 1 GiB device copy:
# fetch x2.000, write x1.000), valid only for the kernel sources they were
# taken on: the sha256 of the listed files must match, else traffic is null.
MEASURED_TRAFFIC = {
    "butterfly_upper": {
        "bytes": (262517 * 2 + 524288) * 1024,
        "sources": ("paper_1803_11301_amd/csrc/k_bf3.h", "paper_1803_11301_amd/csrc/k_bf2.h",
                    "paper_1803_11301_amd/csrc/gf_device.h"),
        "sha256": "a3cd3fe8f5229566408c90f042529d188f42a3fab2d583c1d76c8abac2360db9",
    },
}


def sources_sha256(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None or sources_sha256(rec["sources"]) != rec["sha256"]:
        return None
    return rec["bytes"]


def nominal_bytes(A: int, B: int, N: int) -> int:
    """Nominal algorithmic bytes of one product: each stage of Alg. 5 streams its
    input and output once (BasisCvt 2A+2B, Encode A+B+2N, Butterfly 4N,
    pointwise 3N, iButterfly 2N, Decode 2N, iBasisCvt 2N) = 3A + 3B + 15N."""
    return 3 * A + 3 * B + 15 * N


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(log2_len: int, target_log2: int):
    """The oracle (as it stands) on a bounded sample of the same workload: one
    product of 2^log2_len-bit operands from the same generator, on all host
    threads, projected to 2^target_log2-bit operands by the 3x-per-doubling
    cost of its Karatsuba recursion."""
    import oracle as O
    from paper_1803_11301_amd import synth
    O.build(force=False)
    L = 1 << log2_len
    a, b = synth.single_pair(synth.SEED_LARGE, L)
    threads = O.max_threads()
    t0 = time.perf_counter()
    O.polymul(a, L, b, L, threads=threads)
    sec = time.perf_counter() - t0
    scale = 3 ** (target_log2 - log2_len)
    return {"value": round(sec * 1e3 * scale, 3), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"one 2^{log2_len} x 2^{log2_len}-bit product ({sec:.2f} s on {threads} threads, "
                      f"Karatsuba oracle), x3^{target_log2 - log2_len} for 2^{target_log2}-bit operands"}


def bench_batch(ctx, steps: int):
    """The 4096-product mix (operands log-uniform in [2^10, 2^20] bits, 10%
    sparse, seed 0x5EED4096): products/s of one polymul_batch launch against
    one polymul_ex call per product, on the same resident operands."""
    import numpy as np
    import torch
    from paper_1803_11301_amd import fpmul, synth
    plan = synth.batch_plan()
    As, Bs = zip(*[synth.batch_operands(it) for it in plan])
    las = np.array([it.len_a for it in plan], dtype=np.uint64)
    lbs = np.array([it.len_b for it in plan], dtype=np.uint64)
    a_pool, a_off = fpmul.pack_words(As)
    b_pool, b_off = fpmul.pack_words(Bs)
    out_off, out_words = fpmul.out_layout(las.astype(np.int64), lbs.astype(np.int64))
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x).view(np.int64)).cuda()
    ta, tb, tla, tlb, taoff, tboff, toff = d(a_pool), d(b_pool), d(las), d(lbs), d(a_off), d(b_off), d(out_off)
    out = torch.empty(out_words, dtype=torch.int64, device="cuda")
    status = torch.empty(len(plan), dtype=torch.int32, device="cuda")
    max_bits = int((las + lbs - 1).max())
    stream = torch.cuda.current_stream()
    run = lambda: ctx.polymul_batch(ta, taoff, tla, tb, tboff, tlb, out, toff, max_bits, status, stream)
    run()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        run()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_batch = t0.elapsed_time(t1) / steps
    ok = bool((status == 0).all().item())
    # the same batch with every item over GF(2^64) (the m = 32 path off)
    ctx.set_small_field(0)
    run()
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        run()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_batch_m64 = t0.elapsed_time(t1) / steps
    ctx.set_small_field(20)
    # one stream-ordered call per product on the same operands (views of the pools)
    views = [(ta[int(a_off[k]):], int(las[k]), tb[int(b_off[k]):], int(lbs[k]), out[int(out_off[k]):])
             for k in range(len(plan))]
    for v in views[:64]:
        ctx.polymul(v[0], v[1], v[2], v[3], out=v[4], stream=stream)
    torch.cuda.synchronize()
    t0.record(stream)
    for v in views:
        ctx.polymul(v[0], v[1], v[2], v[3], out=v[4], stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_calls = t0.elapsed_time(t1)
    n = len(plan)
    rec = {"workload": "4096 products, operands log-uniform 2^10..2^20 bits, 10% sparse (density 0.01), "
                       "seed 0x5eed4096", "products": n, "ms_per_batch": round(ms_batch, 4),
           "products_per_s": round(n / (ms_batch / 1e3), 1),
           "small_field": "items with transforms up to 2^20 bits over GF(2^32) (m = 32)",
           "ms_per_batch_all_m64": round(ms_batch_m64, 4), "per_call_ms": round(ms_calls, 3),
           "per_call_products_per_s": round(n / (ms_calls / 1e3), 1),
           "speedup_vs_per_call": round(ms_calls / ms_batch, 2), "all_status_ok": ok, "steps": steps}
    log(f"[bench] batch: {ms_batch:.3f} ms per 4096 products ({rec['products_per_s']:.0f}/s; all over GF(2^64): "
        f"{ms_batch_m64:.3f} ms); per-call {ms_calls:.1f} ms ({rec['per_call_products_per_s']:.0f}/s)")
    return rec


def _time_product(ctx, A, la, B, lb, out, steps: int):
    import torch
    stream = torch.cuda.current_stream()
    ctx.polymul(A, la, B, lb, out=out, stream=stream)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        ctx.polymul(A, la, B, lb, out=out, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def bench_m128(steps: int, log2_len: int = 37, compare: bool = True):
    """The m = 128 variant: a 2^37 x 2^37-bit product, whose 2^38-bit transform
    is past the m = 64 bound and runs over GF(2^128) (operands drawn on the
    device from seeds 0x5eed0037 and 0x5eed0038), timed with its per-kernel
    table; and the 2^30 x 2^30 workload forced onto GF(2^128) for the cost of
    the field at equal size.  (The GPU tests check the products of this path
    against the definition, at this transform size too.)"""
    import torch
    from paper_1803_11301_amd import fpmul, synth
    L = 1 << log2_len
    seed = 0x5EED0037
    A = synth.dense_poly_device(seed, L, "cuda")
    B = synth.dense_poly_device(seed + 1, L, "cuda")
    lc = 2 * L - 1
    out = torch.empty((lc + 63) // 64, dtype=torch.int64, device="cuda")
    torch.cuda.empty_cache()
    ctx = fpmul.Context(0)
    log(f"[bench] m128: 2^{log2_len} x 2^{log2_len} bits over GF(2^128), {steps} steps")
    ms = _time_product(ctx, A, L, B, L, out, steps)
    ctx.profile(True)
    ctx.polymul(A, L, B, L, out=out, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    prof = ctx.profile_report()
    ctx.profile(False)
    kernels = {name: {"launches": cnt, "ms": round(tot, 3)}
               for name, (cnt, tot) in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    for name, k in kernels.items():
        log(f"[bench] m128 {name:22s} {k['launches']:5d} launches {k['ms']:10.2f} ms")
    ctx.close()
    del A, B, out
    torch.cuda.empty_cache()
    ms30 = None
    if compare:
        ms30 = _m128_at_2e30()
    nominal = nominal_bytes(L // 8, L // 8, (1 << (log2_len + 1)) // 8)
    # the inverse BasisCvt steps beyond LDS, two at a time out of place: read
    # and write the whole 2^(log2_len + 1)-bit buffer, 2x its bytes per launch
    # (HBM-bound, the largest kernel of this path); a step left alone updates
    # lo from hi in place, 1.5x
    roof = None
    buf = (1 << (log2_len + 1)) // 8
    for name, per_launch in (("ibasiscvt_wide2", 2 * buf), ("ibasiscvt_wide", 3 * buf // 2)):
        if name not in prof:
            continue
        cnt, tot = prof[name]
        achieved = per_launch / (tot / cnt / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_launch": per_launch,
                "avg_launch_us": round(1e3 * tot / cnt, 1)}
        break
    rec = {"workload": f"single product 2^{log2_len} x 2^{log2_len} bits, uniform random, seeds 0x5eed0037/8, "
                       f"2^{log2_len + 1}-bit transform over GF(2^128)",
           "ms_per_product": round(ms, 2), "steps": steps, "roofline": roof,
           "product_roofline": {"nominal_bytes": nominal, "achieved": round(nominal / (ms / 1e3) / 1e9, 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(nominal / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
           "ms_2e30_product_over_gf2_128": None if ms30 is None else round(ms30, 3),
           "kernels": kernels}
    log(f"[bench] m128: {ms:.1f} ms per 2^{log2_len}-bit product" +
        ("" if ms30 is None else f"; 2^30 over GF(2^128) {ms30:.2f} ms"))
    return rec


def _m128_at_2e30():
    """The large workload (2^30 x 2^30 bits, seed 0x5eed0030) over GF(2^128),
    against its GF(2^64) time in the headline."""
    import numpy as np
    import torch
    from paper_1803_11301_amd import fpmul, synth
    a_np, b_np = synth.single_pair(0x5EED0030, 1 << 30)
    a = torch.from_numpy(a_np.view(np.int64)).cuda()
    b = torch.from_numpy(b_np.view(np.int64)).cuda()
    o = torch.empty(((2 << 30) - 1 + 63) // 64, dtype=torch.int64, device="cuda")
    c2 = fpmul.Context(0)
    c2.set_large_field(31)
    ms30 = _time_product(c2, a, 1 << 30, b, 1 << 30, o, 3)
    c2.close()
    return ms30


def bench_serve(ctx, count: int, warmup: int, rho: float, slots: int = 8, batch_limit_bits: int = 1 << 20,
                max_batch: int = 512):
    """Poisson stream of products, operands log-uniform in [2^12, 2^24] bits
    (seed 0x5EED05E5), through the continuous-batching server: first the
    saturated throughput X (every request submitted at once), then arrivals
    at rate rho * X; latency = submit to completion seen by the server."""
    import numpy as np
    import torch
    from paper_1803_11301_amd import fpmul, synth
    total = warmup + count
    _, la, lb, sa, sb = synth.serve_plan(total, 1.0)
    pool_bits = 1 << 25
    pa = torch.from_numpy(synth.dense_poly(synth.SEED_SERVE + 1, pool_bits).view(np.int64)).cuda()
    pb = torch.from_numpy(synth.dense_poly(synth.SEED_SERVE + 2, pool_bits).view(np.int64)).cuda()
    pw = pool_bits // 64
    aw = (la + 63) // 64
    bw = (lb + 63) // 64
    offa = (sa % np.uint64(1 << 40)).astype(np.int64) % (pw - aw + 1)
    offb = (sb % np.uint64(1 << 40)).astype(np.int64) % (pw - bw + 1)
    ow = (la + lb - 1 + 63) // 64
    oofs = np.concatenate([[0], np.cumsum(ow)[:-1]])
    out = torch.empty(int(ow.sum()), dtype=torch.int64, device="cuda")
    ab, bb, ob = pa.data_ptr(), pb.data_ptr(), out.data_ptr()
    args = [(ab + 8 * int(offa[k]), int(la[k]), bb + 8 * int(offb[k]), int(lb[k]), ob + 8 * int(oofs[k]))
            for k in range(total)]
    torch.cuda.synchronize()
    srv = fpmul.Server(ctx, hbm_budget=8 << 30, slots=slots, batch_limit_bits=batch_limit_bits, max_batch=max_batch)
    # saturation: the warm-up requests plus the first measured ones all at once
    nsat = max(warmup, 1)
    t0 = time.perf_counter()
    tks = [srv.submit(*args[k]) for k in range(nsat)]
    for tk in tks:
        srv.wait(tk)
    X = nsat / (time.perf_counter() - t0)
    # open-loop Poisson arrivals at rho * X
    rate = rho * X
    arr, _, _, _, _ = synth.serve_plan(count, rate)
    tks = []
    t0 = time.perf_counter()
    for k in range(count):
        due = t0 + float(arr[k])
        while True:
            now = time.perf_counter()
            if now >= due:
                break
            if due - now > 2e-4:
                time.sleep((due - now) - 1e-4)
        tks.append(srv.submit(*args[warmup + k]))
    for tk in tks:
        srv.wait(tk)
    wall = time.perf_counter() - t0
    lat = np.array([(lambda s, st, d: (d - s) / 1e6)(*srv.times(tk)) for tk in tks])
    queue = np.array([(lambda s, st, d: (st - s) / 1e6)(*srv.times(tk)) for tk in tks])
    srv.close()
    rec = {"workload": "Poisson stream, operands log-uniform 2^12..2^24 bits, seed 0x5eed05e5",
           "requests": count, "warmup": warmup, "saturated_products_per_s": round(X, 1), "rho": rho,
           "offered_per_s": round(rate, 1), "achieved_products_per_s": round(count / wall, 1),
           "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "mean_ms": round(float(lat.mean()), 3), "p99_queue_ms": round(float(np.percentile(queue, 99)), 3),
           "slots": slots, "batch_limit_bits": batch_limit_bits, "max_batch": max_batch,
           "hbm_budget_bytes": 8 << 30}
    log(f"[bench] serve: saturated {X:.0f}/s; at {rho:.2f}: {count / wall:.0f}/s, p50 {rec['p50_ms']} ms, "
        f"p99 {rec['p99_ms']} ms")
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--cpu-log2", type=int, default=27, help="operand size of the oracle sample")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-products measurement")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-rho", type=float, default=0.8, help="offered load as a fraction of saturation")
    ap.add_argument("--no-m128", action="store_true", help="skip the GF(2^128) measurement")
    ap.add_argument("--m128-steps", type=int, default=2)
    ap.add_argument("--m128-only", action="store_true",
                    help="run only the GF(2^128) measurement (2^37 x 2^37 bits) and print its record")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU; --gpus must be 1 "
              "(independent products shard across GPUs without exchange; one GPU is measured)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1803_11301_amd import fpmul, synth

    if args.m128_only:
        rec = bench_m128(args.m128_steps, compare=False)
        rec.update({"metric": "ms per 2^37-bit x 2^37-bit product over GF(2^128)", "value": rec["ms_per_product"],
                    "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "u64",
                    "data": "synthetic (seeded SplitMix64 bits drawn on the device)"})
        print(json.dumps(rec), flush=True)
        return

    if args.copy_calibrate:
        nbytes = args.copy_calibrate << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)
        return

    L, seed, top, desc = WORKLOADS[args.workload]
    a_np, b_np = synth.single_pair(seed, L, top_bit=top)
    dev = torch.device("cuda:0")
    a = torch.from_numpy(a_np.view(np.int64)).to(dev)
    b = torch.from_numpy(b_np.view(np.int64)).to(dev)
    lc = 2 * L - 1
    out = torch.empty((lc + 63) // 64, dtype=torch.int64, device=dev)
    ctx = fpmul.Context(0)
    stream = torch.cuda.current_stream()

    log(f"[bench] {desc}; warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.polymul(a, L, b, L, out=out, stream=stream)
    torch.cuda.synchronize()

    # the timed steps, as a user runs them (no per-kernel events) ...
    log(f"[bench] timing {args.steps} steps")
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(args.steps):
        ctx.polymul(a, L, b, L, out=out, stream=stream)
    t_stop.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_stop)
    ms = ms_total / args.steps
    # ... and the same steps again with a HIP event pair around every kernel
    # on its launch stream, for the per-kernel times and the roofline
    ctx.profile(True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(args.steps):
        ctx.polymul(a, L, b, L, out=out, stream=stream)
    t_stop.record(stream)
    torch.cuda.synchronize()
    ms_profiled = t_start.elapsed_time(t_stop) / args.steps
    prof = ctx.profile_report()
    ctx.profile(False)

    # nominal bytes of the workload
    A = B = L // 8
    log2n = max(6, (lc - 1).bit_length())
    N = (1 << log2n) // 8
    nominal = nominal_bytes(A, B, N)
    per_kernel = {}
    for name, (cnt, tot) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        per_kernel[name] = {"launches_per_step": cnt / args.steps, "ms_per_step": tot / args.steps,
                            "avg_launch_us": 1e3 * tot / cnt}
        if name in KERNEL_BYTES:
            gbs = KERNEL_BYTES[name](A, B, N) / (tot / cnt / 1e3) / 1e9
            per_kernel[name]["achieved_GBs"] = round(gbs, 1)
        log(f"[bench] {name:26s} {cnt / args.steps:6.1f} launches/step {tot / args.steps:9.4f} ms/step "
            f"{1e3 * tot / cnt:9.2f} us/launch")
    known = [n for n in prof if n in KERNEL_BYTES]
    dom = max(known, key=lambda n: prof[n][1]) if known else None
    roof = None
    if dom:
        cnt, tot = prof[dom]
        bytes_per_launch = KERNEL_BYTES[dom](A, B, N)
        avg_s = tot / cnt / 1e3
        achieved = bytes_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(dom), "bytes_per_launch": int(bytes_per_launch),
                "avg_launch_us": round(avg_s * 1e6, 3)}
    # the butterfly kernels are bound by LDS table lookups rather than HBM:
    # report their rate of multiplications by constants (l/2 * n_p per transform,
    # three transforms) per CU per clock at 2.4 GHz
    bfly = [n for n in prof if "butterfly" in n]
    bfly_ms = sum(prof[n][1] for n in bfly) / args.steps
    l = log2n - 6
    mults = 3 * (l * (1 << l) // 2)
    bfly_rate = None
    if bfly_ms > 0:
        bfly_rate = {"multiplications_per_product": mults, "ms_per_product": round(bfly_ms, 4),
                     "per_cu_per_clock": round(mults / (bfly_ms / 1e3) / (256 * 2.4e9), 3),
                     "lookups_per_multiplication": 8}
    product_gbs = nominal / (ms / 1e3) / 1e9
    log(f"[bench] {ms:.3f} ms/product ({ms_profiled:.3f} with per-kernel events); nominal {nominal / 1e9:.3f} GB -> "
        f"{product_gbs:.1f} GB/s "
        f"({100 * product_gbs / HBM_PEAK_GBS:.1f}% of HBM peak)")

    batch = None
    if not args.no_batch and args.workload == "large":
        batch = bench_batch(ctx, args.batch_steps)

    serve = None
    if not args.no_serve and args.workload == "large":
        serve = bench_serve(ctx, args.serve_requests, args.serve_warmup, args.serve_rho)

    m128 = None
    if not args.no_m128 and args.workload == "large":
        # 2^37-bit operands, a 2^38-bit output and four 2^38-bit workspace
        # buffers: about 192 GiB; the headline line must not depend on it
        free = torch.cuda.mem_get_info()[0]
        if free < (230 << 30):
            m128 = {"skipped": f"needs 230 GiB of free device memory, {free >> 30} GiB free"}
        else:
            try:
                m128 = bench_m128(args.m128_steps)
            except Exception as e:   # reported in the record, not fatal to the headline
                m128 = {"error": f"{type(e).__name__}: {e}"}
                torch.cuda.empty_cache()
        log(f"[bench] m128 record: {'ok' if m128 and 'ms_per_product' in m128 else m128}")

    cpu = None
    if not args.no_cpu:
        log(f"[bench] oracle sample 2^{args.cpu_log2} on the host")
        target = L.bit_length() - 1
        cpu = cpu_baseline(min(args.cpu_log2, target), target)
        log(f"[bench] cpu baseline {cpu}")

    rec = {
        "metric": "ms per 2^30-bit x 2^30-bit product" if args.workload == "large"
        else f"ms per 2^{L.bit_length() - 1}-bit product",
        "value": round(ms, 4), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "ms_per_step_profiled": round(ms_profiled, 4), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (seeded SplitMix64 bits, resident in HBM)",
        "config": {"workload": desc, "len_a": L, "len_b": L, "transform_bits": 1 << log2n,
                   "seed": hex(seed), "field": "GF(2^64)"},
        "roofline": roof,
        "butterfly_rate": bfly_rate,
        "product_roofline": {"nominal_bytes": nominal, "achieved": round(product_gbs, 2), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(product_gbs / HBM_PEAK_GBS, 5)},
        "kernels": per_kernel,
        "batch": batch,
        "serve": serve,
        "m128": m128,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
