#!/usr/bin/env python3
"""Benchmark: ms per product of two 2^30-bit polynomials in GF(2)[x] on one MI355X.

One step = one full product (BasisCvt, Encode, Butterfly for both operands,
pointwise products, iButterfly, Decode, iBasisCvt) with the operands already
resident in HBM.  Prints ONE JSON line on stdout; details go to stderr.

    python bench.py [--steps K] [--warmup W] [--workload large|mid|small] [--no-cpu]

The K timed steps run as a user runs them; then the same K steps run again
with a HIP event pair that the library records around every kernel on its
launch stream (polymul_profile_enable), which gives the per-kernel durations
(those events add about 0.1 ms per product, reported as ms_per_step_profiled).

Byte model (every stage of Alg. 5 streams its input and output once at
natural size; A, B operand bytes, N transform bytes): BasisCvt 2A + 2B,
Encode (A + N) + (B + N), Butterfly 2N per transform (4N for both), pointwise
3N, iButterfly 2N, Decode 2N, iBasisCvt 2N; 3A + 3B + 15N per product.  A
kernel that runs part of a stage is priced at that part's share of the
stage's bytes: a butterfly pass of k of the l layers at k / l of its stage,
and a BasisCvt kernel at the share of the Taylor steps of Alg. 1 it applies
(the superset-sum passes and the final unskew/carry store count the
top-level expansion, the row kernels the inner BasisCvt(2^16), the column
kernels the outer BasisCvt over rows); fused Encode/Decode add their stage.
The `roofline` entry is the kernel with the largest total time, priced so;
`stages` gives the same at stage level and `product_roofline` for the whole
product.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NUM_CU, CLOCK_HZ = 256, 2.4e9            # MI355X: 256 compute units at 2.4 GHz
VALU_LANE_OPS_PEAK = NUM_CU * 64 * CLOCK_HZ   # one wave64 VALU instruction per CU per clock

WORKLOADS = {
    # name: (operand bits, seed, top bit forced, description)
    "small": (1 << 16, 0x5EED0016, False, "single product 2^16 x 2^16 bits, uniform random"),
    "mid": (1 << 24, 0x5EED0024, True, "single product 2^24 x 2^24 bits, uniform random, top bit forced"),
    "large": (1 << 30, 0x5EED0030, False, "single product 2^30 x 2^30 bits, uniform random"),
}


def bcvt_step_count(lg: int) -> int:
    """Number of Taylor steps of BasisCvt(2^lg) in the recursion of Alg. 1
    (tau = 2^(2^k), the largest with tau <= 2^(lg-1); steps for the segment
    lengths 2^lg .. 2 tau; then the outer conversion of 2^lg / tau blocks and
    the inner conversion of tau bits)."""
    if lg <= 1:
        return 0
    lt = 1
    while 2 * lt <= lg - 1:
        lt *= 2
    return (lg - lt) + bcvt_step_count(lg - lt) + bcvt_step_count(lt)


BUTTERFLY_BOTTOM_LAYERS = 7   # layers 0..6 in the bottom pass (transforms of 2^20 values and more)


def kernel_bytes_per_product(A: int, B: int, N: int, log2n: int, la_log2: int) -> dict:
    """Algorithmic bytes per product of each kernel of the fused 2^22..2^31-bit
    schedule, from the stage model in the module docstring."""
    l = log2n - 6
    lb = BUTTERFLY_BOTTOM_LAYERS if l >= 20 else min(l, 11)
    # forward BasisCvt of one 2^la_log2-bit operand: top-level Taylor steps
    # (superset sums over the 2^(la_log2 - 16) rows), outer over rows, inner of 2^16
    lgR_f, lgR_i = max(la_log2 - 16, 0), log2n - 16
    tf, ti = bcvt_step_count(la_log2), bcvt_step_count(log2n)
    top_f, out_f, in_f = la_log2 - 16, bcvt_step_count(lgR_f), bcvt_step_count(16)
    top_i, out_i, in_i = log2n - 16, bcvt_step_count(lgR_i), bcvt_step_count(16)
    assert top_f + out_f + in_f == tf and top_i + out_i + in_i == ti
    bc_f, bc_i = 2 * A + 2 * B, 2 * N
    return {
        "basiscvt_zeta": bc_f * top_f / tf,
        "basiscvt_rows": bc_f * in_f / tf,
        "basiscvt_outer_encode": bc_f * out_f / tf + (A + N) + (B + N),
        "butterfly_upper": 4 * N * (l - lb) / l,
        "butterfly_bottom": 4 * N * lb / l,
        "pointwise": 3 * N,
        "ibutterfly_bottom": 2 * N * lb / l,
        "ibutterfly_upper": 2 * N * (l - lb) / l,
        "decode_outer": 2 * N + bc_i * out_i / ti,
        "ibasiscvt_rows": bc_i * in_i / ti,
        # the top-level inverse expansion: superset-sum passes plus the store (unskew, carry)
        "ibasiscvt_zeta+ibasiscvt_store": bc_i * top_i / ti,
    }


STAGES = [
    # (stage, kernels, nominal bytes from (A, B, N))
    ("BasisCvt + Encode (A and B)", ("basiscvt_zeta", "basiscvt_rows", "basiscvt_outer_encode"),
     lambda A, B, N: 3 * A + 3 * B + 2 * N),
    ("Butterfly (A and B)", ("butterfly_upper", "butterfly_bottom"), lambda A, B, N: 4 * N),
    ("Pointwise", ("pointwise",), lambda A, B, N: 3 * N),
    ("iButterfly", ("ibutterfly_bottom", "ibutterfly_upper"), lambda A, B, N: 2 * N),
    ("Decode + iBasisCvt", ("decode_outer", "ibasiscvt_rows", "ibasiscvt_zeta", "ibasiscvt_store"),
     lambda A, B, N: 4 * N),
]

# Counters per dispatch measured with rocprofv3 on the 2^30 x 2^30-bit product
# (profiles/), and applied to that workload only: FETCH_SIZE and WRITE_SIZE in KiB, each scaled by what the
# counter reads for a plain 1 GiB device copy (fetch x2.000, write x1.000), and
# SQ_INSTS_VALU (wave instructions summed over the chip).  They hold only for
# the kernel sources they were taken on: the sha256 of the listed files must
# match, else the bench reports them as null.
COUNTER_SOURCES = ("paper_1803_11301_amd/csrc/fpmul.hip", "paper_1803_11301_amd/csrc/k_basiscvt.h",
                   "paper_1803_11301_amd/csrc/k_bf3.h", "paper_1803_11301_amd/csrc/k_bf2.h",
                   "paper_1803_11301_amd/csrc/gf_device.h")
COUNTERS_SHA256 = "0fa576d8b43d28be870b1854605f1dd2fcd8ac5fa926cb80bbc653e39e3b076e"
COUNTERS = {
    # kernel: (FETCH_SIZE KiB, WRITE_SIZE KiB, SQ_INSTS_VALU) per dispatch
    "basiscvt_zeta": (213081, 327680, 2.715e+07),
    "basiscvt_rows": (151725, 262144, 1.181e+08),
    "basiscvt_outer_encode": (131399, 524288, 1.463e+08),
    "butterfly_upper": (262514, 524288, 1.475e+08),
    "butterfly_bottom": (262606, 524288, 3.087e+08),
    "pointwise": (262769, 262144, 1.05e+08),
    "ibutterfly_bottom": (131478, 262144, 1.529e+08),
    "ibutterfly_upper": (131371, 262144, 7.336e+07),
    "decode_outer": (131472, 262144, 1.41e+08),
    "ibasiscvt_rows": (132739, 393216, 1.139e+08),
    "ibasiscvt_zeta": (196694, 393216, 2.047e+07),
    "ibasiscvt_store": (168391, 262144, 1.91e+07),
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def sources_sha256(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counters_current() -> bool:
    return COUNTERS_SHA256 is not None and sources_sha256(COUNTER_SOURCES) == COUNTERS_SHA256


def measured_traffic(kernel: str):
    """HBM bytes per dispatch from the committed counters, or None."""
    if not counters_current() or kernel not in COUNTERS:
        return None
    f, w, _ = COUNTERS[kernel]
    return int((f * FETCH_SCALE + w * WRITE_SCALE) * 1024)


def valu_utilisation(kernel: str, avg_launch_s: float):
    """VALU busy fraction of the chip over a launch: wave64 VALU instructions
    (SQ_INSTS_VALU) x 64 lanes / (launch time x 256 CUs x 64 lanes x 2.4 GHz)."""
    if not counters_current() or kernel not in COUNTERS or avg_launch_s <= 0:
        return None
    return COUNTERS[kernel][2] * 64 / (avg_launch_s * VALU_LANE_OPS_PEAK)


def nominal_bytes(A: int, B: int, N: int) -> int:
    """Nominal algorithmic bytes of one product: each stage of Alg. 5 streams its
    input and output once (BasisCvt 2A+2B, Encode A+B+2N, Butterfly 4N,
    pointwise 3N, iButterfly 2N, Decode 2N, iBasisCvt 2N) = 3A + 3B + 15N."""
    return 3 * A + 3 * B + 15 * N


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu() -> dict:
    """CPU model and core counts of the host the oracle runs on."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


# One full-size oracle run on the host of an MI355X machine: `python bench.py --cpu-full`
# (profiles/cpu_oracle_2e30x2e30.md holds its output); the default bench run
# times the bounded sample below and reports this measurement beside it.
CPU_FULL_MEASURED = {"ms": 104283.2, "threads": 16, "cpu_model": "AMD EPYC", "nproc": 16,
                     "matches_stored_digest": True, "record": "profiles/cpu_oracle_2e30x2e30.md"}


def cpu_baseline(log2_len: int, target_log2: int):
    """The oracle (as it stands) on a bounded sample of the same workload: one
    product of 2^log2_len-bit operands from the same generator, on all host
    threads, scaled to 2^target_log2-bit operands by the 3x-per-doubling cost
    of its Karatsuba recursion; beside it the one measured full-size run."""
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
    cpu = host_cpu()
    return {"value": round(sec * 1e3 * scale, 3), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"one 2^{log2_len} x 2^{log2_len}-bit product of the same generator (seed 0x5eed0030) "
                      f"took {sec:.2f} s on {threads} threads; value = that x 3^{target_log2 - log2_len} "
                      f"(Karatsuba: 3x per doubling) for 2^{target_log2}-bit operands",
            "sample_s": round(sec, 3), "cpu_model": cpu["model"], "nproc": cpu["nproc"],
            "usable_cpus": cpu["usable_cpus"], "full_size_measured": CPU_FULL_MEASURED}


def cpu_full(log2_len: int = 30):
    """Time the oracle once on the whole 2^30 x 2^30-bit workload on all host
    threads, and check its output against the stored oracle digest."""
    import numpy as np
    import oracle as O
    from paper_1803_11301_amd import synth
    O.build(force=False)
    L = 1 << log2_len
    a, b = synth.single_pair(synth.SEED_LARGE, L)
    threads = O.max_threads()
    log(f"[bench] oracle 2^{log2_len} x 2^{log2_len} on {threads} threads")
    t0 = time.perf_counter()
    c = O.polymul(a, L, b, L, threads=threads)
    sec = time.perf_counter() - t0
    digest = hashlib.sha256(np.ascontiguousarray(c, dtype="<u8").tobytes()).hexdigest()
    want = None
    gpath = os.path.join(ROOT, "tests", "golden", "digests.json")
    if log2_len == 30 and os.path.exists(gpath):
        with open(gpath) as f:
            want = json.load(f)["large"]["sha256"]
    rec = {"kind": "oracle", "workload": f"single product 2^{log2_len} x 2^{log2_len} bits, seed 0x5eed0030",
           "seconds": round(sec, 2), "ms": round(sec * 1e3, 1), "threads": threads, **host_cpu(),
           "sha256": digest, "matches_stored_digest": None if want is None else digest == want}
    return rec


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


SAT_BURSTS = 3   # bursts behind each saturated rate (their median)
SERVE_TUNE_REQUESTS = 2000
SERVE_TUNE_P99_MS = 2.5


def bench_serve_tune(ctx):
    """The server settings for the serving measurement, chosen by tune_server
    on a mix of SERVE_TUNE_REQUESTS requests of the serving distribution
    (operands log-uniform in [2^12, 2^24] bits, its own seed): the highest
    saturated rate whose p99 at 0.8 of it stays within SERVE_TUNE_P99_MS."""
    from paper_1803_11301_amd import synth
    from paper_1803_11301_amd.serve_tune import tune_server
    _, la, lb, _, _ = synth.serve_plan(SERVE_TUNE_REQUESTS, 1.0, seed=synth.SEED_SERVE + 7)
    t0 = time.perf_counter()
    res = tune_server(ctx, la, lb, rho=0.8, p99_limit_ms=SERVE_TUNE_P99_MS)
    res["seconds"] = round(time.perf_counter() - t0, 2)
    for r in res["table"]:
        log(f"[bench] serve tune: slots {r['slots']} limit 2^{r['batch_limit_bits'].bit_length() - 1} "
            f"max batch {r['max_batch']}: saturated {r['saturated_per_s']:.0f}/s, p50 {r['p50_ms']} ms, "
            f"p99 {r['p99_ms']} ms")
    c = res["choice"]
    log(f"[bench] serve tune: chose slots {c['slots']}, batch limit {c['batch_limit_bits']} bits, "
        f"max batch {c['max_batch']} ({res['seconds']} s)")
    return res


def bench_serve(ctx, count: int, warmup: int, rhos, sat_count: int, slots: int = 8,
                batch_limit_bits: int = 1 << 20, max_batch: int = 512):
    """Poisson stream of products, operands log-uniform in [2^12, 2^24] bits
    (seed 0x5EED05E5), through the continuous-batching server.  First the
    saturated throughput X: the median rate of SAT_BURSTS bursts of the same
    sat_count requests, each submitted at once (one burst alone varied by
    up to 15% from run to run, and the loads below are fractions of X).  Then for
    each offered load rho: `warmup` requests, then `count` timed requests,
    arriving open loop at rate rho * X; latency = submit to completion as the
    server sees it."""
    import numpy as np
    import torch
    from paper_1803_11301_amd import fpmul, synth
    per = warmup + count
    total = sat_count + len(rhos) * per
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
    # outputs of one phase at a time (the phases run one after the other)
    phase_words = max(int(ow[:sat_count].sum()),
                      max(int(ow[sat_count + k * per: sat_count + (k + 1) * per].sum()) for k in range(len(rhos))))
    out = torch.empty(phase_words, dtype=torch.int64, device="cuda")
    ab, bb, ob = pa.data_ptr(), pb.data_ptr(), out.data_ptr()

    def args_for(lo, hi):
        o = 0
        res = []
        for k in range(lo, hi):
            res.append((ab + 8 * int(offa[k]), int(la[k]), bb + 8 * int(offb[k]), int(lb[k]), ob + 8 * o))
            o += int(ow[k])
        return res

    torch.cuda.synchronize()
    srv = fpmul.Server(ctx, hbm_budget=8 << 30, slots=slots, batch_limit_bits=batch_limit_bits, max_batch=max_batch)
    sat = args_for(0, sat_count)
    rates = []
    for _ in range(SAT_BURSTS):
        t0 = time.perf_counter()
        tks = [srv.submit(*x) for x in sat]
        for tk in tks:
            srv.wait(tk)
        rates.append(sat_count / (time.perf_counter() - t0))
    X = float(np.median(rates))
    log(f"[bench] serve: saturated {X:.0f}/s over {sat_count} requests submitted at once "
        f"(median of {SAT_BURSTS} bursts: {', '.join(f'{r:.0f}' for r in rates)})")
    rows = []
    for k, rho in enumerate(rhos):
        lo = sat_count + k * per
        reqs = args_for(lo, lo + per)
        rate = rho * X
        arr = synth.serve_plan(per, rate)[0]
        tks = []
        t0 = time.perf_counter()
        t_meas = None
        for j in range(per):
            due = t0 + float(arr[j])
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                if due - now > 2e-4:
                    time.sleep((due - now) - 1e-4)
            if j == warmup:
                t_meas = time.perf_counter()
            tks.append(srv.submit(*reqs[j]))
        # wait releases each ticket and returns its (submit, launch, done) times
        done = [srv.wait(tk) for tk in tks]
        wall = time.perf_counter() - (t_meas if t_meas is not None else t0)
        tm = done[warmup:]
        lat = np.array([(d - s0) / 1e6 for s0, st, d in tm])
        queue = np.array([(st - s0) / 1e6 for s0, st, d in tm])
        row = {"rho": rho, "offered_per_s": round(rate, 1), "achieved_products_per_s": round(count / wall, 1),
               "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "mean_ms": round(float(lat.mean()), 3), "p99_queue_ms": round(float(np.percentile(queue, 99)), 3)}
        rows.append(row)
        log(f"[bench] serve: rho {rho:.2f}: offered {rate:.0f}/s, achieved {row['achieved_products_per_s']:.0f}/s, "
            f"p50 {row['p50_ms']} ms, p99 {row['p99_ms']} ms")
    srv.close()
    return {"workload": "Poisson stream, operands log-uniform 2^12..2^24 bits, seed 0x5eed05e5",
            "requests_per_load": count, "warmup_per_load": warmup, "saturation_requests": sat_count,
            "saturated_products_per_s": round(X, 1), "saturation_bursts": [round(r, 1) for r in rates],
            "loads": rows, "slots": slots,
            "batch_limit_bits": batch_limit_bits, "max_batch": max_batch, "hbm_budget_bytes": 8 << 30}


def bench_serve_resident(ctx, count: int, warmup: int, rho: float, sat_count: int, n_res: int = 4,
                         la: int = 1 << 20, max_bits: int = 1 << 22, slots: int = 8):
    """Transform reuse in serving: every request multiplies one of n_res
    operands of la bits (seed 0x5EED05E6 + k) by a B of log-uniform 2^12 ..
    2^21 bits, submitted once as ordinary products (polymul_submit) and once
    on the operands kept as forward transforms of max_bits bits
    (polymul_submit_resident).  For each: the saturated rate over sat_count
    requests submitted at once (median of SAT_BURSTS bursts), then count timed
    requests (after warmup)
    arriving open loop at rho times that rate; p50/p99 latency."""
    import numpy as np
    import torch
    from paper_1803_11301_amd import fpmul, synth
    rng = np.random.default_rng(0x5EED05E6)
    total = sat_count + warmup + count
    lbs = np.floor(np.exp2(12 + 9 * rng.random(total))).astype(np.int64)
    which = rng.integers(0, n_res, total)
    A = [torch.from_numpy(synth.dense_poly(0x5EED05E6 + k, la).view(np.int64)).cuda() for k in range(n_res)]
    pool_bits = 1 << 22
    pb = torch.from_numpy(synth.dense_poly(0x5EED05F0, pool_bits).view(np.int64)).cuda()
    pw = pool_bits // 64
    offb = rng.integers(0, pw - (1 << 21) // 64, total)
    ow = (la + lbs - 1 + 63) // 64
    outs = torch.empty(int(ow.sum()), dtype=torch.int64, device="cuda")
    ooff = np.concatenate([[0], np.cumsum(ow)[:-1]])
    res = [fpmul.Resident(ctx, A[k], la, max_bits) for k in range(n_res)]
    torch.cuda.synchronize()
    rows = {}
    for mode in ("plain", "resident"):
        srv = fpmul.Server(ctx, hbm_budget=8 << 30, slots=slots)

        def submit(j):
            b = pb.data_ptr() + 8 * int(offb[j])
            o = outs.data_ptr() + 8 * int(ooff[j])
            k = int(which[j])
            if mode == "resident":
                return srv.submit_resident(res[k], b, int(lbs[j]), o)
            return srv.submit(A[k].data_ptr(), la, b, int(lbs[j]), o)
        rates = []
        for _ in range(SAT_BURSTS):
            t0 = time.perf_counter()
            tks = [submit(j) for j in range(sat_count)]
            for tk in tks:
                srv.wait(tk)
            rates.append(sat_count / (time.perf_counter() - t0))
        X = float(np.median(rates))
        rate = rho * X
        arr = synth.serve_plan(warmup + count, rate)[0]
        tks = []
        t0 = time.perf_counter()
        t_meas = None
        for j in range(warmup + count):
            due = t0 + float(arr[j])
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                if due - now > 2e-4:
                    time.sleep((due - now) - 1e-4)
            if j == warmup:
                t_meas = time.perf_counter()
            tks.append(submit(sat_count + j))
        done = [srv.wait(tk) for tk in tks]
        wall = time.perf_counter() - t_meas
        lat = np.array([(d - s0) / 1e6 for s0, st, d in done[warmup:]])
        rows[mode] = {"saturated_products_per_s": round(X, 1), "saturation_bursts": [round(r, 1) for r in rates],
                      "rho": rho, "offered_per_s": round(rate, 1),
                      "achieved_products_per_s": round(count / wall, 1),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        log(f"[bench] serve {mode}: saturated {X:.0f}/s; rho {rho}: p50 {rows[mode]['p50_ms']} ms, "
            f"p99 {rows[mode]['p99_ms']} ms")
        srv.close()
    for r in res:
        r.close()
    return {"workload": f"{n_res} operands of {la} bits x B log-uniform 2^12..2^21 bits, seed 0x5eed05e6",
            "resident_transform_bits": max_bits, "requests": count, "warmup": warmup,
            "saturation_requests": sat_count, **rows}


def bench_latency(ctx, names=("small", "mid"), runs=(100, 20)):
    """Latency of single products: the median over `runs` products of the
    time between HIP events recorded before and after each polymul_ex call
    on the stream (operands resident), and the same for a replay of the
    product's captured launch chain (polymul_graph_launch)."""
    import numpy as np
    import torch
    from paper_1803_11301_amd import fpmul, synth
    res = {}
    stream = torch.cuda.current_stream()
    for name, nrun in zip(names, runs):
        L, seed, top, desc = WORKLOADS[name]
        a_np, b_np = synth.single_pair(seed, L, top_bit=top)
        a = torch.from_numpy(a_np.view(np.int64)).cuda()
        b = torch.from_numpy(b_np.view(np.int64)).cuda()
        out = torch.empty(((2 * L - 1) + 63) // 64, dtype=torch.int64, device="cuda")
        for _ in range(3):
            ctx.polymul(a, L, b, L, out=out, stream=stream)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nrun)]
        for e0, e1 in ev:
            e0.record(stream)
            ctx.polymul(a, L, b, L, out=out, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
        res[name] = {"workload": desc, "runs": nrun, "median_ms": round(float(np.median(ms)), 4),
                     "p10_ms": round(float(np.percentile(ms, 10)), 4),
                     "p90_ms": round(float(np.percentile(ms, 90)), 4)}
        # the same product replayed from its captured launch chain
        g = fpmul.Graph.product(ctx, a, L, b, L, out)
        for _ in range(3):
            g.launch(stream)
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record(stream)
            g.launch(stream)
            e1.record(stream)
        torch.cuda.synchronize()
        gms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
        g.close()
        res[name].update({"graph_median_ms": round(float(np.median(gms)), 4),
                          "graph_p90_ms": round(float(np.percentile(gms, 90)), 4)})
        log(f"[bench] latency {name}: median {res[name]['median_ms']} ms over {nrun} products, "
            f"{res[name]['graph_median_ms']} ms replayed from the captured graph")
    return res


def kernel_table(prof: dict, steps: int, A: int, B: int, N: int, log2n: int, la_log2: int, fused: bool,
                 counters_apply: bool = True):
    """Per-kernel times with their algorithmic bytes, achieved rate, measured
    traffic and VALU utilisation (the stored counters: only for the workload
    they were taken on, counters_apply); and the dominant kernel's roofline
    entry."""
    kb = kernel_bytes_per_product(A, B, N, log2n, la_log2) if fused else {}
    per_kernel = {}
    for name, (cnt, tot) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        avg_s = tot / cnt / 1e3
        rec = {"launches_per_step": cnt / steps, "ms_per_step": round(tot / steps, 4),
               "avg_launch_us": round(avg_s * 1e6, 2)}
        key = name if name in kb else next((k for k in kb if name in k.split("+")), None)
        if key is not None:
            # launches of every kernel that shares this part of the stage
            share = sum(prof[k][0] for k in key.split("+") if k in prof) / steps
            per_launch = kb[key] / share
            rec["algorithmic_bytes_per_launch"] = int(per_launch)
            rec["achieved_GBs"] = round(per_launch / avg_s / 1e9, 1)
            rec["hbm_frac"] = round(per_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4)
            t = measured_traffic(name) if counters_apply else None
            rec["traffic_bytes_per_launch"] = t
            rec["traffic_over_algorithmic"] = None if t is None else round(t / per_launch, 3)
        v = valu_utilisation(name, avg_s) if counters_apply else None
        rec["valu_utilisation"] = None if v is None else round(v, 3)
        per_kernel[name] = rec
        log(f"[bench] {name:26s} {cnt / steps:6.1f} launches/step {tot / steps:9.4f} ms/step "
            f"{avg_s * 1e6:9.2f} us/launch" + (f"  {rec['achieved_GBs']:8.1f} GB/s algorithmic"
                                               if "achieved_GBs" in rec else ""))
    known = [n for n in per_kernel if "algorithmic_bytes_per_launch" in per_kernel[n]]
    roof = None
    if known:
        dom = max(known, key=lambda n: prof[n][1])
        r = per_kernel[dom]
        roof = {"bound": "hbm", "kernel": dom, "achieved": r["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": r["hbm_frac"], "traffic": r["traffic_bytes_per_launch"],
                "bytes_per_launch": r["algorithmic_bytes_per_launch"], "avg_launch_us": r["avg_launch_us"],
                "traffic_over_algorithmic": r["traffic_over_algorithmic"], "valu_utilisation": r["valu_utilisation"],
                "bytes_model": "share of its stage's nominal bytes (3A+3B+15N per product): a pass of k of the l "
                               "butterfly layers is k/l of the stage's 2N per transform"}
    stages = []
    if fused:
        for stage, kernels, fn in STAGES:
            ks = [k for k in kernels if k in prof]
            if not ks:
                continue
            ms = sum(prof[k][1] for k in ks) / steps
            nb = fn(A, B, N)
            tr = [measured_traffic(k) if counters_apply else None for k in ks]
            traffic = None if any(t is None for t in tr) else sum(t * prof[k][0] / steps for t, k in zip(tr, ks))
            stages.append({"stage": stage, "kernels": ks, "ms_per_product": round(ms, 4), "nominal_bytes": nb,
                           "achieved_GBs": round(nb / (ms / 1e3) / 1e9, 1),
                           "hbm_frac": round(nb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                           "traffic_bytes": None if traffic is None else int(traffic)})
    return per_kernel, roof, stages


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--cpu-log2", type=int, default=28, help="operand size of the oracle sample")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the oracle once on the whole 2^30 x 2^30-bit workload (no GPU)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-products measurement")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=10000, help="timed requests per offered load")
    ap.add_argument("--serve-warmup", type=int, default=500, help="untimed requests before them")
    ap.add_argument("--serve-rhos", default="0.5,0.8,0.95", help="offered loads as fractions of saturation")
    ap.add_argument("--serve-saturation", type=int, default=4000, help="requests submitted at once for X")
    ap.add_argument("--no-resident", action="store_true", help="skip the transform-reuse serving measurement")
    ap.add_argument("--no-serve-tune", action="store_true",
                    help="serve with the server's default settings (no tune_server first)")
    ap.add_argument("--no-tune", action="store_true", help="time the default schedule (no polymul_tune first)")
    ap.add_argument("--tune-reps", type=int, default=3, help="timed products per schedule choice of the tuner")
    ap.add_argument("--tune-cache", default=None,
                    help="schedule cache: load the line for this transform length if present, else tune and append")
    ap.add_argument("--no-latency", action="store_true", help="skip the 2^16 and 2^24 latency lines")
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

    if args.cpu_full:
        print(json.dumps(cpu_full()), flush=True)
        return

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

    lc0 = 2 * L - 1
    log2n0 = max(6, (lc0 - 1).bit_length())
    tune = None
    if not args.no_tune and 22 <= log2n0 <= 31:
        # the schedule the tuner picks for this transform length (layer split
        # of the upper butterfly passes, row and zeta grids), as a user would
        # run after tuning once
        loaded = False
        if args.tune_cache and os.path.exists(args.tune_cache):
            ctx.tune_load(args.tune_cache)
            # applied when the context now uses the cache's last line for this length
            mine = ctx.schedule(log2n0).split()
            want = [ln.split() for ln in open(args.tune_cache) if ln.split()[:3] == mine[:3]]
            loaded = bool(want) and want[-1][3:6] == mine[3:6]
        if loaded:
            tune = {"log2n": log2n0, "loaded_from": args.tune_cache, "schedule": ctx.schedule(log2n0)}
            log(f"[bench] schedule loaded: {tune['schedule']}")
        else:
            t0 = time.perf_counter()
            rep = ctx.tune(log2n0, reps=args.tune_reps, cache_path=args.tune_cache)
            fields = dict(kv.split("=", 1) for kv in rep.replace("|", " ").split() if "=" in kv)
            tune = {"log2n": log2n0, "seconds": round(time.perf_counter() - t0, 2),
                    "default_ms": float(fields.get("default_ms", "nan")),
                    "tuned_ms": float(fields.get("tuned_ms", "nan")),
                    "tried": int(fields.get("tried", "0")), "schedule": ctx.schedule(log2n0)}
            log(f"[bench] tuned: {rep}")

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

    A = B = L // 8
    log2n = max(6, (lc - 1).bit_length())
    N = (1 << log2n) // 8
    nominal = nominal_bytes(A, B, N)
    fused = 22 <= log2n <= 31
    per_kernel, roof, stages = kernel_table(prof, args.steps, A, B, N, log2n, L.bit_length() - 1, fused,
                                            counters_apply=args.workload == "large")
    # multiplications by constants in the butterfly kernels: (l/2) n_p per
    # transform, three transforms; their rate per CU per clock
    bfly = [n for n in prof if "butterfly" in n]
    bfly_ms = sum(prof[n][1] for n in bfly) / args.steps
    l = log2n - 6
    mults = 3 * (l * (1 << l) // 2)
    bfly_rate = None
    if bfly_ms > 0:
        bfly_rate = {"multiplications_per_product": mults, "ms_per_product": round(bfly_ms, 4),
                     "per_cu_per_clock": round(mults / (bfly_ms / 1e3) / (NUM_CU * CLOCK_HZ), 3),
                     "lookups_per_multiplication": 8}
    product_gbs = nominal / (ms / 1e3) / 1e9
    log(f"[bench] {ms:.3f} ms/product ({ms_profiled:.3f} with per-kernel events); nominal {nominal / 1e9:.3f} GB -> "
        f"{product_gbs:.1f} GB/s ({100 * product_gbs / HBM_PEAK_GBS:.1f}% of HBM peak)")

    latency = None
    if not args.no_latency and args.workload == "large":
        latency = bench_latency(ctx)

    batch = None
    if not args.no_batch and args.workload == "large":
        batch = bench_batch(ctx, args.batch_steps)

    serve = serve_tune = None
    if not args.no_serve and args.workload == "large":
        rhos = [float(x) for x in args.serve_rhos.split(",") if x]
        slots, limit, max_batch = 8, 1 << 20, 512   # the server's defaults
        if not args.no_serve_tune:
            serve_tune = bench_serve_tune(ctx)
            c = serve_tune["choice"]
            slots, limit, max_batch = c["slots"], c["batch_limit_bits"], c["max_batch"]
        serve = bench_serve(ctx, args.serve_requests, args.serve_warmup, rhos, args.serve_saturation, slots=slots,
                            batch_limit_bits=limit, max_batch=max_batch)

    serve_resident = None
    if not args.no_serve and not args.no_resident and args.workload == "large":
        serve_resident = bench_serve_resident(ctx, 5000, 500, 0.8, 2000)

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
        target = L.bit_length() - 1
        log(f"[bench] oracle sample 2^{min(args.cpu_log2, target)} on the host")
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
        "product_roofline": {"nominal_bytes": nominal, "achieved": round(product_gbs, 2), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(product_gbs / HBM_PEAK_GBS, 5),
                             "target_frac": 0.5, "ms_at_target": round(nominal / (0.5 * HBM_PEAK_GBS * 1e9) * 1e3, 4)},
        "stages": stages,
        "butterfly_rate": bfly_rate,
        "counters_current": counters_current(),
        "kernels": per_kernel,
        "latency": latency,
        "batch": batch,
        "serve": serve,
        "serve_tune": serve_tune,
        "serve_resident": serve_resident,
        "tune": tune,
        "m128": m128,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
