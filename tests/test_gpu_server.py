"""GPU tests of the continuous-batching product server.

Each product computed in a mix of concurrent requests must equal the same
product computed alone (polymul_ex) and the oracle; memory admission must
serialise requests when the budget is tight and refuse a request larger than
the whole budget.
"""
import random
import sys

import numpy as np
import pytest

import oracle as O
from paper_1803_11301_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_11301_amd import fpmul
    c = fpmul.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev64(arr):
    a = np.ascontiguousarray(arr, dtype=np.uint64)
    if a.size == 0:
        a = np.zeros(1, np.uint64)
    return torch.from_numpy(a.view(np.int64)).cuda()


def host(t, n):
    return t.cpu().numpy().view(np.uint64)[:n]


def check_against_oracle(a, la, b, lb, got, rng):
    n = O.nwords(la + lb - 1)
    if la <= (1 << 16) and lb <= (1 << 16):
        assert np.array_equal(got, O.polymul(a, la, b, lb))
        return
    idx = np.array(sorted({0, n - 1, n // 2} | {rng.randrange(n) for _ in range(5)}), dtype=np.uint64)
    assert np.array_equal(got[idx.astype(np.int64)], O.product_words(a, la, b, lb, idx))
    z = rng.getrandbits(64) | 1
    assert O.gf64_mul(O.eval_at(a, la, z), O.eval_at(b, lb, z)) == O.eval_at(got, la + lb - 1, z)


def test_mix_equals_alone_and_oracle(ctx):
    from paper_1803_11301_amd import fpmul
    t, la, lb, sa, sb = synth.serve_plan(48, 1000.0, lo=12, hi=22)
    lens = list(zip(la.tolist(), lb.tolist()))
    lens += [(1 << 23, 1 << 23), ((1 << 24) - 3, 1 << 22), (1, 1 << 20), (5, 5)]
    say("server mix", len(lens), "requests, largest", max(x + y for x, y in lens))
    rng = random.Random(99)
    ops = []
    for k, (x, y) in enumerate(lens):
        a = synth.dense_poly(int(sa[k % len(sa)]) + k, x)
        b = synth.dense_poly(int(sb[k % len(sb)]) + k, y)
        ops.append((a, x, b, y))
    srv = fpmul.Server(ctx, hbm_budget=2 << 30, slots=4)
    tensors, tickets = [], []
    for a, x, b, y in ops:
        ta, tb = dev64(a), dev64(b)
        out = torch.zeros(O.nwords(x + y - 1), dtype=torch.int64, device="cuda")
        tensors.append((ta, tb, out))
    torch.cuda.synchronize()
    for (a, x, b, y), (ta, tb, out) in zip(ops, tensors):
        tickets.append(srv.submit(ta, x, tb, y, out))
    for tk in tickets:
        s, st, d = srv.wait(tk)
        assert s <= st <= d
    assert srv.outstanding() == 0
    srv.close()
    for (a, x, b, y), (ta, tb, out) in zip(ops, tensors):
        n = O.nwords(x + y - 1)
        got = host(out, n)
        alone = host(ctx.polymul(ta, x, tb, y), n)
        assert np.array_equal(got, alone), (x, y)
        check_against_oracle(a, x, b, y, got, rng)


def test_tight_budget_serialises_and_refuses_too_large(ctx):
    from paper_1803_11301_amd import fpmul
    rng = random.Random(3)
    # 64 MiB holds one 2^24 x 2^24-bit product's workspace (about 18 MiB) at a time with room
    # for small batches, but not a 2^28-bit product
    srv = fpmul.Server(ctx, hbm_budget=64 << 20, slots=3)
    lens = [(1 << 24, 1 << 24), (3000, 4000), (1 << 24, (1 << 24) - 1), (100, 100), (1 << 23, 1 << 23)]
    say("tight budget", lens)
    ops, tickets = [], []
    for k, (x, y) in enumerate(lens):
        a, b = synth.dense_poly(0x5EED7000 + 2 * k, x), synth.dense_poly(0x5EED7001 + 2 * k, y)
        ta, tb = dev64(a), dev64(b)
        out = torch.zeros(O.nwords(x + y - 1), dtype=torch.int64, device="cuda")
        ops.append((a, x, b, y, ta, tb, out))
    torch.cuda.synchronize()
    for a, x, b, y, ta, tb, out in ops:
        tickets.append(srv.submit(ta, x, tb, y, out))
    big = 1 << 28
    tbig = torch.zeros(O.nwords(big), dtype=torch.int64, device="cuda")
    obig = torch.zeros(O.nwords(2 * big), dtype=torch.int64, device="cuda")
    with pytest.raises(fpmul.FpmulError) as ei:
        srv.submit(tbig, big, tbig, big, obig)
    assert ei.value.code == fpmul.ENOMEM
    for tk in tickets:
        srv.wait(tk)
        with pytest.raises(fpmul.FpmulError):   # released by wait
            srv.poll(tk)
    srv.close()
    for a, x, b, y, ta, tb, out in ops:
        check_against_oracle(a, x, b, y, host(out, O.nwords(x + y - 1)), rng)


def test_empty_and_errors(ctx):
    from paper_1803_11301_amd import fpmul
    srv = fpmul.Server(ctx, hbm_budget=16 << 20, slots=1)
    t = torch.zeros(4, dtype=torch.int64, device="cuda")
    o = torch.full((4,), 7, dtype=torch.int64, device="cuda")
    tk = srv.submit(t, 0, t, 100, o)
    assert srv.poll(tk)
    srv.wait(tk)
    assert int(o[0].item()) == 7
    with pytest.raises(fpmul.FpmulError):
        srv.submit(t, 64, t, 64, t)          # out overlaps the inputs
    with pytest.raises(fpmul.FpmulError):
        srv.wait(123456789)                  # unknown ticket
    srv.close()


@pytest.mark.parametrize("limit,max_batch", [(0, 1), (1 << 22, 4096), (1 << 16, 3)])
def test_policy_changes_routing_not_results(ctx, limit, max_batch):
    from paper_1803_11301_amd import fpmul
    lens = [(1000, 3000), (1 << 15, 1 << 15), (1 << 19, 1 << 19), ((1 << 21) - 7, 1 << 20), (64, 64), (65, 1)]
    lens += [(200 + 97 * k, 5000 - 131 * k) for k in range(12)]
    say("policy", limit, max_batch, len(lens), "requests")
    ops = []
    for k, (x, y) in enumerate(lens):
        a, b = synth.dense_poly(0x9011C700 + 2 * k, x), synth.dense_poly(0x9011C701 + 2 * k, y)
        out = torch.zeros(O.nwords(x + y - 1), dtype=torch.int64, device="cuda")
        ops.append((a, x, b, y, dev64(a), dev64(b), out))
    torch.cuda.synchronize()
    srv = fpmul.Server(ctx, hbm_budget=1 << 30, slots=3, batch_limit_bits=limit, max_batch=max_batch)
    tickets = [srv.submit(ta, x, tb, y, out) for a, x, b, y, ta, tb, out in ops]
    with pytest.raises(fpmul.FpmulError):
        fpmul._check(fpmul.lib().polymul_server_set_policy(srv.handle, 1 << 20, 512))
    for tk in tickets:
        srv.wait(tk)
    srv.close()
    rng = random.Random(limit + max_batch)
    for a, x, b, y, ta, tb, out in ops:
        n = O.nwords(x + y - 1)
        got = host(out, n)
        assert np.array_equal(got, host(ctx.polymul(ta, x, tb, y), n)), (x, y)
        check_against_oracle(a, x, b, y, got, rng)


def test_policy_rejects_out_of_range(ctx):
    from paper_1803_11301_amd import fpmul
    for limit, mb in [((1 << 22) + 1, 16), (1 << 20, 0), (1 << 20, 4097)]:
        with pytest.raises(fpmul.FpmulError):
            fpmul.Server(ctx, hbm_budget=16 << 20, slots=1, batch_limit_bits=limit, max_batch=mb)


def test_tickets_are_released_by_wait(ctx):
    """A long run of tickets (empty products, done at submit, and small real
    ones) leaves nothing behind: every wait releases its ticket, after which
    the ticket is unknown; polling keeps a ticket until its wait."""
    from paper_1803_11301_amd import fpmul
    srv = fpmul.Server(ctx, hbm_budget=64 << 20, slots=2)
    say("ticket release, 5000 tickets")
    t = torch.zeros(64, dtype=torch.int64, device="cuda")
    outs = [torch.zeros(4, dtype=torch.int64, device="cuda") for _ in range(16)]
    for rnd in range(250):
        tks = [srv.submit(t, 0, t, 100, outs[0]) for _ in range(12)]
        tks += [srv.submit(t[:2], 100, t[2:4], 90, outs[1 + k]) for k in range(8)]
        assert srv.outstanding() == 20
        srv.poll(tks[0])
        for tk in tks:
            srv.wait(tk)
        assert srv.outstanding() == 0
    with pytest.raises(fpmul.FpmulError):
        srv.wait(tks[-1])
    with pytest.raises(fpmul.FpmulError):
        srv.times(tks[-1])
    srv.close()


def test_resident_operand_in_the_mix(ctx):
    # transform reuse (f2): one operand kept on the device as its forward
    # transform, multiplied by many B inside a mix of ordinary requests; every
    # product equals the same product computed alone (polymul_ex) and the oracle
    from paper_1803_11301_amd import fpmul
    la = (1 << 20) + 333
    say("resident operand", la, "bits in a server mix")
    rng = random.Random(5150)
    a = synth.dense_poly(0x5EED2000, la)
    ta = dev64(a)
    res = fpmul.Resident(ctx, ta, la, 1 << 22)          # transforms of 2^22 bits
    srv = fpmul.Server(ctx, hbm_budget=1 << 30, slots=4)
    try:
        jobs = []
        for k in range(24):
            lb = [1, 63, 64, 4097, (1 << 16) + 5, (1 << 20) - 1, (1 << 21) + 7][k % 7]
            lb = min(lb, (1 << 22) + 1 - la)
            b = synth.dense_poly(0x5EED2100 + k, lb)
            tb = dev64(b)
            out = torch.full((O.nwords(la + lb - 1),), -1, dtype=torch.int64, device="cuda")
            jobs.append((b, lb, tb, out))
            if k % 3 == 2:   # an ordinary request between the resident ones
                x = 1000 + 37 * k
                c = synth.dense_poly(0x5EED2200 + k, x)
                tc = dev64(c)
                o2 = torch.full((O.nwords(x + x - 1),), -1, dtype=torch.int64, device="cuda")
                jobs.append((("plain", c, x), x, tc, o2))
        torch.cuda.synchronize()
        tickets = []
        for b, lb, tb, out in jobs:
            if isinstance(b, tuple):
                tickets.append(srv.submit(tb, lb, tb, lb, out))
            else:
                tickets.append(srv.submit_resident(res, tb, lb, out))
        for tk in tickets:
            srv.wait(tk)
        torch.cuda.synchronize()
        for (b, lb, tb, out) in jobs:
            if isinstance(b, tuple):
                _, c, x = b
                assert np.array_equal(host(out, O.nwords(2 * x - 1)), O.polymul(c, x, c, x))
                continue
            n = O.nwords(la + lb - 1)
            got = host(out, n)
            alone = ctx.polymul(ta, la, tb, lb)
            torch.cuda.synchronize()
            assert np.array_equal(got, host(alone, n)), f"resident x {lb} bits differs from polymul_ex"
            check_against_oracle(a, la, b, lb, got, rng)
        say("resident operand, direct (no server)")
        b = synth.dense_poly(0x5EED2300, 3000000)
        tb = dev64(b)
        got = res.mul(ctx, tb, 3000000)
        torch.cuda.synchronize()
        check_against_oracle(a, la, b, 3000000, host(got, O.nwords(la + 3000000 - 1)), rng)
        say("resident operand errors")
        with pytest.raises(fpmul.FpmulError) as ei:
            res.mul(ctx, tb, (1 << 22) - la + 2)       # longer than the kept transform
        assert ei.value.code == fpmul.EINVAL
    finally:
        srv.close()
        res.close()


def test_server_tuner_on_a_small_mix(ctx):
    # two settings timed on a mix of 300 requests; the choice is one of them,
    # and a server with it computes the same products as polymul_ex
    from paper_1803_11301_amd import fpmul
    from paper_1803_11301_amd.serve_tune import tune_server
    rng = np.random.default_rng(0x5EED0571)
    la = np.floor(np.exp2(10 + 8 * rng.random(300))).astype(np.int64)
    lb = np.floor(np.exp2(10 + 8 * rng.random(300))).astype(np.int64)
    cands = [(4, 1 << 16, 64), (8, 1 << 20, 512)]
    say("server tuner", len(la), "requests,", len(cands), "settings")
    res = tune_server(ctx, la, lb, candidates=cands, bursts=1, p99_limit_ms=1e9)
    assert [(r["slots"], r["batch_limit_bits"], r["max_batch"]) for r in res["table"]] == cands
    assert all(r["saturated_per_s"] > 0 and 0 < r["p50_ms"] <= r["p99_ms"] for r in res["table"])
    c = res["choice"]
    assert c["saturated_per_s"] == max(r["saturated_per_s"] for r in res["table"])
    srv = fpmul.Server(ctx, hbm_budget=1 << 30, slots=c["slots"], batch_limit_bits=c["batch_limit_bits"],
                       max_batch=c["max_batch"])
    ops = []
    for k in range(6):
        x, y = int(la[k]), int(lb[k])
        a, b = synth.dense_poly(0x5EED0572 + 2 * k, x), synth.dense_poly(0x5EED0573 + 2 * k, y)
        ops.append((x, y, dev64(a), dev64(b), torch.zeros(O.nwords(x + y - 1), dtype=torch.int64, device="cuda")))
    torch.cuda.synchronize()
    for tk in [srv.submit(ta, x, tb, y, out) for x, y, ta, tb, out in ops]:
        srv.wait(tk)
    srv.close()
    for x, y, ta, tb, out in ops:
        n = O.nwords(x + y - 1)
        assert np.array_equal(host(out, n), host(ctx.polymul(ta, x, tb, y), n)), (x, y)


def _mixed_requests(seed, count, lo=10, hi=22):
    rng = np.random.default_rng(seed)
    la = np.floor(np.exp2(lo + (hi - lo) * rng.random(count))).astype(np.int64)
    lb = np.floor(np.exp2(lo + (hi - lo) * rng.random(count))).astype(np.int64)
    ops = []
    for k in range(count):
        x, y = int(la[k]), int(lb[k])
        a, b = synth.dense_poly(seed + 2 * k, x), synth.dense_poly(seed + 2 * k + 1, y)
        ops.append((x, y, dev64(a), dev64(b), torch.zeros(O.nwords(x + y - 1), dtype=torch.int64, device="cuda")))
    torch.cuda.synchronize()
    return ops


def test_destroy_completes_outstanding_requests(ctx):
    # the server is destroyed with every request still outstanding: destroy
    # returns once all of them ran (their launcher threads stop after that)
    from paper_1803_11301_amd import fpmul
    ops = _mixed_requests(0x5EED0580, 120)
    say("destroy with", len(ops), "outstanding requests")
    srv = fpmul.Server(ctx, hbm_budget=1 << 30, slots=6)
    for x, y, ta, tb, out in ops:
        srv.submit(ta, x, tb, y, out)
    srv.close()
    for x, y, ta, tb, out in ops[::7]:
        n = O.nwords(x + y - 1)
        assert np.array_equal(host(out, n), host(ctx.polymul(ta, x, tb, y), n)), (x, y)


def test_submits_from_several_host_threads(ctx):
    # four host threads submit and wait at once; every product is right
    import threading
    from paper_1803_11301_amd import fpmul
    ops = _mixed_requests(0x5EED0590, 160)
    say("4 threads x", len(ops) // 4, "requests")
    srv = fpmul.Server(ctx, hbm_budget=1 << 30, slots=8)
    errors = []

    def worker(part):
        try:
            tks = [srv.submit(ta, x, tb, y, out) for x, y, ta, tb, out in part]
            for tk in tks:
                srv.wait(tk)
        except Exception as ex:   # reported below, in the test's own thread
            errors.append(ex)

    threads = [threading.Thread(target=worker, args=(ops[k::4],)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not any(th.is_alive() for th in threads), "a submitting thread did not finish"
    assert not errors, errors
    assert srv.outstanding() == 0
    srv.close()
    for x, y, ta, tb, out in ops[::9]:
        n = O.nwords(x + y - 1)
        assert np.array_equal(host(out, n), host(ctx.polymul(ta, x, tb, y), n)), (x, y)
