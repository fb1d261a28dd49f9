"""GPU parity of polymul_batch: every product of a batch against the CPU oracle.

Every product of every batch is compared word for word with the oracle,
including all 4096 products of the full mix (operand lengths log-uniform in
[2^10, 2^20] bits, 10% sparse), whose oracle products run on a pool of host
threads.
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
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.int64)).cuda()


SENTINEL = np.uint64(0xA5A5A5A5A5A5A5A5)


def oracle_products(As, las, Bs, lbs):
    """The oracle's product of every pair, on up to 16 host threads (the oracle
    call leaves Python, so the threads run in parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(lambda k: O.polymul(As[k], las[k], Bs[k], lbs[k]), range(len(As))))


def run_batch(ctx, As, Bs, las, lbs, max_bits=None, with_status=True):
    """Pack, run one polymul_batch, return (list of output word arrays, status)."""
    from paper_1803_11301_amd import fpmul
    a_pool, a_off = fpmul.pack_words(As)
    b_pool, b_off = fpmul.pack_words(Bs)
    out_off, out_words = fpmul.out_layout(las, lbs)
    out_pool = np.full(max(1, out_words) + 1, SENTINEL, dtype=np.uint64)
    if max_bits is None:
        max_bits = max([la + lb - 1 for la, lb in zip(las, lbs) if la and lb] + [1])
    status = torch.full((len(las),), 7, dtype=torch.int32, device="cuda") if with_status else None
    out_t = dev64(out_pool)
    ctx.polymul_batch(dev64(a_pool), dev64(a_off), dev64(np.asarray(las, np.uint64)), dev64(b_pool), dev64(b_off),
                      dev64(np.asarray(lbs, np.uint64)), out_t, dev64(out_off), max_bits, status)
    torch.cuda.synchronize()
    res = out_t.cpu().numpy().view(np.uint64)
    outs = []
    for k, (la, lb) in enumerate(zip(las, lbs)):
        n = O.nwords(la + lb - 1) if (la and lb) else 0
        outs.append(res[out_off[k]: out_off[k] + max(n, 1)])
    st = status.cpu().numpy() if with_status else None
    assert res[-1] == SENTINEL, "write past the output pool"
    return outs, st


def words(rng, length):
    return O.int_to_words(rng.getrandbits(length) if length else 0, length)


def test_small_mixed_batch_exact(ctx):
    rng = random.Random(1234)
    lens = [(1, 1), (1, 64), (64, 1), (63, 2), (64, 64), (65, 65), (100, 3000), (2048, 2049), (4095, 1),
            (5000, 5000), (31, 33), (7, 4090), (33000, 20000), (1 << 15, 1 << 15), (70000, 70000)]
    for _ in range(40):
        lens.append((rng.randint(1, 9000), rng.randint(1, 9000)))
    say("small mixed batch", len(lens), "items")
    As = [words(rng, la) for la, _ in lens]
    Bs = [words(rng, lb) for _, lb in lens]
    outs, st = run_batch(ctx, As, Bs, [x for x, _ in lens], [y for _, y in lens])
    for k, (la, lb) in enumerate(lens):
        ref = O.polymul(As[k], la, Bs[k], lb)
        assert np.array_equal(outs[k][: ref.size], ref), (k, la, lb)
        assert st[k] == 0


def test_batch_equals_single_products(ctx):
    rng = random.Random(77)
    lens = [(rng.randint(1000, 300000), rng.randint(1000, 300000)) for _ in range(12)]
    say("batch vs single", lens[:3], "...")
    As = [words(rng, la) for la, _ in lens]
    Bs = [words(rng, lb) for _, lb in lens]
    outs, _ = run_batch(ctx, As, Bs, [x for x, _ in lens], [y for _, y in lens])
    for k, (la, lb) in enumerate(lens):
        single = ctx.polymul(dev64(As[k]), la, dev64(Bs[k]), lb)
        torch.cuda.synchronize()
        s = single.cpu().numpy().view(np.uint64)[: O.nwords(la + lb - 1)]
        assert np.array_equal(outs[k][: s.size], s), k


def test_empty_operands_and_rejected_items(ctx):
    rng = random.Random(5)
    lens = [(0, 100), (100, 0), (0, 0), (3000, 3000), (5000, 5000), (10, 10)]
    As = [words(rng, la) for la, _ in lens]
    Bs = [words(rng, lb) for _, lb in lens]
    # max_product_bits 8192: the 5000 x 5000 product (9999 bits) is rejected
    say("empty and rejected items, max_product_bits 8192")
    outs, st = run_batch(ctx, As, Bs, [x for x, _ in lens], [y for _, y in lens], max_bits=8192)
    assert list(st) == [0, 0, 0, 0, -22, 0]
    for k in (0, 1, 2):
        assert outs[k][0] == SENTINEL            # nothing written for an empty product
    assert np.all(outs[4] == SENTINEL)           # rejected: untouched
    for k in (3, 5):
        la, lb = lens[k]
        assert np.array_equal(outs[k], O.polymul(As[k], la, Bs[k], lb))


def test_tail_bits_ignored(ctx):
    rng = random.Random(9)
    lens = [(70, 130), (1000, 1), (129, 129)]
    As, Bs = [], []
    for la, lb in lens:
        a = words(rng, la)
        b = words(rng, lb)
        a[-1] |= np.uint64(~((1 << (la % 64)) - 1) & (2**64 - 1)) if la % 64 else np.uint64(0)
        b[-1] |= np.uint64(~((1 << (lb % 64)) - 1) & (2**64 - 1)) if lb % 64 else np.uint64(0)
        As.append(a)
        Bs.append(b)
    say("tail bits")
    outs, _ = run_batch(ctx, As, Bs, [x for x, _ in lens], [y for _, y in lens])
    for k, (la, lb) in enumerate(lens):
        assert np.array_equal(outs[k], O.polymul(As[k], la, Bs[k], lb)), k


def test_two_batches_in_a_row_smaller_second(ctx):
    rng = random.Random(31)
    for count, hi in ((40, 200000), (7, 3000)):
        lens = [(rng.randint(1, hi), rng.randint(1, hi)) for _ in range(count)]
        say("batch", count, "items up to", hi, "bits")
        As = [words(rng, la) for la, _ in lens]
        Bs = [words(rng, lb) for _, lb in lens]
        outs, st = run_batch(ctx, As, Bs, [x for x, _ in lens], [y for _, y in lens])
        for k, (la, lb) in enumerate(lens):
            assert np.array_equal(outs[k], O.polymul(As[k], la, Bs[k], lb)), (count, k)


def test_full_mixed_batch_4096(ctx):
    """The 4096-product mix at its real sizes, in the launch configuration the benchmark times."""
    plan = synth.batch_plan()
    say("full batch", len(plan), "items, seed", hex(synth.SEED_BATCH))
    As, Bs = zip(*[synth.batch_operands(it) for it in plan])
    las = [it.len_a for it in plan]
    lbs = [it.len_b for it in plan]
    outs, st = run_batch(ctx, list(As), list(Bs), las, lbs, max_bits=1 << 21)
    assert np.all(st == 0)
    refs = oracle_products(As, las, Bs, lbs)
    for k, it in enumerate(plan):
        assert np.array_equal(outs[k], refs[k]), (k, it.len_a, it.len_b, it.sparse)


@pytest.mark.parametrize("limit", [0, 12, 20])
def test_small_field_limit_changes_field_not_products(ctx, limit):
    """Items up to 2^limit transform bits run over GF(2^32), the rest over
    GF(2^64); the products equal the oracle's for every limit."""
    rng = random.Random(4000 + limit)
    lens = [(1, 1), (1, 64), (33, 31), (64, 64), (65, 65), (500, 700), (2048, 2049), (4095, 4097), (9000, 70),
            (1 << 13, 1 << 13), ((1 << 16) - 3, 1 << 16), (1 << 18, 1 << 18), ((1 << 19) - 1, (1 << 19) + 2),
            (1 << 20, 1 << 20)]
    for _ in range(20):
        lens.append((rng.randint(1, 40000), rng.randint(1, 40000)))
    say("small-field limit", limit, len(lens), "items")
    As = [words(rng, la) for la, _ in lens]
    Bs = [words(rng, lb) for _, lb in lens]
    ctx.set_small_field(limit)
    try:
        outs, st = run_batch(ctx, As, Bs, [x for x, _ in lens], [y for _, y in lens])
    finally:
        ctx.set_small_field(20)
    assert (st == 0).all()
    refs = oracle_products(As, [x for x, _ in lens], Bs, [y for _, y in lens])
    for (la, lb), got, ref in zip(lens, outs, refs):
        assert np.array_equal(got[: O.nwords(la + lb - 1)], ref), (la, lb)


def test_small_field_limit_rejects_out_of_range(ctx):
    from paper_1803_11301_amd import fpmul
    for bad in (-1, 21, 64):
        with pytest.raises(fpmul.FpmulError):
            ctx.set_small_field(bad)
