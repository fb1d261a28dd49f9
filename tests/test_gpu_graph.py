"""GPU tests of the captured launch chains (polymul_graph_create,
polymul_batch_graph_create): every replay is compared bit for bit with the
eager product (polymul_ex / polymul_batch) and with the oracle.  Replays are
interleaved with other eager work and host synchronisations, operands are
rewritten in place between replays (a replay reads them when it runs), and
the batch graph is replayed with new lengths written into its device arrays.
Every case prints its name and sizes before touching the GPU.
"""
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


def dev(words):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    return torch.from_numpy(w.view(np.int64)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint64)


# the routes of polymul_ex below 2^32 bits: the one-item batch (<= 2^16-bit
# transform), the fused path with a 2^22-bit transform for a shorter product
# (2^17 .. 2^21 bits), the fused path at its own size (2^22 .. 2^31), and the
# fused path with a 3-bit operand (a single row)
CASES = [("2^15 x 2^15", 1 << 15, 1 << 15), ("2^16 x 2^16", 1 << 16, 1 << 16), ("100000 x 150001", 100000, 150001),
         ("2^24 x 2^24", 1 << 24, 1 << 24), ("3 x 2^20+5", 3, (1 << 20) + 5)]


@pytest.mark.parametrize("name,la,lb", CASES)
def test_product_graph_replays(ctx, name, la, lb):
    from paper_1803_11301_amd import fpmul
    say("graph", name)
    rng = np.random.default_rng(la * 7 + lb)
    nw = (la + lb - 1 + 63) // 64
    a = dev(synth.dense_poly(0x5EED0B00 + la % 97, la))
    b = dev(synth.dense_poly(0x5EED0C00 + lb % 89, lb))
    out = torch.full((nw,), -1, dtype=torch.int64, device="cuda")
    g = fpmul.Graph.product(ctx, a, la, b, lb, out)
    other_a = dev(synth.dense_poly(0x5EED0D00, 5000))
    try:
        for rep in range(3):
            if rep:
                # new operand contents in the same buffers: the replay reads them
                a.copy_(dev(synth.dense_poly(0x5EED0E00 + rep, la)))
                b.copy_(dev(synth.dense_poly(0x5EED0F00 + rep, lb)))
            out.fill_(-1)
            g.launch()
            # eager work of the program between the replay and the check
            scratch = ctx.polymul(other_a, 5000, other_a, 5000)
            torch.cuda.synchronize()
            ref = ctx.polymul(a, la, b, lb)
            torch.cuda.synchronize()
            got, want = host(out), host(ref)
            assert np.array_equal(got, want), f"{name} replay {rep}: word {int(np.nonzero(got != want)[0][0])}"
            if la + lb <= (1 << 21):
                assert np.array_equal(got, O.polymul(host(a), la, host(b), lb, threads=4)), f"{name} replay {rep}"
            del scratch
            _ = rng
    finally:
        g.close()


def test_square_graph_replays(ctx):
    # a square (one buffer for both operands) is captured as one forward
    # transform and the squares; each replay reads the buffer's new contents
    from paper_1803_11301_amd import fpmul
    la = (1 << 20) + 77
    say("graph square", la)
    nw = (2 * la - 1 + 63) // 64
    a = dev(synth.dense_poly(0x5EED0B80, la))
    out = torch.full((nw,), -1, dtype=torch.int64, device="cuda")
    g = fpmul.Graph.product(ctx, a, la, a, la, out)
    try:
        for rep in range(3):
            if rep:
                a.copy_(dev(synth.dense_poly(0x5EED0B80 + rep, la)))
            out.fill_(-1)
            g.launch()
            torch.cuda.synchronize()
            A = host(a)
            got = host(out)
            assert np.array_equal(got, host(ctx.polymul(a, la, a, la))), f"square replay {rep}"
            assert np.array_equal(got, O.polymul(A, la, A, la, threads=4)), f"square replay {rep}"
    finally:
        g.close()


def test_batch_graph_replays_with_new_lengths(ctx):
    from paper_1803_11301_amd import fpmul
    count, max_bits = 96, 1 << 21
    say("batch graph", count, "items, max", max_bits)
    rng = np.random.default_rng(96)
    cap = 1 << 20                     # operand capacity per item, bits
    capw = cap // 64
    a_pool = dev(synth.dense_poly(0x5EED1000, count * cap))
    b_pool = dev(synth.dense_poly(0x5EED1001, count * cap))
    a_off = dev(np.arange(count, dtype=np.uint64) * np.uint64(capw))
    b_off = dev(np.arange(count, dtype=np.uint64) * np.uint64(capw))
    out_off = dev(np.arange(count, dtype=np.uint64) * np.uint64(2 * capw))
    out_pool = torch.full((count * 2 * capw,), -1, dtype=torch.int64, device="cuda")
    la = torch.zeros(count, dtype=torch.int64, device="cuda")
    lb = torch.zeros(count, dtype=torch.int64, device="cuda")
    g = fpmul.Graph.batch(ctx, a_pool, a_off, la, b_pool, b_off, lb, out_pool, out_off, max_bits)
    try:
        A, B = host(a_pool), host(b_pool)
        for rep in range(3):
            las = np.exp2(rng.uniform(1, 20, count)).astype(np.uint64)
            lbs = np.exp2(rng.uniform(1, 20, count)).astype(np.uint64)
            las[rep] = 0                  # an empty operand: nothing written
            la.copy_(dev(las))
            lb.copy_(dev(lbs))
            out_pool.fill_(-1)
            g.launch()
            torch.cuda.synchronize()
            got = host(out_pool)
            # the eager batch on the same arrays
            eager = torch.full_like(out_pool, -1)
            ctx.polymul_batch(a_pool, a_off, la, b_pool, b_off, lb, eager, out_off, max_bits)
            torch.cuda.synchronize()
            assert np.array_equal(got, host(eager)), f"batch graph replay {rep} differs from polymul_batch"
            for k in range(0, count, 7):
                x, y = int(las[k]), int(lbs[k])
                o = k * 2 * capw
                if x == 0:
                    assert np.all(got[o:o + 1] == np.uint64(0xFFFFFFFFFFFFFFFF)), "empty item written"
                    continue
                n = O.nwords(x + y - 1)
                want = O.polymul(A[k * capw: k * capw + O.nwords(x)], x, B[k * capw: k * capw + O.nwords(y)], y)
                assert np.array_equal(got[o:o + n], want), f"replay {rep} item {k} ({x} x {y})"
    finally:
        g.close()


def test_graph_argument_errors(ctx):
    from paper_1803_11301_amd import fpmul
    say("graph argument errors")
    t = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(fpmul.FpmulError) as ei:
        fpmul.Graph.product(ctx, t, 0, t, 5, t)
    assert ei.value.code == fpmul.EINVAL
    with pytest.raises(fpmul.FpmulError) as ei:
        fpmul.Graph.product(ctx, t, 128, t, 128, t[1:])   # out overlaps the inputs
    assert ei.value.code == fpmul.EINVAL
