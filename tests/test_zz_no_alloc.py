"""GPU test of polymul_ex_noalloc, the entry point that allocates nothing:
its products (workspace in the library's device scratch) against polymul_ex
on the same operands, bit for bit, on two calls in a row, the second with a
smaller input; and its size limit.  Every case prints its name and sizes
before touching the GPU.
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


def poisoned(nw):
    return torch.full((max(1, nw),), -1, dtype=torch.int64, device="cuda")


def test_noalloc_equals_polymul_ex_on_two_calls(ctx):
    # the largest product it takes (2^24 x 2^24 bits, top bits set: the fused
    # path), then smaller ragged ones (the fused path with a 2^22-bit
    # transform, then the one-item batch path); each call runs on the scratch
    # the one before left behind
    cases = [("2^24 x 2^24 (top bit set)", synth.SEED_MID, 1 << 24, 1 << 24, True),
             ("12345 x 70001", 0x5EED0A11, 12345, 70001, False),
             ("9999 x 30001", 0x5EED0A14, 9999, 30001, False)]
    for name, seed, la, lb, top in cases:
        say("polymul_ex_noalloc", name, f"seed {seed:#x}")
        a = synth.dense_poly(seed, la, top_bit=top)
        b = synth.dense_poly(seed + 1, lb, top_bit=top)
        ta, tb = dev(a), dev(b)
        nw = (la + lb - 1 + 63) // 64
        ref = poisoned(nw)
        ctx.polymul(ta, la, tb, lb, out=ref)
        got = poisoned(nw)
        ctx.polymul_noalloc(ta, la, tb, lb, got)
        torch.cuda.synchronize()
        r, g = host(ref), host(got)
        assert np.array_equal(g, r), f"{name}: first differing word {int(np.nonzero(g != r)[0][0])}"
        if la + lb <= 1 << 18:
            assert np.array_equal(g, O.polymul(a, la, b, lb, threads=4)), name


def test_noalloc_between_mid_sizes(ctx):
    # a 2^19-bit product (the fused path with a 2^22-bit transform, operands
    # of different row counts) after the other calls
    la, lb = 300000, 200001
    say("polymul_ex_noalloc", f"{la} x {lb}")
    a = synth.dense_poly(0x5EED0A12, la)
    b = synth.dense_poly(0x5EED0A13, lb)
    ta, tb = dev(a), dev(b)
    nw = (la + lb - 1 + 63) // 64
    got = poisoned(nw)
    ctx.polymul_noalloc(ta, la, tb, lb, got)
    torch.cuda.synchronize()
    assert np.array_equal(host(got), O.polymul(a, la, b, lb, threads=4))


def test_noalloc_square(ctx):
    # the same buffer twice: one forward transform in the scratch, squared
    la = (1 << 22) + 3
    say("polymul_ex_noalloc square", la)
    a = synth.dense_poly(0x5EED0A15, la)
    ta = dev(a)
    nw = (2 * la - 1 + 63) // 64
    got, ref = poisoned(nw), poisoned(nw)
    ctx.polymul_noalloc(ta, la, ta, la, got)
    ctx.polymul(ta, la, ta, la, out=ref)
    torch.cuda.synchronize()
    assert np.array_equal(host(got), host(ref))
    spread = np.zeros(2 * nw, dtype=np.uint64)   # bit i of A at bit 2i (Frobenius)
    w = np.asarray(a, dtype=np.uint64)
    for half, sh in ((0, 0), (1, 32)):
        x = (w >> np.uint64(sh)) & np.uint64(0xFFFFFFFF)
        for s_, m in ((16, 0x0000FFFF0000FFFF), (8, 0x00FF00FF00FF00FF), (4, 0x0F0F0F0F0F0F0F0F),
                      (2, 0x3333333333333333), (1, 0x5555555555555555)):
            x = (x | (x << np.uint64(s_))) & np.uint64(m)
        spread[half:2 * w.size:2] = x
    assert np.array_equal(host(got), spread[:nw])


def test_noalloc_rejects_longer_products(ctx):
    from paper_1803_11301_amd import fpmul
    # host-side check: nothing is launched
    la = lb = (1 << 24) + 1
    say("polymul_ex_noalloc size limit", f"{la} x {lb}")
    t = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(fpmul.FpmulError) as ei:
        ctx.polymul_noalloc(t, la, t, lb, t)
    assert ei.value.code == fpmul.EINVAL
    assert "2^25" in str(ei.value)
