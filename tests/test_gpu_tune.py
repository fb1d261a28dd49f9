"""GPU tests of the schedule tuner (polymul_tune, polymul_tune_load,
polymul_tune_get): every schedule it picks, loads or is handed gives the
product the oracle gives (the stored SHA-256 of the oracle's 2^24 x 2^24-bit
product, unique by Prop. 2).  Every case prints its name before touching
the GPU.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_1803_11301_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with open(os.path.join(HERE, "golden", "digests.json")) as f:
        g = json.load(f)["mid"]
    L = g["len_a"]
    a, b = synth.single_pair(synth.SEED_MID, L, top_bit=True)
    ta = torch.from_numpy(a.view(np.int64)).cuda()
    tb = torch.from_numpy(b.view(np.int64)).cuda()
    return ta, tb, L, g["sha256"]


def digest_of(ctx, mid):
    ta, tb, L, _ = mid
    out = ctx.polymul(ta, L, tb, L)
    torch.cuda.synchronize()
    return hashlib.sha256(np.ascontiguousarray(out.cpu().numpy().view(np.uint64), dtype="<u8").tobytes()).hexdigest()


def test_tuned_schedule_gives_the_oracle_product(mid, tmp_path):
    from paper_1803_11301_amd import fpmul
    say("tune 2^25-bit transforms, reps 2")
    cache = tmp_path / "tune.txt"
    ctx = fpmul.Context(0)
    try:
        report = ctx.tune(25, reps=2, cache_path=str(cache))
        print(report)
        assert "tuned_ms=" in report
        line = ctx.schedule(25)
        assert digest_of(ctx, mid) == mid[3]
        say("load the cache into a fresh context")
        c2 = fpmul.Context(0)
        try:
            assert c2.tune_load(str(cache)) == 1
            assert c2.schedule(25) == line
            assert digest_of(c2, mid) == mid[3]
        finally:
            c2.close()
    finally:
        ctx.close()


def test_handed_schedules_give_the_oracle_product(mid, tmp_path):
    from paper_1803_11301_amd import fpmul
    ctx = fpmul.Context(0)
    try:
        arch_line = ctx.schedule(25)            # "<arch> cu=<n> log2n=25 upper=... rows=.. zeta=.. ms=0.0000"
        arch, cu = arch_line.split()[0], arch_line.split()[1]
        # lines for 2^25-bit transforms: they load and their grids apply; a
        # 2^19-value transform's butterflies take the 11-layer bottom pass, so
        # the split itself is exercised in the next test, at 2^20 values
        for upper, rows, zeta in [("7,5", 1, 4), ("5,7", 4, 16), ("5,4,3", 2, 8), ("6,1,5", 1, 16),
                                  ("5,5,2", 4, 4)]:
            say("schedule", upper, rows, zeta)
            p = tmp_path / f"s_{upper.replace(',', '_')}.txt"
            p.write_text(f"{arch} {cu} log2n=25 upper={upper} rows={rows} zeta={zeta} ms=1.0\n")
            assert ctx.tune_load(str(p)) == 1
            assert f"upper={upper} rows={rows} zeta={zeta}" in ctx.schedule(25)
            assert digest_of(ctx, mid) == mid[3], f"schedule {upper} rows={rows} zeta={zeta}"
        say("invalid lines are skipped")
        p = tmp_path / "bad.txt"
        p.write_text(f"{arch} {cu} log2n=25 upper=4,8 rows=2 zeta=8 ms=1.0\n"
                     f"{arch} {cu} log2n=25 upper=6,6 rows=0 zeta=8 ms=1.0\nnot a line\n")
        assert ctx.tune_load(str(p)) == 0
    finally:
        ctx.close()


def test_handed_splits_of_the_resident_table_passes(tmp_path):
    """A 2^25 x 2^25-bit product (2^20-value transforms, the smallest that
    runs the resident-table butterfly passes) under splits of its upper
    layers with a seven-layer bottom pass (13 upper layers) and with a
    six-layer one (14), against the oracle word for word."""
    import oracle as O
    from paper_1803_11301_amd import fpmul
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = 1 << 25
    say("2^25 x 2^25 oracle", hex(synth.SEED_LARGE))
    a, b = synth.single_pair(synth.SEED_LARGE, L)
    want = O.polymul(a, L, b, L, threads=16)
    ta = torch.from_numpy(a.view(np.int64)).cuda()
    tb = torch.from_numpy(b.view(np.int64)).cuda()
    ctx = fpmul.Context(0)
    try:
        arch_line = ctx.schedule(26)
        arch, cu = arch_line.split()[0], arch_line.split()[1]
        for upper in ["7,6", "6,7", "5,4,4", "7,7", "6,4,4", "6,7,1"]:
            say("split", upper, "bottom layers", 20 - sum(int(k) for k in upper.split(",")))
            p = tmp_path / f"s26_{upper.replace(',', '_')}.txt"
            p.write_text(f"{arch} {cu} log2n=26 upper={upper} rows=2 zeta=8 ms=1.0\n")
            assert ctx.tune_load(str(p)) == 1
            assert f"upper={upper} " in ctx.schedule(26)
            out = ctx.polymul(ta, L, tb, L)
            torch.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint64)
            assert np.array_equal(got[: want.size], want), f"split {upper}"
        say("a six-layer bottom split whose lowest pass is too short is refused")
        p = tmp_path / "bad26.txt"
        p.write_text(f"{arch} {cu} log2n=26 upper=5,5,4 rows=2 zeta=8 ms=1.0\n")
        assert ctx.tune_load(str(p)) == 0
    finally:
        ctx.close()


def test_tune_argument_errors():
    from paper_1803_11301_amd import fpmul
    say("tune argument errors")
    ctx = fpmul.Context(0)
    try:
        for lg in (21, 32):
            with pytest.raises(fpmul.FpmulError) as ei:
                ctx.tune(lg)
            assert ei.value.code == fpmul.EINVAL
        with pytest.raises(fpmul.FpmulError):
            ctx.tune(25, reps=0)
    finally:
        ctx.close()
