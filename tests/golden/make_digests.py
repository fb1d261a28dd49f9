#!/usr/bin/env python3
"""Write tests/golden/digests.json: SHA-256 of the oracle's product for the
single-product workloads (2^16, 2^24 with the top bit forced, 2^30 bits).

The product in GF(2)[x] has exactly one value (the plain definition
c_k = XOR_{i+j=k} a_i b_j, Sec. 2.1; the method's interpolation is exact,
Prop. 2), so a digest of the oracle's output words pins the whole output of
any implementation.  Only ``oracle/`` computes here; ``synth`` draws the
seeded inputs.  The 2^30-bit product takes a few minutes on all host threads.

    python tests/golden/make_digests.py [--only small,mid,large]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "digests.json")

# name: (operand bits, seed, top bit forced)
CASES = {
    "small": (1 << 16, 0x5EED0016, False),
    "mid": (1 << 24, 0x5EED0024, True),
    "large": (1 << 30, 0x5EED0030, False),
}


def digest_words(words) -> str:
    """SHA-256 of the product's words as little-endian 64-bit integers."""
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


def main():
    import oracle as O
    from paper_1803_11301_amd import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=",".join(CASES))
    args = ap.parse_args()
    O.build(force=False)
    rec = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            rec = json.load(f)
    threads = O.max_threads()
    for name in args.only.split(","):
        L, seed, top = CASES[name]
        a, b = synth.single_pair(seed, L, top_bit=top)
        t0 = time.perf_counter()
        c = O.polymul(a, L, b, L, threads=threads)
        sec = time.perf_counter() - t0
        rec[name] = {"len_a": L, "len_b": L, "seed_a": hex(seed), "seed_b": hex(seed + 1), "top_bit": top,
                     "words": int(c.size), "sha256": digest_words(c),
                     "source": "oracle.polymul (Karatsuba over carry-less word products), "
                               f"{sec:.1f} s on {threads} threads"}
        print(f"{name}: {rec[name]['sha256']} ({sec:.1f} s)", flush=True)
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
