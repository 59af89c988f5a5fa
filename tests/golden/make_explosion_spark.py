"""Write tests/golden/explosion_spark.json: explosion-spark coordinates worked
out in exact rational arithmetic (test fixture generator; calls only oracle/).

The explosion step of Alg. 1 moves every coordinate of a firework x by the
amplitude A times a uniform draw in [-1, 1) (the build's reading: one fused
multiply-add, s = fma(A, 2u - 1, x), rounded once to binary32), and maps a
coordinate that leaves the box to a fresh uniform position in it (the random
mapping: fma(u', ub - lb, lb), clamped).  Here the random words come from the
oracle's Philox4x32-10 (pinned separately against rocRAND's engine); every
arithmetic step after them is done on exact fractions and rounded to binary32
by hand, round-to-nearest-even, so the stored values do not depend on the
oracle's C arithmetic.  The case is chosen so that one coordinate lands outside
the box and at least one differs between a single rounding (fma) and two
(multiply, round, add, round): a spark written as a multiply and an add fails.

Run: python tests/golden/make_explosion_spark.py
"""
import json
import os
import struct
import sys
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as O  # noqa: E402

SEED, ROW, T, DIM = 20250107, 37, 3, 8
LB, UB = -5.0, 5.0


def round32(q: Fraction) -> float:
    """q rounded to the nearest binary32 (ties to even), normal range only."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while a / Fraction(2) ** e >= 2:
        e += 1
    while a / Fraction(2) ** e < 1:
        e -= 1
    assert -126 <= e <= 127, "outside the normal binary32 range"
    scaled = a / Fraction(2) ** (e - 23)            # in [2^23, 2^24)
    n, rem = divmod(scaled.numerator, scaled.denominator)
    twice = 2 * rem
    if twice > scaled.denominator or (twice == scaled.denominator and n % 2 == 1):
        n += 1
    v = sign * n * 2.0 ** (e - 23)
    assert float(np.float32(v)) == v
    return v


def f32(v: float) -> Fraction:
    return Fraction(float(np.float32(v)))


def hexf(v: float) -> str:
    return "0x%08x" % struct.unpack("<I", struct.pack("<f", v))[0]


def u01(r: int) -> Fraction:
    return Fraction(r >> 8, 1 << 24)


def work(x, A):
    out, rows = [], []
    span, lb, ub = f32(UB) - f32(LB), f32(LB), f32(UB)
    assert span == 10
    for d in range(DIM):
        r = O.word(SEED, "expl", ROW, T, d)
        v = 2 * u01(r) - 1                          # exact in binary32
        assert round32(v) == float(v) if v != 0 else True
        fused = round32(A * v + x[d])
        two = round32(Fraction(round32(A * v)) + x[d])
        mapped = not (lb <= Fraction(fused) <= ub)
        final = fused
        r2 = None
        if mapped:
            r2 = O.word(SEED, "expl_map", ROW, T, d)
            final = min(max(round32(u01(r2) * span + lb), float(lb)), float(ub))
        out.append(final)
        rows.append(dict(d=d, word=r, map_word=r2, unmapped=hexf(fused),
                         two_roundings=hexf(two), fma_differs=fused != two, mapped=mapped,
                         value=hexf(final)))
    return out, rows


def main():
    rng = np.random.default_rng(7)
    A = f32(3.7)                                   # not a power of two
    for _ in range(10000):
        x = [f32(v) for v in rng.uniform(-4.5, 4.5, DIM)]
        out, rows = work(x, A)
        if any(r["mapped"] for r in rows) and any(r["fma_differs"] and not r["mapped"]
                                                  for r in rows):
            break
    else:
        raise RuntimeError("no discriminating case found")
    doc = {
        "about": ("Explosion-spark coordinates (Alg. 1, explosion and mapping steps; reading "
                  "s = fma(A, 2u - 1, x), out-of-box coordinates mapped to fma(u', ub - lb, lb) "
                  "clamped), worked in exact rational arithmetic from the oracle's Philox words "
                  "by tests/golden/make_explosion_spark.py.  Values are binary32 bit patterns."),
        "seed": SEED, "row": ROW, "t": T, "lb": LB, "ub": UB, "A": hexf(float(A)),
        "x": [hexf(float(v)) for v in x], "coordinates": rows,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "explosion_spark.json")
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")
    print(path, sum(r["fma_differs"] for r in rows), "fma-sensitive,",
          sum(r["mapped"] for r in rows), "mapped")


if __name__ == "__main__":
    main()
