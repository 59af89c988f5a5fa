"""Pins of the oracle's counter-based generator (no GPU).

The oracle's Philox4x32-10 is checked against rocRAND's own implementation of
the same block function (Salmon et al., SC'11), built here for the host from
rocRAND's installed header-only engine and run as a separate program; the
uniform conversion is checked on its exact edge cases and for uniformity.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_blocks():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp(prefix="rpb")
    exe = os.path.join(d, "rpb")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950",
                    os.path.join(HERE, "pins", "rocrand_philox_blocks.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(rows):
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [[int(v) for v in line.split()] for line in out.strip().splitlines()]

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand_block_function(rocrand_blocks):
    rng = np.random.default_rng(1234)
    rows = [[0] * 6, [0xFFFFFFFF] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 1, 0, 0], [0, 0, 0, 0, 0, 1]]
    rows += rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).tolist()
    # the layout the method uses: small d/4, row, generation and tag
    for _ in range(200):
        rows.append([int(rng.integers(0, 60000)), int(rng.integers(0, 5000)),
                     int(rng.integers(0, 600)), int(rng.integers(0, 5)),
                     int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))])
    want = rocrand_blocks(rows)
    got = [O.philox(r[:4], r[4:]) for r in rows]
    assert got == want


def test_word_layout_uses_counter_words():
    # coordinate d of (row, t, tag) takes word d % 4 of block (d/4, row, t, tag)
    seed = 0x0123456789ABCDEF
    for (tag, row, t, d) in [(0, 0, 0, 0), (1, 7, 3, 5), (2, 4095, 499, 203529), (4, 15, 1, 3)]:
        blk = O.philox([d // 4, row, t, tag], [seed & 0xFFFFFFFF, seed >> 32])
        assert O.word(seed, tag, row, t, d) == blk[d % 4]


def test_u01_edges_exact():
    assert O.u01(0) == 0.0
    assert O.u01(0xFF) == 0.0                      # low 8 bits are dropped
    assert O.u01(0x100) == 2.0 ** -24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24   # never reaches 1
    assert O.u01(0x80000000) == 0.5
    r = np.random.default_rng(5).integers(0, 2**32, size=2000, dtype=np.uint64)
    for v in r[:200]:
        u = O.u01(int(v))
        assert u == (int(v) >> 8) / 2.0 ** 24       # exact 24-bit grid value


def test_uniformity_chi_square():
    # 64-bin chi-square of 2^15 draws across rows, generations and coordinates
    n = 1 << 15
    vals = np.array([O.u01(O.word(99, 1, i // 64, 3, i % 64)) for i in range(n)])
    hist, _ = np.histogram(vals, bins=64, range=(0.0, 1.0))
    expect = n / 64
    chi2 = float(((hist - expect) ** 2 / expect).sum())
    # 63 degrees of freedom: P(chi2 > 120) < 1e-5
    assert chi2 < 120.0, chi2
    assert abs(vals.mean() - 0.5) < 0.01
