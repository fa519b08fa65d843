"""Pins for the oracle's counter-based generator and normal transform.

Philox4x32-10 is pinned against ROCm's rocRAND engine (an independent
implementation, run here, not copied); the log and sincos it uses are pinned
against the C library; the Box-Muller mapping against numpy; the normals
by their moments and a Kolmogorov-Smirnov test.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "philox_rocrand_ref.cpp")


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, HELPER], check=True, cwd="/tmp")

    def run(queries):
        txt = "\n".join(" ".join(f"{v & 0xffffffff:x}" for v in q) for q in queries) + "\n"
        out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
        return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]
    return run


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(123)
    queries = [[0, 0, 0, 0, 0, 0], [0xffffffff] * 6]
    queries += [list(map(int, rng.integers(0, 2 ** 32, size=6, dtype=np.uint64))) for _ in range(500)]
    # the counter layouts the filter uses: (j, n, tag<<28|blk<<20|iter, b)
    for j, n, tag, blk, it, b in [(5, 17, 2, 3, 0, 0), (65535, 1600, 1, 9, 7, 511), (0, 500, 3, 0, 1999, 63)]:
        queries.append([j, n, (tag << 28) | (blk << 20) | it, b, 0x12345678, 0x9abcdef0])
    ref = rocrand_ref(queries)
    for q, r in zip(queries, ref):
        assert list(orc.philox(q[:4], q[4:])) == r, q


def test_philox_is_injective_on_a_counter_range(orc):
    seen = set()
    for j in range(1 << 14):
        w = tuple(orc.philox([j, 3, 2 << 28, 0], [0, 0]))
        seen.add(w)
    assert len(seen) == 1 << 14


def test_u01_exact_cell_centres(orc):
    assert orc.u01(0) == 0.5 * 2.0 ** -32
    assert orc.u01(0xffffffff) == 1.0 - 0.5 * 2.0 ** -32
    assert 0.0 < orc.u01(0) < orc.u01(1) < orc.u01(0xffffffff) < 1.0


def _ulp_err(a, b):
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a)


def test_ln_against_libm(orc):
    rng = np.random.default_rng(7)
    xs = list(rng.uniform(0, 1, 4000)) + list(np.exp(rng.uniform(-700, 700, 2000)))
    xs += [2.0 ** e for e in range(-1000, 1000, 37)] + [0.5 * 2.0 ** -32, 1.0 - 2.0 ** -33,
                                                        0.7071067811865475, 0.7071067811865476,
                                                        1.0, 1.4142135623730951, 3.0]
    worst = 0.0
    for x in xs:
        if x <= 0 or x < 2.2250738585072014e-308:
            continue
        ref = math.log(x)
        got = orc.ln(x)
        if ref == 0.0:
            assert got == 0.0
            continue
        worst = max(worst, _ulp_err(got, ref))
    assert worst <= 2.0, worst


def test_sincos2pi_against_libm(orc):
    rng = np.random.default_rng(8)
    us = list(rng.uniform(0, 1, 5000)) + [k / 8 for k in range(8)] + [orc.u01(0), orc.u01(2 ** 32 - 1)]
    for u in us:
        s, c = orc.sincos2pi(u)
        # reference in extended form: 2*pi*u rounded once, so allow a few 1e-16
        assert abs(s - math.sin(2 * math.pi * u)) < 2e-15
        assert abs(c - math.cos(2 * math.pi * u)) < 2e-15
    assert orc.sincos2pi(0.25) == (1.0, pytest.approx(0.0, abs=1e-16))
    s, c = orc.sincos2pi(0.5)
    assert c == -1.0 and abs(s) < 1e-16


def test_box_muller_mapping(orc):
    """z0,z1 from words (w0,w1), z2,z3 from (w2,w3); radius from the first word."""
    seed = 0x0123456789abcdef
    for (tag, blk, it, j, n, b) in [(2, 0, 0, 0, 1, 0), (2, 9, 0, 77, 123, 4), (1, 1, 5, 1000, 0, 9)]:
        w = orc.philox([j, n, (tag << 28) | (blk << 20) | it, b], [seed & 0xffffffff, seed >> 32])
        u = (w.astype(np.float64) + 0.5) * 2.0 ** -32
        ref = np.empty(4)
        for p in range(2):
            r = np.sqrt(-2.0 * np.log(u[2 * p]))
            ref[2 * p] = r * np.cos(2 * np.pi * u[2 * p + 1])
            ref[2 * p + 1] = r * np.sin(2 * np.pi * u[2 * p + 1])
        z = orc.normals4(seed, tag, blk, it, j, n, b)
        np.testing.assert_allclose(z, ref, rtol=0, atol=1e-13 * (1 + np.abs(ref)).max())


def test_normal_moments_and_ks(orc):
    z = orc.normals_bulk(42, 2, 0, 0, 1, 1 << 18).ravel()  # 2^20 normals
    n = z.size
    assert abs(z.mean()) < 4 / math.sqrt(n)
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / n)
    assert abs(scipy.stats.skew(z)) < 4 * math.sqrt(6 / n)
    assert abs(scipy.stats.kurtosis(z)) < 4 * math.sqrt(24 / n)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # the four positions of a call are independent
    zz = z.reshape(-1, 4)
    c = np.corrcoef(zz.T)
    assert np.abs(c - np.eye(4)).max() < 5 / math.sqrt(zz.shape[0])
