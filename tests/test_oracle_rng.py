"""Pins of the oracle's random-number generator and logarithm.

Philox4x32-10 is checked against rocRAND's independent implementation (the
ROCm header, compiled here for the host); the logarithm against the C
library's to within one unit in the last place; the constants against
high-precision values computed in the test.
"""
import math
import os
import re
import shutil
import struct
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
    probe p; unsigned a[6];
    while (scanf("%u %u %u %u %u %u", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
        uint4 o = p.run(make_uint4(a[0], a[1], a[2], a[3]), make_uint2(a[4], a[5]));
        printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
}
"""


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND header or hipcc not available")
    d = tmp_path_factory.mktemp("probe")
    src = d / "probe.cpp"
    src.write_text(PROBE_SRC)
    exe = d / "probe"
    subprocess.run([hipcc, "-O1", "-o", str(exe), str(src)], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(11)
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6]
    cases += rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64).tolist()
    inp = "\n".join(" ".join(str(int(x)) for x in c) for c in cases) + "\n"
    res = subprocess.run([str(rocrand_probe)], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for c, line in zip(cases, lines):
        want = [int(x) for x in line.split()]
        got = orc.philox4x32_10(c[:4], c[4:])
        assert got == want, (c, got, want)


def test_uniform_grid_and_word_use(orc):
    # draw j uses block j>>1; even j -> words (0,1), odd j -> words (2,3)
    for j in range(6):
        blk = orc.philox4x32_10([j >> 1, 7, 123, 9], [5, 0])
        a, b = (blk[0], blk[1]) if j % 2 == 0 else (blk[2], blk[3])
        want = ((a >> 5) * 67108864 + (b >> 6)) / 2.0**53
        got = orc.uniform(5, 0, 7, 123, 9, j)
        assert got == want
        assert 0.0 <= got < 1.0
        assert (got * 2.0**53) == int(got * 2.0**53)
    # realization enters the key's high word
    blk = orc.philox4x32_10([0, 1, 2, 3], [9, 4])
    assert orc.uniform(9, 4, 1, 2, 3, 0) == ((blk[0] >> 5) * 67108864 + (blk[1] >> 6)) / 2.0**53


def test_uniform_moments(orc):
    u = np.array([orc.uniform(3, 0, 0, t, 0, 0) for t in range(20000)])
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 0.005


def _ulp(x):
    return math.ulp(x)


def test_ln_within_one_ulp(orc):
    rng = np.random.default_rng(5)
    xs = np.concatenate([
        rng.uniform(0, 1, 20000),                       # SSA: ln(1 - u)
        np.exp(rng.uniform(-700, 700, 20000)),           # whole exponent range
        rng.uniform(0.5, 2.0, 20000),                    # near 1, both reduction branches
        1.0 + rng.uniform(-1e-6, 1e-6, 2000),
        np.array([2.0**-1074, 2.0**-1060, 2.0**-1022 * 0.75, 1.0 - 2.0**-53, 2.0**-53,
                  math.sqrt(2.0), math.nextafter(math.sqrt(2.0), 2), math.nextafter(math.sqrt(2.0), 0)]),
    ])
    worst = 0.0
    for x in xs:
        if x <= 0:
            continue
        got = orc.ln(float(x))
        want = math.log(float(x))
        err = abs(got - want) / _ulp(want) if want != 0 else abs(got)
        worst = max(worst, err)
    assert worst <= 1.0, worst


def test_ln_exact_points(orc):
    assert orc.ln(1.0) == 0.0
    for k in range(-60, 61):
        assert abs(orc.ln(2.0**k) - k * math.log(2.0)) <= _ulp(k * math.log(2.0) or 1.0)


def _read_source(path):
    with open(os.path.join(ROOT, path)) as f:
        return f.read()


def _hex_consts(src, name):
    m = re.search(name + r"\s*=\s*(0x[0-9a-fp.+-]+)", src)
    return float.fromhex(m.group(1))


def test_ln_constants_are_the_stated_values():
    getcontext().prec = 50
    src = _read_source("oracle/oracle.c")
    hi = _hex_consts(src, "ORC_LN2_HI")
    lo = _hex_consts(src, "ORC_LN2_LO")
    ln2 = Decimal(2).ln()
    bits = struct.unpack("<Q", struct.pack("<d", hi))[0]
    assert bits & ((1 << 21) - 1) == 0                    # e * hi is exact for |e| < 2^11
    assert abs(Decimal(hi) - ln2) < Decimal(2) ** -32
    assert lo == float(ln2 - Decimal(hi))
    assert _hex_consts(src, "ORC_SQRT2") == math.sqrt(2.0)


def test_stirling_table_is_exact():
    """fc(k) = ln k! - (k+1/2) ln(k+1) + (k+1) - ln(2 pi)/2, correctly rounded."""
    getcontext().prec = 60
    src = _read_source("oracle/oracle.c")
    body = re.search(r"ORC_FC\[10\]\s*=\s*\{([^}]*)\}", src).group(1)
    table = [float.fromhex(x.strip()) for x in body.split(",") if x.strip()]
    assert len(table) == 10
    pi = Decimal("3.14159265358979323846264338327950288419716939937510582097494459")
    half_ln2pi = (2 * pi).ln() / 2
    fact = Decimal(1)
    for k in range(10):
        if k:
            fact *= k
        v = fact.ln() - (Decimal(k) + Decimal("0.5")) * Decimal(k + 1).ln() + Decimal(k + 1) - half_ln2pi
        assert table[k] == float(v), k
