"""The exact sign test behind the rounding of dequantised reconstructions near
a half (Sec. 6.1.1 inverse with a quantiser step that admits exact halves):
the kernels decide the sign of (a + b sqrt p) + (c + d sqrt p) sqrt q with
128-bit integers and 256-bit squares.  The same source
(`paper_1808_02950_amd/csrc/settle.hpp`) is compiled here for the host and
checked against 150-digit decimal arithmetic on random components up to 2^52,
on near-cancelling ones, and on exact zeros, for the generator pairs of the
built-in matrices (sqrt 10; sqrt 3; sqrt 6, sqrt 10; sqrt 2, sqrt 3; sqrt 3,
sqrt 10)."""

import os
import random
import shutil
import subprocess
from decimal import Decimal, getcontext

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
PAIRS = [(10, 1), (3, 1), (6, 10), (2, 3), (3, 10)]

getcontext().prec = 150


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    out = str(tmp_path_factory.mktemp("settle") / "settle_check")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
                    f"-I{os.path.join(ROOT, 'paper_1808_02950_amd', 'csrc')}",
                    os.path.join(ROOT, "tests", "settle_check.hip"), "-o", out],
                   check=True, capture_output=True)
    return out


def _exact_sign(a, b, c, d, p, q):
    sp, sq = Decimal(p).sqrt(), Decimal(q).sqrt()
    v = Decimal(a) + Decimal(b) * sp + (Decimal(c) + Decimal(d) * sp) * sq
    if a == b == c == d == 0:
        return 0
    assert abs(v) > Decimal(10) ** -100       # nonzero in the field: far from 0 at this precision
    return 1 if v > 0 else -1


def _run(driver, cases):
    text = "".join(f"{a} {b} {c} {d} {p} {q}\n" for a, b, c, d, p, q in cases)
    r = subprocess.run([driver], input=text, capture_output=True, text=True, check=True)
    return [int(x) for x in r.stdout.split()]


def _cases(seed):
    rng = random.Random(seed)
    lim = 1 << 52
    out = []
    for p, q in PAIRS:
        two = q > 1
        for _ in range(300):                     # random
            c = rng.randrange(-lim, lim) if two else 0
            d = rng.randrange(-lim, lim) if two else 0
            out.append((rng.randrange(-lim, lim), rng.randrange(-lim, lim), c, d, p, q))
        for _ in range(300):                     # a chosen to cancel the rest to within 1/2
            b = rng.randrange(-lim // 8, lim // 8)
            c = rng.randrange(-lim // 8, lim // 8) if two else 0
            d = rng.randrange(-lim // 8, lim // 8) if two else 0
            rest = Decimal(b) * Decimal(p).sqrt() + (Decimal(c) + Decimal(d) * Decimal(p).sqrt()) * Decimal(q).sqrt()
            a = int((-rest).to_integral_value())
            out.append((a, b, c, d, p, q))
        if two:
            for _ in range(200):                 # X close to -Y sqrt q with X, Y of opposite signs
                c = rng.randrange(1, lim // 16)
                d = rng.randrange(-lim // 16, lim // 16)
                y = (Decimal(c) + Decimal(d) * Decimal(p).sqrt()) * Decimal(q).sqrt()
                b = rng.randrange(-lim // 16, lim // 16)
                a = int((-y - Decimal(b) * Decimal(p).sqrt()).to_integral_value())
                out.append((a, b, c, d, p, q))
        out.append((0, 0, 0, 0, p, q))
        out.append((lim - 1, -(lim - 1), (lim - 1) if two else 0, -(lim - 1) if two else 0, p, q))
    return out


def test_signs_match_exact_arithmetic(driver):
    cases = _cases(1)
    got = _run(driver, cases)
    assert len(got) == len(cases)
    bad = [(c, g) for c, g in zip(cases, got) if g != _exact_sign(*c)]
    assert not bad, bad[:5]


def test_planted_error_is_caught(driver):
    """A wrong answer for one case must be visible to the comparison: flip the
    expected sign of a near-cancelling case."""
    cases = [c for c in _cases(2) if c[2] == 0][:50]
    got = _run(driver, cases)
    exact = [_exact_sign(*c) for c in cases]
    assert got == exact
    flipped = [-e for e in exact]
    assert got != flipped
