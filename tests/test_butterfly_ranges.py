"""The exactness argument of the NTT butterflies, pinned on the CPU: the
library's own butterfly code (csrc/butterfly.h, compiled for the host)
against exact 128-bit integer arithmetic for every prime of every chain the
library runs, at the extremes of each input range (forward inputs in
(-2q-1, 4q+1), inverse inputs in (-q, 2q+1], multiplicands at +-4q with
twiddles 0, 1, q-1, the fold over |x| < 2^52) and at multiplicands whose
product with the twiddle lies next to a multiple of q, where the floating
quotient estimate is off by one.  Primes below 2^50 run the FP64 form and
the integer form, larger ones the integer form; the largest prime below
2^50 with q = 1 mod 2^15 is included."""
import os
import subprocess

import pytest
import sympy

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHAINS = [
    (12, [40, 20, 40]), (13, [60] + [40] * 6 + [60]), (14, [50] * 9), (12, [50] * 9), (13, [50] * 9),
    (13, [60, 40, 40, 60]), (12, [60, 40, 40, 40, 60]), (12, [60, 40, 40, 40, 40, 60]), (14, [60, 40, 40, 60]),
    (13, [60, 40, 60]), (14, [50, 50, 50]), (14, [60] + [40] * 11 + [60]), (12, [60, 40, 40, 60]),
]


def largest_prime_below_2_50():
    m = 1 << 15
    q = ((1 << 50) - 2) // m * m + 1
    while not sympy.isprime(q):
        q -= m
    return q


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("bf") / "butterfly_check")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-Xclang",
                           "-target-feature", "-Xclang", "-packed-fp32-ops",
                           os.path.join(ROOT, "tests", "butterfly_check.cpp"), "-o", out],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out


def test_butterflies_exact_at_range_extremes(checker):
    primes = set()
    for log_n, bits in CHAINS:
        primes.update(O.Oracle(log_n, bits, 2.0 ** 20, 1).primes)
    q50 = largest_prime_below_2_50()
    assert (1 << 50) - (1 << 22) < q50 < 1 << 50
    primes.add(q50)
    r = subprocess.run([checker] + [str(q) for q in sorted(primes)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "ALL OK" in r.stdout
    fp = [l for l in r.stdout.splitlines() if " fp+int ok" in l]
    assert len(fp) >= 20 and str(q50) + " fp+int ok" in r.stdout
    off = int([l for l in r.stdout.splitlines() if l.startswith("quotient estimates off by one")][0].split()[-1])
    assert off > 0  # the off-by-one quotient case was exercised
