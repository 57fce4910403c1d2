"""Pins of the oracle's primitives against things other than itself:
published test vectors (ChaCha20, RFC 8439), brute-force primality (sympy),
a 60-digit recomputation of the Gaussian CDT (mpmath), schoolbook negacyclic
products, closed forms for monomials, and sampler moments."""
import os

import mpmath as mp
import numpy as np
import pytest
from sympy import isprime

from oracle import oracle as O
from paper_2104_03152_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_chacha():
    rows = []
    with open(os.path.join(GOLDEN, "chacha20_rfc8439.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, ctr, nonce, out = line.split("|")
            rows.append((bytes.fromhex(key), int(ctr), bytes.fromhex(nonce), bytes.fromhex(out)))
    return rows


@pytest.mark.parametrize("row", _golden_chacha())
def test_chacha20_block_rfc8439(row):
    key, ctr, nonce, want = row
    kw = [int.from_bytes(key[4 * i:4 * i + 4], "little") for i in range(8)]
    nw = [int.from_bytes(nonce[4 * i:4 * i + 4], "little") for i in range(3)]
    out = O.chacha20_block(kw, ctr, nw)
    got = b"".join(int(w).to_bytes(4, "little") for w in out)
    assert got == want


def test_stream_words_layout():
    # stream word w is the little-endian u64 at byte 8*(w%8) of block w//8
    seed, tag, a, b = 0x0123456789ABCDEF, 7, 11, 13
    words = O.stream_words(seed, tag, a, b, 24)
    key = [seed & 0xFFFFFFFF, seed >> 32, 0, 0, 0, 0, 0, 0]
    for blk in range(3):
        out = O.chacha20_block(key, blk, [tag, a, b])
        raw = b"".join(int(w).to_bytes(4, "little") for w in out)
        for r in range(8):
            assert int(words[blk * 8 + r]) == int.from_bytes(raw[8 * r:8 * r + 8], "little")


CHAINS = [(I.SMALL["log_n"], I.SMALL["bits"]), (I.CNN["log_n"], I.CNN["bits"]),
          (I.RAW["log_n"], I.RAW["bits"]), (13, [21] * 6), (12, [50] * 9), (13, [50] * 9)]


@pytest.mark.parametrize("log_n,bits", CHAINS)
def test_prime_chain_brute_force(log_n, bits):
    primes = O.gen_primes(log_n, bits)
    m = 2 << log_n
    assert len(set(primes)) == len(primes)
    for i, (q, b) in enumerate(zip(primes, bits)):
        assert isprime(q) and O.is_prime(q)
        assert q % m == 1 and (1 << (b - 1)) < q < (1 << b)
        # every larger candidate below 2^b is composite or already taken
        c = q + m
        while c < (1 << b):
            assert (not isprime(c)) or c in primes[:i]
            c += m


def test_prime_values_small_chain():
    # the 3-prime N=4096 chain [40, 20 | 40]
    assert O.gen_primes(12, [40, 20, 40]) == [1099511480321, 1032193, 1099511390209]


def test_is_prime_matches_sympy():
    rng = np.random.default_rng(5)
    for x in list(rng.integers(1, 1 << 62, 3000, dtype=np.uint64)) + [2, 3, 4, 561, 2 ** 61 - 1]:
        assert O.is_prime(int(x)) == isprime(int(x))


def test_cdt_table_60_digits():
    mp.mp.dps = 60
    s = mp.mpf("3.2")
    rho = [mp.e ** (-(mp.mpf(x) ** 2) / (2 * s * s)) for x in range(-19, 20)]
    z = mp.fsum(rho)
    want = []
    for k in range(20):
        p = mp.fsum(rho[19 - k:19 + k + 1]) / z
        want.append(int(mp.floor(p * mp.mpf(2) ** 63)))
    assert O.cdt_table() == want


def test_sampler_moments():
    n = 1 << 16
    g = O.sample_gaussian(9, 3, 0, n)
    assert np.abs(g).max() <= 19
    var = g.astype(np.float64).var()
    # truncated variance 10.24; std error of the variance ~ sqrt(2/n)*10.24
    assert abs(var - 10.24) < 6 * np.sqrt(2.0 / n) * 10.24
    assert abs(g.mean()) < 6 * np.sqrt(10.24 / n)
    t = O.sample_ternary(9, 1, 0, n)
    counts = np.array([(t == v).sum() for v in (-1, 0, 1)])
    chi2 = ((counts - n / 3) ** 2 / (n / 3)).sum()
    assert chi2 < 20  # 2 dof, p ~ 5e-5
    q = 1099511480321
    u = O.sample_uniform(9, 2, 0, 0, q, n)
    assert int(u.max()) < q
    buckets = np.bincount((u.astype(np.float64) / q * 16).astype(int), minlength=16)
    chi2 = ((buckets - n / 16) ** 2 / (n / 16)).sum()
    assert chi2 < 50  # 15 dof


def _schoolbook(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += ai * int(b[j])
            else:
                c[k - n] -= ai * int(b[j])
    return np.array([x % q for x in c], dtype=np.uint64)


ALL_PRIMES = sorted({q for lg, b in CHAINS for q in O.gen_primes(lg, b)})


@pytest.mark.parametrize("q", ALL_PRIMES)
def test_negacyclic_vs_schoolbook_every_prime(q):
    rng = np.random.default_rng(q % 1000)
    for log_n in (2, 3, 5, 6):
        n = 1 << log_n
        a = rng.integers(0, q, n, dtype=np.uint64)
        b = rng.integers(0, q, n, dtype=np.uint64)
        assert np.array_equal(O.negacyclic_mul(a, b, log_n, q), _schoolbook(a, b, q))


def test_negacyclic_vs_schoolbook_n1024():
    q = 1152921504606830593
    rng = np.random.default_rng(1)
    a = rng.integers(0, q, 1024, dtype=np.uint64)
    b = rng.integers(0, 1 << 20, 1024, dtype=np.uint64)
    assert np.array_equal(O.negacyclic_mul(a, b, 10, q), _schoolbook(a, b, q))


@pytest.mark.parametrize("log_n,bits", CHAINS[:3])
def test_monomial_closed_form_full_size(log_n, bits):
    # a * X^k shifts coefficients up by k with sign flips on wrap-around;
    # X^k * X^(N-k) = X^N = -1.
    n = 1 << log_n
    rng = np.random.default_rng(log_n)
    for q in O.gen_primes(log_n, bits)[:3]:
        a = rng.integers(0, q, n, dtype=np.uint64)
        for k in (1, 7, n // 2 + 3, n - 1):
            xk = np.zeros(n, dtype=np.uint64)
            xk[k] = 1
            got = O.negacyclic_mul(a, xk, log_n, q)
            want = np.empty(n, dtype=object)
            for i in range(n):
                j = i + k
                if j < n:
                    want[j] = int(a[i])
                else:
                    want[j - n] = (q - int(a[i])) % q
            assert np.array_equal(got, want.astype(np.uint64))
            xnk = np.zeros(n, dtype=np.uint64)
            xnk[n - k] = 1
            m1 = O.negacyclic_mul(xk, xnk, log_n, q)
            assert int(m1[0]) == q - 1 and not m1[1:].any()


def _xpow(e, log_n, q):
    # X^e in Z_q[X]/(X^N+1) by square-and-multiply through the ring product
    n = 1 << log_n
    r = np.zeros(n, dtype=np.uint64)
    r[0] = 1
    x = np.zeros(n, dtype=np.uint64)
    x[1 % n] = 1 if n > 1 else 0
    while e:
        if e & 1:
            r = O.negacyclic_mul(r, x, log_n, q)
        x = O.negacyclic_mul(x, x, log_n, q)
        e >>= 1
    return r


def test_automorphism_ring_homomorphism():
    # tau_g is the ring map fixing Z_q and sending X to X^g: check tau_g(X^i)
    # = (X^g)^i for every i (so by linearity on every a), plus
    # multiplicativity on random products.
    q = 1099511480321
    log_n = 5
    n = 1 << log_n
    rng = np.random.default_rng(3)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    for g in (5, 25, 2 * n - 1, 3, 5 ** 7 % (2 * n)):
        want = np.zeros(n, dtype=object)
        for i in range(n):
            xi = np.zeros(n, dtype=np.uint64)
            xi[i] = 1
            img = _xpow(g * i, log_n, q)
            assert np.array_equal(O.automorphism(xi, log_n, g, q), img)
            want = want + img.astype(object) * int(a[i])
        want = np.array([int(v) % q for v in want], dtype=np.uint64)
        ta = O.automorphism(a, log_n, g, q)
        assert np.array_equal(ta, want)
        ab = O.negacyclic_mul(a, b, log_n, q)
        assert np.array_equal(O.automorphism(ab, log_n, g, q),
                              O.negacyclic_mul(ta, O.automorphism(b, log_n, g, q), log_n, q))
