"""Oracle pins for the remaining vector operations of section 3: sub_plain,
power (minimum multiplicative depth) and polyval.  Each is checked against
plaintext arithmetic after decryption, against the depth its circuit must
consume, and (sub_plain) against an independent composition that the
correctly rounded encoder makes bit-identical."""
import math

import numpy as np
import pytest

from oracle import oracle as O

BITS = [60, 40, 40, 40, 40, 60]  # five data primes: four rescales


@pytest.fixture(scope="module")
def ctx():
    o = O.Oracle(12, BITS, 2.0 ** 40, 11)
    o.keygen()
    return o


def _enc(o, v, level):
    return o.encrypt(o.encode(v, o.scale, level), 3, True)


def _dec(o, ct, n):
    return o.decode(o.decrypt(ct), n)


@pytest.fixture(scope="module")
def x():
    return np.random.default_rng(5).uniform(-1, 1, 2048)


def test_sub_plain(ctx, x):
    o = ctx
    top = o.L - 1
    v = np.random.default_rng(6).uniform(-1, 1, 2048)
    cx = _enc(o, x, top)
    r = o.sub_plain(cx, o.encode(v, o.scale, top))
    assert np.abs(_dec(o, r, 2048) - (x - v)).max() < 1e-6
    # encoding is correctly rounded with ties away from zero, so encode(-v)
    # is exactly -encode(v) and the two compositions agree bit for bit
    alt = o.add_plain(cx, o.encode(-v, o.scale, top))
    assert np.array_equal(r.data(), alt.data())


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 7, 8, 11, 16])
def test_power_matches_plaintext_at_minimum_depth(ctx, x, k):
    o = ctx
    top = o.L - 1
    r = o.power(_enc(o, x, top), k)
    assert r.level == top - math.ceil(math.log2(k))
    assert np.abs(_dec(o, r, 2048) - x ** k).max() < 1e-5


def test_power_errors(ctx, x):
    o = ctx
    cx = _enc(o, x, o.L - 1)
    with pytest.raises(O.OracleError):
        o.power(cx, 0)
    with pytest.raises(O.OracleError):  # depth 5 > four levels
        o.power(cx, 17)


def test_polyval_paper_polynomial(ctx, x):
    # 2X^2 + X, the polynomial of the unary-operation table of the appendix
    o = ctx
    top = o.L - 1
    r = o.polyval(_enc(o, x, top), [0.0, 1.0, 2.0])
    assert r.level == top - 2
    assert abs(r.scale / o.scale - 1) < 2.0 ** -20
    assert np.abs(_dec(o, r, 2048) - (2 * x ** 2 + x)).max() < 1e-5


def test_polyval_degree_five(ctx, x):
    o = ctx
    top = o.L - 1
    c = [0.5, -1.0, 0.0, 0.25, 0.0, 0.1]
    r = o.polyval(_enc(o, x, top), c)
    assert r.level == top - 4  # ceil(log2 5) + 1
    want = np.polynomial.polynomial.polyval(x, c)
    assert np.abs(_dec(o, r, 2048) - want).max() < 1e-5


def test_polyval_errors(ctx, x):
    o = ctx
    cx = _enc(o, x, o.L - 1)
    with pytest.raises(O.OracleError):
        o.polyval(cx, [1.0])
    with pytest.raises(O.OracleError):
        o.polyval(cx, [1.0, 0.0, 0.0])
