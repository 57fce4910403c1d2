"""GPU parity of sub_plain, power and polyval (section 3) against the
oracle's circuits, bit for bit, and of the decrypted results against
plaintext arithmetic."""
import math

import numpy as np
import pytest

from tests.gpu_common import Pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def deep():
    return Pair(12, [60, 40, 40, 40, 40, 60], 2.0 ** 40, 11)


@pytest.fixture(scope="module")
def xs(deep):
    P = deep
    x = np.random.default_rng(5).uniform(-1, 1, 2048)
    top = P.o.L - 1
    g = P.H.he_encrypt(P.g, P.H.he_encode(P.g, x, P.scale, top), 3, True)
    o = P.o.encrypt(P.o.encode(x, P.scale, top), 3, True)
    P.ct_equal(g, o, "input")
    return x, g, o


def test_sub_plain_bit_exact(deep, xs):
    P = deep
    x, g, o = xs
    top = P.o.L - 1
    v = np.random.default_rng(6).uniform(-1, 1, 2048)
    P.ct_equal(P.H.he_sub_plain(P.g, g, P.H.he_encode(P.g, v, P.scale, top)),
               P.o.sub_plain(o, P.o.encode(v, P.scale, top)), "sub_plain")


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7, 8, 11, 16])
def test_power_bit_exact(deep, xs, k):
    P = deep
    x, g, o = xs
    say("power", k)
    r = P.H.he_power(P.g, g, k)
    P.ct_equal(r, P.o.power(o, k), "power %d" % k)
    assert r.info()[0] == P.o.L - 1 - math.ceil(math.log2(k))
    assert np.abs(P.H.he_decode(P.g, P.H.he_decrypt(P.g, r), 2048) - x ** k).max() < 1e-5


@pytest.mark.parametrize("coeffs", [[0.0, 1.0, 2.0], [0.5, -1.0, 0.0, 0.25, 0.0, 0.1], [0.0, 0.0, 0.0, 1.5]])
def test_polyval_bit_exact(deep, xs, coeffs):
    P = deep
    x, g, o = xs
    say("polyval", coeffs)
    r = P.H.he_polyval(P.g, g, coeffs)
    P.ct_equal(r, P.o.polyval(o, coeffs), "polyval")
    want = np.polynomial.polynomial.polyval(x, coeffs)
    assert np.abs(P.H.he_decode(P.g, P.H.he_decrypt(P.g, r), 2048) - want).max() < 1e-5


def test_power_polyval_errors(deep, xs):
    P = deep
    _, g, _ = xs
    for bad in (lambda: P.H.he_power(P.g, g, 0), lambda: P.H.he_power(P.g, g, 17),
                lambda: P.H.he_polyval(P.g, g, [1.0]), lambda: P.H.he_polyval(P.g, g, [1.0, 0.0])):
        with pytest.raises(P.H.HeError):
            bad()
