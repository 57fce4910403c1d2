"""Pins of the oracle's encoder and decoder (canonical embedding, section 3:
a CKKSVector holds N/2 real values).

The encoder's integer coefficients must be round(scale * m_k), ties away from
zero, where m is the unique real polynomial whose value at zeta^(5^j) is z_j
(zeta = exp(i pi / N)).  The pins solve that interpolation problem as a
linear system in 50-digit arithmetic (no cosine formula involved), check the
embedding at full size by evaluating the encoded polynomial, and check the
closed-form special cases (constant vectors, exact ties)."""
import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O


def _ctx(log_n, bits=(40, 40), scale=2.0 ** 30):
    return O.Oracle(log_n, list(bits), scale, 7)


def _round_half_away(x):
    f = mp.floor(abs(x) + mp.mpf("0.5"))
    return int(f) if x >= 0 else -int(f)


@pytest.mark.parametrize("log_n", [3, 4, 5])
def test_encode_solves_interpolation(log_n):
    mp.mp.dps = 50
    n = 1 << log_n
    o = _ctx(log_n)
    rng = np.random.default_rng(log_n)
    for trial in range(3):
        nz = n // 2 if trial else n // 2 - 1
        z = rng.uniform(-1, 1, nz)
        zf = list(z) + [0.0] * (n // 2 - nz)
        scale = 2.0 ** 30 * (1 + trial * 0.37)
        # unknown real coefficients m_0..m_{N-1}; equations Re/Im of
        # m(zeta^(5^j)) = z_j, j < N/2
        A = mp.matrix(n, n)
        rhs = mp.matrix(n, 1)
        for j in range(n // 2):
            e = pow(5, j, 2 * n)
            for k in range(n):
                ang = mp.pi * e * k / n
                A[2 * j, k] = mp.cos(ang)
                A[2 * j + 1, k] = mp.sin(ang)
            rhs[2 * j] = mp.mpf(zf[j])
            rhs[2 * j + 1] = 0
        m = mp.lu_solve(A, rhs)
        want = [_round_half_away(mp.mpf(scale) * m[k]) for k in range(n)]
        got = o.encode_coeffs(z, scale)
        assert [int(v) for v in got] == want


def test_encode_constant_vector_closed_form():
    # a constant vector c in all N/2 slots is the constant polynomial c
    for log_n in (6, 12, 13):
        o = _ctx(log_n)
        n = 1 << log_n
        for c in (0.75, -1.25, 0.1):
            got = o.encode_coeffs(np.full(n // 2, c), 2.0 ** 30)
            assert int(got[0]) == _round_half_away(mp.mpf(c) * 2 ** 30)
            assert not got[1:].any()


def test_encode_ties_away_from_zero():
    o = _ctx(6)
    n = 64
    for k in (0, 3, 1000):
        c = (k + 0.5) / 2 ** 20  # scale * c is exactly k + 1/2
        got = o.encode_coeffs(np.full(n // 2, c), 2.0 ** 20)
        assert int(got[0]) == k + 1
        got = o.encode_coeffs(np.full(n // 2, -c), 2.0 ** 20)
        assert int(got[0]) == -(k + 1)


def test_encode_range_error():
    o = _ctx(6)
    with pytest.raises(O.OracleError) as e:
        o.encode_coeffs(np.ones(33), 2.0 ** 20)  # more than N/2 slots
    assert e.value.code == O.ORC_ERANGE
    with pytest.raises(O.OracleError) as e:
        o.encode_coeffs(np.full(32, 2.0 ** 40), 2.0 ** 30)
    assert e.value.code == O.ORC_ERANGE


@pytest.mark.parametrize("log_n", [12, 13])
def test_encoded_polynomial_embeds_the_slots_full_size(log_n):
    # evaluate the integer polynomial at zeta^(5^j) in 30 digits: it must be
    # scale * z_j up to the rounding of the N coefficients (each <= 1/2)
    mp.mp.dps = 30
    n = 1 << log_n
    o = _ctx(log_n)
    rng = np.random.default_rng(11)
    z = rng.uniform(-1, 1, n // 2)
    scale = 2.0 ** 40
    c = o.encode_coeffs(z, scale)
    for j in (0, 1, 17, n // 2 - 1):
        e = pow(5, j, 2 * n)
        val = mp.fsum(int(c[k]) * mp.cos(mp.pi * e * k / n) for k in range(n) if c[k])
        im = mp.fsum(int(c[k]) * mp.sin(mp.pi * e * k / n) for k in range(n) if c[k])
        # the rounding errors r_k (|r_k| <= 1/2) enter as sum r_k cos(.),
        # a sum of N terms: allow 6 sigma of that random walk
        bound = 6 * 0.5 * np.sqrt(n / 3.0)
        assert abs(val - mp.mpf(scale) * mp.mpf(z[j])) < bound
        assert abs(im) < bound


def test_decode_inverts_encode():
    o = O.Oracle(13, [60, 60], 2.0 ** 40, 1)
    n = 8192
    rng = np.random.default_rng(2)
    z = rng.uniform(-3, 3, n // 2)
    pt = o.encode(z, 2.0 ** 40, 0)
    back = o.decode(pt, n // 2)
    assert np.abs(back - z).max() < 2.0 ** -30
    # fewer slots: the rest decode to ~0
    pt = o.encode(z[:100], 2.0 ** 40, 0)
    back = o.decode(pt, n // 2)
    assert np.abs(back[:100] - z[:100]).max() < 2.0 ** -30
    assert np.abs(back[100:]).max() < 2.0 ** -30
